"""GPU parity of the supervised trainer (rs_trainer_*) against the FP64 oracle:
the reconstruction loss of Sec. 3.2 (Eq. form-vanilla-supervised-construction)
with its encoder and decoder gradients, the Lipschitz term of Sec. 4.2 (Eq.
form-unconstrained-lipschitz-optimization) over pairs of the batch's encodings,
the encodings themselves, and the Adam update."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2409_03807_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_03807_amd import binding as rb  # noqa: E402

DEV = "cuda:0"


def problem(name):
    if name == "tinyb":
        return I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3)
    if name == "c1b":
        return I.config("c1", bias_scale=0.1)
    return I.config(name, bias_scale=0.05)


def encoder(p, hidden, seed=7):
    return I.glorot_decoder(p.n, hidden, p.r, seed=seed, bias_scale=0.1)


def snapshots(p, N, scale=0.05, seed=8):
    """Synthetic displacement snapshots (N x 3 nv), zero on pinned vertices."""
    d = scale * np.random.default_rng(seed).normal(size=(N, p.nv, 3))
    d[:, p.pinned.astype(bool)] = 0.0
    return d.reshape(N, -1)


def setup(name, prec, enc_hidden, N=10, max_batch=8):
    p = problem(name)
    eW, eb = encoder(p, enc_hidden)
    ctx = rb.Context(p, prec=prec, max_batch=16)
    tr = rb.Trainer(ctx, eW, eb, p.Ws, p.bs, max_batch=max_batch)
    d = snapshots(p, N)
    store = torch.tensor(d, dtype=ctx.tdtype, device=DEV)
    if prec == rb.PREC_F32:
        d = d.astype(np.float32).astype(np.float64)   # the oracle sees the values the GPU stores
    return p, ctx, tr, d, store, O.Mlp(eW, eb)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


CASES = [("tinyb", rb.PREC_F64, [6], 1e-10), ("tinyb", rb.PREC_F64, [], 1e-10),
         ("tinyb", rb.PREC_F32, [6, 6], 1e-4), ("c1b", rb.PREC_F64, [32, 32], 1e-10)]


@pytest.mark.parametrize("name,prec,enc_hidden,tol", CASES)
def test_reconstruction_grad_matches_oracle(name, prec, enc_hidden, tol):
    p, ctx, tr, d, store, enc = setup(name, prec, enc_hidden)
    idx = np.array([7, 2, 9, 0, 4, 5], dtype=np.int32)
    losses, ge, gd = tr.grad(store, torch.tensor(idx, device=DEV), want_grads=True)
    lo, geo, gdo = O.Oracle(p).recon_loss_grad(enc, p.X.ravel()[None] + d[idx])
    torch.cuda.synchronize()
    losses = losses.cpu().numpy()
    assert abs(losses[0] - lo) <= tol * lo and losses[1] == 0.0
    assert rel(ge.cpu().numpy(), geo) <= tol
    assert rel(gd.cpu().numpy(), gdo) <= tol
    # rows 0..B-1 of the store without an index list
    losses, ge, gd = tr.grad(store, None, B=5, want_grads=True)
    lo, geo, gdo = O.Oracle(p).recon_loss_grad(enc, p.X.ravel()[None] + d[:5])
    torch.cuda.synchronize()
    assert abs(losses[0].item() - lo) <= tol * lo
    assert rel(ge.cpu().numpy(), geo) <= tol and rel(gd.cpu().numpy(), gdo) <= tol


@pytest.mark.parametrize("name,prec,enc_hidden,tol", CASES[:1] + CASES[2:])
def test_lipschitz_term_on_encoded_pairs(name, prec, enc_hidden, tol):
    p, ctx, tr, d, store, enc = setup(name, prec, enc_hidden)
    idx = np.array([1, 3, 8, 6, 2, 0, 5], dtype=np.int32)
    lam = 0.37
    losses, ge, gd = tr.grad(store, torch.tensor(idx, device=DEV), lambda_ls=lam, n_pairs=3, want_grads=True)
    o = O.Oracle(p)
    lo, geo, gdo = o.recon_loss_grad(enc, p.X.ravel()[None] + d[idx])
    z = enc.encode(d[idx])
    z1, z2 = z[0:6:2], z[1:6:2]
    llo, glo = o.lipschitz_param_grad(z1, z2)
    torch.cuda.synchronize()
    losses = losses.cpu().numpy()
    gd = gd.cpu().numpy()
    if prec == rb.PREC_F64:
        assert abs(losses[1] - llo) <= tol * llo
        assert rel(gd, gdo + lam * glo) <= tol
    else:
        # the float32 Lipschitz bar: the Hessian's 1e-4 amplified by the pairs' cancellation
        fl = O.EXACT | O.ELASTIC_ONLY
        H1 = o.reduced(z1, flags=fl)[2].reshape(3, -1)
        H2 = o.reduced(z2, flags=fl)[2].reshape(3, -1)
        amp = ((np.linalg.norm(H1, axis=1) + np.linalg.norm(H2, axis=1)) / np.linalg.norm(H1 - H2, axis=1)).max()
        bar = tol * amp
        assert abs(losses[1] - llo) <= bar * llo
        assert np.linalg.norm(gd - gdo - lam * glo) <= tol * np.linalg.norm(gdo) + bar * lam * np.linalg.norm(glo)
    # the encoder gradient carries no Lipschitz term (the pairs are held fixed)
    assert rel(ge.cpu().numpy(), geo) <= tol


@pytest.mark.parametrize("name,prec,enc_hidden,tol", CASES)
def test_encode_matches_oracle(name, prec, enc_hidden, tol):
    p, ctx, tr, d, store, enc = setup(name, prec, enc_hidden, N=20, max_batch=4)
    z = tr.encode(store)                                   # 20 rows in chunks of 4
    idx = np.array([19, 3, 3, 11], dtype=np.int32)
    zi = tr.encode(store, torch.tensor(idx, device=DEV))
    zo = enc.encode(d)
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), zo) <= tol
    assert rel(zi.cpu().numpy(), zo[idx]) <= tol


def test_adam_step_and_decoder_reload():
    p, ctx, tr, d, store, enc = setup("tinyb", rb.PREC_F64, [6])
    e0, d0 = (a.cpu().numpy() for a in tr.params())
    lam = 0.5
    _, ge, gd = tr.grad(store, None, B=6, lambda_ls=lam, n_pairs=3, want_grads=True)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    tr.adam(lr, b1, b2, eps)
    e1, d1 = (a.cpu().numpy() for a in tr.params())
    for p0, g, p1 in ((e0, ge.cpu().numpy(), e1), (d0, gd.cpu().numpy(), d1)):
        m = (1 - b1) * g
        v = (1 - b2) * g * g
        want = p0 - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps)
        assert np.allclose(p1, want, rtol=1e-12, atol=1e-15)
    # the context now evaluates the updated decoder
    parts = ctx.unpack_params(torch.tensor(d1))
    q = I.Problem(**{**p.__dict__})
    q.Ws = [W.numpy() for W, _ in parts]
    q.bs = [b.numpy() for _, b in parts]
    zt = torch.tensor(I.latent_batch(3, p.r), device=DEV)
    a = ctx.energy_grad_hess(zt)
    b = rb.Context(q, prec=rb.PREC_F64, max_batch=4).energy_grad_hess(zt)
    torch.cuda.synchronize()
    for u, w in zip(a, b):
        assert rel(u.cpu().numpy(), w.cpu().numpy()) <= 1e-12


def test_training_reduces_the_reconstruction_loss():
    p, ctx, tr, d, store, enc = setup("tinyb", rb.PREC_F32, [6], N=16, max_batch=16)
    l0 = tr.grad(store)[0][0].item()
    for _ in range(200):
        tr.grad(store)
        tr.adam(1e-2)
    l1 = tr.grad(store)[0][0].item()
    assert np.isfinite(l1) and l1 < 0.5 * l0, (l0, l1)


def test_trainer_argument_errors():
    p, ctx, tr, d, store, enc = setup("tinyb", rb.PREC_F64, [6])
    with pytest.raises(RuntimeError):
        tr.grad(store, None, B=9)                       # beyond max_batch
    with pytest.raises(RuntimeError):
        tr.grad(store, None, B=4, lambda_ls=1.0, n_pairs=3)   # 2 n_pairs > B
    with pytest.raises(RuntimeError):
        rb.Trainer(rb.Context(p, prec=rb.PREC_BF16, max_batch=4), *encoder(p, [6]), p.Ws, p.bs)


def test_c4_block_float32_sampled():
    """The learned part's workload: 16^3 block (n = 14739), r = 12, decoder 4 x 256,
    encoder 14739 -> 256 -> 256 -> 12, float32, eight snapshots (the long
    reductions over n take the split-K path)."""
    p, ctx, tr, d, store, enc = setup("c4", rb.PREC_F32, [256, 256], N=8, max_batch=8)
    losses, ge, gd = tr.grad(store, None, B=8, want_grads=True)
    lo, geo, gdo = O.Oracle(p).recon_loss_grad(enc, p.X.ravel()[None] + d)
    torch.cuda.synchronize()
    assert abs(losses[0].item() - lo) <= 1e-4 * lo
    assert rel(ge.cpu().numpy(), geo) <= 1e-4
    assert rel(gd.cpu().numpy(), gdo) <= 1e-4
