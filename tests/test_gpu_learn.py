"""GPU parity of the learned part's building blocks against the FP64 oracle:
the device-side decoder load and the decoder-parameter gradient of the
Lipschitz loss (Sec. 4.1, Eq. form-L-LS-E, on the cubature elastic Hessian of
Sec. 4.3).  The oracle's gradient is the chain rule written out and pinned by
central differences of its own forward-over-forward loss on the CPU."""
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


def t64(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def problem(name, **kw):
    if name == "tinyb":
        return I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3, **kw)
    if name == "lin":
        return I.make_problem("lin", 2, 1, 1, 4, [], 8, bend=True, bias_scale=0.3, **kw)
    if name == "c1b":
        return I.config("c1", bias_scale=0.1, **kw)
    return I.config(name, **kw)


def flat(p):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(p.Ws, p.bs)])


def with_flat(p, theta):
    parts, off, Ws, bs = [], 0, [], []
    for W, b in zip(p.Ws, p.bs):
        nw, nb = W.size, b.size
        Ws.append(theta[off:off + nw].reshape(W.shape).copy())
        bs.append(theta[off + nw:off + nw + nb].copy())
        off += nw + nb
    q = I.Problem(**{**p.__dict__})
    q.Ws, q.bs = Ws, bs
    return q


@pytest.mark.parametrize("name,prec", [("tinyb", rb.PREC_F64), ("tinyb", rb.PREC_F32), ("lin", rb.PREC_F64),
                                       ("c1b", rb.PREC_F64), ("c2", rb.PREC_F32), ("tinyb", rb.PREC_BF16)])
def test_device_decoder_load_matches_host_load(name, prec):
    """Weights loaded from a device buffer give the evaluation of a context created with them."""
    p = problem(name)
    rng = np.random.default_rng(11)
    theta = flat(p) * (1.0 + 0.1 * rng.standard_normal(flat(p).size))
    q = with_flat(p, theta)
    ref = rb.Context(q, prec=prec, max_batch=8)
    ctx = rb.Context(p, prec=prec, max_batch=8)
    for dt in (torch.float64, torch.float32):
        th = torch.tensor(theta, dtype=dt, device=DEV)
        if dt == torch.float32:
            ref.set_decoder(*[[a.astype(np.float32).astype(np.float64) for a in arr] for arr in (q.Ws, q.bs)])
        ctx.set_decoder_device(th)
        z = t64(I.latent_batch(5, p.r))
        tg, fo = I.loads_for(p, 5)
        tg, fo = (None if a is None else t64(a) for a in (tg, fo))
        a = ctx.energy_grad_hess(z, tg, fo, flags=rb.HESS_EXACT)
        b = ref.energy_grad_hess(z, tg, fo, flags=rb.HESS_EXACT)
        x1, J1 = ctx.decode(z)
        x2, J2 = ref.decode(z)
        torch.cuda.synchronize()
        # the same weights folded by a different summation order: equal to rounding
        tol = 1e-12 if prec == rb.PREC_F64 else 1e-5 if prec == rb.PREC_F32 else 1e-2
        for u, v in list(zip(a, b)) + [(x1, x2), (J1, J2)]:
            u, v = u.double().cpu().numpy(), v.double().cpu().numpy()
            assert np.linalg.norm(u - v) <= tol * np.linalg.norm(v) + 1e-300, (name, prec, dt)


def lip_bar_f32(o, z1, z2, tol):
    """Float32 bar of the Lipschitz gradient, derived from the Hessian's bar: the
    loss differences H(z1) - H(z2); a relative error tol of each Hessian (and of
    each of its parameter derivatives) is amplified by (|H1| + |H2|) / |H1 - H2|."""
    fl = O.EXACT | O.ELASTIC_ONLY
    H1 = o.reduced(z1, flags=fl)[2].reshape(len(z1), -1)
    H2 = o.reduced(z2, flags=fl)[2].reshape(len(z2), -1)
    valid = np.linalg.norm(z1 - z2, axis=1) > 0
    amp = (np.linalg.norm(H1, axis=1) + np.linalg.norm(H2, axis=1)) / np.maximum(np.linalg.norm(H1 - H2, axis=1), 1e-300)
    return tol * amp[valid].max()


@pytest.mark.parametrize("name,prec,B,mb", [("tinyb", rb.PREC_F64, 5, 4), ("tinyb", rb.PREC_F32, 5, 4),
                                            ("lin", rb.PREC_F64, 3, 8), ("c1b", rb.PREC_F64, 4, 8),
                                            ("c1b", rb.PREC_F32, 4, 8)])
def test_lipschitz_param_grad(name, prec, B, mb):
    p = problem(name)
    z1 = I.latent_batch(B, p.r, seed=21)
    z2 = I.latent_batch(B, p.r, seed=22)
    z2[1] = z1[1]   # excluded pair
    ctx = rb.Context(p, prec=prec, max_batch=mb)   # max_batch 4: two pairs per pass, three passes
    loss, grad = ctx.lipschitz_param_grad(t64(z1), t64(z2))
    lref = ctx.lipschitz_loss(t64(z1), t64(z2))["loss"]
    o = O.Oracle(p)
    oloss, ograd = o.lipschitz_param_grad(z1, z2)
    torch.cuda.synchronize()
    loss, grad, lref = loss.item(), grad.cpu().numpy(), lref.item()
    # the loss of the gradient pass is the loss of rs_lipschitz_loss, by the same kernels' Hessians
    assert loss == pytest.approx(lref, rel=1e-12)
    if prec == rb.PREC_F64:
        bar = 1e-10
    else:
        bar = lip_bar_f32(o, z1, z2, 1e-4)
        assert bar < 1e-2   # not vacuous for these pairs
    assert abs(loss - oloss) <= bar * abs(oloss)
    # per layer (W and b flattened)
    off = 0
    for W, b in zip(p.Ws, p.bs):
        for n in (W.size, b.size):
            g, go = grad[off:off + n], ograd[off:off + n]
            assert np.linalg.norm(g - go) <= bar * np.linalg.norm(ograd) + 1e-300, (name, prec, off)
            off += n
    assert np.linalg.norm(grad - ograd) <= bar * np.linalg.norm(ograd)


def test_lipschitz_param_grad_edges():
    p = problem("tinyb")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    z = t64(I.latent_batch(3, p.r))
    loss, grad = ctx.lipschitz_param_grad(z, z.clone())        # no valid pair
    assert loss.item() == 0.0 and not grad.any().item()
    e = torch.empty((0, p.r), dtype=torch.float64, device=DEV)
    loss, grad = ctx.lipschitz_param_grad(e, e)                # B = 0
    assert loss.item() == 0.0 and not grad.any().item()
    with pytest.raises(RuntimeError):
        rb.Context(p, prec=rb.PREC_BF16, max_batch=4).lipschitz_param_grad(z, z)


def test_lipschitz_param_grad_c4_sampled():
    """The learned part's own workload (16^3 block, r = 12, 4 x 256, 512 cubature
    tets), float32, 64 pairs in one pass: the gradient against the oracle's on the
    first four pairs, by linearity of the mean (the pass's gradient over four pairs
    is what the oracle computes over them)."""
    p = I.config("c4", bias_scale=0.05)
    P = 4
    z1 = I.latent_batch(P, p.r, seed=31)
    z2 = I.latent_batch(P, p.r, seed=32)
    ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=128)
    loss, grad = ctx.lipschitz_param_grad(t64(z1), t64(z2))
    o = O.Oracle(p)
    oloss, ograd = o.lipschitz_param_grad(z1, z2)
    torch.cuda.synchronize()
    bar = lip_bar_f32(o, z1, z2, 1e-4)
    assert bar < 1e-2
    assert abs(loss.item() - oloss) <= bar * abs(oloss)
    assert np.linalg.norm(grad.cpu().numpy() - ograd) <= bar * np.linalg.norm(ograd)


def test_dynamics_subspace_training_small():
    """The dynamics workload's subspace construction end to end on a small beam:
    full-space equilibria of end-face poses, reconstruction training, and a
    context built from the trained decoder evaluates the rest shape's
    coordinates to a finite energy and a small displacement."""
    from paper_2409_03807_amd import learn

    p = I.make_problem("small", 6, 2, 2, 4, [32, 32], 48, wlo=1.0, whi=3.0, twist=False)
    p.dt = 1.0 / 60.0
    out = learn.train_dynamics_subspace(p, n_snap=32, epochs=60, batch=16, bend_deg=20.0, twist_deg=20.0,
                                        log=lambda *a, **k: None)
    assert out["snapshot_solve"]["converged"] == 32 and out["train_snapshots"] == 32
    assert [W.shape for W in out["Ws"]] == [W.shape for W in p.Ws]
    assert np.isfinite(out["loss"])
    q = I.Problem(**{**p.__dict__})
    q.Ws, q.bs = out["Ws"], out["bs"]
    ctx = rb.Context(q, prec=rb.PREC_F64, max_batch=4)
    z = out["z_rest"].reshape(1, -1).contiguous()
    E, g, H = ctx.energy_grad_hess(z)
    x, _ = ctx.decode(z, want_J=False)
    assert torch.isfinite(E).all() and torch.isfinite(g).all() and torch.isfinite(H).all()
    # the rest shape's coordinates decode to a displacement of the snapshots' size, not a blow-up
    assert np.abs(x.double().cpu().numpy() - q.X).max() < 0.5
