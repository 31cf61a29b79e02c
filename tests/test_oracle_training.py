"""Pins of the oracle's training gradients (the learned part): the decoder-
parameter gradient of the Lipschitz loss (Sec. 4.1, Eq. form-L-LS-E) and the
encoder/decoder gradients of the supervised reconstruction loss (Sec. 3.2,
Eq. form-vanilla-supervised-construction), each against central differences
of the oracle's own loss.  The Lipschitz loss itself is computed from
forward-over-forward second derivatives of the decoder, a different algorithm
from the gradient's contracted jets, so the differences check the gradient
against the definition."""
import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I


def _problem(hidden=(8, 8), bias_scale=0.3, r=4):
    return I.make_problem("tl", 2, 1, 1, r, list(hidden), 8, bend=True, bias_scale=bias_scale)


def _flat(o):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(o.p.Ws, o.p.bs)])


def _set_flat(O, p, flat):
    o = O.Oracle(p)
    parts = o.unpack_params(flat)
    p2 = I.Problem(**{**p.__dict__})
    p2.Ws = [W.copy() for W, _ in parts]
    p2.bs = [b.copy() for _, b in parts]
    return O.Oracle(p2)


def _sample_indices(o, rng, per_block=3):
    """A few entries of every W and b block of the packed parameters."""
    idx, off = [], 0
    for (ws, bs) in o.param_shapes():
        nw, nb = ws[0] * ws[1], bs[0]
        idx += list(off + rng.choice(nw, size=min(per_block, nw), replace=False))
        idx += list(off + nw + rng.choice(nb, size=min(per_block, nb), replace=False))
        off += nw + nb
    return np.array(idx)


@pytest.mark.parametrize("hidden", [(8, 8), (6,), ()])
def test_lipschitz_param_grad_matches_central_differences(oracle_mod, hidden):
    O = oracle_mod
    p = _problem(hidden)
    o = O.Oracle(p)
    B = 3
    z1 = I.latent_batch(B, p.r, seed=41)
    z2 = I.latent_batch(B, p.r, seed=42)
    z2[1] = z1[1]   # an excluded pair
    loss, grad = o.lipschitz_param_grad(z1, z2)
    ref = o.lipschitz(z1, z2)
    assert loss == pytest.approx(ref["loss"], rel=1e-12)
    theta = _flat(o)
    rng = np.random.default_rng(5)
    idx = _sample_indices(o, rng)
    scale = np.abs(grad).max()
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (_set_flat(O, p, tp).lipschitz(z1, z2)["loss"] - _set_flat(O, p, tm).lipschitz(z1, z2)["loss"]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * scale + 1e-5 * abs(fd), (i, fd, grad[i])


def test_lipschitz_param_grad_zero_without_valid_pairs(oracle_mod):
    p = _problem()
    o = oracle_mod.Oracle(p)
    z = I.latent_batch(2, p.r)
    loss, grad = o.lipschitz_param_grad(z, z)
    assert loss == 0.0 and not grad.any()


def test_lipschitz_param_grad_is_a_mean_over_pairs(oracle_mod):
    """The loss and its gradient are means over the valid pairs (Eq. form-L-LS-E)."""
    p = _problem()
    o = oracle_mod.Oracle(p)
    z1 = I.latent_batch(4, p.r, seed=3)
    z2 = I.latent_batch(4, p.r, seed=4)
    la, ga = o.lipschitz_param_grad(z1[:2], z2[:2])
    lb, gb = o.lipschitz_param_grad(z1[2:], z2[2:])
    l, g = o.lipschitz_param_grad(z1, z2)
    assert l == pytest.approx(0.5 * (la + lb), rel=1e-12)
    assert np.allclose(g, 0.5 * (ga + gb), rtol=1e-10, atol=1e-12 * np.abs(g).max())
    # symmetric in the two points of a pair
    l2, g2 = o.lipschitz_param_grad(z2, z1)
    assert l2 == pytest.approx(l, rel=1e-12)
    assert np.allclose(g2, g, rtol=1e-10, atol=1e-12 * np.abs(g).max())


def _encoder(n, r, width, seed=7):
    Ws, bs = I.glorot_decoder(n, [width] if width else [], r, seed=seed, bias_scale=0.2)
    return Ws, bs


@pytest.mark.parametrize("enc_width", [6, 0])
def test_reconstruction_grad_matches_central_differences(oracle_mod, enc_width):
    O = oracle_mod
    p = _problem()
    o = O.Oracle(p)
    Ws, bs = _encoder(p.n, p.r, enc_width)
    enc = O.Mlp(Ws, bs)
    rng = np.random.default_rng(8)
    B = 3
    q = p.X[None] + 0.05 * rng.normal(size=(B,) + p.X.shape)
    q[:, p.pinned.astype(bool)] = p.X[p.pinned.astype(bool)]
    q = q.reshape(B, -1)
    loss, ge, gd = o.recon_loss_grad(enc, q)
    # the loss by its definition: mass-weighted squared distance of the reconstruction
    z = enc.encode(q - p.X.ravel())
    x, _ = o.decode(z, want_J=False)
    m = np.repeat(o.lumped_mass(), 3)
    want = np.mean([(m * (x[i].ravel() - q[i]) ** 2).sum() for i in range(B)])
    assert loss == pytest.approx(want, rel=1e-12)
    # decoder parameters
    theta = _flat(o)
    for i in _sample_indices(o, np.random.default_rng(9)):
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (_set_flat(O, p, tp).recon_loss_grad(enc, q)[0] - _set_flat(O, p, tm).recon_loss_grad(enc, q)[0]) / (2 * h)
        assert abs(fd - gd[i]) <= 1e-7 * np.abs(gd).max() + 1e-6 * abs(fd), (i, fd, gd[i])
    # encoder parameters
    phi = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])
    shapes = [(W.shape, b.shape) for W, b in zip(Ws, bs)]

    def enc_from(flat):
        out, off = ([], []), 0
        for ws, bsh in shapes:
            nw, nb = ws[0] * ws[1], bsh[0]
            out[0].append(flat[off:off + nw].reshape(ws))
            out[1].append(flat[off + nw:off + nw + nb])
            off += nw + nb
        return O.Mlp(*out)

    rng = np.random.default_rng(10)
    for i in rng.choice(phi.size, size=12, replace=False):
        h = 1e-6 * max(1.0, abs(phi[i]))
        tp, tm = phi.copy(), phi.copy()
        tp[i] += h
        tm[i] -= h
        fd = (o.recon_loss_grad(enc_from(tp), q)[0] - o.recon_loss_grad(enc_from(tm), q)[0]) / (2 * h)
        assert abs(fd - ge[i]) <= 1e-7 * np.abs(ge).max() + 1e-6 * abs(fd), (i, fd, ge[i])
