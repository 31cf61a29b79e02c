"""GPU parity: every ABI entry point against the FP64 CPU oracle on the same
seeded inputs.

Tolerances (per item, |a - b|_2 / max(|b|_2, tau)): 1e-10 for float64
contexts, 1e-4 for float32 contexts (element physics and decoder in float32,
float64 accumulation).  Newton solves are compared by exit status, iteration
count and energy, and by stationarity of the GPU solution under the oracle's
own gradient (several local minima can be correct).
"""
import math

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
# BF16 contexts carry every decoder operand as three BF16 parts (float32 accuracy)
TOL = {rb.PREC_F64: 1e-10, rb.PREC_F32: 1e-4, rb.PREC_BF16: 1e-4}


def energy_scale(p):
    """mu * total volume: the scale of energies that cancel to ~0 (rest, balanced loads)."""
    mu = p.young / (2 * (1 + p.poisson))
    return mu * p.meta["h"] ** 3 * p.ne / 5


def relerr(a, b, tau=0.0):
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    den = np.maximum(np.linalg.norm(b, axis=1), tau)
    return np.linalg.norm(a - b, axis=1) / den


def t64(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def problem(name, **kw):
    if name == "tinyb":
        return I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3, **kw)
    if name == "tiny":
        return I.config("tiny", bias_scale=0.3, **kw)
    return I.config(name, **kw)


CASES = [("tinyb", rb.PREC_F64), ("tinyb", rb.PREC_F32), ("c1", rb.PREC_F64), ("c2", rb.PREC_F32),
         ("c2", rb.PREC_F64)]


# ------------------------------------------------------------------- decode
@pytest.mark.parametrize("name,prec", CASES)
def test_decode(name, prec):
    p = problem(name)
    B = 5
    ctx = rb.Context(p, prec=prec, max_batch=8)
    z = I.latent_batch(B, p.r)
    x, J = ctx.decode(t64(z))
    xo, Jo = O.Oracle(p).decode(z)
    tol = TOL[prec]
    assert relerr(x.cpu().numpy() - p.X, xo - p.X, tau=1e-3).max() < tol
    assert relerr(J.cpu().numpy(), Jo).max() < tol
    xv, Jn = ctx.decode(t64(z), want_J=False)
    assert Jn is None and relerr(xv.cpu().numpy() - p.X, xo - p.X, tau=1e-3).max() < tol


# ------------------------------------------------------------------- E, g, H
@pytest.mark.parametrize("name,prec", CASES)
@pytest.mark.parametrize("flags", [rb.HESS_EXACT, 0, rb.HESS_EXACT | rb.ELASTIC_ONLY])
def test_energy_grad_hess(name, prec, flags):
    p = problem(name)
    B = 5
    ctx = rb.Context(p, prec=prec, max_batch=8)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=flags)
    oflags = (O.EXACT if flags & rb.HESS_EXACT else 0) | (O.ELASTIC_ONLY if flags & rb.ELASTIC_ONLY else 0)
    Eo, go, Ho = O.Oracle(p).reduced(z, tg, fo, flags=oflags)
    tol = TOL[prec]
    # the energy is always evaluated in float64
    assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), go).max() < tol
    assert relerr(H.cpu().numpy(), Ho).max() < tol


@pytest.mark.parametrize("name,prec", [("tinyb", rb.PREC_F64), ("c2", rb.PREC_F32)])
def test_energy_only_and_chunking(name, prec):
    """B above max_batch is processed in chunks; ragged last chunk."""
    p = problem(name)
    B = 11
    ctx = rb.Context(p, prec=prec, max_batch=4)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=rb.HESS_EXACT)
    E2, g2, H2 = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=rb.ENERGY_ONLY)
    assert g2 is None and H2 is None
    Eo, go, Ho = O.Oracle(p).reduced(z, tg, fo)
    assert relerr(E2.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), go).max() < TOL[prec]
    assert relerr(H.cpu().numpy(), Ho).max() < TOL[prec]


@pytest.mark.parametrize("n_cub", [16, 45, 100])
@pytest.mark.parametrize("flags", [rb.HESS_EXACT, 0])
def test_element_two_column_path_ragged_rounds(n_cub, flags):
    """r = 16 in float32 with J_R through device memory (the two-kernel path,
    which ground contact, inertia and the element options use): the element
    kernel runs 8 lanes per tet with two columns each, 32 tets a round;
    cubature sets that end inside a round, and small batches whose items are
    split over several workgroups."""
    p = I.make_problem(f"two{n_cub}", 6, 2, 2, 16, [32, 32], n_cub, bend=True, bias_scale=0.3)
    o = O.Oracle(p)
    for B in (3, 40):
        ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=B)
        assert ctx.set_fused(False)
        z = I.latent_batch(B, p.r)
        tg, fo = I.loads_for(p, B)
        E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=flags)
        Eo, go, Ho = o.reduced(z, tg, fo, flags=O.EXACT if flags & rb.HESS_EXACT else 0)
        assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
        assert relerr(g.cpu().numpy(), go).max() < TOL[rb.PREC_F32]
        assert relerr(H.cpu().numpy(), Ho).max() < TOL[rb.PREC_F32]


def test_empty_batch_is_a_no_op():
    p = problem("tiny")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    z = torch.zeros((0, p.r), dtype=torch.float64, device=DEV)
    E, g, H = ctx.energy_grad_hess(z)
    assert E.numel() == 0
    res = ctx.newton_solve(z)
    assert res["z"].numel() == 0
    lip = ctx.lipschitz_loss(z, z)
    torch.cuda.synchronize()
    assert lip["n_valid"].item() == 0 and lip["loss"].item() == 0.0


def test_argument_errors():
    p = problem("tiny")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    z = torch.zeros((5, p.r), dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError, match="max_batch"):
        ctx.newton_solve(z)
    with pytest.raises(TypeError):
        ctx.energy_grad_hess(z.float())
    # a BF16 context needs hidden layers for its BF16 products
    q = I.make_problem("lin", 2, 1, 1, 4, [], 8)
    with pytest.raises(RuntimeError):
        rb.Context(q, prec=rb.PREC_BF16, max_batch=4)


# ------------------------------------------------------------------- Newton
def _compare_newton(p, prec, z0, tg=None, fo=None, opts_kw=None, exact_iters=True):
    opts_kw = opts_kw or {}
    ctx = rb.Context(p, prec=prec, max_batch=max(len(z0), 2))
    res = ctx.newton_solve(t64(z0), t64(tg), t64(fo), opts=rb.default_opts(**opts_kw))
    o = O.Oracle(p)
    ores = o.newton(z0, tg, fo, opts=O.default_opts(**opts_kw))
    r = {k: v.cpu().numpy() for k, v in res.items()}
    return r, ores, o


@pytest.mark.parametrize("name", ["c1", "tinyb"])
def test_newton_float64_matches_oracle_iterates(name):
    p = problem(name)
    B = 6
    z0 = np.vstack([np.zeros((2, p.r)), I.latent_batch(B - 2, p.r)])
    tg, fo = I.loads_for(p, B)
    r, ores, o = _compare_newton(p, rb.PREC_F64, z0, tg, fo)
    assert np.array_equal(r["status"], ores["status"])
    assert np.array_equal(r["iters"], ores["iters"])
    assert relerr(r["E"][:, None], ores["E"][:, None], tau=1e-6 * energy_scale(p)).max() < 1e-9
    assert np.abs(r["z"] - ores["z"]).max() < 1e-6
    conv = r["status"] == rb.CONVERGED
    assert np.all(r["relgrad"][conv] <= 1e-6)


def test_newton_float32_c2_stationary_for_oracle():
    p = problem("c2")
    B = 10
    z0 = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    r, ores, o = _compare_newton(p, rb.PREC_F32, z0, tg, fo)
    assert np.all(np.isin(r["status"], [rb.CONVERGED, rb.LS_MAX, rb.ITER_MAX]))
    assert (r["status"] == rb.CONVERGED).mean() >= 0.8
    # the GPU solution is stationary for the oracle's float64 gradient
    g0 = np.abs(o.reduced(z0, tg, fo)[1]).max(axis=1)
    Eg, gg, _ = o.reduced(r["z"], tg, fo)
    conv = r["status"] == rb.CONVERGED
    # 1e-6 on the float32 gradient plus its measured noise floor (5e-7 of |g_0|)
    assert np.all(np.abs(gg[conv]).max(axis=1) <= 1.5e-6 * g0[conv])
    # its reported energy is the float64 energy of that point
    assert relerr(r["E"][:, None], Eg[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    # and it is no worse than the oracle's own solve from the same start, up to local minima
    same = np.abs(r["E"] - ores["E"]) <= 1e-6 * np.abs(ores["E"]) + 1e-9
    assert same.mean() >= 0.8
    assert np.abs(r["iters"][same] - ores["iters"][same]).max() <= 2


def test_newton_forced_statuses():
    p = problem("tinyb")
    z0 = I.latent_batch(1, p.r)
    tg, fo = I.loads_for(p, 1, twist_deg=[120.0])
    r, ores, _ = _compare_newton(p, rb.PREC_F64, z0, tg, fo, dict(max_iter=0))
    assert r["status"][0] == rb.ITER_MAX == ores["status"][0] and r["iters"][0] == 0
    r, ores, _ = _compare_newton(p, rb.PREC_F64, z0, tg, fo, dict(ls_max=0))
    assert r["status"][0] == rb.LS_MAX == ores["status"][0]
    zn = z0.copy(); zn[0, 1] = np.nan
    r, ores, _ = _compare_newton(p, rb.PREC_F64, zn, tg, fo)
    assert r["status"][0] == rb.NONFINITE == ores["status"][0]
    # an indefinite start without projection ends as the saddle exit
    o = O.Oracle(p)
    rng = np.random.default_rng(11)
    for _ in range(200):
        z = rng.normal(scale=1.5, size=(1, p.r))
        Hh = o.reduced(z, tg, fo)[2][0]
        if np.linalg.eigvalsh(0.5 * (Hh + Hh.T)).min() < 0:
            break
    r, ores, _ = _compare_newton(p, rb.PREC_F64, z, tg, fo, dict(proj=rb.PROJ_NONE))
    assert r["status"][0] == rb.NOT_DESCENT == ores["status"][0]
    # with the projection both converge identically
    r, ores, _ = _compare_newton(p, rb.PREC_F64, z, tg, fo)
    assert r["status"][0] == ores["status"][0] and r["iters"][0] == ores["iters"][0]


def test_newton_gauss_newton_and_abs_projection():
    p = problem("c1", bias_scale=0.1)
    z0 = I.latent_batch(4, p.r)
    for kw in (dict(hess=0), dict(proj=rb.PROJ_ABS)):
        r, ores, _ = _compare_newton(p, rb.PREC_F64, z0, None, None, kw)
        assert np.array_equal(r["status"], ores["status"])
        assert np.array_equal(r["iters"], ores["iters"])
        assert relerr(r["E"][:, None], ores["E"][:, None], tau=1e-6 * energy_scale(p)).max() < 1e-9


@pytest.mark.parametrize("r", [5, 7, 16, 20])
def test_newton_projection_across_latent_sizes(r):
    """Indefinite starts force the eigen-projection: odd r (the round-robin gets
    a dummy index), the register-resident Jacobi (r <= 16) and the LDS one (r > 16)."""
    # hidden layers wider than r and 36 free DOFs keep the reduced Hessian well posed
    p = I.make_problem(f"proj{r}", 3, 1, 1, r, [32, 32], 16, bend=True, bias_scale=0.3)
    o = O.Oracle(p)
    rng = np.random.default_rng(17 + r)
    Z = rng.normal(scale=1.5, size=(64, r))
    tg, fo = I.loads_for(p, 64)
    H = o.reduced(Z, tg, fo)[2]
    indef = [b for b in range(64) if np.linalg.eigvalsh(0.5 * (H[b] + H[b].T)).min() < 0][:4]
    assert len(indef) >= 2
    sel = np.array(indef)
    z0 = Z[sel]
    tgs = None if tg is None else tg[sel]
    fos = None if fo is None else fo[sel]
    # the projected Newton steps themselves (the eigen-decompositions differ
    # only by rounding, so the first iterates agree to rounding)
    for k in (1, 3):
        r_, ores, _ = _compare_newton(p, rb.PREC_F64, z0, tgs, fos, dict(max_iter=k))
        assert np.array_equal(r_["status"], ores["status"])
        assert np.array_equal(r_["iters"], ores["iters"])
        assert relerr(r_["z"], ores["z"]).max() < 1e-9
    # whole solves: a trajectory that wanders through indefinite regions for
    # tens of steps amplifies rounding, so compare the end points by stationarity
    r_, ores, o = _compare_newton(p, rb.PREC_F64, z0, tgs, fos, dict(max_iter=200))
    assert np.all(r_["status"] == rb.CONVERGED)
    g0 = np.abs(o.reduced(z0, tgs, fos)[1]).max(axis=1)
    gg = o.reduced(r_["z"], tgs, fos)[1]
    assert np.all(np.abs(gg).max(axis=1) <= 2e-6 * g0)


def test_identity_decoder_linear_path():
    """No hidden layer (a linear decoder selecting every free DOF, r = 24)."""
    p = I.make_problem("ident", 2, 1, 1, 1, [], 10 ** 9)
    free = np.nonzero(np.repeat(p.pinned == 0, 3))[0]
    p.Ws, p.bs = I.identity_decoder(free, p.n)
    p.r = len(free)
    rng = np.random.default_rng(3)
    z = 0.01 * rng.normal(size=(3, p.r))
    tg, fo = I.loads_for(p, 3, twist_deg=[40.0, 10.0, 0.0])
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg))
    Eo, go, Ho = O.Oracle(p).reduced(z, tg)
    assert relerr(g.cpu().numpy(), go).max() < 1e-10
    assert relerr(H.cpu().numpy(), Ho).max() < 1e-10
    r, ores, _ = _compare_newton(p, rb.PREC_F64, z, tg, None, dict(rel_tol=1e-9, max_iter=60))
    assert np.array_equal(r["status"], ores["status"]) and np.array_equal(r["iters"], ores["iters"])


# ------------------------------------------------------------------- Lipschitz
@pytest.mark.parametrize("name,prec", CASES)
def test_lipschitz(name, prec):
    p = problem(name)
    B = 5
    z1 = I.latent_batch(B, p.r, seed=5)
    z2 = I.latent_batch(B, p.r, seed=6)
    z2[3] = z1[3]
    ctx = rb.Context(p, prec=prec, max_batch=4)  # 2 pairs per pass: 3 chunks
    res = ctx.lipschitz_loss(t64(z1), t64(z2))
    o = O.Oracle(p)
    ores = o.lipschitz(z1, z2)
    tol = TOL[prec]
    assert res["n_valid"].item() == ores["n_valid"] == B - 1
    per = res["per_pair"].cpu().numpy()
    assert per[3] == 0.0
    # Bars derived from the Hessian's: with |H_gpu(z) - H(z)|_F <= tol |H(z)|_F at
    # both points of a pair, e_H = tol (|H1|_F + |H2|_F) bounds the error of
    # D = H1 - H2, and | |a|^2 - |b|^2 | <= |a - b| (2 |b| + |a - b|) gives
    # |l_gpu - l| <= (2 e_H |D|_F + e_H^2) / |dz|^2 per pair; the mean takes the
    # mean bound and sqrt(l) (the max-pair estimator) moves by at most e_H / |dz|.
    fl = O.EXACT | O.ELASTIC_ONLY
    H1 = o.reduced(z1, flags=fl)[2].reshape(B, -1)
    H2 = o.reduced(z2, flags=fl)[2].reshape(B, -1)
    n1, n2, nd = (np.linalg.norm(a, axis=1) for a in (H1, H2, H1 - H2))
    dz = np.linalg.norm(z1 - z2, axis=1)
    valid = dz > 0
    eH = tol * (n1 + n2)
    bound = np.zeros(B)
    bound[valid] = (2 * eH[valid] * nd[valid] + eH[valid] ** 2) / dz[valid] ** 2
    assert np.all(np.abs(per - ores["per_pair"]) <= bound)
    assert abs(res["loss"].item() - ores["loss"]) <= bound[valid].mean()
    assert abs(res["lip_max"].item() - ores["lip_max"]) <= (eH[valid] / dz[valid]).max()
    # for pairs this far apart the bars are a few tol relative, not vacuous
    assert np.all(bound[valid] <= 50 * tol * ores["per_pair"][valid])


# ------------------------------------------------------------------- BF16 decoder
@pytest.mark.parametrize("name", ["tinyb", "c1", "c2"])
def test_bf16_decode(name):
    """BF16 decoder products (float32 accumulation) against the float64 oracle at the BF16 bar."""
    p = problem(name)
    B = 5
    ctx = rb.Context(p, prec=rb.PREC_BF16, max_batch=8)
    z = I.latent_batch(B, p.r)
    x, J = ctx.decode(t64(z))
    assert x.dtype == torch.float32 and J.dtype == torch.float32
    xo, Jo = O.Oracle(p).decode(z)
    tol = TOL[rb.PREC_BF16]
    assert relerr(x.cpu().numpy() - p.X, xo - p.X, tau=1e-3).max() < tol
    assert relerr(J.cpu().numpy(), Jo).max() < tol


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("flags", [rb.HESS_EXACT, rb.HESS_EXACT | rb.ELASTIC_ONLY])
def test_bf16_energy_grad_hess(name, flags):
    p = problem(name)
    B = 5
    ctx = rb.Context(p, prec=rb.PREC_BF16, max_batch=8)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=flags)
    oflags = O.EXACT | (O.ELASTIC_ONLY if flags & rb.ELASTIC_ONLY else 0)
    Eo, go, Ho = O.Oracle(p).reduced(z, tg, fo, flags=oflags)
    tol = TOL[rb.PREC_BF16]
    # the energy is evaluated with the float64 decoder
    assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), go).max() < tol
    assert relerr(H.cpu().numpy(), Ho).max() < tol


def test_bf16_full_size_sampled():
    """c3: BF16 decoder at B = 4096 in the launch configuration of the benchmark, sampled items."""
    p = problem("c3")
    B = 4096
    ctx = rb.Context(p, prec=rb.PREC_BF16, max_batch=B)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo))
    idx = np.array([0, 1, 17, B // 2 + 3, B - 1])
    Eo, go, Ho = O.Oracle(p).reduced(z[idx], tg[idx], None)
    tol = TOL[rb.PREC_BF16]
    assert relerr(g.cpu().numpy()[idx], go).max() < tol
    assert relerr(H.cpu().numpy()[idx], Ho).max() < tol
    assert relerr(E.cpu().numpy()[idx, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert torch.isfinite(H).all()


def test_bf16_newton_c2_stationary_for_oracle():
    """BF16 search directions (three-part operands) and the float64 line-search
    energies belong to one function: solves converge at 1e-6 on the BF16
    gradient and are stationary for the oracle's float64 gradient to 1e-6 plus
    the float32 noise floor, with the exact float64 energy reported."""
    p = problem("c2")
    B = 16
    z0 = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    r, ores, o = _compare_newton(p, rb.PREC_BF16, z0, tg, fo)
    assert np.all(r["status"] == rb.CONVERGED), r["status"]
    g0 = np.abs(o.reduced(z0, tg, fo)[1]).max(axis=1)
    Eg, gg, _ = o.reduced(r["z"], tg, fo)
    assert np.all(np.abs(gg).max(axis=1) <= 1.5e-6 * g0)
    assert relerr(r["E"][:, None], Eg[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    same = np.abs(r["E"] - ores["E"]) <= 1e-6 * np.abs(ores["E"]) + 1e-9
    assert same.mean() >= 0.8
    assert np.abs(r["iters"][same] - ores["iters"][same]).max() <= 2


# ------------------------------------------------------ parameter gradient
def _layer_errs(ctx, grad, go):
    """Per-layer relative errors (W and b, flattened) of a packed gradient."""
    errs = []
    o = O.Oracle(ctx.p)
    for (gW, gb), (oW, ob) in zip(ctx.unpack_params(grad.cpu()), o.unpack_params(go)):
        for a, b in ((gW.numpy().ravel(), oW.ravel()), (gb.numpy(), ob)):
            errs.append(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return errs


@pytest.mark.parametrize("name,prec", [("tinyb", rb.PREC_F64), ("tinyb", rb.PREC_F32), ("c1", rb.PREC_F64),
                                       ("c2", rb.PREC_F32)])
@pytest.mark.parametrize("flags", [0, rb.ELASTIC_ONLY])
def test_energy_param_grad(name, prec, flags):
    """dE/dtheta of the summed energy (Sec. 3.2's potential loss) against the
    oracle's hand-applied chain rule, layer by layer."""
    p = problem(name)
    B = 5
    ctx = rb.Context(p, prec=prec, max_batch=8)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, grad = ctx.energy_param_grad(t64(z), t64(tg), t64(fo), flags=flags)
    assert grad.numel() == ctx.param_count()
    o = O.Oracle(p)
    oflags = O.ELASTIC_ONLY if flags & rb.ELASTIC_ONLY else 0
    Eo, go = o.energy_param_grad(z, tg, fo, flags=oflags)
    _, gzo, _ = o.reduced(z, tg, fo, flags=oflags)
    assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), gzo).max() < TOL[prec]
    assert max(_layer_errs(ctx, grad, go)) < TOL[prec]


def test_energy_param_grad_chunks_and_empty_batch():
    """B above max_batch accumulates over chunks (ragged last chunk); B = 0 gives zeros."""
    p = problem("tinyb")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    B = 11
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, grad = ctx.energy_param_grad(t64(z), t64(tg), t64(fo))
    Eo, go = O.Oracle(p).energy_param_grad(z, tg, fo)
    assert max(_layer_errs(ctx, grad, go)) < 1e-10
    grad.fill_(7.0)
    ld, _ = ctx._load(0, None, None)
    rc = rb.load_library().rs_energy_param_grad(ctx.ctx, 0, None, rb.C.byref(ld), 0, None, None, rb._ptr(grad),
                                                rb._stream())
    assert rc == rb.RS_OK
    torch.cuda.synchronize()
    assert torch.count_nonzero(grad).item() == 0


def test_energy_param_grad_errors():
    p = problem("tinyb")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    z = t64(I.latent_batch(2, p.r))
    with pytest.raises(RuntimeError, match="code 1"):
        ctx.energy_param_grad(z, flags=rb.HESS_EXACT)
    bctx = rb.Context(problem("c1"), prec=rb.PREC_BF16, max_batch=4)
    with pytest.raises(RuntimeError, match="code 5"):
        bctx.energy_param_grad(t64(I.latent_batch(2, 8)))


def test_cubature_energy_autograd_function():
    """torch.autograd through the library's reverse pass: theta.grad and z.grad
    against the oracle, and a directional finite difference of the GPU's own
    float64 energy along a random parameter direction."""
    p = problem("tinyb")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=8)
    o = O.Oracle(p)
    B = 4
    zn = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    theta0 = torch.cat([torch.cat([torch.tensor(W).ravel(), torch.tensor(b)]) for W, b in zip(p.Ws, p.bs)])
    theta = theta0.to(DEV).clone().requires_grad_(True)
    z = t64(zn).requires_grad_(True)
    loss = rb.CubatureEnergy.apply(ctx, z, theta, t64(tg), t64(fo), 0)
    loss.backward()
    Eo, go = o.energy_param_grad(zn, tg, fo)
    _, gzo, _ = o.reduced(zn, tg, fo, flags=0)
    assert abs(loss.item() - Eo.sum()) <= 1e-10 * abs(Eo).sum()
    assert max(_layer_errs(ctx, theta.grad.detach(), go)) < 1e-10
    assert relerr(z.grad.cpu().numpy(), gzo).max() < 1e-10
    d = torch.tensor(np.random.default_rng(3).normal(size=theta0.numel()), dtype=torch.float64, device=DEV)
    h = 1e-6
    with torch.no_grad():
        Ep = rb.CubatureEnergy.apply(ctx, z, theta + h * d, t64(tg), t64(fo), 0).item()
        Em = rb.CubatureEnergy.apply(ctx, z, theta - h * d, t64(tg), t64(fo), 0).item()
    fd = (Ep - Em) / (2 * h)
    an = float((theta.grad * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)


# ------------------------------------------------------------------- misc
def test_set_decoder_matches_fresh_context():
    p = problem("tinyb")
    q = problem("tinyb", decoder_seed=7)
    z = I.latent_batch(3, p.r)
    tg, fo = I.loads_for(p, 3)
    a = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    a.set_decoder(q.Ws, q.bs)
    b = rb.Context(q, prec=rb.PREC_F64, max_batch=4)
    ra = a.energy_grad_hess(t64(z), t64(tg), t64(fo))
    rbb = b.energy_grad_hess(t64(z), t64(tg), t64(fo))
    for x, y in zip(ra, rbb):
        assert torch.equal(x, y)


def test_profile_records_kernels():
    p = problem("c1")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=4)
    ctx.profile(True)
    ctx.newton_solve(torch.zeros((2, p.r), dtype=torch.float64, device=DEV))
    ctx.profile(False)
    prof = ctx.profile_read()
    for k in ("gemm_out", "elem", "newton_dir", "energy_f64"):
        assert prof[k]["launches"] > 0 and prof[k]["ms"] > 0
    # only the requested kind is bracketed
    ctx.profile(True, kinds=["elem"])
    ctx.newton_solve(torch.zeros((2, p.r), dtype=torch.float64, device=DEV))
    ctx.profile(False)
    prof = ctx.profile_read()
    assert set(prof) == {"elem"} and prof["elem"]["bytes"] > 0


# ------------------------------------------------------------------- full size
@pytest.mark.parametrize("name,B", [("c2", 1024), ("c3", 4096)])
def test_full_size_sampled(name, B):
    """Launch configuration of the benchmark; sampled items against the oracle."""
    p = problem(name)
    ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=B)
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo))
    idx = np.array([0, 1, 17, B // 2 + 3, B - 1])
    Eo, go, Ho = O.Oracle(p).reduced(z[idx], tg[idx], None)
    assert relerr(g.cpu().numpy()[idx], go).max() < 1e-4
    assert relerr(H.cpu().numpy()[idx], Ho).max() < 1e-4
    assert relerr(E.cpu().numpy()[idx, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert torch.isfinite(H).all()


# ------------------------------------------------------------------- L-BFGS
def _compare_lbfgs(p, prec, z0, tg=None, fo=None, opts_kw=None):
    opts_kw = opts_kw or {}
    ctx = rb.Context(p, prec=prec, max_batch=max(len(z0), 2))
    res = ctx.lbfgs_solve(t64(z0), t64(tg), t64(fo), opts=rb.default_lbfgs_opts(**opts_kw))
    o = O.Oracle(p)
    ores = o.lbfgs(z0, tg, fo, opts=O.default_lbfgs_opts(**opts_kw))
    r = {k: v.cpu().numpy() for k, v in res.items()}
    return r, ores, o


@pytest.mark.parametrize("name", ["c1", "tinyb"])
@pytest.mark.parametrize("history", [0, 1, 10, 16])
def test_lbfgs_float64_first_iterates_match_oracle(name, history):
    """The first L-BFGS steps (history update, two-loop direction, Armijo) to rounding."""
    p = problem(name)
    B = 6
    z0 = np.vstack([np.zeros((1, p.r)), I.latent_batch(B - 1, p.r)])
    tg, fo = I.loads_for(p, B)
    for k in (1, 3, 8):
        r, ores, _ = _compare_lbfgs(p, rb.PREC_F64, z0, tg, fo, dict(max_iter=k, history=history))
        assert np.array_equal(r["status"], ores["status"])
        assert np.array_equal(r["iters"], ores["iters"])
        assert relerr(r["z"], ores["z"], tau=1e-3).max() < 1e-9
        assert relerr(r["E"][:, None], ores["E"][:, None], tau=1e-6 * energy_scale(p)).max() < 1e-9


@pytest.mark.parametrize("name", ["c1", "tinyb"])
def test_lbfgs_float64_solves_converge_like_oracle(name):
    p = problem(name)
    B = 6
    z0 = np.vstack([np.zeros((1, p.r)), I.latent_batch(B - 1, p.r)])
    tg, fo = I.loads_for(p, B)
    r, ores, o = _compare_lbfgs(p, rb.PREC_F64, z0, tg, fo)
    assert np.all(r["status"] == rb.CONVERGED) and np.all(ores["status"] == O.CONVERGED)
    # whole trajectories of tens of steps amplify rounding: compare the end points
    g0 = np.abs(o.reduced(z0, tg, fo)[1]).max(axis=1)
    Eg, gg, _ = o.reduced(r["z"], tg, fo)
    assert np.all(np.abs(gg).max(axis=1) <= 1e-6 * g0 * (1 + 1e-6))
    assert relerr(r["E"][:, None], Eg[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    same = np.abs(r["E"] - ores["E"]) <= 1e-8 * np.abs(ores["E"]) + 1e-9 * energy_scale(p)
    assert same.mean() >= 0.8
    assert np.abs(r["iters"][same] - ores["iters"][same]).max() <= max(3, 0.1 * ores["iters"].max())


def test_lbfgs_float32_c2_stationary_for_oracle():
    p = problem("c2")
    B = 8
    z0 = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=B)
    res = ctx.lbfgs_solve(t64(z0), t64(tg), t64(fo))
    r = {k: v.cpu().numpy() for k, v in res.items()}
    o = O.Oracle(p)
    assert np.all(np.isin(r["status"], [rb.CONVERGED, rb.LS_MAX]))
    assert (r["status"] == rb.CONVERGED).mean() >= 0.75
    g0 = np.abs(o.reduced(z0, tg, fo)[1]).max(axis=1)
    Eg, gg, _ = o.reduced(r["z"], tg, fo)
    conv = r["status"] == rb.CONVERGED
    # 1e-6 on the float32 reverse-mode gradient plus the float32 noise floor (5e-7 of |g_0|)
    assert np.all(np.abs(gg[conv]).max(axis=1) <= 1.5e-6 * g0[conv])
    assert relerr(r["E"][:, None], Eg[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10


def test_lbfgs_forced_statuses_and_errors():
    p = problem("tinyb")
    z0 = I.latent_batch(1, p.r)
    tg, fo = I.loads_for(p, 1, twist_deg=[120.0])
    r, ores, _ = _compare_lbfgs(p, rb.PREC_F64, z0, tg, fo, dict(max_iter=0))
    assert r["status"][0] == rb.ITER_MAX == ores["status"][0] and r["iters"][0] == 0
    r, ores, _ = _compare_lbfgs(p, rb.PREC_F64, z0, tg, fo, dict(ls_max=0))
    assert r["status"][0] == rb.LS_MAX == ores["status"][0]
    zn = z0.copy(); zn[0, 1] = np.nan
    r, ores, _ = _compare_lbfgs(p, rb.PREC_F64, zn, tg, fo)
    assert r["status"][0] == rb.NONFINITE == ores["status"][0]
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=2)
    with pytest.raises(RuntimeError, match="invalid solver options"):
        ctx.lbfgs_solve(t64(z0), t64(tg), t64(fo), opts=rb.default_lbfgs_opts(history=rb.MAX_HISTORY + 1))
    # the history lives in the context: a second solve from the same start repeats the first
    a = ctx.lbfgs_solve(t64(z0), t64(tg), t64(fo))
    b = ctx.lbfgs_solve(t64(z0), t64(tg), t64(fo))
    assert torch.equal(a["z"], b["z"]) and torch.equal(a["iters"], b["iters"])


@pytest.mark.parametrize("name,prec", [("tinyb", rb.PREC_F64), ("c1", rb.PREC_F64), ("c2", rb.PREC_F32),
                                       ("c2", rb.PREC_F64), ("tinyb", rb.PREC_F32)])
@pytest.mark.parametrize("flags", [0, rb.ELASTIC_ONLY])
def test_reverse_mode_gradient(name, prec, flags):
    """g = J^T grad_q E formed backwards (value pass, adjoint seeds, reverse pass) against the oracle."""
    p = problem(name)
    B = 7
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    ctx = rb.Context(p, prec=prec, max_batch=4)  # B > max_batch: chunked, ragged last chunk
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=flags | rb.GRAD_REVERSE)
    assert H is None
    Eo, go, _ = O.Oracle(p).reduced(z, tg, fo, flags=O.ELASTIC_ONLY if flags else 0)
    assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), go).max() < TOL[prec]


# ------------------------------------------------------------------- largest sizes
MAXCASES = {
    # the largest latent size (32: the 32-lane element path, two-tile curvature, LDS Jacobi) and width 256
    "r32w256": dict(nx=4, ny=2, nz=1, r=32, hidden=[256, 256], n_cub=40),
    # the most hidden layers (8)
    "l8": dict(nx=3, ny=1, nz=1, r=12, hidden=[64] * 8, n_cub=15),
}


def max_problem(name):
    c = MAXCASES[name]
    return I.make_problem(name, c["nx"], c["ny"], c["nz"], c["r"], c["hidden"], c["n_cub"], bend=True,
                          bias_scale=0.3)


@pytest.mark.parametrize("name", sorted(MAXCASES))
@pytest.mark.parametrize("prec", [rb.PREC_F64, rb.PREC_F32])
def test_largest_sizes_evaluation(name, prec):
    p = max_problem(name)
    B = 5
    z = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    ctx = rb.Context(p, prec=prec, max_batch=8)
    o = O.Oracle(p)
    tol = TOL[prec]
    x, J = ctx.decode(t64(z))
    xo, Jo = o.decode(z)
    assert relerr(x.cpu().numpy() - p.X, xo - p.X, tau=1e-3).max() < tol
    assert relerr(J.cpu().numpy(), Jo).max() < tol
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo))
    Eo, go, Ho = o.reduced(z, tg, fo, flags=O.EXACT)
    assert relerr(E.cpu().numpy()[:, None], Eo[:, None], tau=1e-6 * energy_scale(p)).max() < 1e-10
    assert relerr(g.cpu().numpy(), go).max() < tol
    assert relerr(H.cpu().numpy(), Ho).max() < tol
    Er, gr, _ = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=rb.GRAD_REVERSE)
    assert relerr(gr.cpu().numpy(), go).max() < tol
    # decoder-parameter gradient at the widest layers and the deepest decoder
    _, _, grad = ctx.energy_param_grad(t64(z), t64(tg), t64(fo))
    _, pgo = o.energy_param_grad(z, tg, fo)
    assert max(_layer_errs(ctx, grad, pgo)) < tol


@pytest.mark.parametrize("name", sorted(MAXCASES))
def test_largest_sizes_solvers(name):
    """Newton steps and L-BFGS steps at the largest sizes against the oracle's (float64)."""
    p = max_problem(name)
    B = 4
    z0 = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    for k in (1, 2):
        r, ores, _ = _compare_newton(p, rb.PREC_F64, z0, tg, fo, dict(max_iter=k))
        assert np.array_equal(r["status"], ores["status"]) and np.array_equal(r["iters"], ores["iters"])
        assert relerr(r["z"], ores["z"], tau=1e-3).max() < 1e-8
        r, ores, _ = _compare_lbfgs(p, rb.PREC_F64, z0, tg, fo, dict(max_iter=2 * k))
        assert np.array_equal(r["status"], ores["status"]) and np.array_equal(r["iters"], ores["iters"])
        assert relerr(r["z"], ores["z"], tau=1e-3).max() < 1e-8
