"""GPU parity of the optional element treatments: the per-element
positive-semi-definite projection (RS_ELEM_PSD; supplement, projective Newton)
and the 12x12 element-Hessian dump (RS_DEBUG_ELEM_HESS), against the float64
oracle, which projects each 12x12 element Hessian itself with its own Jacobi
eigen-decomposition (the library projects the equivalent 9x9 matrix)."""
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
TOL = {rb.PREC_F64: 1e-10, rb.PREC_F32: 1e-4, rb.PREC_BF16: 1e-4}


def t64(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def relerr(a, b, tau=0.0):
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), tau)


def problem(name):
    if name == "tinyb":
        return I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3)
    if name == "c1":
        return I.config("c1", bias_scale=0.1)
    return I.config(name)


CASES = [("tinyb", rb.PREC_F64), ("tinyb", rb.PREC_F32), ("c1", rb.PREC_F64), ("c2", rb.PREC_F32),
         ("c2", rb.PREC_BF16)]


def _z(p, B, scale):
    return scale * np.random.default_rng(23).normal(size=(B, p.r))


@pytest.mark.parametrize("name,prec", CASES)
@pytest.mark.parametrize("exact", [0, 1])
def test_elem_psd_reduced_hessian(name, prec, exact):
    p = problem(name)
    B = 6
    z = _z(p, B, 1.5)   # large latent values: strongly deformed, indefinite elements
    tg, fo = I.loads_for(p, B)
    ctx = rb.Context(p, prec=prec, max_batch=4)   # B > max_batch: chunked
    flags = rb.ELEM_PSD | (rb.HESS_EXACT if exact else 0)
    E, g, H = ctx.energy_grad_hess(t64(z), t64(tg), t64(fo), flags=flags)
    o = O.Oracle(p)
    oflags = O.ELEM_PSD | (O.EXACT if exact else 0)
    Eo, go, Ho = o.reduced(z, tg, fo, flags=oflags)
    _, _, Hraw = o.reduced(z, tg, fo, flags=O.EXACT if exact else 0)
    # the projection changes these Hessians well beyond the bar
    assert relerr(Ho, Hraw).max() > min(100 * TOL[prec], 0.2)
    assert relerr(g.cpu().numpy(), go).max() < TOL[prec]
    assert relerr(H.cpu().numpy(), Ho).max() < TOL[prec]


@pytest.mark.parametrize("name,prec", [("tinyb", rb.PREC_F64), ("c1", rb.PREC_F64), ("c2", rb.PREC_F32)])
def test_debug_element_hessians(name, prec):
    p = problem(name)
    B = 3
    z = _z(p, B, 0.8)
    ctx = rb.Context(p, prec=prec, max_batch=2)   # two chunks, the second ragged
    S = len(p.cub_elem)
    He = torch.full((B, S, 12, 12), np.nan, dtype=torch.float64, device=DEV)
    ctx.set_elem_hess_dump(He)
    ctx.energy_grad_hess(t64(z), flags=rb.HESS_EXACT | rb.DEBUG_ELEM_HESS)
    o = O.Oracle(p)
    x, _ = o.decode(z, want_J=False)
    mu, lam = O.lame(p.young, p.poisson)
    got = He.cpu().numpy()
    want = np.empty_like(got)
    for b in range(B):
        for s, e in enumerate(p.cub_elem):
            t = p.tets[e]
            want[b, s] = O.elem_hess(p.X[t], x[b][t], mu, lam)
    err = relerr(got.reshape(B * S, -1), want.reshape(B * S, -1))
    assert err.max() < TOL[prec]
    # registering nothing and asking for the dump is an argument error
    ctx.set_elem_hess_dump(None)
    with pytest.raises(RuntimeError, match="RS_DEBUG_ELEM_HESS"):
        ctx.energy_grad_hess(t64(z), flags=rb.DEBUG_ELEM_HESS)


@pytest.mark.parametrize("hess", [rb.HESS_GN_ELEM_PSD, rb.HESS_EXACT_ELEM_PSD])
def test_newton_elem_psd_float64_matches_oracle(hess):
    """Projected element Hessians inside the Newton solve (c1, float64): the
    oracle's statuses, iteration counts and iterates."""
    p = problem("c1")
    B = 6
    z0 = np.vstack([np.zeros((2, p.r)), I.latent_batch(B - 2, p.r)])
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=B)
    res = ctx.newton_solve(t64(z0), opts=rb.default_opts(hess=hess))
    r = {k: v.cpu().numpy() for k, v in res.items()}
    ores = O.Oracle(p).newton(z0, opts=O.default_opts(hess=hess))
    assert np.array_equal(r["status"], ores["status"])
    assert np.array_equal(r["iters"], ores["iters"])
    assert np.abs(r["z"] - ores["z"]).max() < 1e-6


def test_newton_gn_elem_psd_float32_c2_stationary():
    p = problem("c2")
    B = 8
    z0 = I.latent_batch(B, p.r)
    tg, fo = I.loads_for(p, B)
    ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=B)
    res = ctx.newton_solve(t64(z0), t64(tg), t64(fo), opts=rb.default_opts(hess=rb.HESS_GN_ELEM_PSD))
    r = {k: v.cpu().numpy() for k, v in res.items()}
    conv = r["status"] == rb.CONVERGED
    assert conv.mean() >= 0.75
    o = O.Oracle(p)
    g0 = np.abs(o.reduced(z0, tg, fo, flags=0)[1]).max(axis=1)
    gg = o.reduced(r["z"], tg, fo, flags=0)[1]
    assert np.all(np.abs(gg[conv]).max(axis=1) <= 1e-5 * g0[conv])


def test_solver_rejects_unknown_hessian_mode():
    p = problem("tinyb")
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=2)
    with pytest.raises(RuntimeError, match="invalid solver options"):
        ctx.newton_solve(t64(np.zeros((1, p.r))), opts=rb.default_opts(hess=4))
