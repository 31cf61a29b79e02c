"""GPU solve parity at the benchmark's batch and beyond it.

The device-resident solve control splits its work by batch size: the
line-search candidate points over eight workgroups, and the Armijo test over
chunks of 1024 searching items.  These tests run whole batches of 1024 and
2048 items (duplicated start points in the second half, so every item has a
twin that must end identically) and compare sampled items with the float64
oracle: exact statuses, iteration counts and iterates for float64 contexts;
stationarity under the oracle's gradient and the exact float64 energy for
float32 and BF16 contexts.
"""
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

# Float32 gradient noise floor: |g_fp32(z*) - g(z*)|_inf / |g(z_0)|_inf at the
# oracle's float64 minimisers z* of the c2 workload (twist sweep, z0 ~ N(0, 0.5^2)).
# Measured on one MI355X over 64 such points: median 2.4e-8, max 2.0e-7.  The
# float32 solver stops at 1e-6 on its own gradient, so the oracle's gradient at
# a float32 solution is at most 1e-6 plus this floor, relative to |g_0|
# (measured over the 1024 bench items: max 9.9e-7, all 1024 below 1e-6).
FP32_FLOOR_C2 = 5e-7


def t64(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def energy_scale(p):
    mu = p.young / (2 * (1 + p.poisson))
    return mu * p.meta["h"] ** 3 * p.ne / 5


def _solve(p, prec, z0, tg, fo, **kw):
    ctx = rb.Context(p, prec=prec, max_batch=len(z0))
    res = ctx.newton_solve(t64(z0), t64(tg), t64(fo), opts=rb.default_opts(**kw))
    return {k: v.cpu().numpy() for k, v in res.items()}


def _twin(a):
    """Inputs whose second half repeats the first."""
    return None if a is None else np.concatenate([a, a], axis=0)


def test_newton_float64_c1_batch_2048_matches_oracle():
    """c1 in float64 with 2048 items (more than 1024 searching items: the
    Armijo kernel's chunk loop; the candidate points over eight workgroups)."""
    p = I.config("c1", bias_scale=0.1)
    half = 1024
    z0 = _twin(np.vstack([np.zeros((1, p.r)), I.latent_batch(half - 1, p.r)]))
    r = _solve(p, rb.PREC_F64, z0, None, None)
    # twins end identically (items are independent of their place in the batch)
    for k in ("status", "iters"):
        assert np.array_equal(r[k][:half], r[k][half:])
    assert np.array_equal(r["z"][:half], r["z"][half:])
    assert np.array_equal(r["E"][:half], r["E"][half:])
    # sampled items in both halves against the oracle's own solves
    idx = np.array([0, 1, 2, 511, 1023, 1024, 1300, 2047])
    ores = O.Oracle(p).newton(z0[idx])
    assert np.array_equal(r["status"][idx], ores["status"])
    assert np.array_equal(r["iters"][idx], ores["iters"])
    assert np.abs(r["z"][idx] - ores["z"]).max() < 1e-6
    E = r["E"][idx]
    assert np.all(np.abs(E - ores["E"]) <= 1e-9 * np.maximum(np.abs(ores["E"]), 1e-6 * energy_scale(p)))


@pytest.mark.parametrize("name,prec,B", [("c2", rb.PREC_F32, 1024), ("c2", rb.PREC_F32, 2048),
                                         ("c3", rb.PREC_BF16, 4096)])
def test_newton_float32_full_batch_oracle_stationary(name, prec, B):
    """The benchmark workloads (c2 in float32 at B = 1024, and at B = 2048 with
    duplicated starts; c3 with the BF16 decoder at B = 4096): every item
    converges, sampled items are stationary for the oracle's float64 gradient
    to 1e-6 plus the float32 floor, and their reported energies are the
    float64 energies of the returned points."""
    p = I.config(name)
    half = min(B, 1024) if prec == rb.PREC_F32 else B
    z0 = I.latent_batch(half, p.r)
    tg, fo = I.loads_for(p, half)
    if B > half:
        z0, tg, fo = _twin(z0), _twin(tg), _twin(fo)
    r = _solve(p, prec, z0, tg, fo)
    st = r["status"]
    assert np.all(st == rb.CONVERGED), np.unique(st, return_counts=True)
    if B > half:
        for k in ("status", "iters"):
            assert np.array_equal(r[k][:half], r[k][half:])
        assert np.array_equal(r["z"][:half], r["z"][half:])
    rng = np.random.default_rng(7 + B)
    idx = np.sort(rng.choice(B, size=24, replace=False))
    idx = idx[st[idx] == rb.CONVERGED]
    o = O.Oracle(p)
    sel = lambda a: None if a is None else a[idx]
    g0 = np.abs(o.reduced(z0[idx], sel(tg), sel(fo), flags=0)[1]).max(axis=1)
    Eg, gg, _ = o.reduced(r["z"][idx], sel(tg), sel(fo), flags=0)
    rel = np.abs(gg).max(axis=1) / g0
    assert np.all(rel <= 1e-6 + FP32_FLOOR_C2), rel.max()
    den = np.maximum(np.abs(Eg), 1e-6 * energy_scale(p))
    assert np.all(np.abs(r["E"][idx] - Eg) <= 1e-10 * den)


@pytest.mark.parametrize("prec", [rb.PREC_F32, rb.PREC_BF16])
def test_fp32_gradient_noise_floor_c2(prec):
    """The float32 reduced gradient at the oracle's float64 minimisers (c2),
    from the float32 decoder and from the BF16 decoder (three-part operands):
    the floor the solver's 1e-6 test sits on, measured, not assumed."""
    p = I.config("c2")
    n = 8
    z0 = I.latent_batch(n, p.r)
    tg, fo = I.loads_for(p, n)
    o = O.Oracle(p)
    ores = o.newton(z0, tg, fo)
    ok = ores["status"] == O.CONVERGED
    assert ok.sum() >= 6
    g0 = np.abs(o.reduced(z0, tg, fo, flags=0)[1]).max(axis=1)
    ctx = rb.Context(p, prec=prec, max_batch=n)
    _, g, _ = ctx.energy_grad_hess(t64(ores["z"]), t64(tg), t64(fo))
    gor = o.reduced(ores["z"], tg, fo, flags=0)[1]
    floor = np.abs(g.cpu().numpy() - gor).max(axis=1) / g0
    print("gradient floor", prec, np.median(floor[ok]), floor[ok].max(), flush=True)
    assert np.all(floor[ok] <= FP32_FLOOR_C2), floor[ok].max()
    # the oracle's own minimisers sit below 1e-6, so the float32 gradient there does too, up to the floor
    assert np.all(np.abs(g.cpu().numpy()[ok]).max(axis=1) / g0[ok] <= 1e-6 + FP32_FLOOR_C2)
