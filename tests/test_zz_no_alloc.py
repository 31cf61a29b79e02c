"""The allocation-free Lipschitz-gradient entry point (its pass workspace is the
library's static device array) against the allocating one, through the C ABI:
two calls in a row on one context, the second with fewer pairs, at the
context's parity bar (1e-10 in float64, 1e-4 in float32); and the size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2409_03807_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_03807_amd import binding as rb  # noqa: E402

DEV = "cuda:0"


def t64(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _pairs(B, r, seed):
    z1 = I.latent_batch(B, r, seed=seed)
    z2 = I.latent_batch(B, r, seed=seed + 1)
    z2[0] = z1[0]   # one excluded pair
    return t64(z1), t64(z2)


@pytest.mark.parametrize("name,prec,sizes,tol", [
    ("tinyb", rb.PREC_F64, (5, 3), 1e-10),
    ("c4", rb.PREC_F32, (64, 20), 1e-4),
])
def test_noalloc_matches_allocating_variant(name, prec, sizes, tol):
    if name == "tinyb":
        p = I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3)
        mb = 4
    else:
        p = I.config("c4", bias_scale=0.05)
        mb = 128
    ctx = rb.Context(p, prec=prec, max_batch=mb)
    n = ctx.param_count()
    # preallocated outputs, reused by both noalloc calls (the second call must overwrite them)
    loss_na = torch.empty(1, dtype=torch.float64, device=DEV)
    grad_na = torch.empty(n, dtype=torch.float64, device=DEV)
    for call, B in enumerate(sizes):
        z1, z2 = _pairs(B, p.r, seed=40 + 2 * call)
        print(f"noalloc case {name} prec={prec} call={call} B={B}", flush=True)
        ctx.lipschitz_param_grad(z1, z2, out=(loss_na, grad_na), noalloc=True)
        loss, grad = ctx.lipschitz_param_grad(z1, z2)
        torch.cuda.synchronize()
        a, b = grad_na.cpu().numpy(), grad.cpu().numpy()
        assert np.isfinite(a).all()
        assert abs(loss_na.item() - loss.item()) <= tol * abs(loss.item())
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b)
        assert np.linalg.norm(b) > 0


def test_noalloc_rejects_a_pair_beyond_the_static_array():
    """The c2 beam in float64 with r = 20 and every tet as cubature: one pair's
    element rows alone need 9 * 12800 * 44 * 8 * 2 bytes (81 MB), more than the
    64 MiB array."""
    p = I.make_problem("c2all", 40, 8, 8, 20, [128] * 4, 10 ** 9)
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=2)
    z1, z2 = _pairs(1, p.r, seed=50)
    with pytest.raises(RuntimeError, match="static"):
        ctx.lipschitz_param_grad(z1, z2, noalloc=True)
