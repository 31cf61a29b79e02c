"""The stream-ordered Newton solve (rs_newton_solve_async): with enough
super-steps it ends every item where the adaptive solve does; with too few it
leaves items running; captured into a HIP graph it replays to the eager result."""
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


def _outs(B, r):
    return (torch.empty((B, r), dtype=torch.float64, device=DEV), torch.empty(B, dtype=torch.int32, device=DEV),
            torch.empty(B, dtype=torch.int32, device=DEV), torch.empty(B, dtype=torch.float64, device=DEV),
            torch.empty(B, dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("name,prec", [("c1", rb.PREC_F64), ("c2", rb.PREC_F32)])
def test_async_solve_matches_adaptive(name, prec):
    p = I.config(name, bias_scale=0.1) if name == "c1" else I.config(name)
    B = 64
    z0 = t64(I.latent_batch(B, p.r))
    tg, fo = I.loads_for(p, B)
    tg, fo = (None if a is None else t64(a) for a in (tg, fo))
    ctx = rb.Context(p, prec=prec, max_batch=B)
    a = ctx.newton_solve(z0, tg, fo)
    b = ctx.newton_solve(z0, tg, fo, super_steps=60)
    torch.cuda.synchronize()
    sa, sb = a["status"].cpu().numpy(), b["status"].cpu().numpy()
    assert np.all(sa == rb.CONVERGED)
    assert np.array_equal(sa, sb)
    assert np.array_equal(a["iters"].cpu().numpy(), b["iters"].cpu().numpy())
    za, zb = a["z"].cpu().numpy(), b["z"].cpu().numpy()
    assert np.abs(za - zb).max() <= 1e-12 * max(np.abs(za).max(), 1.0)
    assert np.array_equal(a["E"].cpu().numpy(), b["E"].cpu().numpy()) or \
        np.abs(a["E"].cpu().numpy() - b["E"].cpu().numpy()).max() <= 1e-12 * np.abs(a["E"].cpu().numpy()).max()


def test_async_solve_too_few_steps_leaves_items_running():
    p = I.config("c1", bias_scale=0.1)
    B = 16
    z0 = t64(I.latent_batch(B, p.r))
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=B)
    b = ctx.newton_solve(z0, super_steps=2)
    torch.cuda.synchronize()
    st = b["status"].cpu().numpy()
    assert (st == rb.RUNNING).all()
    assert np.all(b["iters"].cpu().numpy() <= 2)
    assert torch.isfinite(b["z"]).all() and torch.isfinite(b["E"]).all()
    with pytest.raises(RuntimeError):
        ctx.newton_solve(z0, super_steps=0)


def test_async_solve_graph_replays():
    """Captured once, replayed three times with eager work in between: every
    replay reproduces the eager stream-ordered solve exactly."""
    p = I.config("c1", bias_scale=0.1)
    B = 32
    z0 = t64(I.latent_batch(B, p.r))
    ctx = rb.Context(p, prec=rb.PREC_F64, max_batch=B)
    out = _outs(B, p.r)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.newton_solve(z0, out=out, super_steps=40)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = [t.clone() for t in out]
    assert (ref[2] == rb.CONVERGED).all()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.newton_solve(z0, out=out, super_steps=40)
    for rep in range(3):
        for t in out:
            t.fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t, u in zip(out, ref):
            assert torch.equal(t, u), rep
        # eager work of the program's own between replays
        ctx.newton_solve(z0 + 0.01, super_steps=5)
        torch.cuda.synchronize()
