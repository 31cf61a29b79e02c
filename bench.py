"""Benchmark of the reduced-Newton hot path on one MI355X.

One step = one pass of the whole hot path over one batch: a batched projective
Newton solve (decoder value + Jacobian, cubature element physics, reductions,
exact Hessian, r x r solve, float64 line search, convergence test) of every item
from its start point, then the Lipschitz loss of the exact cubature elastic
Hessian over the batch taken as pairs.

Workload (default): 40x8x8 cube-grid beam (3321 vertices, 12800 tets,
n = 9963), stable Neo-Hookean E = 1e5 Pa, nu = 0.45, gravity, x = 0 face fixed,
end twist 0-180 deg as penalty targets (k_c = 1e6 N/m) on the x = L face;
decoder r = 16 -> 4 x 128 ELU -> 9963 (Glorot init, untrained: the plain
subspace); 256 cubature tets, weights U[20, 80]; batch of 1024 latent start
points z0 ~ N(0, 0.5^2); float32 decoder and element physics, float64
reductions, r x r solve, line-search energies and convergence test.

Metric: converged reduced solves per second (items ending with
|g|_inf <= 1e-6 |g_0|_inf), whole job, inputs resident in HBM.

Batching: by default the solve lines (Newton and L-BFGS) stream the timed
steps' batches (copies of the same batch) through one solve with the batch size
(1024) in flight: an item that finishes gives its place to the next one, so no
super-step runs with only the slowest items of a batch (continuous batching;
every launch still holds at most 1024 items).  --batching per-batch solves each
step's batch on its own, as the other paths always do.

Other lines of the same script:
* --config c1 / c3: the 10x2x2 beam in float64, or c2 at a batch of 4096 with
  the BF16 decoder (three-part BF16 operands, float32 accuracy);
* --solver lbfgs: the same solves by L-BFGS; --hess / --proj: other Hessian
  policies; --z0 zero / --twist T: start points and loads of one kind;
* --path param_grad: the gradient of the summed cubature energy of the batch
  with respect to every decoder parameter (the potential loss of the
  unsupervised subspace construction), in items per second;
* --path learned: the learned part on the 16^3 block (snapshots, training
  with and without the Lipschitz term, PCA, held-out solves);
* --path simulate: implicit-Euler simulations with ground contact (c5), with
  --train-epochs to train their subspace first.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# "bf16": the BF16 contexts' decoder products take six BF16 MFMAs per float32
# product (three-part operands), so their float32-equivalent peak is the dense
# BF16 peak (2.5 PFLOP/s) over six
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0 / 6}
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2409_03807_amd", "csrc", "rs_kernels.hip")


def recorded_traffic(kind, workload):
    """HBM bytes per launch of `kind` measured by rocprofv3 --pmc (FETCH_SIZE and
    WRITE_SIZE, each scaled by what it reads for a plain copy of known size), from
    the `traffic-json:` line of a summary under profiles/.  None when no summary
    covers this kind and workload, or when the kernel source changed since the
    counters were taken."""
    with open(KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-json:"):
                    continue
                rec = json.loads(line[len("traffic-json:"):])
                if rec.get("kind") == kind and rec.get("workload") == workload and rec.get("source_sha256") == sha:
                    return rec["bytes_per_launch"]
    return None


# the bound of each launch kind: contractions on the matrix cores, the r x r
# solves on the float64 vector ALUs, everything else on HBM bandwidth
MFMA_KINDS = {"gemm_hidden", "gemm_out", "gemm_adjoint", "decode_hidden", "decode_out", "elem_fused"}
MFMA_F64_KINDS = {"ls_gemm_hidden", "ls_gemm_out"}
ALU_F64_KINDS = {"newton_dir", "param_grad"}
VALU_F64_PEAK_TFLOPS = 78.6


def kernel_roofline(kind, rec, dtype):
    """Achieved rate of one launch kind (algorithmic bytes or flops over its
    summed event-timed duration) against the peak of its bound."""
    secs = rec["ms"] * 1e-3
    if kind in MFMA_KINDS or kind in MFMA_F64_KINDS:
        # BF16 contexts run only the forward decoder products in BF16; the adjoint product stays float32
        kd = "f64" if kind in MFMA_F64_KINDS else ("f32" if dtype == "bf16" and kind == "gemm_adjoint" else dtype)
        peak = MFMA_PEAK_TFLOPS[kd]
        ach = rec["flops"] / secs / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak}
    if kind in ALU_F64_KINDS:
        ach = rec["flops"] / secs / 1e12
        return {"bound": "alu", "achieved": ach, "peak": VALU_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / VALU_F64_PEAK_TFLOPS}
    ach = rec["bytes"] / secs / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c5"],
                    help="c5 (with --path simulate): implicit-Euler simulations with ground contact")
    ap.add_argument("--batch", type=int, default=0, help="override the batch size")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="oracle solves timed for cpu_baseline (0 = skip; default 320 Newton, 64 L-BFGS)")
    ap.add_argument("--no-profile", action="store_true", help="do not bracket launches with HIP events")
    ap.add_argument("--solver", default="newton", choices=["newton", "lbfgs"],
                    help="projective Newton (default) or L-BFGS (the paper's main solver)")
    ap.add_argument("--path", default="solve", choices=["solve", "param_grad", "simulate", "learned"],
                    help="solve: the reduced solves (default); param_grad: the decoder-parameter gradient of the "
                         "summed cubature energy over the batch (the potential loss of unsupervised training); "
                         "simulate: implicit-Euler steps of a batch of simulations (c5); learned: snapshots, "
                         "two-stage training, PCA and held-out solves of the c4 block (Lipschitz vs plain vs PCA)")
    ap.add_argument("--prec", default="", choices=["", "f64", "f32", "bf16"], help="override the precision")
    ap.add_argument("--z0", default="random", choices=["random", "zero"], help="start points of the solves")
    ap.add_argument("--twist", type=float, default=None, help="one twist angle (deg) for every item")
    ap.add_argument("--epochs", type=int, nargs=2, default=[400, 400], help="learned path: stage epochs")
    ap.add_argument("--train-epochs", type=int, default=0,
                    help="simulate path: train the subspace on static snapshots for this many epochs first (0: untrained)")
    ap.add_argument("--train-snapshots", type=int, default=512, help="simulate path: snapshots for --train-epochs")
    ap.add_argument("--lam-rel", type=float, nargs="+", default=[0.1], help="learned path: lambda_LS factors")
    ap.add_argument("--proj", default="abs", choices=["clamp", "abs"], help="Hessian eigen-projection")
    ap.add_argument("--eig-floor", type=float, default=1e-8)
    ap.add_argument("--hess", default="exact", choices=["exact", "gn", "gn_psd", "exact_psd"],
                    help="Newton Hessian: exact or Gauss-Newton, optionally with per-element PSD projection")
    ap.add_argument("--batching", default="auto", choices=["auto", "continuous", "per-batch"],
                    help="continuous (the default for the solves): the timed steps' batches (copies of the base "
                         "batch) go through one solve with the batch size in flight, a finished item's place "
                         "taken by the next one, plus one Lipschitz evaluation per step; per-batch: one solve per "
                         "step (the default for the other paths)")
    ap.add_argument("--fused", default="auto", choices=["auto", "on", "off"],
                    help="output map and element physics in one kernel (on) or two (off); auto: the "
                         "context's default (on for BF16, off for float32)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the reduced solves of a batch "
                                   "are independent and would shard by item across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_03807_amd import binding as rb
    from paper_2409_03807_amd import inputs as I

    torch.cuda.set_device(0)
    if args.path == "learned":
        return main_learned(args)
    if args.path == "simulate" or args.config == "c5":
        return main_simulate(args)
    name = args.config
    p = I.config(name)
    B = args.batch or {"c1": 1024, "c2": 1024, "c3": 4096}[name]
    # c1 float64, c2 float32, c3 the BF16 decoder variant of c2
    prec = {"c1": rb.PREC_F64, "c2": rb.PREC_F32, "c3": rb.PREC_BF16}[name]
    if args.prec:
        prec = {"f64": rb.PREC_F64, "f32": rb.PREC_F32, "bf16": rb.PREC_BF16}[args.prec]
    dtype = {rb.PREC_F64: "f64", rb.PREC_F32: "f32", rb.PREC_BF16: "bf16"}[prec]
    # continuous batching: the timed steps' batches go through one solve, B items in flight
    solve_path = args.path == "solve"
    if args.batching == "continuous" and not solve_path:
        raise SystemExit("--batching continuous applies to the solve path")
    args.stream = args.batching == "continuous" or (args.batching == "auto" and solve_path)
    nstream = max(args.steps, args.warmup, 1) if args.stream else 1
    ctx = rb.Context(p, prec=prec, max_batch=B * nstream)
    if args.fused == "auto":
        fused = prec == rb.PREC_BF16 and ctx.set_fused(True)
    else:
        fused = ctx.set_fused(args.fused == "on") and args.fused == "on"
    info = ctx.info()
    dev = "cuda:0"
    z0 = torch.tensor(I.latent_batch(B, p.r), device=dev)
    if args.z0 == "zero":
        z0.zero_()
    tg_np, fo_np = I.loads_for(p, B, twist_deg=args.twist)
    tg = torch.tensor(tg_np, device=dev) if tg_np is not None else None
    fo = torch.tensor(fo_np, device=dev) if fo_np is not None else None
    out = (torch.empty_like(z0), torch.empty(B, dtype=torch.int32, device=dev),
           torch.empty(B, dtype=torch.int32, device=dev), torch.empty(B, dtype=torch.float64, device=dev),
           torch.empty(B, dtype=torch.float64, device=dev))
    hess = {"exact": rb.HESS_EXACT_OPT, "gn": rb.HESS_GN, "gn_psd": rb.HESS_GN_ELEM_PSD,
            "exact_psd": rb.HESS_EXACT_ELEM_PSD}[args.hess]
    opts = rb.default_opts(proj=rb.PROJ_CLAMP if args.proj == "clamp" else rb.PROJ_ABS, eig_floor=args.eig_floor,
                           hess=hess)
    if args.stream:
        opts.window = B
    lbfgs = args.solver == "lbfgs"
    lopts = rb.default_lbfgs_opts()
    if args.stream:
        lopts.window = B
    npair = B // 2
    z1, z2 = z0[0:2 * npair:2].contiguous(), z0[1:2 * npair:2].contiguous()

    # per-step bookkeeping stays on the device (no host sync inside the timed
    # region beyond what the solver itself does)
    conv_acc = torch.zeros((), dtype=torch.int64, device=dev)
    iter_acc = torch.zeros((), dtype=torch.int64, device=dev)

    pgrad = args.path == "param_grad"

    def stream_steps(n):
        """n batches (copies of the base batch) through one solve with B items in flight,
        plus n Lipschitz evaluations: the work of n steps."""
        N = n * B
        zs = z0.repeat(n, 1)
        tgs = tg.repeat(n, 1, 1) if tg is not None else None
        fos = fo.repeat(n, 1) if fo is not None else None
        res = ctx.lbfgs_solve(zs, tgs, fos, opts=lopts) if lbfgs else ctx.newton_solve(zs, tgs, fos, opts=opts)
        lip = None
        for _ in range(n):
            lip = ctx.lipschitz_loss(z1, z2, want_per_pair=False) if npair else None
        conv_acc.add_((res["status"] == rb.CONVERGED).sum())
        iter_acc.add_(res["iters"].sum())
        assert res["status"].shape[0] == N
        return res, lip

    def step():
        if pgrad:
            E, g, grad = ctx.energy_param_grad(z0, tg, fo, want_g=False)
            conv_acc.add_(B)
            return {"status": torch.zeros(B, dtype=torch.int32, device=dev), "grad": grad}, None
        if lbfgs:
            res = ctx.lbfgs_solve(z0, tg, fo, opts=lopts, out=out)
        else:
            res = ctx.newton_solve(z0, tg, fo, opts=opts, out=out)
        lip = ctx.lipschitz_loss(z1, z2, want_per_pair=False) if npair else None
        conv_acc.add_((res["status"] == rb.CONVERGED).sum())
        iter_acc.add_(res["iters"].sum())
        return res, lip

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.stream:
        if args.warmup:
            stream_steps(args.warmup)
    else:
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    dominant = None
    if not args.no_profile:
        # a profiled pass picks the dominant kernel kind; the timed region then
        # brackets only that kind with HIP events (one event pair per launch)
        ctx.profile(True)
        if args.stream:
            stream_steps(1)
        else:
            step()
        ctx.profile(False)
        warm = ctx.profile_read()
        dominant = max(warm.items(), key=lambda kv: kv[1]["ms"])[0]
        ctx.profile(True, kinds=[dominant])
    conv_acc.zero_()
    iter_acc.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.stream:
        res, lip = stream_steps(args.steps)
    else:
        for _ in range(args.steps):
            res, lip = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    conv = int(conv_acc.item())
    mean_iters = int(iter_acc.item()) / (args.steps * B)
    prof = {}
    if not args.no_profile:
        ctx.profile(False)
        prof = ctx.profile_read()
    st = res["status"].cpu().numpy()

    # dominant kernel: the launch kind with the largest summed duration
    roof = None
    if prof:
        kind, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
        roof = kernel_roofline(kind, rec, dtype)
        roof["kernel"] = kind
        roof["avg_us"] = rec["ms"] / rec["launches"] * 1e3
        roof["launches"] = rec["launches"]
        roof["algorithmic_bytes"] = rec["bytes"] / rec["launches"]
        roof["algorithmic_flops"] = rec["flops"] / rec["launches"]
        roof["traffic"] = recorded_traffic(kind, f"{name}_b{B}")
        # every kind of the profiled warm pass against its own bound
        roof["kernels_warm_pass"] = {}
        for k, v in warm.items():
            kr = kernel_roofline(k, v, dtype)
            roof["kernels_warm_pass"][k] = {"ms": round(v["ms"], 3), "launches": v["launches"], "bound": kr["bound"],
                                            "achieved": round(kr["achieved"], 2), "unit": kr["unit"],
                                            "frac": round(kr["frac"], 4)}

    cpu = None
    if args.cpu_sample < 0:
        args.cpu_sample = 64 if lbfgs else 320
    if args.cpu_sample > 0 and pgrad:
        from oracle import oracle as O
        n = min(args.cpu_sample, B)
        o = O.Oracle(p)
        t1 = time.perf_counter()
        o.energy_param_grad(z0[:n].cpu().numpy(), tg_np[:n] if tg_np is not None else None,
                            fo_np[:n] if fo_np is not None else None)
        cdt = time.perf_counter() - t1
        cpu = {"value": n / cdt, "unit": "items/s", "cores": 1, "kind": "oracle",
               "sample": f"{n} items of the same batch through the float64 oracle's chain rule (serial), {cdt:.1f} s"}
    elif args.cpu_sample > 0:
        from oracle import oracle as O
        n = min(args.cpu_sample, B)
        o = O.Oracle(p)
        zs = z0[:n].cpu().numpy()
        t1 = time.perf_counter()
        solve = o.lbfgs if lbfgs else o.newton
        ores = solve(zs, tg_np[:n] if tg_np is not None else None, fo_np[:n] if fo_np is not None else None)
        cdt = time.perf_counter() - t1
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        cores = min(cores, len(os.sched_getaffinity(0)))
        cpu = {"value": int((ores["status"] == O.CONVERGED).sum()) / cdt, "unit": "solves/s", "cores": cores,
               "kind": "oracle", "sample": f"{n} float64 oracle {'L-BFGS' if lbfgs else 'Newton'} solves of the same workload "
                                          f"(first {n} start points), {cdt:.1f} s"}
        # the same oracle on one thread, on a sixteenth of the sample
        n1 = max(1, n // 16)
        O.set_threads(1)
        t1 = time.perf_counter()
        ores1 = solve(zs[:n1], tg_np[:n1] if tg_np is not None else None, fo_np[:n1] if fo_np is not None else None)
        cdt1 = time.perf_counter() - t1
        O.set_threads(cores)
        cpu["single_thread"] = {"value": int((ores1["status"] == O.CONVERGED).sum()) / cdt1, "unit": "solves/s",
                                "cores": 1, "sample": f"first {n1} start points, {cdt1:.1f} s"}

    line = {
        "metric": ("potential-loss parameter-gradient items/s" if pgrad else
                   "converged reduced solves/s at rel. grad 1e-6, Lipschitz vs plain subspace"),
        "value": conv / dt,
        "unit": "items/s" if pgrad else "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{name}: {p.meta['nx']}x{p.meta['ny']}x{p.meta['nz']} beam, nv={p.nv}, ne={p.ne}, "
                        f"r={p.r}, hidden={p.hidden}, |S|={len(p.cub_elem)}, B={B}, plain (untrained Glorot) "
                        f"decoder, " + (f"twist {args.twist:g} deg" if args.twist is not None else "twist 0-180 deg")
                        + " penalty targets" + (", z0 = 0" if args.z0 == "zero" else ", z0 ~ N(0, 0.5^2)"),
            "batch": B, "rows": info.rows, "subspace": "plain", "solver": "none" if pgrad else args.solver,
            "path": args.path, "hessian": args.hess, "projection": args.proj,
            "output_map": "fused with the element physics" if fused else "separate kernel (J_R through HBM)",
            "batching": (f"continuous: the {args.steps} batches through one solve, {B} items in flight"
                         if args.stream else "one solve per batch"),
        },
        "converged_frac": float((st == rb.CONVERGED).mean()),
        "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
        "mean_iters": mean_iters,
        "lipschitz_loss": None if (pgrad or lip is None) else float(lip["loss"].item()),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def profile_line(ctx, dtype):
    """Every launch kind of a profiled pass against its own bound, and the dominant one."""
    prof = ctx.profile_read()
    if not prof:
        return None
    kind, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    roof = kernel_roofline(kind, rec, dtype)
    roof.update(kernel=kind, avg_us=rec["ms"] / rec["launches"] * 1e3, launches=rec["launches"],
                algorithmic_bytes=rec["bytes"] / rec["launches"], algorithmic_flops=rec["flops"] / rec["launches"],
                traffic=None)
    roof["kernels"] = {}
    for k, v in prof.items():
        kr = kernel_roofline(k, v, dtype)
        roof["kernels"][k] = {"ms": round(v["ms"], 3), "launches": v["launches"], "bound": kr["bound"],
                              "achieved": round(kr["achieved"], 2), "unit": kr["unit"], "frac": round(kr["frac"], 4)}
    return roof


def main_simulate(args):
    """Implicit-Euler simulations with ground contact (c5): one step of the bench is
    one time step of every simulation of the batch."""
    import numpy as np
    import torch

    from paper_2409_03807_amd import binding as rb
    from paper_2409_03807_amd import inputs as I

    p = I.config("c5")
    B = args.batch or 64
    prec = {"f64": rb.PREC_F64, "f32": rb.PREC_F32, "bf16": rb.PREC_BF16}[args.prec or "f32"]
    dtype = {rb.PREC_F64: "f64", rb.PREC_F32: "f32", rb.PREC_BF16: "bf16"}[prec]
    dev = "cuda:0"
    subspace = "plain (untrained Glorot) decoder"
    trained = None
    if args.train_epochs > 0:
        from paper_2409_03807_amd import learn
        trained = learn.train_dynamics_subspace(p, n_snap=args.train_snapshots, epochs=args.train_epochs,
                                                log=lambda *a, **k: print(*a, **k, file=sys.stderr))
        p.Ws, p.bs = trained["Ws"], trained["bs"]
        subspace = (f"decoder trained on {trained['train_snapshots']} static snapshots (gravity, {trained['poses']}), "
                    f"{args.train_epochs} epochs")
    ctx = rb.Context(p, prec=prec, max_batch=B)
    z0 = torch.zeros((B, p.r), dtype=torch.float64, device=dev)
    if trained is not None:
        z0[:] = trained["z_rest"]
    v0 = torch.tensor(I.swing_velocities(p, B), device=dev)
    # convergence floor: 1e-6 of the first step's start gradient (largest over the batch)
    x0, _ = ctx.decode(z0, want_J=False)
    free = torch.tensor(~p.pinned.astype(bool), device=dev)[None, :, None]
    qb1 = ((x0.double() - torch.tensor(p.X, device=dev)[None]) + p.dt * v0) * free
    _, g1, _ = ctx.energy_grad_hess(z0, qbar=qb1.contiguous(), dt=p.dt, flags=0)
    opts = rb.default_opts(abs_tol=1e-6 * float(g1.abs().max().item()))
    if args.warmup:
        ctx.simulate(z0, args.warmup, p.dt, v0=v0, opts=opts, want_traj=False)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.simulate(z0, 2, p.dt, v0=v0, opts=opts, want_traj=False)
    ctx.profile(False)
    roof = profile_line(ctx, dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.simulate(z0, args.steps, p.dt, v0=v0, opts=opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    failed = res["failed"].cpu().numpy()
    iters = res["iters"].cpu().numpy()
    conv = B * args.steps - int(failed.sum())
    x, _ = ctx.decode(res["traj"][-1].contiguous(), want_J=False)
    # how the simulations move: lowest point and mean end-face displacement every 20 steps
    tip = torch.tensor(I.face_vertices(p.X, 0, p.X[:, 0].max()), device=dev)
    Xd = torch.tensor(p.X, device=dev)
    motion = {"step": [], "min_y": [], "tip_disp_mean": []}
    for k in list(range(0, args.steps, 20)) + [args.steps - 1]:
        xk, _ = ctx.decode(res["traj"][k].contiguous(), want_J=False)
        xk = xk.double()
        motion["step"].append(k + 1)
        motion["min_y"].append(round(float(xk[..., 1].min().item()), 4))
        motion["tip_disp_mean"].append(round(float((xk[:, tip] - Xd[tip]).norm(dim=-1).mean().item()), 4))
    line = {
        "metric": "converged reduced solves/s at rel. grad 1e-6 (implicit-Euler steps)",
        "value": conv / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / max(args.steps, 1) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"c5: 50x10x10 beam, nv={p.nv}, ne={p.ne}, r={p.r}, hidden={p.hidden}, "
                               f"|S|={len(p.cub_elem)}, {B} simulations x {args.steps} steps, dt=1/60, ground "
                               f"y={p.ground_y} m, k_ground={p.k_ground:g} N/m, {subspace}, "
                               f"seeded swing velocities", "batch": B, "path": "simulate"},
        "failed_steps": int(failed.sum()), "mean_iters_per_step": float(iters.sum() / (B * max(args.steps, 1))),
        "min_y_last_step": float(x[..., 1].min().item()), "motion": motion,
        "subspace_training": None if trained is None else {
            k: trained[k] for k in ("snapshot_solve", "train_snapshots", "epochs", "loss", "train_seconds", "poses")},
        "roofline": roof, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main_learned(args):
    """The learned part at the c4 block: full-space snapshots, two-stage training,
    PCA and held-out reduced solves; value is the Lipschitz subspace's held-out
    converged solves/s (first lambda factor), beside the plain and PCA subspaces."""
    import numpy as np  # noqa: F401

    from paper_2409_03807_amd import learn

    t0 = time.perf_counter()
    out = learn.run(epochs1=args.epochs[0], epochs2=args.epochs[1], lam_rels=tuple(args.lam_rel),
                    log=lambda *a, **k: print(*a, **k, file=sys.stderr))
    total = time.perf_counter() - t0
    lip = f"lipschitz_{args.lam_rel[0]:g}"
    h = out["heldout"]
    line = {
        "metric": "converged reduced solves/s at rel. grad 1e-6, Lipschitz vs plain subspace",
        "value": h[lip]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": h[lip]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": out["workload"], "path": "learned", "subspace": lip,
                   "held_out": out["heldout_snapshots"], "train": out["train_snapshots"],
                   "epochs": out["epochs"], "lambda_ls": out["lambda_ls"]},
        "comparison": h, "snapshot_solve": out["snapshot_solve"], "pipeline_seconds": total,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
