"""The learned part on one GPU, end to end, every step in librs:

1. snapshots: full-space equilibria of random twist and bend loads on the 16^3
   block (rs_full_solve), split into training and held-out sets;
2. the supervised construction (Sec. 3.2, Eq. form-vanilla-supervised-construction):
   encoder and decoder trained on the training snapshots with the reconstruction
   loss (rs_trainer_*);
3. Lipschitz optimisation (Sec. 4.2, Eq. form-unconstrained-lipschitz-optimization):
   from the same start, one branch continues with the reconstruction loss alone
   (the plain, "vanilla" subspace) and one with the reconstruction loss plus
   lambda times the Lipschitz loss over pairs of encoded training snapshots;
4. the PCA subspace of the same snapshots (rs_pca) as the linear baseline;
5. held-out reduced solves (rs_newton_solve) of every subspace from the
   reduced coordinates of the rest shape: converged solves per second, Newton
   iterations, and the subspace error against the held-out full-space
   equilibria; with the max-pair estimate of the Lipschitz constant of the
   cubature elastic Hessian over encoded held-out pairs (the paper's Table 1
   statistic).

This module orchestrates library calls (device buffers, seeds, loops); it holds
none of the method's arithmetic."""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import binding as rb
from . import inputs as I

DEV = "cuda:0"


def _t64(a):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def generate_snapshots(ctx, targets, force, chunk=256, opts=None, log=print):
    """Full-space equilibria (N x nv x 3 displacements, float64 device) of the load
    cases, solved in batches of `chunk` from the rest shape."""
    N = (targets if targets is not None else force).shape[0]
    out = torch.empty((N, ctx.nv, 3), dtype=torch.float64, device=DEV)
    status = torch.empty(N, dtype=torch.int32, device=DEV)
    iters = torch.empty(N, dtype=torch.int32, device=DEV)
    t0 = time.time()
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        res = ctx.full_solve(torch.zeros((c1 - c0, ctx.nv, 3), dtype=torch.float64, device=DEV),
                             None if targets is None else _t64(targets[c0:c1]),
                             None if force is None else _t64(force[c0:c1]), opts)
        out[c0:c1] = res["u"]
        status[c0:c1] = res["status"]
        iters[c0:c1] = res["iters"]
        torch.cuda.synchronize()
        log(f"snapshots {c1}/{N}: {time.time() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    it = iters.cpu().numpy()
    return out, dict(seconds=time.time() - t0, converged=int((st == rb.CONVERGED).sum()), n=N,
                     mean_iters=float(it.mean()), max_iters=int(it.max()), status=st)


def _epoch_indices(rng, n, B):
    perm = rng.permutation(n).astype(np.int32)
    return [torch.tensor(perm[i:i + B], device=DEV) for i in range(0, n - B + 1, B)]


def run_epochs(tr, store, n, epochs, B, lr, rng, lam=0.0, n_pairs=0, log=print, tag=""):
    """Adam epochs over the store's rows with a cosine learning-rate decay from lr
    to 0 over the stage; returns the last epoch's mean (L_C, L_LS)."""
    acc = torch.zeros(2, dtype=torch.float64, device=DEV)
    losses = torch.empty(2, dtype=torch.float64, device=DEV)
    last = (float("nan"), float("nan"))
    steps = epochs * (n // B)
    step = 0
    for ep in range(epochs):
        acc.zero_()
        batches = _epoch_indices(rng, n, B)
        for idx in batches:
            tr.grad(store, idx, lambda_ls=lam, n_pairs=n_pairs, losses=losses)
            tr.adam(lr * 0.5 * (1.0 + math.cos(math.pi * step / max(steps, 1))))
            step += 1
            acc += losses
        if ep == epochs - 1 or ep % max(1, epochs // 5) == 0:
            v = (acc / len(batches)).cpu().numpy()
            last = (float(v[0]), float(v[1]))
            log(f"{tag} epoch {ep + 1}/{epochs}: L_C {v[0]:.4e} L_LS {v[1]:.4e}", flush=True)
    return last


def heldout_solves(ctx, z0, targets, force, reps=5, solver="newton"):
    """Solves (projective Newton or L-BFGS) of the held-out loads from z0: converged
    count, mean iterations, median wall time of `reps` calls (after one warm-up),
    and the final z."""
    B = targets.shape[0]
    tg, fo = _t64(targets), _t64(force)
    z0b = z0.reshape(1, -1).expand(B, -1).contiguous()
    solve = ctx.newton_solve if solver == "newton" else ctx.lbfgs_solve
    res = solve(z0b, tg, fo)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = solve(z0b, tg, fo)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = res["status"].cpu().numpy()
    it = res["iters"].cpu().numpy()
    ms = float(np.median(times)) * 1e3
    conv = int((st == rb.CONVERGED).sum())
    return dict(converged=conv, items=B, mean_iters=float(it.mean()), median_iters=float(np.median(it)),
                ms=ms, solves_per_s=conv / (ms * 1e-3), status_counts={int(k): int(v) for k, v in
                                                                      zip(*np.unique(st, return_counts=True))}), res


def subspace_error(ctx, z, u_full):
    """mean over items of |u_red - u_full|_2 / |u_full|_2 (a reported statistic)."""
    x, _ = ctx.decode(z, want_J=False)
    u_red = (x.double().cpu().numpy() - ctx.p.X[None]).reshape(len(z), -1)
    uf = u_full.reshape(len(z), -1)
    return float(np.mean(np.linalg.norm(u_red - uf, axis=1) / np.maximum(np.linalg.norm(uf, axis=1), 1e-300)))


def lipschitz_estimate(ctx, z):
    """max-pair and mean estimates of the Lipschitz constant of the cubature elastic
    Hessian over disjoint pairs of the latent points z (Eq. form-H-Lipschitz-estimation)."""
    P = len(z) // 2
    res = ctx.lipschitz_loss(z[0:2 * P:2].contiguous(), z[1:2 * P:2].contiguous(), want_per_pair=True)
    per = res["per_pair"].cpu().numpy()
    return dict(lip_max=float(res["lip_max"].item()), lip_mean=float(np.sqrt(per).mean()))


def run(n_snap=2048, n_test=256, epochs1=100, epochs2=100, batch=128, pairs=64, lr1=1e-3, lr2=3e-4,
        lam_rels=(1.0,), enc_hidden=(256, 256), pca_iters=60, reps=5, log=print):
    """The whole learned part at the c4 workload; returns a dict of results.
    Snapshots whose full-space solve did not converge are left out of both sets.
    lam_rels: one Lipschitz branch per value, lambda_LS = lam_rel times the ratio
    of the reconstruction loss to the Lipschitz loss at the end of stage 1."""
    torch.cuda.set_device(0)
    p = I.config("c4")
    out = dict(workload="c4: 16^3 block, nv=4913, ne=20480, n=14739, r=12, decoder 4x256 ELU, "
                        "|S|=512 (weights U[20,60]), twist U[-180,180] deg + bend U[0,2000] N",
               snapshots=n_snap, held_out=n_test, epochs=[epochs1, epochs2], batch=batch, pairs=pairs)
    ctx = rb.Context(p, prec=rb.PREC_F32, max_batch=max(2 * batch, 256))
    # 1. snapshots
    twist, targets, force = I.snapshot_loads(p, n_snap)
    u, info = generate_snapshots(ctx, targets, force, log=log)
    out["snapshot_solve"] = info
    tr_idx, te_idx = I.heldout_split(n_snap, n_test)
    ok = info.pop("status") == rb.CONVERGED
    tr_idx, te_idx = tr_idx[ok[tr_idx]], te_idx[ok[te_idx]]
    out["train_snapshots"], out["heldout_snapshots"] = int(len(tr_idx)), int(len(te_idx))
    n_test = len(te_idx)
    store = u.reshape(n_snap, -1)[torch.tensor(tr_idx, device=DEV)].float().contiguous()
    u_test = u[torch.tensor(te_idx, device=DEV)].cpu().numpy()
    n_train = len(tr_idx)
    # 2. stage 1: reconstruction loss
    eW, eb = I.glorot_decoder(p.n, list(enc_hidden), p.r, seed=I.SEED_ENCODER)
    tr = rb.Trainer(ctx, eW, eb, p.Ws, p.bs, max_batch=batch)
    rng = np.random.default_rng(7)
    t0 = time.time()
    out["stage1_loss"] = run_epochs(tr, store, n_train, epochs1, batch, lr1, rng, log=log, tag="stage 1")
    torch.cuda.synchronize()
    out["stage1_seconds"] = time.time() - t0
    enc1, dec1 = (a.double().cpu().numpy() for a in tr.params())
    # the Lipschitz weight: lam_rel times the ratio of the two losses on a training batch
    idx0 = torch.tensor(np.arange(batch, dtype=np.int32), device=DEV)
    l0, _, _ = tr.grad(store, idx0, lambda_ls=1.0, n_pairs=pairs)
    l0 = l0.cpu().numpy()
    ratio = float(l0[0] / max(l0[1], 1e-300))
    branches = [("plain", 0.0)] + [(f"lipschitz_{lr:g}", lr * ratio) for lr in lam_rels]
    out["lambda_ls"] = {name: lam_b for name, lam_b in branches}
    tr.close()
    # 3. the branches from the stage-1 parameters
    ctxs, encs = {}, {}
    for name, lam_b in branches:
        c_b = rb.Context(p, prec=rb.PREC_F32, max_batch=max(2 * batch, 256))
        parts = c_b.unpack_params(torch.tensor(dec1))
        e_parts = []
        off = 0
        for W, b in zip(eW, eb):
            e_parts.append((enc1[off:off + W.size].reshape(W.shape), enc1[off + W.size:off + W.size + b.size]))
            off += W.size + b.size
        t_b = rb.Trainer(c_b, [w for w, _ in e_parts], [b for _, b in e_parts], [W.numpy() for W, _ in parts],
                         [b.numpy() for _, b in parts], max_batch=batch)
        rng_b = np.random.default_rng(8)
        t0 = time.time()
        out[f"{name}_loss"] = run_epochs(t_b, store, n_train, epochs2, batch, lr2, rng_b, lam=lam_b,
                                         n_pairs=pairs if lam_b > 0 else 0, log=log, tag=name)
        torch.cuda.synchronize()
        out[f"{name}_seconds"] = time.time() - t0
        # held-out reconstruction loss
        te_store = torch.tensor(u_test.reshape(n_test, -1), dtype=torch.float32, device=DEV)
        lt, _, _ = t_b.grad(te_store, None, B=min(batch, n_test))
        out[f"{name}_heldout_recon"] = float(lt[0].item())
        zr = t_b.encode(torch.zeros((1, p.n), dtype=torch.float32, device=DEV))[0]
        zt = t_b.encode(te_store)
        encs[name] = (zr, zt)
        ctxs[name] = c_b
        t_b.close()
    # 4. PCA of the training snapshots
    W, mean, ev, zr = ctx.pca(store, p.r, iters=pca_iters)
    Wn, mn = W.cpu().numpy(), mean.cpu().numpy()
    pp = I.Problem(**{**p.__dict__})
    pp.Ws, pp.bs, pp.hidden = [Wn], [mn], []
    ctx_pca = rb.Context(pp, prec=rb.PREC_F32, max_batch=max(2 * batch, 256))
    # 5. held-out solves from the reduced coordinates of the rest shape
    tg_te, fo_te = targets[te_idx], force[te_idx]
    res = {}
    for name in [b for b, _ in branches] + ["pca"]:
        c_e = ctx_pca if name == "pca" else ctxs[name]
        z0 = zr if name == "pca" else encs[name][0]
        r_e, sol = heldout_solves(c_e, z0, tg_te, fo_te, reps=reps)
        r_e["subspace_error"] = subspace_error(c_e, sol["z"], u_test)
        r_l, sol_l = heldout_solves(c_e, z0, tg_te, fo_te, reps=reps, solver="lbfgs")
        r_e["lbfgs"] = {k: r_l[k] for k in ("converged", "mean_iters", "median_iters", "ms", "solves_per_s",
                                             "status_counts")}
        if name != "pca":
            r_e.update(lipschitz_estimate(c_e, encs[name][1]))
        res[name] = r_e
        log(f"held-out {name}: {r_e}", flush=True)
    out["heldout"] = res
    return out


def train_dynamics_subspace(p, n_snap=512, epochs=300, batch=128, lr=1e-3, bend_deg=45.0, twist_deg=60.0,
                            enc_hidden=(256, 256), log=print):
    """A subspace for the implicit-Euler workload: full-space static equilibria of
    the beam under gravity with its end face held by penalty targets in random
    rigid poses (bends about y and z, twist about x; rs_full_solve), then the
    supervised construction with the reconstruction loss alone (Sec. 3.2).
    Returns the trained decoder (Ws, bs), the rest shape's reduced coordinates
    and the snapshot and training statistics."""
    torch.cuda.set_device(0)
    q = I.end_pose_problem(p)
    ctx = rb.Context(q, prec=rb.PREC_F32, max_batch=max(2 * batch, 256))
    targets = I.end_pose_targets(p, q.target_vtx, n_snap, bend_deg=bend_deg, twist_deg=twist_deg)
    u, info = generate_snapshots(ctx, targets, None, log=log)
    ok = info.pop("status") == rb.CONVERGED
    idx = torch.tensor(np.nonzero(ok)[0], device=DEV)
    store = u.reshape(n_snap, -1)[idx].float().contiguous()
    n = len(idx)
    eW, eb = I.glorot_decoder(p.n, list(enc_hidden), p.r, seed=I.SEED_ENCODER)
    tr = rb.Trainer(ctx, eW, eb, p.Ws, p.bs, max_batch=batch)
    t0 = time.time()
    loss = run_epochs(tr, store, n, epochs, min(batch, n), lr, np.random.default_rng(7), log=log, tag="c5 subspace")
    torch.cuda.synchronize()
    seconds = time.time() - t0
    z_rest = tr.encode(torch.zeros((1, p.n), dtype=torch.float32, device=DEV))[0].double()
    _, dec = tr.params()
    parts = ctx.unpack_params(dec.double().cpu())
    tr.close()
    return dict(Ws=[W.numpy() for W, _ in parts], bs=[b.numpy() for _, b in parts], z_rest=z_rest,
                snapshot_solve=info, train_snapshots=n, epochs=epochs, loss=loss[0], train_seconds=seconds,
                poses=f"end face bent U[-{bend_deg:g}, {bend_deg:g}] deg about y and z, twisted "
                      f"U[-{twist_deg:g}, {twist_deg:g}] deg")
