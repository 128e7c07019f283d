"""Train and evaluate the learned warm start (python -m paper_2110_00733_amd.warmstart_train --help).

Training data are fields the solver itself produces: for each seeded synthetic 64^3 octet lattice
with manufacturing defects, solve_rve on the six unit Mandel macro strains gives the 36 channels
(6 cases x 6 components) of fluctuation strain the network learns to predict from phi.  Every
sample is drawn from its own seed (10000 + i):
  strut radius r with r^2 uniform between the radii of relative density 3% and 30% (density then
  spans about 3-30%), roughness amplitude U[0, 1.5] voxels with Gaussian std U[1, 3] voxels, and
  U{0..8} pores with lognormal radii of median U[1, 2] voxels (log-std 0.5).
Training runs entirely in the rve_nn kernels (forward, backward, Adam); evaluation compares
solve_rve from zero with solve_rve from the network's start at larger grids.
"""
from __future__ import annotations

import argparse
import functools
import json
import math
import os
import sys
import time

import numpy as np

import lattice_inputs as li

from . import solve, last_solve_info
from .nn import N_TARGET, WarmStartNet

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_octet64.npz")
C_SOLID = li.isotropic_mandel(1.0, 0.3)


@functools.lru_cache(maxsize=None)
def _radius_range(n: int):
    """Strut radii of the ideal octet at 3% and 30% relative density (density searches, cached)."""
    return li.octet_radius(n, 0.03), li.octet_radius(n, 0.30)


def sample_spec(i: int, seed0: int = 10000, n: int = 64) -> dict:
    u = li.uniforms(seed0 + i, 8)
    r_lo, r_hi = _radius_range(n)
    r = math.sqrt(r_lo ** 2 + (r_hi ** 2 - r_lo ** 2) * float(u[0]))
    return dict(radius=r, rough_amp=1.5 * float(u[1]), rough_sigma=1.0 + 2.0 * float(u[2]),
                n_pores=min(int(9 * float(u[3])), 8), pore_median_vox=1.0 + float(u[4]),
                seed_rough=2 * (seed0 + i) + 1, seed_pores=2 * (seed0 + i) + 2)


def make_phi(i: int, n: int = 64, seed0: int = 10000) -> np.ndarray:
    sp = sample_spec(i, seed0, n)
    phi, _ = li.octet_defect_phase_map(n, rho=0.0, radius=sp["radius"], rough_amp=sp["rough_amp"],
                                       rough_sigma=sp["rough_sigma"], n_pores=sp["n_pores"],
                                       pore_median_vox=sp["pore_median_vox"], pore_s=0.5,
                                       seed_rough=sp["seed_rough"], seed_pores=sp["seed_pores"])
    return phi


def log(msg):
    print(msg, flush=True)


def generate(count: int, n: int = 64, seed0: int = 10000, tol: float = 1e-5, device="cuda:0"):
    """phi [count, n, n, n] and targets [count, 36, n^3] (float32, device) plus per-sample stats."""
    import torch
    t0 = time.time()
    phis = np.empty((count, n, n, n), dtype=np.float32)
    for i in range(count):
        phis[i] = make_phi(i, n, seed0)
        if (i + 1) % 50 == 0 or i + 1 == count:
            log(f"  generated {i + 1}/{count} geometries ({time.time() - t0:.0f} s)")
    phi_t = torch.from_numpy(phis).to(device)
    targets = torch.empty((count, N_TARGET, n ** 3), dtype=torch.float32, device=device)
    E = li.unit_mandel_cases()
    iters = np.zeros((count, 6), dtype=np.int32)
    t1 = time.time()
    for i in range(count):
        out = solve(phi_t[i], C_SOLID, E, tol=tol, want_stress=False)
        targets[i].copy_(out["strain"].reshape(N_TARGET, n ** 3))
        iters[i] = out["iterations"]
        if (i + 1) % 50 == 0 or i + 1 == count:
            log(f"  solved {i + 1}/{count} ({time.time() - t1:.0f} s, mean iterations per case {iters[:i + 1].mean():.0f})")
    return phi_t, targets, dict(rho=phis.reshape(count, -1).mean(axis=1), iterations=iters, phis=phis,
                                gen_s=t1 - t0, solve_s=time.time() - t1)


def weight_sums(phis: np.ndarray, weight3) -> np.ndarray:
    """Per-sample sum of the loss voxel weights w0 + w1 phi + w2 [0 < phi < 1] (host bookkeeping)."""
    p = phis.reshape(phis.shape[0], -1).astype(np.float64)
    return (weight3[0] + weight3[1] * p + weight3[2] * ((p > 0) & (p < 1))).sum(axis=1)


def train(net: WarmStartNet, phi_t, targets, wsum, *, batch: int = 4, seconds: float = 300.0, lr: float = 1e-3,
          weight3=(0.1, 1.0, 0.0), n_val: int = 16, seed: int = 0):
    """Adam with a cosine learning rate over a step budget fitted to `seconds` after a timing epoch.
    The last n_val samples are held out for validation."""
    import torch
    count = phi_t.shape[0]
    n_train = count - n_val
    rng = np.random.default_rng(seed)
    hist = []

    def batches():
        perm = rng.permutation(n_train)
        for k in range(0, n_train - batch + 1, batch):
            yield perm[k:k + batch]

    def run_batch(idx, lr_now):
        ix = torch.from_numpy(np.sort(idx)).to(phi_t.device)
        inv = 1.0 / (N_TARGET * float(wsum[idx].sum()))
        part = net.train_step(phi_t.index_select(0, ix), targets.index_select(0, ix), inv, lr_now, weight3=weight3)
        return part, inv

    def val_loss():
        tot = 0.0
        for k in range(n_train, count, batch):
            idx = np.arange(k, min(k + batch, count))
            ix = torch.from_numpy(idx).to(phi_t.device)
            inv = 1.0 / (N_TARGET * float(wsum[idx].sum()))
            n = phi_t.shape[-1]
            B = net.pack(phi_t.index_select(0, ix), n)
            net.forward(B, n)
            part = net.loss(B, n, targets.index_select(0, ix), phi_t.index_select(0, ix), weight3, inv)
            tot += inv * float(part.cpu().numpy().sum()) * len(idx)
        return tot / max(1, count - n_train)

    steps_per_epoch = n_train // batch
    torch.cuda.synchronize()
    t0 = time.time()
    total_steps = None
    step = 0
    epoch = 0
    while True:
        losses = []
        for idx in batches():
            if total_steps is None:
                lr_now = lr
            else:
                lr_now = 0.5 * lr * (1 + math.cos(math.pi * min(1.0, step / total_steps)))
            part, inv = run_batch(idx, lr_now)
            losses.append((part, inv))
            step += 1
            if total_steps is not None and step >= total_steps:
                break
        tr = float(np.mean([inv * float(p.cpu().numpy().sum()) for p, inv in losses]))
        epoch += 1
        el = time.time() - t0
        if total_steps is None:
            total_steps = max(steps_per_epoch, int(seconds / el * steps_per_epoch))
            log(f"  epoch 1 took {el:.1f} s ({steps_per_epoch} steps): training {total_steps} steps")
        vl = val_loss() if n_val > 0 else float("nan")
        hist.append(dict(epoch=epoch, step=step, train_loss=tr, val_loss=vl, seconds=time.time() - t0))
        log(f"  epoch {epoch} step {step}/{total_steps} train {tr:.4e} val {vl:.4e} ({time.time() - t0:.0f} s)")
        if step >= total_steps:
            break
    return hist


def evaluate(net: WarmStartNet, phi, E, *, tol: float = 1e-6, precision: int = 0, repeats: int = 1, grid: int = 64):
    """Zero start against the network's start on one RVE: iterations, wall time to tolerance (network
    inference included), initial relative residual, C_eff agreement."""
    import torch
    res = {}
    for mode in ("zero", "learned"):
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eps0 = net.predict(phi, E, grid=grid) if mode == "learned" else None
            out = solve(phi, C_SOLID, E, tol=tol, precision=precision, eps0=eps0, want_stress=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        info = last_solve_info()
        res[mode] = dict(iterations=out["iterations"].tolist(), seconds=min(times),
                         initial_rel_residual=info["initial_rel_residual"].tolist(),
                         warm_rejected=info["warm_rejected"].tolist(), rel_residual=out["rel_residual"].tolist(),
                         eff_stress=out["eff_stress"].tolist())
    z, w = np.array(res["zero"]["eff_stress"]), np.array(res["learned"]["eff_stress"])
    res["eff_stress_rel_diff"] = float(np.max(np.abs(z - w)) / max(np.max(np.abs(z)), 1e-300))
    res["iteration_ratio"] = float(np.sum(res["learned"]["iterations"]) / max(1, np.sum(res["zero"]["iterations"])))
    res["time_ratio"] = res["learned"]["seconds"] / res["zero"]["seconds"]
    return res


def eval_suite(net, device="cuda:0", repeats=2, heldout=(), n=64, seed0=10000, sets=("128", "256")):
    """Held-out training-distribution geometries at the training grid, the 128^3 ideal octets
    (rho 5/10/20 %, 6 unit cases) and the 256^3 defect octet (uniaxial), the larger grids with the
    network run at their own resolution ("native") and at the training grid ("coarse")."""
    import torch
    out = {}

    def show(key, r):
        out[key] = r
        log(f"  {key}: iterations {sum(r['zero']['iterations'])} -> {sum(r['learned']['iterations'])}, "
            f"time {r['zero']['seconds']:.3f} -> {r['learned']['seconds']:.3f} s, "
            f"r0 {np.mean(r['learned']['initial_rel_residual']):.3f}, rejected {sum(r['learned']['warm_rejected'])}")

    for i in heldout:
        phi = torch.from_numpy(make_phi(i, n, seed0)).to(device)
        show(f"heldout{n}_{i}", evaluate(net, phi, li.unit_mandel_cases(), repeats=repeats, grid=n))
    for rho in (0.05, 0.10, 0.20) if "128" in sets else ():
        phi = torch.from_numpy(li.octet_phase_map(128, rho)[0]).to(device)
        for g in (128, 64):
            show(f"octet128_rho{rho:.2f}_{'native' if g == 128 else 'coarse'}",
                 evaluate(net, phi, li.unit_mandel_cases(), repeats=repeats, grid=g))
    phi = torch.from_numpy(li.octet_defect_phase_map(256)[0]).to(device) if "256" in sets else None
    for g in (256, 64) if "256" in sets else ():
        show(f"octet256_defects_{'native' if g == 256 else 'coarse'}",
             evaluate(net, phi, li.uniaxial_strain(1e-3), repeats=repeats, grid=g))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--count", type=int, default=334, help="geometries (6 unit-case solves each)")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--seed0", type=int, default=10000)
    ap.add_argument("--train-seconds", type=float, default=300.0)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight", default="0.1,1,0", help="loss voxel weight w0,w1,w2: w0 + w1 phi + w2 [0<phi<1]")
    ap.add_argument("--variants", default=None,
                    help="';'-separated loss weights to train one after another on the same data "
                         "(each saved as <out>.<k>.npz); overrides --weight")
    ap.add_argument("--n-val", type=int, default=16)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None, help="JSON file for the training history and evaluation")
    ap.add_argument("--eval-only", action="store_true", help="load --out and only evaluate")
    ap.add_argument("--eval", default="heldout,128,256", help="evaluation sets: heldout, 128, 256 (comma list)")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        sys.exit("the warm-start network trains on the GPU only")
    sets = set(args.eval.split(",")) if args.eval else set()
    heldout = range(args.count, args.count + 4) if "heldout" in sets else ()
    report = dict(args=vars(args), runs=[])
    if args.eval_only:
        net = WarmStartNet(seed=args.init_seed).load(args.out)
        report["runs"].append(dict(weights=args.out, eval=eval_suite(net, heldout=heldout, n=args.n, seed0=args.seed0,
                                                                      sets=sets)))
    else:
        log(f"generating {args.count} geometries at {args.n}^3 and solving 6 unit cases each")
        phi_t, targets, stats = generate(args.count, args.n, args.seed0)
        report["data"] = dict(count=args.count, fields=6 * args.count, rho_min=float(stats["rho"].min()),
                              rho_max=float(stats["rho"].max()), mean_iterations=float(stats["iterations"].mean()),
                              generate_s=stats["gen_s"], solve_s=stats["solve_s"])
        variants = args.variants.split(";") if args.variants else [args.weight]
        for k, v in enumerate(variants):
            w3 = tuple(float(x) for x in v.split(","))
            out = args.out if len(variants) == 1 else f"{os.path.splitext(args.out)[0]}.{k}.npz"
            net = WarmStartNet(seed=args.init_seed)
            log(f"training with loss weight {w3} for about {args.train_seconds:.0f} s")
            hist = train(net, phi_t, targets, weight_sums(stats["phis"], w3), batch=args.batch,
                         seconds=args.train_seconds, lr=args.lr, weight3=w3, n_val=args.n_val)
            meta = dict(grid=args.n, count=args.count, seed0=args.seed0, steps=hist[-1]["step"],
                        train_loss=hist[-1]["train_loss"], val_loss=hist[-1]["val_loss"], weight3=list(w3))
            os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
            net.save(out, meta)
            log(f"saved {out}")
            log("evaluating zero start against the learned start")
            report["runs"].append(dict(weights=out, weight3=list(w3), history=hist,
                                       eval=eval_suite(net, heldout=heldout, n=args.n, seed0=args.seed0, sets=sets)))
            del net
            torch.cuda.empty_cache()
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
