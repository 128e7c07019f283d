#!/usr/bin/env python3
"""Benchmark of the gfx950 Galerkin-FFT homogenization hot path on one GPU.

A step is one complete solve of the benchmark workload to the residual tolerance: FP64 right-hand
side, FP32 MINRES iterations (operator apply = 5 FFT/projection passes + Krylov updates), FP64 true
residual and refinement, post-processing.  Workload (default): a 256^3 octet-truss RVE at 15%
relative density with synthetic manufacturing defects (Gaussian-filtered roughness of amplitude
1.5 voxels, sigma 2 voxels; 200 lognormal pores, median radius 2 voxels), uniaxial macro strain
eps_11 = 1e-3, isotropic solid E = 1, nu = 0.3, empty phase of zero stiffness, tolerance 1e-6.

Prints one JSON line: voxel-iterations/s (value), wall time per solve (ms_per_step), the roofline
entry of the dominant kernel (HIP-event durations recorded on the solve stream inside the timed
solves) and the FP64 CPU oracle's rate on a bounded sample of the same problem.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import lattice_inputs as li
    if name == "octet256_defects":
        n = (256, 256, 256)
        phi, info = li.octet_defect_phase_map(n, 0.15)
        cfg = {"workload": "octet256_defects", "grid": list(n), "rho_target": 0.15, "rho_actual": info.rho_actual,
               "pores": info.n_pores, "roughness_amp_vox": 1.5, "roughness_sigma_vox": 2.0, "load": "eps11=1e-3",
               "load_cases": 1, "tol": 1e-6, "precision": "fp32-mixed"}
        E = li.uniaxial_strain(1e-3)[None]
    elif name == "octet128_6cases":
        n = (128, 128, 128)
        phi, _ = li.octet_phase_map(n, 0.10)
        cfg = {"workload": "octet128_6cases", "grid": list(n), "rho_target": 0.10,
               "rho_actual": float(phi.mean(dtype=np.float64)), "load": "6 unit Mandel strains", "load_cases": 6,
               "tol": 1e-6, "precision": "fp32-mixed"}
        E = np.eye(6)
    elif name == "octet32_fp64":
        n = (32, 32, 32)
        phi, _ = li.octet_phase_map(n, 0.10)
        cfg = {"workload": "octet32_fp64", "grid": list(n), "rho_target": 0.10,
               "rho_actual": float(phi.mean(dtype=np.float64)), "load": "eps11=1e-3", "load_cases": 1,
               "tol": 1e-8, "precision": "fp64"}
        E = li.uniaxial_strain(1e-3)[None]
    elif name == "octet_batch64":
        rv = li.heterogeneous_rves(64)
        phis = [li.octet_phase_map(nn, rho)[0] for nn, rho in rv]
        cfg = {"workload": "octet_batch64", "rves": 64, "sizes_per_axis": [32, 48, 64, 96], "rho_range": [0.03, 0.30],
               "seeds": "1000+i", "load": "6 unit Mandel strains per RVE", "load_cases": 6, "tol": 1e-6,
               "precision": "fp32-mixed", "voxels_total": int(sum(np.prod(nn) for nn, _ in rv))}
        return [tuple(nn) for nn, _ in rv], phis, np.eye(6), cfg
    elif name == "octet_j2":
        # the paper's nonlinear test: octet VA map at relative density 0.1 and about 15 voxels per strut
        # diameter (162^3), uniaxial compression to -10 % in 20 increments, lateral stress-free
        n = (162, 162, 162)
        cfg = {"workload": "octet_j2", "grid": list(n), "rho_target": 0.10, "representation": "VA",
               "material": {"young_MPa": 1700.0, "poisson": 0.4, "yield_MPa": 70.0},
               "load": "uniaxial compression eps11 -> -0.1, sigma_22..12 = 0", "increments": 20,
               "newton_tol": 5e-3, "lin_tol": 1e-6, "precision": "fp32-mixed"}
        return n, None, None, cfg
    elif name == "octet_modbfft":
        # the paper's solver comparison: plain-voxel octet at density 0.1 and about 20 voxels per strut
        # diameter (216^3, the paper's 215^3), uniaxial strain, tolerance 1e-6; MoDBFFT (FP64 CG) beside
        # the Galerkin MINRES solver on the same map
        n = (216, 216, 216)
        cfg = {"workload": "octet_modbfft", "grid": list(n), "rho_target": 0.10, "representation": "PV",
               "load": "eps11=1e-3", "tol": 1e-6, "alpha": "1e-4 E", "precision": "fp64"}
        return n, None, None, cfg
    elif name == "density_study":
        cfg = {"workload": "density_study", "rho_target": 0.1, "timed": "phase-field smoothening (PFS) of the "
               "octet at 108^3 coarse voxels on its 540^3 fine grid (ratio 5), FP64",
               "grid": [108, 108, 108], "ratio": 5, "fine": [540, 540, 540], "precision": "fp64"}
        return (108, 108, 108), None, None, cfg
    else:
        raise SystemExit(f"unknown workload {name}")
    return n, phi, E, cfg


def method_bytes_per_voxel_iteration(n2, elem):
    """The method's own HBM bytes per voxel and MINRES iteration, each operand counted once: the
    forward half (strain and phase map read, half spectrum written), the inverse half (half spectrum
    read, A v written) and the MINRES vector update (p, v_k, v_k-1, w_k-1, w_k-2, x read; v_k+1, w_k,
    x written).  The half spectrum holds 6 (n2/2 + 1) complex values per n2 voxels.  FP32 fields at
    n2 = 256: 316.4 B; FP64: 628.8 B."""
    spec = 6 * 2 * elem * (n2 // 2 + 1) / n2
    forward = 6 * elem + 4 + spec
    inverse = spec + 6 * elem
    update = 9 * 6 * elem
    return forward + inverse + update


def method_bytes_per_voxel_apply(n2, elem):
    """The operator apply alone (forward + inverse halves above): 100.4 B per voxel in FP32 at n2 = 256."""
    spec = 6 * 2 * elem * (n2 // 2 + 1) / n2
    return (6 * elem + 4 + spec) + (spec + 6 * elem)


def algorithmic_bytes(kind, n, nc, elem, plain_apply=False):
    """Bytes one launch of a pass must move (each of its operands read or written once), FP32/FP64
    fields.  plain_apply: the operator apply of a residual check, whose P5 writes A x without the
    Lanczos combination (no u_k, u_k-1 reads).  Summed over the passes of one iteration this is the implementation's operand traffic
    (406 B per voxel-iteration in FP32 at 256^3), about 1.3 times the method's own count above: the
    five-pass transform writes and reads the spectrum between passes."""
    n0, n1, n2 = n
    nv = n0 * n1 * n2
    spec = 6 * (n2 // 2 + 1) * n0 * n1 * 2 * elem
    field = 6 * nv * elem
    table = {
        "P1_stiffness_fft_axis2_alpha": field + 4 * nv + spec,   # u_k, phi -> spectrum
        "P2_fft_axis1": 2 * spec,
        "P3_fft_axis0_projection": 2 * spec,
        "P4_ifft_axis1": 2 * spec,
        "P5_ifft_axis2_lanczos": spec + (1 if plain_apply else 3) * field,  # spectrum, u_k, u_k-1 -> u_k+1
        # u_k, d_k-1, d_k-2 -> d_k every iteration; x read and written every third one (4 2/3 fields on average)
        "U2_direction_update": 14 * field // 3,
    }
    return table.get(kind, 0) * nc


KIND_TO_KERNEL = {  # profiler kind -> rocprofv3 kernel name prefix (FP32 fields)
    "P1_stiffness_fft_axis2_alpha": "rve::k_fwd_axis2<{t},",
    "P2_fft_axis1": "rve::k_axis1<{t},*,-1>",
    "P3_fft_axis0_projection": "rve::k_axis0_project_split<{t},",  # the variant the tuner keeps at 256^3
    "P4_ifft_axis1": "rve::k_axis1<{t},*,1>",
    "P5_ifft_axis2_lanczos": "rve::k_inv_axis2<{t},",
    "U2_direction_update": "rve::k_direction<{t},",
}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("rve_kernels.h", "rve_device.h", "rve_solver_kernels.h", "rve_solver.hip"):
        h.update(open(os.path.join(ROOT, "paper_2110_00733_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, kind, tname):
    """HBM bytes per launch of `kind` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or
    None when there is none or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_pmc_traffic.md")
    if not os.path.exists(path) or kind not in KIND_TO_KERNEL:
        return None
    txt = open(path).read()
    if f"kernel sources hash: {kernel_sources_hash()}" not in txt:
        return None
    data = json.loads(txt.split("machine-readable (bytes per launch): ", 1)[1].strip().splitlines()[0])
    pat = KIND_TO_KERNEL[kind].format(t=tname).replace(" ", "")
    for name, b in data.items():
        nm = name.replace(" ", "")
        if "*" in pat:
            head, tail = pat.split("*")
            if nm.startswith(head) and nm.endswith(tail):
                return b
        elif nm.startswith(pat):
            return b
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="octet256_defects")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3, help="timed oracle MINRES iterations")
    ap.add_argument("--cpu-warmup", type=int, default=1, help="untimed oracle MINRES iterations before them")
    ap.add_argument("--profile-steps", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--inner-floor", type=float, default=None,
                    help="FP32-mixed: relative reduction at which an inner FP32 sweep stops (library default 1e-5)")
    ap.add_argument("--precision", choices=["fp32-mixed", "fp64"], default=None,
                    help="override the workload's precision (fp64 = the plain FP64 GPU MINRES)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the wall-time comparison plain FP64 / FP32-mixed / learned warm start")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs each RVE on a single MI355X (load cases and "
              "RVEs are independent solves; a multi-GPU run would split them); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_00733_amd as rve
    import lattice_inputs as li

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    t0 = time.time()
    n, phi, E, cfg = workload(args.workload)
    if args.precision:
        cfg["precision"] = args.precision
    C1 = li.isotropic_mandel(1.0, 0.3)
    if cfg["workload"] == "octet_batch64":
        return bench_batch(args, n, phi, E, cfg, C1)
    if cfg["workload"] == "density_study":
        return bench_density(args, cfg)
    if cfg["workload"] == "octet_j2":
        return bench_j2(args, n, cfg)
    if cfg["workload"] == "octet_modbfft":
        return bench_modbfft(args, n, cfg, C1)
    log(f"workload {cfg['workload']} built in {time.time() - t0:.1f}s, rho={cfg['rho_actual']:.5f}")
    prec = rve.FP64 if cfg["precision"] == "fp64" else rve.FP32_MIXED
    d = torch.as_tensor(phi, device="cuda:0")
    ws = rve.Workspace()
    nvox = int(np.prod(n))
    nc = E.shape[0]

    extra = {}
    if args.inner_floor:
        extra["inner_floor"] = args.inner_floor
        cfg["inner_floor"] = args.inner_floor

    def one():
        return rve.solve(d, C1, E, tol=cfg["tol"], precision=prec, workspace=ws, want_stress=True, **extra)

    apply_ms = None  # tuned operator apply (P1-P5, no Lanczos work), own precision
    if not args.no_autotune:
        ta = time.time()
        precs = [rve.FP64] if prec == rve.FP64 else [rve.FP32_MIXED, rve.FP64]
        for p_ in precs:
            r_ = rve.autotune(n, n_cases=nc, precision=p_, workspace=ws)
            log(f"autotune prec={p_}: tiles {r_['tiles']} apply {r_['ms']:.3f} ms")
            if p_ == prec:
                apply_ms = r_["ms"]
        cfg["tiles"] = {"fp32": list(rve.tuned_tiles(n, rve.FP32_MIXED)[0]), "fp64": list(rve.tuned_tiles(n, rve.FP64)[0])}
        log(f"autotune took {time.time() - ta:.1f}s")

    for i in range(args.warmup):
        out = one()
        log(f"warmup {i}: status {out['status']} iters {out['iterations'].tolist()} res {out['rel_residual'].tolist()}")
    torch.cuda.synchronize()
    times, iters, res = [], [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        out = one()
        torch.cuda.synchronize()
        te = time.perf_counter()
        times.append(te - ts)
        iters.append(int(out["iterations"].sum()))
        res.append(float(out["rel_residual"].max()))
        log(f"step {i}: {1e3 * (te - ts):.1f} ms, iters {out['iterations'].tolist()}, res {out['rel_residual'].tolist()}")
    total_t = sum(times)
    value = nvox * sum(iters) / total_t
    ms_per_step = 1e3 * total_t / args.steps
    # per-kernel durations: the same solve with every launch bracketed by HIP events on the solve
    # stream (profiled solves launch directly instead of replaying the captured graph)
    rve.profile_reset()
    rve.profile_enable(True)
    tp = time.perf_counter()
    prof_iters = 0
    for i in range(args.profile_steps):
        out = one()
        prof_iters += int(out["iterations"].sum())
    torch.cuda.synchronize()
    log(f"profiled steps: {1e3 * (time.perf_counter() - tp) / max(args.profile_steps, 1):.1f} ms per solve")
    rve.profile_enable(False)
    prof = rve.profile_read()

    # roofline entry for the kernel with the largest share of the timed loop among those that do not
    # share the GPU with another kernel
    # Kinds of the solve's own precision run once per MINRES iteration; a launch of a chunk's iterations
    # after convergence returns at once, so the time of a working launch is the kind's total over the
    # iteration count (per case when the cases share a launch).  The other precision's kinds are the
    # FP64 residual applies of the FP32-mixed solver, every launch of which works.
    elem = 8 if prec == rve.FP64 else 4
    kernels = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        is64 = k.endswith("_f64")
        own = is64 == (elem == 8)
        work = prof_iters / nc if own else cnt
        if work <= 0:
            continue
        avg = ms / work
        ab = algorithmic_bytes(k[:-4] if is64 else k, n, nc, 8 if is64 else 4, plain_apply=not own)
        kernels[k] = {"total_ms": ms, "launches": cnt, "working_launches": round(work, 1), "avg_us": 1e3 * avg,
                      "alg_bytes": ab, "gbs": (ab / (avg * 1e-3) / 1e9) if ab else None}
    # U2 runs on a second stream beside the next iteration's P3 in the timed solve, so its time there
    # is shared and no profiler average of a lone launch describes it; the roofline kernel is the
    # longest of those that run alone.
    alone = [k for k in kernels if kernels[k]["alg_bytes"] and not k.startswith("U2_")]
    dom = max(alone, key=lambda k: kernels[k]["total_ms"]) if alone else None
    roof = None
    if dom:
        kd = kernels[dom]
        ach = kd["gbs"] or 0.0
        traffic = measured_traffic(cfg["workload"], dom.removesuffix("_f64"), "double" if prec == rve.FP64 else "float")
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_us": round(kd["avg_us"], 2),
                "launches": kd["launches"], "working_launches": kd["working_launches"],
                "alg_bytes_per_launch": kd["alg_bytes"]}
    log(json.dumps({k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()}))

    learned = None
    if not args.no_learned and cfg["workload"] == "octet256_defects" and prec == rve.FP32_MIXED:
        learned = learned_vs_plain(d, C1, E, cfg["tol"], ws, 1e-3 * ms_per_step, iters[-1])

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.time()
        secs = oracle.time_minres(n, phi, C1, iters=args.cpu_iters, warmup=args.cpu_warmup)
        cpu = {"value": nvox * args.cpu_iters / secs, "unit": "voxel-iterations/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_iters} timed FP64 MINRES iterations (operator apply + vector updates, "
                         f"{secs:.1f} s) of the CPU oracle on the same {n[0]}x{n[1]}x{n[2]} grid and phase map, "
                         f"zero start, after {args.cpu_warmup} untimed warm-up iteration(s); all vectors "
                         f"allocated and first touched before timing; the right-hand side is a seeded random "
                         f"field (an iteration's cost does not depend on it)"}
        log(f"cpu baseline {cpu['value']:.3e} voxel-it/s in {time.time() - t1:.1f}s wall")

    # whole-solve average: the MINRES iterations' algorithmic bytes over the timed wall time, which
    # also holds the setup, the FP64 refinement applies and the post-processing (so a lower bound)
    iter_kinds = ("P1_stiffness_fft_axis2_alpha", "P2_fft_axis1", "P3_fft_axis0_projection", "P4_ifft_axis1",
                  "P5_ifft_axis2_lanczos", "U2_direction_update")
    iter_bytes = sum(algorithmic_bytes(k, n, 1, elem) for k in iter_kinds)
    solve_gbs = iter_bytes * sum(iters) / total_t / 1e9
    # the method's own bytes (each operand once, the spectrum written and read once per half):
    # per voxel-iteration over the whole timed solve, and per voxel over the tuned plain apply
    bvi = method_bytes_per_voxel_iteration(n[2], elem)
    alg_iter_gbs = bvi * nvox * sum(iters) / total_t / 1e9
    bva = method_bytes_per_voxel_apply(n[2], elem)
    method = {"bytes_per_voxel_iteration": round(bvi, 2), "alg_iteration_gbs": round(alg_iter_gbs, 1),
              "alg_frac_iteration": round(alg_iter_gbs / HBM_PEAK_GBS, 4),
              "operand_bytes_per_voxel_iteration": round(iter_bytes / nvox, 2),
              "operand_over_method_bytes": round(iter_bytes / nvox / bvi, 3),
              "bytes_per_voxel_apply": round(bva, 2)}
    if apply_ms:
        method.update({"apply_ms": round(apply_ms, 4),
                       "alg_frac_apply": round(bva * nvox * nc / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    if roof is not None:
        roof.update({"alg_frac_iteration": method["alg_frac_iteration"],
                     "alg_frac_apply": method.get("alg_frac_apply")})
    cfg.update({"iterations_per_solve": iters[-1] // nc if nc else 0, "rel_residual": max(res),
                "wall_time_to_tol_ms": round(ms_per_step, 2), "minres_iterations_per_s": sum(iters) / total_t / nc,
                "solve_avg_operand_gbs": round(solve_gbs, 1),
                "solve_avg_operand_frac": round(solve_gbs / HBM_PEAK_GBS, 4),
                "method_bytes": method, "parallelism": "single-gpu"})
    line = {"metric": "voxel-iterations/s + wall time to 1e-6 residual at 256^3, learned vs plain",
            "value": value, "unit": "voxel-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prec == rve.FP64 else "f32", "data": "synthetic", "config": cfg,
            "roofline": roof, "cpu_baseline": cpu, "learned_vs_plain": learned, "kernels": kernels}
    print(json.dumps(line), flush=True)


def bench_modbfft(args, n, cfg, C1):
    """MoDBFFT solve (FP64 CG) on a plain-voxel octet: wall time to the tolerance, CG voxel-iterations/s,
    per-pass times of a second, timed solve, the roofline of the longest pass, the Galerkin solver on the
    same map for comparison, and the oracle's CG iterations as CPU baseline."""
    import torch
    import paper_2110_00733_amd as rve
    from paper_2110_00733_amd import density_study as ds, geometry as geo
    import lattice_inputs as li
    r = ds.target_radius(cfg["rho_target"])
    S = li.octet_struts(r)
    phi64, phi = geo.phase_map(n, S, geo.PV, want_f32=True)
    cfg.update({"radius": r, "rho_actual": float(phi64.mean().item()), "voxels_per_diameter": round(2 * r * n[0], 2)})
    del phi64
    E = li.uniaxial_strain(1e-3)
    ws = rve.Workspace()
    for _ in range(args.warmup):
        rve.solve_modbfft(phi, C1, E, tol=cfg["tol"], max_iter=200, workspace=ws, check=False)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    out = rve.solve_modbfft(phi, C1, E, tol=cfg["tol"], max_iter=5000, workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - ts
    its = out["iterations"]
    nvox = int(np.prod(n))
    log(f"modbfft: {its} iterations, {wall:.2f}s, residual {out['rel_residual']:.2e}, <s11> {out['eff_stress'][0]:.4e}")
    prof = rve.solve_modbfft(phi, C1, E, tol=cfg["tol"], max_iter=min(its, 60), workspace=ws, timed=True, check=False)
    K = n[2] // 2 + 1
    comp = n[0] * n[1] * K * 16  # one component of the FP64 half spectrum
    alg = {"expand": 3 * comp + 9 * comp, "ifft_axis0": 18 * comp, "ifft_axis1": 18 * comp,
           "axis2_stress": 18 * comp + 4 * nvox, "fft_axis1": 18 * comp, "fft_axis0": 18 * comp,
           "contract": 9 * comp + 3 * comp + 3 * comp, "cg_update": 4 * 3 * comp + 2 * 3 * comp + 2 * 3 * comp}
    kernels = {}
    for k, (ms, cnt) in prof["pass_ms"].items():
        if cnt:
            avg = ms / cnt
            kernels[k] = {"avg_us": round(1e3 * avg, 2), "launches": cnt, "alg_bytes": alg[k],
                          "gbs": round(alg[k] / (avg * 1e-3) / 1e9, 1)}
    log(json.dumps(kernels))
    dom = max((k for k in kernels if k != "cg_update"), key=lambda k: kernels[k]["avg_us"])
    kd = kernels[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4), "traffic": None, "avg_us": kd["avg_us"],
            "alg_bytes_per_launch": kd["alg_bytes"],
            "iteration_bytes": sum(alg.values()),
            "iteration_frac": round(sum(alg.values()) * its / wall / 1e9 / HBM_PEAK_GBS, 4)}
    # the Galerkin MINRES solver on the same plain-voxel map (FP32-mixed and FP64)
    gal = {}
    for name, prec in (("galerkin_fp32_mixed", rve.FP32_MIXED), ("galerkin_fp64", rve.FP64)):
        if not args.no_autotune:
            rve.autotune(n, n_cases=1, precision=prec)
        rve.solve(phi, C1, E[None], tol=cfg["tol"], precision=prec, workspace=ws, want_stress=False)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        o = rve.solve(phi, C1, E[None], tol=cfg["tol"], precision=prec, workspace=ws, want_stress=False)
        torch.cuda.synchronize()
        gal[name] = {"wall_s": round(time.perf_counter() - tg, 4), "iterations": int(o["iterations"][0]),
                     "eff_stress_11": float(o["eff_stress"][0][0])}
        log(f"{name}: {gal[name]}")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import modbfft as mb
        import oracle
        nn = (96, 96, 96)
        p96 = geo.phase_map(nn, S, geo.PV).cpu().numpy()
        tc = time.perf_counter()
        ro = mb.solve(nn, p96, C1, E, tol=1e-30, maxit=5)
        secs = time.perf_counter() - tc
        cpu = {"value": int(np.prod(nn)) * ro["iterations"] / secs, "unit": "voxel-iterations/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{ro['iterations']} preconditioned CG iterations of the MoDBFFT oracle (numpy FFTs, one "
                         f"thread per transform) on the same octet at 96^3, {secs:.1f} s including the right-hand "
                         f"side and the final fields"}
        log(f"cpu baseline {cpu['value']:.3e} voxel-it/s")
    cfg.update({"iterations": its, "rel_residual": out["rel_residual"], "wall_s": round(wall, 3),
                "eff_stress": [float(v) for v in out["eff_stress"]], "alpha_used": out["alpha"],
                "galerkin_same_map": gal, "parallelism": "single-gpu"})
    line = {"metric": "MoDBFFT voxel-iterations/s and wall time to 1e-6 (octet PV 216^3)",
            "value": nvox * its / wall, "unit": "voxel-iterations/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
            "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic", "config": cfg, "roofline": roof, "cpu_baseline": cpu,
            "kernels": kernels}
    print(json.dumps(line), flush=True)


def bench_j2(args, n, cfg):
    """Nonlinear J2 ramp: wall time of the whole stress-strain curve (Newton + MINRES, FP32-mixed),
    MINRES voxel-iterations per second over it, per-kernel times of a profiled two-increment ramp,
    the stress-strain curve, and the oracle's per-voxel-tangent MINRES iterations as CPU baseline."""
    import torch
    import paper_2110_00733_amd as rve
    from paper_2110_00733_amd import density_study as ds, geometry as geo
    import lattice_inputs as li
    m = cfg["material"]
    t0 = time.time()
    r = ds.target_radius(cfg["rho_target"])
    S = li.octet_struts(r)
    phi64, phi = geo.phase_map(n, S, geo.VA, want_f32=True)
    cfg["radius"] = r
    cfg["rho_actual"] = float(phi64.mean().item())
    cfg["voxels_per_diameter"] = round(2 * r * n[0], 2)
    del phi64
    log(f"octet VA map {n} radius {r:.6f} rho {cfg['rho_actual']:.5f} built in {time.time() - t0:.1f}s")
    prec = rve.FP32_MIXED if cfg["precision"] == "fp32-mixed" else rve.FP64
    if not args.no_autotune:
        rve.autotune(n, n_cases=1, precision=prec)
        if prec == rve.FP32_MIXED:
            rve.autotune(n, n_cases=1, precision=rve.FP64)
    ws = rve.Workspace()
    E = [-0.1, 0, 0, 0, 0, 0]
    kw = dict(increments=cfg["increments"], newton_tol=cfg["newton_tol"], lin_tol=cfg["lin_tol"], stress_mask=0b111110,
              macro_stress_final=np.zeros(6), precision=prec, workspace=ws, max_iter=5000)

    def ramp(first=None, ph=None, **over):
        """The ramp; first=k: only its first k increments (same increment size)."""
        k = dict(kw)
        k.update(over)
        Ek = E
        if first:
            Ek = [e * first / k["increments"] for e in E]
            k["increments"] = first
        return rve.solve_j2(phi if ph is None else ph, m["young_MPa"], m["poisson"], m["yield_MPa"], Ek, **k)

    for _ in range(args.warmup):
        ramp(first=2)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    out = ramp()
    torch.cuda.synchronize()
    wall = time.perf_counter() - ts
    hist = out["history"]
    minres = sum(h["minres"] for h in hist)
    nvox = int(np.prod(n))
    value = nvox * minres / wall
    curve = [[round(float(h["strain_mean"][0]), 5), round(float(h["stress_mean"][0]), 4)] for h in hist]
    log(f"ramp {wall:.2f}s, newton {[h['newton'] for h in hist]}, minres {minres}, status {out['status']}")
    # the paper's other densities at about 15 voxels per diameter (untimed curves)
    others = {}
    for rho_o, n_o in ((0.2, 108), (0.3, 90)):
        r_o = ds.target_radius(rho_o)
        p_o = geo.phase_map(n_o, li.octet_struts(r_o), geo.VA, want_f32=True)
        if not args.no_autotune:
            rve.autotune((n_o,) * 3, n_cases=1, precision=prec)
        to = time.perf_counter()
        o = ramp(ph=p_o[1])
        torch.cuda.synchronize()
        others[str(rho_o)] = {"grid": n_o, "radius": r_o, "rho_actual": float(p_o[0].mean().item()),
                              "voxels_per_diameter": round(2 * r_o * n_o, 2), "wall_s": round(time.perf_counter() - to, 3),
                              "newton_per_increment": [h["newton"] for h in o["history"]],
                              "minres_total": sum(h["minres"] for h in o["history"]), "status": o["status"],
                              "stress_strain_curve": [[round(float(h["strain_mean"][0]), 5),
                                                       round(float(h["stress_mean"][0]), 4)] for h in o["history"]]}
        log(f"rho {rho_o}: {others[str(rho_o)]['wall_s']}s newton {others[str(rho_o)]['newton_per_increment']}")
        del p_o
    cfg["other_densities"] = others
    # per-kernel: the first two increments again with every launch timed alone (no graphs)
    rve.profile_reset()
    rve.profile_enable(True)
    ramp(first=2)
    torch.cuda.synchronize()
    rve.profile_enable(False)
    prof = rve.profile_read()
    kernels = {}
    elem = 4 if prec == rve.FP32_MIXED else 8
    for k, (ms, cnt) in prof.items():
        if cnt == 0 or k[0] in "GM":
            continue
        is64 = k.endswith("_f64")
        own = is64 == (elem == 8)
        ab = algorithmic_bytes(k[:-4] if is64 else k, n, 1, 8 if is64 else 4, plain_apply=not own)
        if k.startswith("P1_"):
            ab += 7 * nvox * (8 if is64 else 4)  # the tangent's data
        avg = ms / cnt
        kernels[k] = {"total_ms": ms, "launches": cnt, "avg_us": 1e3 * avg, "alg_bytes": ab,
                      "gbs": (ab / (avg * 1e-3) / 1e9) if ab else None}
    log(json.dumps({k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()}))
    alone = [k for k in kernels if kernels[k]["alg_bytes"] and not k.startswith("U2_")]
    dom = max(alone, key=lambda k: kernels[k]["total_ms"])
    kd = kernels[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(kd["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4), "traffic": None, "avg_us": round(kd["avg_us"], 2),
            "alg_bytes_per_launch": kd["alg_bytes"]}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import plasticity as opl
        nn = (96, 96, 96)
        p96 = geo.phase_map(nn, S, geo.VA).cpu().numpy()
        eps = np.zeros((6,) + nn)
        eps[0] = -0.05
        sig, Ct, _, _ = opl.return_map(eps, np.zeros_like(eps), p96, m["young_MPa"], m["poisson"], m["yield_MPa"])
        b = -oracle.project(nn, sig, stress_mask=0b111110)
        tc = time.perf_counter()
        opl.minres_tangent(nn, Ct, b, 1e-30, 3, stress_mask=0b111110)
        secs = time.perf_counter() - tc
        cpu = {"value": int(np.prod(nn)) * 3 / secs, "unit": "voxel-iterations/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"3 FP64 MINRES iterations with the per-voxel tangent (a 6x6 matrix per voxel) of the CPU "
                         f"oracle on the same octet at 96^3, plastic state at 5 % compression, {secs:.1f} s "
                         f"including setup and the final true-residual apply"}
        log(f"cpu baseline {cpu['value']:.3e} voxel-it/s")
    cfg.update({"wall_s": round(wall, 3), "newton_per_increment": [h["newton"] for h in hist],
                "minres_per_increment": [h["minres"] for h in hist], "minres_total": minres,
                "status": out["status"], "stress_strain_curve": curve,
                "plastic_voxel_fraction": float((out["ep_acc"] > 0).double().mean().item()),
                "parallelism": "single-gpu"})
    line = {"metric": "J2 stress-strain curve: MINRES voxel-iterations/s and wall time (20 increments)",
            "value": value, "unit": "voxel-iterations/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
            "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec == rve.FP32_MIXED else "f64", "data": "synthetic", "config": cfg,
            "roofline": roof, "cpu_baseline": cpu, "kernels": kernels}
    print(json.dumps(line), flush=True)


def bench_density(args, cfg):
    """Surface-smoothening study (densities of PV / VFG / VA / PFS / CS over seven grids, untimed),
    then the timed phase-field pipeline at one density-study size: fine voxels per second, per-kernel
    times from the library's event timing, the roofline of the longest kernel and the oracle on a
    432^3 fine grid as CPU baseline."""
    import torch
    import paper_2110_00733_amd as rve
    from paper_2110_00733_amd import density_study as ds, geometry as geo
    import lattice_inputs as li
    t0 = time.time()
    study = ds.run(cfg["rho_target"], log=log)
    log(f"density study in {time.time() - t0:.1f}s, radius {study['radius']:.6f}")
    S = li.octet_struts(study["radius"])
    n, ratio = tuple(cfg["grid"]), cfg["ratio"]
    m = [v * ratio for v in n]
    ws = rve.Workspace()
    for _ in range(max(args.warmup, 1)):
        geo.phase_field(n, S, ratio, workspace=ws)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        geo.phase_field(n, S, ratio, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - ts) / args.steps
    fine = int(np.prod(m))
    rve.profile_reset()
    rve.profile_enable(True)
    for _ in range(max(args.profile_steps, 1)):
        geo.phase_field(n, S, ratio, workspace=ws)
    torch.cuda.synchronize()
    rve.profile_enable(False)
    prof = {k: v for k, v in rve.profile_read().items() if k.startswith("G") and v[1] > 0}
    spec = m[0] * m[1] * (m[2] // 2 + 1) * 16
    coarse = int(np.prod(n)) * 16  # phi and the value before the threshold, FP64
    alg = {"G1_source_fft_axis2": spec, "G2_fft_axis1": 2 * spec, "G3_fft_axis0_helmholtz": 2 * spec,
           "G4_ifft_axis1": 2 * spec, "G5_ifft_axis2_coarsen": spec + coarse}
    kernels = {}
    for k, (ms, cnt) in prof.items():
        avg = ms / cnt
        kernels[k] = {"avg_us": round(1e3 * avg, 2), "launches": cnt, "alg_bytes": alg[k],
                      "gbs": round(alg[k] / (avg * 1e-3) / 1e9, 1)}
    log(json.dumps(kernels))
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    kd = kernels[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4), "traffic": None, "avg_us": kd["avg_us"],
            "alg_bytes_per_launch": kd["alg_bytes"],
            "pipeline_frac": round(sum(alg.values()) / dt / 1e9 / HBM_PEAK_GBS, 4)}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import geometry as og
        import oracle
        tc = time.time()
        og.phase_field(54, S, 8)
        secs = time.time() - tc
        cpu = {"value": 432 ** 3 / secs, "unit": "fine voxels/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"one oracle phase-field smoothening of the same octet at 54^3 coarse voxels on a 432^3 "
                         f"fine grid (ratio 8; C distance loops on all cores, numpy FFTs), {secs:.1f} s"}
        log(f"cpu baseline {cpu['value']:.3e} fine voxels/s")
    cfg.update({"radius": study["radius"], "study": study["rows"], "study_seconds": study["seconds"],
                "ms_per_call": round(1e3 * dt, 3), "parallelism": "single-gpu"})
    line = {"metric": "phase-field smoothening fine voxels/s (density study)", "value": fine / dt,
            "unit": "fine voxels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic", "config": cfg, "roofline": roof, "cpu_baseline": cpu,
            "kernels": kernels}
    print(json.dumps(line), flush=True)


def learned_vs_plain(d, C1, E, tol, ws, fp32_s, fp32_iters, repeats=2):
    """Wall time to the tolerance for the plain FP64 GPU MINRES (zero start), the FP32-mixed solver
    (zero start, the timed steps) and the FP32-mixed solver started from the trained network's
    prediction (network inference, prolongation and projection included)."""
    import torch
    import paper_2110_00733_amd as rve
    from paper_2110_00733_amd.nn import WarmStartNet
    from paper_2110_00733_amd.warmstart_train import DEFAULT_WEIGHTS

    def timed(fn):
        best, out = None, None
        for _ in range(repeats):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        return best, out

    t64, o64 = timed(lambda: rve.solve(d, C1, E, tol=tol, precision=rve.FP64, workspace=ws, want_stress=True))
    res = {"plain_fp64_s": round(t64, 4), "plain_fp64_iterations": int(o64["iterations"].sum()),
           "fp32_mixed_s": round(fp32_s, 4), "fp32_mixed_iterations": int(fp32_iters)}
    if not os.path.exists(DEFAULT_WEIGHTS):
        res["learned"] = None
        return res
    net = WarmStartNet().load(DEFAULT_WEIGHTS)
    tl, ol = timed(lambda: rve.solve(d, C1, E, tol=tol, workspace=ws, want_stress=True, eps0=net.predict(d, E, grid=64)))
    info = rve.last_solve_info()
    torch.cuda.synchronize()
    ti = time.perf_counter()
    net.predict(d, E, grid=64)
    torch.cuda.synchronize()
    res.update({"learned_fp32_mixed_s": round(tl, 4), "learned_iterations": int(ol["iterations"].sum()),
                "learned_inference_s": round(time.perf_counter() - ti, 4),
                "learned_initial_rel_residual": float(info["initial_rel_residual"][0]),
                "learned_start_rejected": bool(info["warm_rejected"][0]),
                "eff_stress_rel_diff_learned_vs_fp64": float(np.max(np.abs(ol["eff_stress"] - o64["eff_stress"])) /
                                                             np.max(np.abs(o64["eff_stress"]))),
                "speedup_fp32_mixed_vs_plain_fp64": round(t64 / fp32_s, 3),
                "speedup_learned_vs_plain_fp64": round(t64 / tl, 3),
                "speedup_learned_vs_fp32_mixed": round(fp32_s / tl, 3),
                "weights": os.path.relpath(DEFAULT_WEIGHTS, ROOT)})
    log("learned vs plain: " + json.dumps(res))
    return res


def bench_batch(args, grids, phis, E, cfg, C1):
    """Heterogeneous batch: every RVE with 6 unit load cases, one solve_rve_batch call (RVEs grouped by
    grid, the groups' MINRES iterations in one captured graph)."""
    import torch
    import paper_2110_00733_amd as rve
    rves = [(torch.as_tensor(p, device="cuda:0"), E) for p in phis]
    ws = rve.Workspace()
    if not args.no_autotune:
        ta = time.time()
        prec_t = rve.FP64 if cfg["precision"] == "fp64" else rve.FP32_MIXED
        for g in sorted(set(grids)):
            rve.autotune(g, n_cases=E.shape[0], precision=prec_t, workspace=ws)
        cfg["autotuned_grids"] = len(set(grids))
        log(f"autotuned {len(set(grids))} grids in {time.time() - ta:.1f}s")

    prec = rve.FP64 if cfg["precision"] == "fp64" else rve.FP32_MIXED

    def one():
        return rve.solve_batch(rves, C1, tol=cfg["tol"], precision=prec, workspace=ws)

    for i in range(args.warmup):
        out = one()
        log(f"warmup {i}: status {out['status']}")
    times, tot_vit, its = [], 0, None
    for i in range(args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        out = one()
        torch.cuda.synchronize()
        te = time.perf_counter()
        times.append(te - ts)
        tot_vit += sum(int(np.prod(g)) * int(r["iterations"].sum()) for g, r in zip(grids, out["results"]))
        its = [r["iterations"].tolist() for r in out["results"]]
        log(f"step {i}: {1e3 * (te - ts):.1f} ms, status {out['status']}")
    total_t = sum(times)
    cfg.update({"per_rve_iterations": its, "rve_grids": [list(g) for g in grids],
                "max_rel_residual": max(float(r["rel_residual"].max()) for r in out["results"])})
    line = {"metric": "voxel-iterations/s + wall time to 1e-6 residual at 256^3, learned vs plain",
            "value": tot_vit / total_t, "unit": "voxel-iterations/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * total_t / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == rve.FP64 else "f32", "data": "synthetic",
            "config": cfg,
            "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
