"""Density misrepresentation of the surface-smoothening approaches (section "Analysis of the surface
smoothening approaches", figure calcdens): relative density of the octet-truss phase map built by
plain voxels (PV), Voigt fine grid (VFG), Voigt analytic (VA), phase-field smoothening (PFS) and
combined smoothening (CS), against the target density, over grids of about 5 to 25 voxels per strut
diameter.  Every map is computed by the library's kernels (include/rve_geometry.h); the densities
are voxel means of those maps.

Settings of the paper: target density 0.1; VA width one voxel; phase field with eps = 1, ell = half a
coarse voxel, threshold 0.05, on a fine grid of ratio fine voxels per coarse voxel; VFG with the same
ratio as sub-grid.  The paper keeps the fine grid near a fixed size; here ratio * n stays near 540
and is 5-smooth (the coarse lengths are 5-smooth too: 270 stands in for the paper's 269).
The target radius comes from a VFG map of 1024^3 points (256^3 voxels, 4^3 sub-points each).

Run: python -m paper_2110_00733_amd.density_study [--rho 0.1] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

# (coarse voxels per axis, fine voxels per coarse voxel): fine grids 432-540
GRIDS = ((54, 10), (81, 6), (108, 5), (135, 4), (162, 3), (216, 2), (270, 2))


def _octet(r):
    import lattice_inputs as li
    return li.octet_struts(r)


def density(phi) -> float:
    return float(phi.double().mean().item())


def target_radius(rho: float = 0.1, n_ref: int = 256, sub: int = 4, tol: float = 1e-7) -> float:
    """Strut radius at which the octet's VFG density on n_ref^3 voxels x sub^3 points equals rho
    (bisection; the density grows monotonically with the radius)."""
    from . import geometry as geo
    lo, hi = 0.0, 0.25
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if density(geo.phase_map(n_ref, _octet(mid), geo.VFG, sub=sub)) < rho:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def run(rho: float = 0.1, grids=GRIDS, radius: float | None = None, log=print) -> dict:
    import torch
    from . import geometry as geo
    t0 = time.time()
    r = target_radius(rho) if radius is None else float(radius)
    S = _octet(r)
    rows = []
    for n, ratio in grids:
        pv = geo.phase_map(n, S, geo.PV)
        vfg = geo.phase_map(n, S, geo.VFG, sub=ratio)
        va = geo.phase_map(n, S, geo.VA)
        pfs, pfs_raw = geo.phase_field(n, S, ratio)
        cs, cs_raw = geo.phase_field(n, S, ratio, source=va)
        row = {"n": n, "ratio": ratio, "fine": n * ratio, "voxels_per_diameter": round(2 * r * n, 2),
               "PV": density(pv), "VFG": density(vfg), "VA": density(va), "PFS": density(pfs),
               "CS": density(cs), "PFS_before_threshold": density(pfs_raw), "CS_before_threshold": density(cs_raw)}
        row["rel_err"] = {k: (row[k] - rho) / rho for k in ("PV", "VFG", "VA", "PFS", "CS")}
        rows.append(row)
        log(f"n={n:3d} ratio={ratio:2d} d/h={row['voxels_per_diameter']:5.2f}  " +
            "  ".join(f"{k} {100 * v:+.3f}%" for k, v in row["rel_err"].items()))
        del pv, vfg, va, pfs, pfs_raw, cs, cs_raw
        torch.cuda.empty_cache()
    return {"rho_target": rho, "radius": r, "reference": "VFG 256^3 x 4^3 points", "rows": rows,
            "seconds": round(time.time() - t0, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rho", type=float, default=0.1)
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    out = run(args.rho)
    txt = json.dumps(out, indent=1)
    if args.json:
        with open(args.json, "w") as f:
            f.write(txt)
    else:
        print(txt)


if __name__ == "__main__":
    main()
