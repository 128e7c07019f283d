"""Write oracle-only effective stiffness goldens for ideal octet lattices.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generator (lattice_inputs/).  The
ideal octet is exactly cubic-symmetric on the voxel grid (checked by the CPU tests), so the oracle
solves the two independent unit load cases e_11 and sqrt2*e_23 and the 6x6 Mandel matrix is assembled
from C11, C12, C44.  Material: isotropic E = 1, nu = 0.3, empty phase of zero stiffness; 4^3
sub-voxel Voigt fractions; rotated scheme, natural Nyquist reading; MINRES to tol 1e-10.

usage: python tests/golden/make_golden_ceff.py N rho [rho ...]   -> tests/golden/ceff_octet_N.json
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lattice_inputs as li  # noqa: E402
import oracle  # noqa: E402


def main():
    n = int(sys.argv[1])
    rhos = [float(v) for v in sys.argv[2:]]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"ceff_octet_{n}.json")
    data = json.load(open(out)) if os.path.exists(out) else {}
    C1 = li.isotropic_mandel(1.0, 0.3)
    for rho in rhos:
        key = f"{rho:.4f}"
        if key in data:
            continue
        phi, r = li.octet_phase_map(n, rho)
        t0 = time.time()
        cols = {}
        infos = {}
        for J in (0, 3):
            E = np.zeros(6)
            E[J] = 1.0
            res = oracle.solve(n, phi, C1, E, tol=1e-10, maxit=20000, want_sigma=False)
            cols[J] = res["sigma_mean"]
            infos[J] = {k: res[k] for k in ("iterations", "status", "rel_residual", "true_residual")}
        c11, c12, c44 = cols[0][0], cols[0][1], cols[3][3]
        C = np.zeros((6, 6))
        C[:3, :3] = c12
        for i in range(3):
            C[i, i] = c11
            C[3 + i, 3 + i] = c44
        data[key] = dict(n=n, rho_target=rho, rho_actual=float(phi.mean(dtype=np.float64)), radius=r,
                         C=C.tolist(), col_e11=list(map(float, cols[0])), col_e23=list(map(float, cols[3])),
                         info_e11=infos[0], info_e23=infos[3], seconds=time.time() - t0,
                         threads=oracle.num_threads())
        json.dump(data, open(out + ".tmp", "w"), indent=1)
        os.replace(out + ".tmp", out)
        print(n, rho, data[key]["info_e11"], data[key]["info_e23"], flush=True)


if __name__ == "__main__":
    main()
