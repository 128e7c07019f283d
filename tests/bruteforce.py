"""Dense brute-force references for tiny grids (numpy only; independent of the FFT oracle).

The rotated forward-difference scheme of eq. (freqrot) is, in real space, the "8-corner" stencil:
the centre strain of voxel v is built from periodic nodal displacements u at the 8 voxel corners,
    d_p u_i (centre) = 1/(4 h_p) * sum over the 4 voxel edges parallel to axis p of [u_i(end) - u_i(start)].
Its Fourier symbol is i (2/h_p) e^{i sum q/2} sin(q_p/2) prod_{m!=p} cos(q_m/2), i.e. the modified
frequency of eq. (freqrot) times a common phase.  Assembling B densely gives the compatible strain
space range(B) without any FFT, so the minimum-energy problem of the Galerkin method can be solved
by dense linear algebra: minimise <(E + eps) C (E + eps)> over eps in range(B).
"""
from __future__ import annotations

import itertools

import numpy as np

SQ2 = np.sqrt(2.0)


def stencil_B(n, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Dense B (6N x 3N): Mandel strain [6][N] at voxel centres from nodal displacements [3][N]."""
    n = tuple(int(v) for v in n)
    N = n[0] * n[1] * n[2]
    h = [L[p] / n[p] for p in range(3)]
    grad = np.zeros((3, 3, N, N))  # grad[p][i] maps u_i (nodes) -> d_p u_i (voxels), same for each i

    def nid(a, b, c):
        return ((a % n[0]) * n[1] + (b % n[1])) * n[2] + (c % n[2])

    D = np.zeros((3, N, N))  # D[p]: nodal scalar -> d_p at centres
    for a, b, c in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        v = nid(a, b, c)
        for p in range(3):
            others = [q for q in range(3) if q != p]
            for o1, o2 in itertools.product((0, 1), (0, 1)):
                off = [0, 0, 0]
                off[others[0]] = o1
                off[others[1]] = o2
                start = nid(a + off[0], b + off[1], c + off[2])
                off[p] = 1
                end = nid(a + off[0], b + off[1], c + off[2])
                D[p, v, end] += 1.0 / (4 * h[p])
                D[p, v, start] -= 1.0 / (4 * h[p])
    del grad
    B = np.zeros((6, N, 3, N))
    # Mandel: 00, 11, 22, sqrt2*12, sqrt2*02, sqrt2*01 with eps_ij = (d_i u_j + d_j u_i)/2
    B[0, :, 0, :] = D[0]
    B[1, :, 1, :] = D[1]
    B[2, :, 2, :] = D[2]
    for m, (i, j) in zip((3, 4, 5), ((1, 2), (0, 2), (0, 1))):
        B[m, :, j, :] += SQ2 * 0.5 * D[i]
        B[m, :, i, :] += SQ2 * 0.5 * D[j]
    return B.reshape(6 * N, 3 * N)


def stiffness_matrix(phi, C1, C0=None) -> np.ndarray:
    """Dense block operator (6N x 6N) acting on [6][N] Mandel fields: C(x) = phi C1 + (1-phi) C0."""
    phi = np.asarray(phi, dtype=np.float64).reshape(-1)
    N = phi.size
    C0 = np.zeros((6, 6)) if C0 is None else np.asarray(C0, dtype=np.float64)
    K = np.zeros((6, N, 6, N))
    idx = np.arange(N)
    for a in range(6):
        for b in range(6):
            K[a, idx, b, idx] = phi * C1[a, b] + (1.0 - phi) * C0[a, b]
    return K.reshape(6 * N, 6 * N)


def compatible_basis(n, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Orthonormal basis (columns) of range(B), the periodic compatible zero-mean strain fields."""
    B = stencil_B(n, L)
    U, s, _ = np.linalg.svd(B, full_matrices=False)
    return U[:, s > 1e-10 * s.max()]


def min_norm_solution(n, phi, C1, Ebar, C0=None, L=(1.0, 1.0, 1.0)):
    """Minimum-norm compatible fluctuation eps minimising the energy of E + eps, and its stress.

    Returns (eps [6,*n], sigma [6,*n], sigma_mean [6])."""
    n = tuple(int(v) for v in n)
    N = n[0] * n[1] * n[2]
    Q = compatible_basis(n, L)
    C = stiffness_matrix(phi, C1, C0)
    E = np.repeat(np.asarray(Ebar, dtype=np.float64).reshape(6, 1), N, axis=1).reshape(-1)
    M = Q.T @ C @ Q
    rhs = -Q.T @ (C @ E)
    y = np.linalg.lstsq(M, rhs, rcond=1e-12)[0]
    eps = Q @ y
    sig = C @ (E + eps)
    return eps.reshape((6,) + n), sig.reshape((6,) + n), sig.reshape(6, N).mean(axis=1)


def laminate_closed_form(profile, axis: int, E: float, nu: float) -> np.ndarray:
    """Effective Mandel stiffness of a laminate phi(x_axis) of an isotropic solid (C = phi C_m).

    Layers normal to `axis`: in-plane strains are uniform and tractions sigma_{axis,j} uniform, so
    with A = <phi> and H = 1/<1/phi> (H = 0 with a void layer) C_eff = H C_m + (A - H) S, S being the
    plane-stress stiffness E/(1-nu^2)[[1,nu],[nu,1]] plus the in-plane Mandel shear 2 mu."""
    prof = np.asarray(profile, dtype=np.float64)
    A = prof.mean()
    H = 0.0 if np.any(prof == 0) else 1.0 / np.mean(1.0 / prof)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    Cm = np.zeros((6, 6))
    Cm[:3, :3] = lam
    Cm += 2 * mu * np.eye(6)
    S = np.zeros((6, 6))
    inplane = [q for q in range(3) if q != axis]
    shear = {0: 3, 1: 4, 2: 5}[axis]  # Mandel index of the in-plane shear component
    Ep = E / (1 - nu * nu)
    S[inplane[0], inplane[0]] = S[inplane[1], inplane[1]] = Ep
    S[inplane[0], inplane[1]] = S[inplane[1], inplane[0]] = nu * Ep
    S[shear, shear] = 2 * mu
    return H * Cm + (A - H) * S


def mixed_solution(n, phi, C1, Ebar, stress_components, Sbar, C0=None, L=(1.0, 1.0, 1.0)):
    """Mixed macroscopic control by dense minimisation: the strain is Ebar (strain-controlled
    components only) + m + eps, with eps a compatible zero-mean stencil strain and m a uniform strain
    in the stress-controlled components; (eps, m) minimise the energy 1/2 <(E + m + eps) C (E + m + eps)>
    minus the work <Sbar . m> of the prescribed macroscopic stress.  Minimum-norm least squares where
    empty voxels make it singular.

    Returns (fluctuation eps + m [6,*n], sigma [6,*n], sigma_mean [6], strain_mean [6])."""
    n = tuple(int(v) for v in n)
    N = n[0] * n[1] * n[2]
    KL = sorted(int(a) for a in stress_components)
    Q = compatible_basis(n, L)
    M = np.zeros((6 * N, len(KL)))
    for j, a in enumerate(KL):
        M[a * N:(a + 1) * N, j] = 1.0
    Z = np.concatenate([Q, M], axis=1)
    C = stiffness_matrix(phi, C1, C0)
    Eb = np.array([0.0 if a in KL else float(Ebar[a]) for a in range(6)])
    E = np.repeat(Eb.reshape(6, 1), N, axis=1).reshape(-1)
    Sb = np.array([float(Sbar[a]) if a in KL else 0.0 for a in range(6)])
    s = np.repeat(Sb.reshape(6, 1), N, axis=1).reshape(-1)  # the uniform prescribed stress field
    Kz = Z.T @ C @ Z
    rhs = -Z.T @ (C @ E) + Z.T @ s
    y = np.linalg.lstsq(Kz, rhs, rcond=1e-12)[0]
    fl = Z @ y
    sig = C @ (E + fl)
    return (fl.reshape((6,) + n), sig.reshape((6,) + n), sig.reshape(6, N).mean(axis=1),
            Eb + fl.reshape(6, N).mean(axis=1))
