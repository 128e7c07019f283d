"""FP64 CPU oracle of the lattice surface-smoothening phase maps.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark, never by the solver package.  Plain numpy in float64; numpy's real FFT serves as the
one library step (the Fourier transform of eq. phase3).

Paper sections followed:
  * "Voigt approaches": C = phi C_m with phi the solid volume fraction of the voxel; the Voigt
    fine-grid map (VFG) counts sub-grid points inside the solid, the Voigt analytic map (VA) is
    linear in the signed distance D of the voxel centre to the strut surface over a width ell
    (eq. phaselin), clipped to [0, 1].
  * "Phase-field smoothening" (eqs. phase, phase2, phase3): phi minimises
    int 1/2 ell^2 |grad phi|^2 + eps/2 (phi - omega)^2 over periodic fields, solved in Fourier space
    on a fine grid (voxel d_coarse / ratio) from the solid indicator omega at the fine voxel centres,
    then averaged over each coarse voxel; values below 5 % are set to zero.
  * "Combined smoothening": the phase-field step applied to the VA coefficient map.
  * "Analysis of the surface smoothening approaches": relative density = voxel mean of phi.

Readings where the text is garbled or silent:
  * eq. phaselin: the printed sign of D makes phi fall towards the strut axis; the definition that
    gives phi = 1 deep in the solid and the exact volume fraction at a planar interface is
    phi = 1/2 - D/ell with D < 0 inside the solid, i.e. phi = 1/2 + d/ell inside, 1/2 - d/ell outside.
  * eq. phase3: the printed denominator 1 - (ell^2/eps) xi.xi has the wrong sign for a real
    frequency xi; the minimiser of eq. phase has phi_hat = omega_hat / (1 + (ell^2/eps) |xi|^2),
    with xi the continuous frequency 2 pi k / L of eq. freq.  eq. phase2's (ell/eps)^2 is read as
    ell^2/eps, the Euler-Lagrange coefficient of eq. phase (the same for the paper's eps = 1).
  * The strut surface is the boundary of the union of capsules (cylinders with spherical ends);
    D(x) = min over struts of (distance to the strut axis segment - radius), which is the exact
    signed distance outside the solid and inside a single strut.  Each strut is measured at its
    periodic image nearest to the strut midpoint.
  * Sub-grid points of VFG and the fine grid of the phase-field step are the same points: the
    centres of the voxels of the grid ratio * n.
  * Combined smoothening: the fine-grid source is the VA map of the coarse grid, constant over each
    coarse voxel, so the coarse mean is kept (the paper: CS has the density of VA).

Pins (tests/test_geometry_pins.py): closed-form distances of the octet's octahedral and
tetrahedral sites, brute-force segment distance, VA at a planar slab (exact voxel fractions),
Fourier eigenmodes of the smoothing, the periodic slab's hyperbolic closed form, mean conservation.
"""
from __future__ import annotations

import numpy as np

PV, VFG, VA = 0, 1, 2


def _n3(n):
    if isinstance(n, int):
        n = (n, n, n)
    return tuple(int(v) for v in n)


def voxel_centres(n, L=(1.0, 1.0, 1.0), sub: int = 1) -> list[np.ndarray]:
    """Axis coordinates of the voxel centres of the grid sub * n: x_p = (j + 1/2) * L_p / (sub n_p)."""
    n = _n3(n)
    return [(np.arange(sub * n[p], dtype=np.float64) + 0.5) * (float(L[p]) / (sub * n[p])) for p in range(3)]


def segment_distance(points: np.ndarray, a, b, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Euclidean distance from points (M, 3) to the segment a-b (endpoints in fractions of the cell),
    taking for each point the periodic image of the segment nearest to the segment midpoint."""
    Lv = np.asarray(L, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64) * Lv
    b = np.asarray(b, dtype=np.float64) * Lv
    mid = 0.5 * (a + b)
    half = 0.5 * (b - a)
    dx = points - mid
    dx = dx - Lv * np.floor(dx / Lv + 0.5)
    hh = float(half @ half)
    t = np.clip((dx @ half) / hh, -1.0, 1.0) if hh > 0 else np.zeros(len(points))
    e = dx - t[:, None] * half
    return np.sqrt(np.sum(e * e, axis=1))


def signed_distance(points: np.ndarray, struts: np.ndarray, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """D(x) = min over struts of (segment distance - radius); struts rows are (a[3], b[3], radius)."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    D = np.full(len(points), np.inf)
    for s in np.asarray(struts, dtype=np.float64).reshape(-1, 7):
        D = np.minimum(D, segment_distance(points, s[0:3], s[3:6], L) - s[6])
    return D


def distance_map(n, struts, L=(1.0, 1.0, 1.0), sub: int = 1) -> np.ndarray:
    """Signed distance at every voxel centre of the grid sub * n, shape sub * n (axis 2 fastest);
    the same arithmetic as signed_distance, as plain C loops (geometry_oracle.c) for large grids."""
    import ctypes
    from . import _load, _dp
    n = _n3(n)
    st = np.ascontiguousarray(np.asarray(struts, dtype=np.float64).reshape(-1, 7))
    out = np.empty(tuple(sub * v for v in n))
    Lv = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
    _load().og_distance_map((ctypes.c_int * 3)(*n), _dp(Lv), int(sub), _dp(st), int(st.shape[0]), _dp(out))
    return out


def indicator(D: np.ndarray) -> np.ndarray:
    """Solid indicator omega = 1 where D <= 0 (the closed solid), else 0."""
    return (D <= 0.0).astype(np.float64)


def coarsen(f: np.ndarray, ratio: int) -> np.ndarray:
    """Mean over each ratio^3 block of voxels (the fine voxels of one coarse voxel)."""
    m = f.shape
    n = tuple(v // ratio for v in m)
    assert all(v * ratio == w for v, w in zip(n, m))
    return f.reshape(n[0], ratio, n[1], ratio, n[2], ratio).mean(axis=(1, 3, 5))


def upsample(f: np.ndarray, ratio: int) -> np.ndarray:
    """Piecewise-constant copy of a coarse map on the grid ratio * n."""
    return np.repeat(np.repeat(np.repeat(f, ratio, axis=0), ratio, axis=1), ratio, axis=2)


def phase_pv(n, struts, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Plain voxelization: the solid indicator at the voxel centres."""
    return indicator(distance_map(n, struts, L))


def phase_vfg(n, struts, sub: int, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Voigt fine grid: fraction of the sub^3 sub-voxel centres of each voxel that lie in the solid."""
    return coarsen(indicator(distance_map(n, struts, L, sub)), sub)


def va_from_distance(D: np.ndarray, ell: float) -> np.ndarray:
    """eq. phaselin (sign reading above): phi = clip(1/2 - D/ell, 0, 1)."""
    return np.clip(0.5 - np.asarray(D, dtype=np.float64) / ell, 0.0, 1.0)


def phase_va(n, struts, L=(1.0, 1.0, 1.0), ell: float | None = None) -> np.ndarray:
    """Voigt analytic map at the voxel centres; ell defaults to one voxel length (L_0 / n_0)."""
    n = _n3(n)
    if ell is None:
        ell = float(L[0]) / n[0]
    return va_from_distance(distance_map(n, struts, L), ell)


def helmholtz_smooth(omega: np.ndarray, L=(1.0, 1.0, 1.0), ell: float = 0.0, eps: float = 1.0) -> np.ndarray:
    """eq. phase3 (reading above): phi_hat(xi) = omega_hat(xi) / (1 + (ell^2/eps) |xi|^2), xi = 2 pi k / L."""
    m = omega.shape
    k0 = np.fft.fftfreq(m[0], d=1.0 / m[0])
    k1 = np.fft.fftfreq(m[1], d=1.0 / m[1])
    k2 = np.fft.rfftfreq(m[2], d=1.0 / m[2])
    xi2 = ((2 * np.pi * k0 / L[0]) ** 2)[:, None, None] + ((2 * np.pi * k1 / L[1]) ** 2)[None, :, None] \
        + ((2 * np.pi * k2 / L[2]) ** 2)[None, None, :]
    spec = np.fft.rfftn(omega) / (1.0 + (ell * ell / eps) * xi2)
    return np.fft.irfftn(spec, s=m, axes=(0, 1, 2))


def threshold(phi: np.ndarray, thr: float) -> np.ndarray:
    """Values below thr are set to zero (detached material, section "Phase-field smoothening")."""
    return np.where(phi < thr, 0.0, phi)


def phase_field(n, struts, ratio: int, L=(1.0, 1.0, 1.0), ell: float | None = None, eps: float = 1.0,
                thr: float = 0.05, source: np.ndarray | None = None):
    """Phase-field smoothening on the grid ratio * n, averaged to n and thresholded.

    source None: omega = solid indicator at the fine voxel centres (PFS).  source = a coarse map
    (the VA map for the combined smoothening): omega = that map, constant over each coarse voxel.
    ell defaults to half a coarse voxel (L_0 / (2 n_0)).  Returns (phi, phi before the threshold)."""
    n = _n3(n)
    if ell is None:
        ell = 0.5 * float(L[0]) / n[0]
    if source is None:
        omega = indicator(distance_map(n, struts, L, ratio))
    else:
        omega = upsample(np.asarray(source, dtype=np.float64).reshape(n), ratio)
    raw = coarsen(helmholtz_smooth(omega, L, ell, eps), ratio)
    return threshold(raw, thr), raw


def relative_density(phi: np.ndarray) -> float:
    """Relative density of a phase map: its voxel mean."""
    return float(np.mean(phi, dtype=np.float64))
