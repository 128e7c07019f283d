"""Seeded synthetic inputs for the lattice homogenization solver and its CPU oracle.

Octet-truss voxel phase maps (Voigt fine-grid fractions, plain voxelization as S=1), manufacturing
defects (roughness + pores), simple analytic patterns (laminates, inclusions) and the macro strain
load cases.  Nothing here performs any step of the homogenization method itself; both the GPU path
and the FP64 oracle only read what this module produces.

Geometry: the octet truss of the section "Lattice geometry and simulation parameters" (all 24 FCC
nearest-neighbour struts of the cubic cell, capsules of radius r); voxel fractions by the Voigt
fine-grid rule of the section "Voigt approaches"; relative density as the voxel mean of phi
(section "Analysis of the surface smoothening approaches").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lattice_gen.c")
_SO = os.path.join(_HERE, "liblattice_gen.so")
_lib = None

SQRT2 = float(np.sqrt(2.0))


def build(force: bool = True) -> str:
    """Compile the generator with gcc + OpenMP (portable x86-64 code, no -march=native)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i3 = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.lg_octet_radius.restype = ctypes.c_double
        lib.lg_octet_radius.argtypes = [i3, ctypes.c_int, ctypes.c_double]
        lib.lg_octet_phi.restype = None
        lib.lg_octet_phi.argtypes = [i3, ctypes.c_int, ctypes.c_double, fp, ctypes.c_double, dp, ctypes.c_int, fp]
        lib.lg_roughness.restype = ctypes.c_int
        lib.lg_roughness.argtypes = [i3, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, fp]
        lib.lg_place_pores.restype = ctypes.c_int
        lib.lg_place_pores.argtypes = [i3, ctypes.c_double, fp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, ctypes.c_int, dp]
        lib.lg_splitmix64.restype = ctypes.c_uint64
        lib.lg_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp]
        lib.lg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _n3(n):
    if isinstance(n, int):
        n = (n, n, n)
    n = tuple(int(v) for v in n)
    assert len(n) == 3 and all(v >= 1 for v in n)
    return n, (ctypes.c_int * 3)(*n)


def uniforms(seed: int, count: int) -> np.ndarray:
    """`count` splitmix64 uniforms in [0,1) (53-bit) from `seed`."""
    out = np.empty(count, dtype=np.float64)
    _load().lg_splitmix64(ctypes.c_uint64(seed), count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def octet_struts(radius: float) -> np.ndarray:
    """Strut list of the octet truss (input description of the lattice): 24 rows (a[3], b[3], r) with
    endpoints in fractions of the cubic cell: the FCC basis points joined to their nearest neighbours
    along the six face diagonals, as in the section "Lattice geometry and simulation parameters"."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    dirs = np.array([[0.5, 0.5, 0], [0.5, -0.5, 0], [0.5, 0, 0.5], [0.5, 0, -0.5], [0, 0.5, 0.5], [0, 0.5, -0.5]],
                    dtype=np.float64)
    out = np.zeros((24, 7))
    k = 0
    for b in basis:
        for d in dirs:
            out[k, 0:3] = b
            out[k, 3:6] = b + d
            out[k, 6] = radius
            k += 1
    return out


def octet_radius(n, rho: float, sub: int = 4) -> float:
    """Strut radius (unit cell = 1) whose S^3-subsampled phase map has mean exactly round(rho*N*S^3)/(N*S^3)."""
    _, c = _n3(n)
    r = _load().lg_octet_radius(c, int(sub), float(rho))
    if r < 0:
        raise ValueError("density out of range for the octet generator")
    return r


def octet_phi(n, r: float, sub: int = 4, eta: np.ndarray | None = None, rough_h: float = 0.0,
              pores: np.ndarray | None = None) -> np.ndarray:
    """Voxel solid fractions (float32, shape n, axis 2 contiguous) of the octet with strut radius r."""
    n, c = _n3(n)
    phi = np.empty(n, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    eta_p = None
    if eta is not None:
        eta = np.ascontiguousarray(eta, dtype=np.float32)
        assert eta.shape == n
        eta_p = eta.ctypes.data_as(fp)
    npores = 0
    pores_p = None
    if pores is not None and len(pores):
        pores = np.ascontiguousarray(pores, dtype=np.float64)
        npores = pores.shape[0]
        pores_p = pores.ctypes.data_as(dp)
    _load().lg_octet_phi(c, int(sub), float(r), eta_p, float(rough_h), pores_p, npores, phi.ctypes.data_as(fp))
    return phi


def octet_phase_map(n, rho: float, sub: int = 4):
    """Ideal octet at target relative density rho: returns (phi, r)."""
    r = octet_radius(n, rho, sub)
    return octet_phi(n, r, sub), r


def roughness_field(n, sigma: float, amp: float, seed: int) -> np.ndarray:
    """Zero-mean smooth noise (voxel units, max |eta| = amp): U(-1,1) per voxel, Gaussian std sigma."""
    n, c = _n3(n)
    eta = np.empty(n, dtype=np.float32)
    rc = _load().lg_roughness(c, float(sigma), float(amp), ctypes.c_uint64(seed),
                              eta.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if rc != 0:
        raise MemoryError("roughness field allocation failed")
    return eta


@dataclass
class DefectInfo:
    radius: float
    n_pores: int
    pores: np.ndarray
    rho_ideal: float
    rho_actual: float


def octet_defect_phase_map(n, rho: float = 0.15, rough_amp: float = 1.5, rough_sigma: float = 2.0,
                           n_pores: int = 200, pore_median_vox: float = 2.0, pore_s: float = 0.5,
                           seed_rough: int = 20211001, seed_pores: int = 20211002, sub: int = 4,
                           radius: float | None = None):
    """Octet with synthetic manufacturing defects.

    The radius is chosen for `rho` on the ideal geometry; the strut signed distance is then perturbed
    by rough_amp-voxel roughness (Gaussian-filtered U(-1,1) noise, std rough_sigma voxels), and
    `n_pores` spherical pores with lognormal radii (median pore_median_vox voxels, log-std pore_s)
    are carved from the solid (centres drawn until n_pores land inside the perturbed solid).
    A given `radius` (unit cell = 1) replaces the density search (rho is then only recorded).
    """
    n, c = _n3(n)
    r = float(radius) if radius is not None else octet_radius(n, rho, sub)
    h = 1.0 / n[0]
    eta = roughness_field(n, rough_sigma, rough_amp, seed_rough) if rough_amp > 0 else None
    pores = np.zeros((max(n_pores, 1), 4), dtype=np.float64)
    got = 0
    if n_pores > 0:
        got = _load().lg_place_pores(c, float(r), eta.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if eta is not None else None,
                                     h, int(n_pores), pore_median_vox * h, float(pore_s), ctypes.c_uint64(seed_pores),
                                     int(200 * n_pores + 1000), pores.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    pores = pores[:got]
    phi = octet_phi(n, r, sub, eta=eta, rough_h=h, pores=pores)
    return phi, DefectInfo(radius=r, n_pores=got, pores=pores, rho_ideal=rho, rho_actual=float(phi.mean(dtype=np.float64)))


def heterogeneous_rves(count: int = 64, sizes=(32, 48, 64, 96), rho_range=(0.03, 0.30), seed0: int = 1000):
    """Per-RVE (grid, rho) for a batch of uneven octet RVEs: RVE i draws each axis length
    independently from `sizes` and rho uniformly from rho_range, all from seed seed0 + i."""
    out = []
    for i in range(count):
        u = uniforms(seed0 + i, 4)
        n = tuple(int(sizes[min(int(u[p] * len(sizes)), len(sizes) - 1)]) for p in range(3))
        rho = rho_range[0] + (rho_range[1] - rho_range[0]) * u[3]
        out.append((n, float(rho)))
    return out


# ------------------------------------------------------------------ simple analytic patterns
def laminate_phi(n, axis: int, profile) -> np.ndarray:
    """phi varying only along `axis`, with the given per-layer profile (length n[axis])."""
    n, _ = _n3(n)
    prof = np.asarray(profile, dtype=np.float32)
    assert prof.shape == (n[axis],)
    shape = [1, 1, 1]
    shape[axis] = n[axis]
    return np.ascontiguousarray(np.broadcast_to(prof.reshape(shape), n)).astype(np.float32)


def random_phi(n, seed: int, void_fraction: float = 0.5) -> np.ndarray:
    """Seeded random phase map: a void fraction of exact zeros, the rest U(0,1] values."""
    n, _ = _n3(n)
    N = n[0] * n[1] * n[2]
    u = uniforms(seed, 2 * N)
    phi = np.where(u[:N] < void_fraction, 0.0, 1.0 - u[N:])
    return phi.reshape(n).astype(np.float32)


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded U(-scale, scale) float64 array (e.g. strain fields for operator parity)."""
    shape = tuple(int(s) for s in shape)
    N = int(np.prod(shape))
    return (scale * (2.0 * uniforms(seed, N) - 1.0)).reshape(shape)


def unit_mandel_cases() -> np.ndarray:
    """The six unit macro strains in Mandel notation (11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12)."""
    return np.eye(6, dtype=np.float64)


def uniaxial_strain(eps11: float = 1e-3) -> np.ndarray:
    e = np.zeros(6)
    e[0] = eps11
    return e


def isotropic_mandel(E: float, nu: float) -> np.ndarray:
    """6x6 Mandel stiffness of an isotropic solid (input description of the material)."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for i in range(6):
        C[i, i] += 2 * mu
    return C
