"""FP64 CPU oracle for the Galerkin-FFT homogenization solver.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark, never by the solver package.  The arithmetic lives in ``galerkin_oracle.c`` (plain C,
FP64, OpenMP over FFT lines); this module converts between the Mandel vectors used at the solver's
interface and the Cartesian tensor components used inside the oracle.

Paper sections followed: "Galerkin-FFT with discrete differences and mixed loading control"
(eqs. freq, galop, gallin, linearOp, galres, freqrot) and "Voigt approaches" (C = phi C_m).  The
surface-smoothening phase maps (VFG, VA, phase field, combined) are in ``oracle.geometry``.
Every function is pinned by CPU tests against closed forms, brute force or invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "galerkin_oracle.c"), os.path.join(_HERE, "geometry_oracle.c")]
_SO = os.path.join(_HERE, "libgalerkin_oracle.so")
_lib = None

ROTATED, CONTINUOUS = 0, 1
NYQ_NATURAL, NYQ_ZERO_ALL = 0, 1
MINRES, CG = 0, 1
_SHEAR_SCALE = np.array([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, *_SRCS, "-lm"],
                       check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.or_dft_naive.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int]
        lib.or_fft.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int]
        lib.or_fft3.argtypes = [dp, ip, ctypes.c_int]
        lib.or_projection_matrix.argtypes = [ctypes.c_void_p, ip, dp, dp]
        lib.or_modified_frequency.argtypes = [ctypes.c_void_p, ip, dp, dp]
        lib.or_apply.argtypes = [ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.or_project.argtypes = [ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.or_solve.argtypes = [ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_time_minres.argtypes = [ip, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int]
        lib.or_time_minres.restype = ctypes.c_double
        lib.or_apply_field.argtypes = [ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.or_minres_field.argtypes = [ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double,
                                        ctypes.c_int, dp, dp]
        lib.og_distance_map.argtypes = [ip, dp, ctypes.c_int, dp, ctypes.c_int, dp]
        lib.og_distance_map.restype = None
        _lib = lib
    return _lib


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3), ("scheme", ctypes.c_int),
                ("nyquist", ctypes.c_int), ("stress_mask", ctypes.c_int)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _n3(n):
    if isinstance(n, int):
        n = (n, n, n)
    return tuple(int(v) for v in n)


def num_threads() -> int:
    return int(_load().or_num_threads())


# ------------------------------------------------------------------ Mandel <-> tensor components
def mandel_to_tensor(x: np.ndarray) -> np.ndarray:
    """Mandel (.., 6 leading axis first) -> Cartesian components (00,11,22,12,02,01)."""
    x = np.asarray(x, dtype=np.float64)
    return x / _SHEAR_SCALE.reshape((6,) + (1,) * (x.ndim - 1))


def tensor_to_mandel(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return x * _SHEAR_SCALE.reshape((6,) + (1,) * (x.ndim - 1))


# ------------------------------------------------------------------ transforms
def dft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """O(n^2) DFT, y_k = sum_j x_j exp(sign 2 pi i jk/n)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().or_dft_naive(_dp(x.view(np.float64)), _dp(y.view(np.float64)), x.size, sign)
    return y


def fft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Recursive mixed-radix FFT (unnormalised both ways)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().or_fft(_dp(x.view(np.float64)), _dp(y.view(np.float64)), x.size, sign)
    return y


def fft3(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """3-D transform; forward unnormalised, inverse (sign=+1) scaled by 1/N."""
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    n = (ctypes.c_int * 3)(*a.shape)
    _load().or_fft3(_dp(a.view(np.float64)), n, sign)
    return a


# ------------------------------------------------------------------ frequencies and projection
def _grid(n, L, scheme, nyquist, stress_mask=0):
    g = _Grid()
    g.n[:] = _n3(n)
    g.L[:] = tuple(float(v) for v in L)
    g.scheme = scheme
    g.nyquist = nyquist
    g.stress_mask = int(stress_mask)
    return g


def mask_of(components) -> int:
    """Bit mask of stress-controlled Mandel components (indices 0..5 = 11, 22, 33, 23, 13, 12)."""
    m = 0
    for a in components:
        m |= 1 << int(a)
    return m


def modified_frequency(n, m, L=(1.0, 1.0, 1.0), scheme=ROTATED) -> np.ndarray:
    g = _grid(n, L, scheme, NYQ_NATURAL)
    re, im = np.zeros(3), np.zeros(3)
    _load().or_modified_frequency(ctypes.byref(g), (ctypes.c_int * 3)(*m), _dp(re), _dp(im))
    return re + 1j * im


def projection_matrix(n, m, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL, mandel=True,
                      stress_mask=0) -> np.ndarray:
    """Ghat at storage frequency m as a 6x6 complex matrix.  mandel=True: acting on Mandel vectors
    (then symmetric for real Ghat); else acting on the six Cartesian components.  stress_mask: the
    stress-controlled components (mixed control), which only change Ghat at m = 0."""
    g = _grid(n, L, scheme, nyquist, stress_mask)
    re, im = np.zeros(36), np.zeros(36)
    _load().or_projection_matrix(ctypes.byref(g), (ctypes.c_int * 3)(*m), _dp(re), _dp(im))
    G = (re + 1j * im).reshape(6, 6)
    if mandel:
        # out_mandel = S out_tensor ; in_tensor = in_mandel / S  (S = shear scale) and the
        # Cartesian-component matrix already accounts for S_kl = S_lk (each off-diagonal appears twice)
        s = _SHEAR_SCALE
        G = (s[:, None] * G) / s[None, :]
    return G


# ------------------------------------------------------------------ operator and solve
def _fields_in(x, N):
    x = mandel_to_tensor(np.asarray(x, dtype=np.float64).reshape(6, N))
    return np.ascontiguousarray(x)


def apply(n, phi, C1, x, C0=None, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL,
          stress_mask=0) -> np.ndarray:
    """A(x) of eq. (linearOp) on a Mandel strain field x [6, *n]; returns Mandel [6, *n]."""
    n = _n3(n)
    N = int(np.prod(n))
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(N)
    C1 = np.ascontiguousarray(C1, dtype=np.float64).reshape(36)
    C0 = np.zeros(36) if C0 is None else np.ascontiguousarray(C0, dtype=np.float64).reshape(36)
    xt = _fields_in(x, N)
    y = np.empty_like(xt)
    _load().or_apply((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), scheme, nyquist,
                     int(stress_mask), _dp(phi), _dp(C1), _dp(C0), _dp(xt), _dp(y))
    return tensor_to_mandel(y).reshape((6,) + n)


def project(n, x, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL, stress_mask=0) -> np.ndarray:
    """Re F^{-1} Ghat F x on a Mandel field (projection onto compatible strain fields; under mixed
    control the uniform stress-controlled components are kept)."""
    n = _n3(n)
    N = int(np.prod(n))
    xt = _fields_in(x, N)
    y = np.empty_like(xt)
    _load().or_project((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), scheme, nyquist,
                       int(stress_mask), _dp(xt), _dp(y))
    return tensor_to_mandel(y).reshape((6,) + n)


def solve(n, phi, C1, Ebar, tol=1e-8, maxit=1000, C0=None, L=(1.0, 1.0, 1.0), scheme=ROTATED,
          nyquist=NYQ_NATURAL, solver=MINRES, x0=None, want_sigma=True, stress_mask=0, Sbar=None) -> dict:
    """Galerkin solve of eq. (gallin) for the strain fluctuation (Mandel in, Mandel out): strain
    control by default; with stress_mask, mixed control (those components stress-controlled at the
    macroscopic stress Sbar, the others strain-controlled at Ebar).

    Returns dict(eps [6,*n], sigma [6,*n] or None, sigma_mean [6], strain_mean [6] (total macroscopic
    strain), iterations, status, rel_residual (recurrence), true_residual, bnorm, history)."""
    n = _n3(n)
    N = int(np.prod(n))
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(N)
    C1 = np.ascontiguousarray(C1, dtype=np.float64).reshape(36)
    C0 = np.zeros(36) if C0 is None else np.ascontiguousarray(C0, dtype=np.float64).reshape(36)
    E = np.ascontiguousarray(mandel_to_tensor(np.asarray(Ebar, dtype=np.float64).reshape(6)))
    S = np.ascontiguousarray(mandel_to_tensor(np.zeros(6) if Sbar is None else np.asarray(Sbar, np.float64).reshape(6)))
    eps = np.zeros((6, N))
    sig = np.zeros((6, N)) if want_sigma else None
    smean = np.zeros(6)
    hist = np.zeros(max(maxit, 1))
    info = np.zeros(8)
    x0p = None
    if x0 is not None:
        x0t = _fields_in(x0, N)
        x0p = _dp(x0t)
    _load().or_solve((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), scheme, nyquist, int(stress_mask),
                     _dp(phi), _dp(C1), _dp(C0), _dp(E), _dp(S), float(tol), int(maxit), int(solver), x0p, _dp(eps),
                     _dp(sig) if sig is not None else None, _dp(smean), _dp(hist), _dp(info))
    it = int(info[0])
    Eused = np.array([0.0 if (int(stress_mask) >> a) & 1 else float(np.asarray(Ebar).reshape(6)[a]) for a in range(6)])
    emean = tensor_to_mandel(eps).mean(axis=1)
    return dict(eps=tensor_to_mandel(eps).reshape((6,) + n), strain_mean=Eused + emean,
                sigma=tensor_to_mandel(sig).reshape((6,) + n) if sig is not None else None,
                sigma_mean=tensor_to_mandel(smean), iterations=it, status=int(info[1]),
                rel_residual=float(info[2]), true_residual=float(info[3]), bnorm=float(info[4]),
                history=hist[:it].copy())


def time_minres(n, phi, C1, iters=3, warmup=1, C0=None, L=(1.0, 1.0, 1.0)) -> float:
    """Wall seconds of `iters` MINRES iterations (operator + vector work) on this problem, after all
    vectors are allocated and first touched and `warmup` iterations have run (those are not timed).
    The right-hand side is a seeded random field: an iteration's cost does not depend on it."""
    n = _n3(n)
    N = int(np.prod(n))
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(N)
    C1 = np.ascontiguousarray(C1, dtype=np.float64).reshape(36)
    C0 = np.zeros(36) if C0 is None else np.ascontiguousarray(C0, dtype=np.float64).reshape(36)
    return float(_load().or_time_minres((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), _dp(phi),
                                        _dp(C1), _dp(C0), int(iters), int(warmup)))


def effective_stiffness(n, phi, C1, tol=1e-10, maxit=5000, cases=range(6), **kw) -> tuple[np.ndarray, list]:
    """C_eff (Mandel 6x6): column J is <sigma> for the unit Mandel macro strain e_J."""
    Ceff = np.full((6, 6), np.nan)
    infos = []
    for J in cases:
        E = np.zeros(6)
        E[J] = 1.0
        r = solve(n, phi, C1, E, tol=tol, maxit=maxit, want_sigma=False, **kw)
        Ceff[:, J] = r["sigma_mean"]
        infos.append({k: r[k] for k in ("iterations", "status", "rel_residual", "true_residual")})
    return Ceff, infos
