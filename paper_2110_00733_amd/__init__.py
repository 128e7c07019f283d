"""Python binding of librve.so, the gfx950 Galerkin-FFT homogenization solver (C ABI in include/rve.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.  PyTorch
supplies device memory (workspace, fields) and the current HIP stream.  There is no CPU fallback:
importing works without a GPU (so the ABI can be inspected), but any solve or apply needs the built
library and a ROCm device, and raises otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librve.so")

RVE_OK, RVE_NOT_CONVERGED, RVE_BREAKDOWN = 0, 1, 2
RVE_EINVAL, RVE_EUNSUPPORTED_SIZE, RVE_ENONFINITE, RVE_ENOMEM, RVE_EDEVICE = -1, -2, -3, -4, -5
FP32_MIXED, FP64 = 0, 1
ROTATED, CONTINUOUS = 0, 1
NYQ_NATURAL, NYQ_ZERO_ALL = 0, 1
APPLY_OPERATOR, APPLY_PROJECTION, APPLY_STIFFNESS_ROUNDTRIP = 0, 1, 2

# every symbol include/rve.h declares
ABI_SYMBOLS = ("rve_default_options", "rve_supported_length", "rve_validate", "rve_workspace_bytes", "solve_rve",
               "rve_apply_workspace_bytes", "rve_apply", "rve_profile_enable", "rve_profile_reset", "rve_profile_read",
               "rve_profile_kind_name", "rve_batch_workspace_bytes", "solve_rve_batch", "rve_autotune", "rve_load_tuning", "rve_tuned_tiles", "rve_last_error",
               "rve_last_solve_info", "rve_last_mean_strain", "rve_release_caches", "rve_cache_counts", "solve_rve_noalloc",
               "rve_noalloc_scratch_bytes", "rve_status_string", "rve_j2_workspace_bytes", "solve_rve_j2",
               "rve_j2_return_map", "rve_modbfft_workspace_bytes", "solve_rve_modbfft")


class RveError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        extra = ""
        if status == RVE_EDEVICE:
            extra = ": " + load_library().rve_last_error().decode()
        super().__init__(f"{where}: {status_string(status)} ({status}){extra}")


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3)]


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("nyquist", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("inner_floor", ctypes.c_double), ("inner_safety", ctypes.c_double),
                ("stress_mask", ctypes.c_int32), ("macro_stress", ctypes.POINTER(ctypes.c_double))]


class J2Material(ctypes.Structure):
    _fields_ = [("young", ctypes.c_double), ("poisson", ctypes.c_double), ("yield_stress", ctypes.c_double)]


class J2Options(ctypes.Structure):
    _fields_ = [("increments", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("newton_tol", ctypes.c_double),
                ("lin_tol", ctypes.c_double)]


class J2Increment(ctypes.Structure):
    _fields_ = [("strain_mean", ctypes.c_double * 6), ("stress_mean", ctypes.c_double * 6), ("r_newton", ctypes.c_double),
                ("newton", ctypes.c_int32), ("minres", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


MODBFFT_PASSES = ("expand", "ifft_axis0", "ifft_axis1", "axis2_stress", "fft_axis1", "fft_axis0", "contract",
                  "cg_update")


class ModbfftStats(ctypes.Structure):
    _fields_ = [("timed", ctypes.c_int32), ("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("alpha", ctypes.c_double), ("pass_ms", ctypes.c_double * 8), ("pass_launches", ctypes.c_int64 * 8)]


class BatchItem(ctypes.Structure):
    _fields_ = [("grid", Grid), ("voxel_fraction_field", ctypes.c_void_p),
                ("phase_stiffness", ctypes.POINTER(ctypes.c_double)), ("macro_strain", ctypes.POINTER(ctypes.c_double)),
                ("n_cases", ctypes.c_int32), ("eps0", ctypes.c_void_p), ("strain_out", ctypes.c_void_p),
                ("stress_out", ctypes.c_void_p), ("eff_stress", ctypes.POINTER(ctypes.c_double)),
                ("iterations", ctypes.POINTER(ctypes.c_int32)), ("rel_residual", ctypes.POINTER(ctypes.c_double)),
                ("macro_stress", ctypes.POINTER(ctypes.c_double)), ("mean_strain", ctypes.POINTER(ctypes.c_double)),
                ("status", ctypes.c_int32)]


_lib = None


def load_library():
    """Load librve.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2110_00733_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    gp, op = ctypes.POINTER(Grid), ctypes.POINTER(Options)
    lib.rve_default_options.argtypes = [op]
    lib.rve_default_options.restype = None
    lib.rve_supported_length.argtypes = [ctypes.c_int32]
    lib.rve_supported_length.restype = ctypes.c_int32
    lib.rve_validate.argtypes = [gp, dp, dp, ctypes.c_int32, op]
    lib.rve_validate.restype = ctypes.c_int
    lib.rve_workspace_bytes.argtypes = [gp, ctypes.c_int32, op]
    lib.rve_workspace_bytes.restype = ctypes.c_size_t
    lib.solve_rve.argtypes = [gp, vp, dp, dp, ctypes.c_int32, op, vp, vp, vp, dp, ip, dp, vp, ctypes.c_size_t, vp]
    lib.solve_rve.restype = ctypes.c_int
    lib.rve_apply_workspace_bytes.argtypes = [gp, ctypes.c_int32, ctypes.c_int32]
    lib.rve_apply_workspace_bytes.restype = ctypes.c_size_t
    lib.rve_apply.argtypes = [gp, vp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, vp, vp, vp, ctypes.c_size_t, vp]
    lib.rve_apply.restype = ctypes.c_int
    lib.rve_profile_enable.argtypes = [ctypes.c_int32]
    lib.rve_profile_enable.restype = None
    lib.rve_profile_reset.argtypes = []
    lib.rve_profile_reset.restype = None
    lib.rve_profile_read.argtypes = [dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    lib.rve_profile_read.restype = ctypes.c_int32
    lib.rve_profile_kind_name.argtypes = [ctypes.c_int32]
    lib.rve_profile_kind_name.restype = ctypes.c_char_p
    bp = ctypes.POINTER(BatchItem)
    lib.rve_batch_workspace_bytes.argtypes = [bp, ctypes.c_int32, op]
    lib.rve_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.solve_rve_batch.argtypes = [bp, ctypes.c_int32, op, vp, ctypes.c_size_t, vp]
    lib.solve_rve_batch.restype = ctypes.c_int
    lib.rve_autotune.argtypes = [gp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.c_char_p, dp]
    lib.rve_autotune.restype = ctypes.c_int
    lib.rve_j2_workspace_bytes.argtypes = [gp, op]
    lib.rve_j2_workspace_bytes.restype = ctypes.c_size_t
    lib.solve_rve_j2.argtypes = [gp, vp, ctypes.POINTER(J2Material), dp, dp, op, ctypes.POINTER(J2Options), vp, vp, vp,
                                 vp, ctypes.POINTER(J2Increment), vp, ctypes.c_size_t, vp]
    lib.solve_rve_j2.restype = ctypes.c_int
    lib.rve_j2_return_map.argtypes = [ctypes.c_int64, vp, ctypes.POINTER(J2Material), vp, vp, vp, vp, vp]
    lib.rve_j2_return_map.restype = ctypes.c_int
    lib.rve_modbfft_workspace_bytes.argtypes = [gp]
    lib.rve_modbfft_workspace_bytes.restype = ctypes.c_size_t
    lib.solve_rve_modbfft.argtypes = [gp, vp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp, dp,
                                      ctypes.POINTER(ModbfftStats), vp, ctypes.c_size_t, vp]
    lib.solve_rve_modbfft.restype = ctypes.c_int
    lib.rve_load_tuning.argtypes = [ctypes.c_char_p]
    lib.rve_load_tuning.restype = ctypes.c_int32
    lib.rve_tuned_tiles.argtypes = [gp, ctypes.c_int32, ip]
    lib.rve_tuned_tiles.restype = ctypes.c_int32
    lib.rve_last_error.argtypes = []
    lib.rve_last_error.restype = ctypes.c_char_p
    lib.rve_last_solve_info.argtypes = [dp, ip, ctypes.c_int32]
    lib.rve_last_mean_strain.argtypes = [dp, ctypes.c_int32]
    lib.rve_last_mean_strain.restype = ctypes.c_int32
    lib.rve_last_solve_info.restype = ctypes.c_int32
    lib.solve_rve_noalloc.argtypes = [gp, vp, dp, dp, ctypes.c_int32, op, vp, vp, vp, dp, ip, dp, vp]
    lib.solve_rve_noalloc.restype = ctypes.c_int
    lib.rve_noalloc_scratch_bytes.argtypes = []
    lib.rve_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.rve_release_caches.argtypes = []
    lib.rve_release_caches.restype = ctypes.c_int32
    lib.rve_cache_counts.argtypes = [ctypes.POINTER(ctypes.c_int64)]
    lib.rve_cache_counts.restype = ctypes.c_int32
    lib.rve_status_string.argtypes = [ctypes.c_int]
    lib.rve_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def profile_enable(on: bool = True) -> None:
    load_library().rve_profile_enable(1 if on else 0)


def profile_reset() -> None:
    load_library().rve_profile_reset()


def profile_read() -> dict:
    """{kernel kind: (total ms, launches)} accumulated since the last reset."""
    lib = load_library()
    kinds = int(lib.rve_profile_read(None, None, 0))
    ms = np.zeros(kinds)
    cnt = np.zeros(kinds, dtype=np.int64)
    k = lib.rve_profile_read(_dp(ms), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), kinds)
    return {lib.rve_profile_kind_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}


def autotune(n, n_cases: int = 1, precision: int = FP32_MIXED, cache_path: str | None = None,
             L=(1.0, 1.0, 1.0), device="cuda:0", workspace: Workspace | None = None) -> dict:
    """rve_autotune for a grid: returns {"ms": tuned apply time, "tiles": (P1/P5 rows, P3 pencils, P2/P4 rows)}."""
    torch = _torch()
    lib = load_library()
    g = make_grid(n, L)
    opt = default_options(precision=precision)
    nbytes = lib.rve_workspace_bytes(ctypes.byref(g), int(n_cases), ctypes.byref(opt))
    if nbytes == 0:
        raise RveError(RVE_EUNSUPPORTED_SIZE, "rve_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, torch.device(device))
    ms = np.zeros(1)
    ss = _solver_stream(torch, ws.device)
    st = lib.rve_autotune(ctypes.byref(g), int(n_cases), int(precision), ctypes.c_void_p(ws.data_ptr()),
                          ctypes.c_size_t(ws.numel()), ctypes.c_void_p(ss.cuda_stream),
                          cache_path.encode() if cache_path else None, _dp(ms))
    if st != RVE_OK:
        raise RveError(st, "rve_autotune")
    return {"ms": float(ms[0]), "tiles": tuned_tiles(n, precision, L)[0]}


def tuned_tiles(n, precision: int = FP32_MIXED, L=(1.0, 1.0, 1.0)):
    """((P1/P5 rows, P3 pencils, P2/P4 rows, P3 component split, NA axis 0, NA axis 1, NA axis 2), from_tuner)"""
    g = make_grid(n, L)
    t = (ctypes.c_int32 * 7)()
    f = load_library().rve_tuned_tiles(ctypes.byref(g), int(precision), t)
    return tuple(t), bool(f)


def load_tuning(path: str) -> int:
    return int(load_library().rve_load_tuning(path.encode()))


def last_solve_info(max_cases: int = 64) -> dict:
    """Start of the last solve on this thread: initial relative residual and warm-start rejection per case."""
    r0 = np.zeros(max_cases)
    rej = np.zeros(max_cases, dtype=np.int32)
    n = load_library().rve_last_solve_info(_dp(r0), rej.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), max_cases)
    n = min(int(n), max_cases)
    return dict(initial_rel_residual=r0[:n].copy(), warm_rejected=rej[:n].astype(bool))


def release_caches() -> int:
    """Free the cached graphs, side streams and events (rve_release_caches); returns the sets freed."""
    return int(load_library().rve_release_caches())


def cache_counts() -> dict:
    """Cached runtime objects: {"sets", "streams", "events", "graphs"} (rve_cache_counts)."""
    c = np.zeros(4, dtype=np.int64)
    load_library().rve_cache_counts(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return dict(zip(("sets", "streams", "events", "graphs"), (int(v) for v in c)))


def last_mean_strain(max_cases: int = 64) -> np.ndarray:
    """Total macroscopic strain [n_cases, 6] of the last solve on this thread (rve_last_mean_strain)."""
    out = np.zeros((max_cases, 6))
    n = int(load_library().rve_last_mean_strain(_dp(out), max_cases))
    return out[:min(n, max_cases)].copy()


def stress_mask_of(components) -> int:
    """Bit mask of stress-controlled Mandel components (0..5 = 11, 22, 33, 23, 13, 12)."""
    m = 0
    for a in components:
        m |= 1 << int(a)
    return m


def status_string(s: int) -> str:
    return load_library().rve_status_string(int(s)).decode()


def make_grid(n, L=(1.0, 1.0, 1.0)) -> Grid:
    if isinstance(n, int):
        n = (n, n, n)
    g = Grid()
    g.n[:] = tuple(int(v) for v in n)
    g.L[:] = tuple(float(v) for v in L)
    return g


def default_options(**kw) -> Options:
    o = Options()
    load_library().rve_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def supported_length(n: int) -> bool:
    return bool(load_library().rve_supported_length(int(n)))


def _stiffness(C_solid, C_void=None) -> np.ndarray:
    C = np.zeros((2, 6, 6))
    if C_void is not None:
        C[0] = np.asarray(C_void, dtype=np.float64)
    C[1] = np.asarray(C_solid, dtype=np.float64)
    return np.ascontiguousarray(C.reshape(72))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def validate(n, C_solid, macro_strain, opt: Options | None = None, C_void=None, L=(1.0, 1.0, 1.0)) -> int:
    """Host-side argument check (no GPU needed)."""
    g = make_grid(n, L)
    C = _stiffness(C_solid, C_void)
    E = np.ascontiguousarray(np.asarray(macro_strain, dtype=np.float64).reshape(-1, 6))
    opt = opt or default_options()
    return int(load_library().rve_validate(ctypes.byref(g), _dp(C), _dp(E), E.shape[0], ctypes.byref(opt)))


def workspace_bytes(n, n_cases: int, opt: Options | None = None, L=(1.0, 1.0, 1.0)) -> int:
    g = make_grid(n, L)
    return int(load_library().rve_workspace_bytes(ctypes.byref(g), int(n_cases), ctypes.byref(opt or default_options())))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no ROCm GPU visible: the solver has no CPU path")
    return torch


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_solver_streams = {}


def _solver_stream(torch, device):
    """A dedicated (default-priority) stream per device: solve_rve captures its iteration chunks into
    HIP graphs, which needs a non-NULL stream."""
    key = torch.device(device).index
    if key not in _solver_streams:
        _solver_streams[key] = torch.cuda.Stream(device=device)
    return _solver_streams[key]


class Workspace:
    """Reusable device workspace (a torch uint8 buffer), grown on demand."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def solve(phi, C_solid, macro_strain, *, C_void=None, L=(1.0, 1.0, 1.0), opt: Options | None = None, eps0=None,
          want_stress: bool = True, workspace: Workspace | None = None, check: bool = True, macro_stress=None,
          **opt_kw) -> dict:
    """solve_rve on a device phase map `phi` (torch float32 [n0,n1,n2]) for each macro strain row; with
    stress_mask=... (and macro_stress rows [nc,6], default zero) under mixed strain/stress control.

    Returns dict(strain [nc,6,*n], stress [nc,6,*n] or None, eff_stress [nc,6], mean_strain [nc,6],
    iterations [nc], rel_residual [nc], status)."""
    torch = _torch()
    lib = load_library()
    if not (phi.is_cuda and phi.dtype == torch.float32 and phi.dim() == 3 and phi.is_contiguous()):
        raise ValueError("phi must be a contiguous float32 CUDA tensor of shape (n0, n1, n2)")
    n = tuple(phi.shape)
    opt = opt or default_options(**opt_kw)
    E = np.ascontiguousarray(np.asarray(macro_strain, dtype=np.float64).reshape(-1, 6))
    nc = E.shape[0]
    S = None
    if macro_stress is not None:
        S = np.ascontiguousarray(np.broadcast_to(np.asarray(macro_stress, dtype=np.float64).reshape(-1, 6), (nc, 6)))
        opt.macro_stress = _dp(S)
    C = _stiffness(C_solid, C_void)
    g = make_grid(n, L)
    fdt = torch.float32 if opt.precision == FP32_MIXED else torch.float64
    strain = torch.empty((nc, 6) + n, dtype=fdt, device=phi.device)
    stress = torch.empty((nc, 6) + n, dtype=fdt, device=phi.device) if want_stress else None
    if eps0 is not None:
        eps0 = eps0.to(device=phi.device, dtype=fdt).contiguous()
        if tuple(eps0.shape) != (nc, 6) + n:
            raise ValueError("eps0 must have shape (n_cases, 6, n0, n1, n2)")
    nbytes = lib.rve_workspace_bytes(ctypes.byref(g), nc, ctypes.byref(opt))
    if nbytes == 0:
        s = lib.rve_validate(ctypes.byref(g), _dp(C), _dp(E), nc, ctypes.byref(opt))
        raise RveError(s if s != 0 else RVE_EINVAL, "rve_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, phi.device)
    eff = np.zeros((nc, 6))
    its = np.zeros(nc, dtype=np.int32)
    res = np.zeros(nc)
    cur = torch.cuda.current_stream(phi.device)
    ss = _solver_stream(torch, phi.device)
    ss.wait_stream(cur)  # inputs written on the caller's stream are ready
    st = lib.solve_rve(ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()), _dp(C), _dp(E), nc, ctypes.byref(opt),
                       ctypes.c_void_p(eps0.data_ptr()) if eps0 is not None else None,
                       ctypes.c_void_p(strain.data_ptr()),
                       ctypes.c_void_p(stress.data_ptr()) if stress is not None else None,
                       _dp(eff), its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(res),
                       ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), ctypes.c_void_p(ss.cuda_stream))
    cur.wait_stream(ss)  # solve_rve returns after synchronising its stream; keep torch's ordering explicit
    if check and st < 0:
        raise RveError(st, "solve_rve")
    mean = last_mean_strain(nc) if st >= 0 else np.full((nc, 6), np.nan)
    del S
    return dict(strain=strain, stress=stress, eff_stress=eff, mean_strain=mean, iterations=its, rel_residual=res,
                status=int(st))


def solve_j2(phi, young: float, poisson: float, yield_stress: float, macro_strain_final, *, increments: int = 20,
             newton_tol: float = 5e-3, lin_tol: float = 1e-6, max_newton: int = 25, macro_stress_final=None,
             L=(1.0, 1.0, 1.0), opt: Options | None = None, workspace: Workspace | None = None, check: bool = True,
             **opt_kw) -> dict:
    """solve_rve_j2: J2 perfectly plastic solid on the device phase map `phi` (float32 [n0,n1,n2]),
    load ramp to macro_strain_final (and macro_stress_final on the stress_mask components).
    Returns dict(strain, stress, plastic_strain [6,*n] FP64, ep_acc [*n], history: list of dicts per
    increment (strain_mean, stress_mean, newton, minres, r_newton, status), status)."""
    torch = _torch()
    lib = load_library()
    if not (phi.is_cuda and phi.dtype == torch.float32 and phi.dim() == 3 and phi.is_contiguous()):
        raise ValueError("phi must be a contiguous float32 CUDA tensor of shape (n0, n1, n2)")
    n = tuple(phi.shape)
    opt = opt or default_options(**opt_kw)
    g = make_grid(n, L)
    mat = J2Material(float(young), float(poisson), float(yield_stress))
    jo = J2Options(int(increments), int(max_newton), float(newton_tol), float(lin_tol))
    E = np.ascontiguousarray(np.asarray(macro_strain_final, dtype=np.float64).reshape(6))
    S = None if macro_stress_final is None else np.ascontiguousarray(np.asarray(macro_stress_final, np.float64).reshape(6))
    nbytes = lib.rve_j2_workspace_bytes(ctypes.byref(g), ctypes.byref(opt))
    if nbytes == 0:
        raise RveError(RVE_EINVAL, "rve_j2_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, phi.device)
    f = lambda: torch.empty((6,) + n, dtype=torch.float64, device=phi.device)  # noqa: E731
    strain, stress, eps_p = f(), f(), f()
    ep = torch.empty(n, dtype=torch.float64, device=phi.device)
    hist = (J2Increment * int(increments))()
    cur = torch.cuda.current_stream(phi.device)
    ss = _solver_stream(torch, phi.device)
    ss.wait_stream(cur)
    st = lib.solve_rve_j2(ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()), ctypes.byref(mat), _dp(E),
                          _dp(S) if S is not None else None, ctypes.byref(opt), ctypes.byref(jo),
                          ctypes.c_void_p(strain.data_ptr()), ctypes.c_void_p(stress.data_ptr()),
                          ctypes.c_void_p(eps_p.data_ptr()), ctypes.c_void_p(ep.data_ptr()), hist,
                          ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), ctypes.c_void_p(ss.cuda_stream))
    cur.wait_stream(ss)
    if check and st < 0:
        raise RveError(st, "solve_rve_j2")
    history = [dict(strain_mean=np.array(h.strain_mean[:]), stress_mean=np.array(h.stress_mean[:]), newton=h.newton,
                    minres=h.minres, r_newton=h.r_newton, status=h.status) for h in hist]
    return dict(strain=strain, stress=stress, plastic_strain=eps_p, ep_acc=ep, history=history, status=int(st))


def solve_modbfft(phi, C_solid, macro_strain, *, alpha: float | None = None, tol: float = 1e-6,
                  max_iter: int = 5000, L=(1.0, 1.0, 1.0), want_fields: bool = True, timed: bool = False,
                  workspace: Workspace | None = None, check: bool = True) -> dict:
    """solve_rve_modbfft (one macroscopic strain, FP64): returns dict(strain, stress [6,*n] FP64 or None,
    eff_stress [6], iterations, rel_residual, alpha, pass_ms {pass: ms} when timed, status)."""
    torch = _torch()
    lib = load_library()
    if not (phi.is_cuda and phi.dtype == torch.float32 and phi.dim() == 3 and phi.is_contiguous()):
        raise ValueError("phi must be a contiguous float32 CUDA tensor of shape (n0, n1, n2)")
    n = tuple(phi.shape)
    g = make_grid(n, L)
    C = np.ascontiguousarray(np.asarray(C_solid, dtype=np.float64).reshape(36))
    E = np.ascontiguousarray(np.asarray(macro_strain, dtype=np.float64).reshape(6))
    nbytes = lib.rve_modbfft_workspace_bytes(ctypes.byref(g))
    if nbytes == 0:
        raise RveError(RVE_EUNSUPPORTED_SIZE, "rve_modbfft_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, phi.device)
    strain = torch.empty((6,) + n, dtype=torch.float64, device=phi.device) if want_fields else None
    stress = torch.empty((6,) + n, dtype=torch.float64, device=phi.device) if want_fields else None
    eff = np.zeros(6)
    st = ModbfftStats()
    st.timed = 1 if timed else 0
    cur = torch.cuda.current_stream(phi.device)
    ss = _solver_stream(torch, phi.device)
    ss.wait_stream(cur)
    rc = lib.solve_rve_modbfft(ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()), _dp(C), _dp(E),
                               float(alpha) if alpha is not None else 0.0, float(tol), int(max_iter),
                               ctypes.c_void_p(strain.data_ptr()) if strain is not None else None,
                               ctypes.c_void_p(stress.data_ptr()) if stress is not None else None, _dp(eff),
                               ctypes.byref(st), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                               ctypes.c_void_p(ss.cuda_stream))
    cur.wait_stream(ss)
    if check and rc < 0:
        raise RveError(rc, "solve_rve_modbfft")
    out = dict(strain=strain, stress=stress, eff_stress=eff, iterations=int(st.iterations),
               rel_residual=float(st.rel_residual), alpha=float(st.alpha), status=int(rc))
    if timed:
        out["pass_ms"] = {k: (float(st.pass_ms[i]), int(st.pass_launches[i])) for i, k in enumerate(MODBFFT_PASSES)}
    return out


def j2_return_map(phi, young: float, poisson: float, yield_stress: float, strain, plastic_strain):
    """rve_j2_return_map on device fields (FP64 [6, ...], phi float32): returns (stress [6, ...],
    tangent data [7, ...]: a and m of C_t = phi (C_e - a I_dev - m m))."""
    torch = _torch()
    lib = load_library()
    nv = int(phi.numel())
    mat = J2Material(float(young), float(poisson), float(yield_stress))
    sig = torch.empty_like(strain)
    tan = torch.empty((7,) + tuple(strain.shape[1:]), dtype=torch.float64, device=strain.device)
    st = lib.rve_j2_return_map(nv, ctypes.c_void_p(phi.data_ptr()), ctypes.byref(mat),
                               ctypes.c_void_p(strain.data_ptr()), ctypes.c_void_p(plastic_strain.data_ptr()),
                               ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(tan.data_ptr()),
                               _stream_ptr(torch, strain.device))
    if st != RVE_OK:
        raise RveError(st, "rve_j2_return_map")
    return sig, tan


def solve_batch(rves, C_solid, *, C_void=None, opt: Options | None = None, want_stress: bool = False,
                workspace: Workspace | None = None, check: bool = True, **opt_kw) -> dict:
    """solve_rve_batch: `rves` is a list of (phi [n0,n1,n2] float32 CUDA tensor, macro strains [nc,6]) or
    (phi, macro strains, macro stresses) under mixed control; grids may differ.  Returns
    dict(results=[per-RVE dict like solve()], status)."""
    torch = _torch()
    lib = load_library()
    opt = opt or default_options(**opt_kw)
    fdt = torch.float32 if opt.precision == FP32_MIXED else torch.float64
    C = _stiffness(C_solid, C_void)
    keep = [C]
    items = (BatchItem * len(rves))()
    results = []
    dev = rves[0][0].device
    for i, rv in enumerate(rves):
        phi, E = rv[0], rv[1]
        if not (phi.is_cuda and phi.dtype == torch.float32 and phi.dim() == 3 and phi.is_contiguous()):
            raise ValueError("each phi must be a contiguous float32 CUDA tensor (n0, n1, n2)")
        E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, 6))
        n = tuple(phi.shape)
        nc = E.shape[0]
        r = dict(strain=torch.empty((nc, 6) + n, dtype=fdt, device=dev),
                 stress=torch.empty((nc, 6) + n, dtype=fdt, device=dev) if want_stress else None,
                 eff_stress=np.zeros((nc, 6)), mean_strain=np.zeros((nc, 6)), iterations=np.zeros(nc, dtype=np.int32),
                 rel_residual=np.zeros(nc))
        results.append(r)
        keep.append(E)
        it = items[i]
        it.grid = make_grid(n)
        it.voxel_fraction_field = phi.data_ptr()
        it.phase_stiffness = _dp(C)
        it.macro_strain = _dp(E)
        it.n_cases = nc
        it.eps0 = None
        it.strain_out = r["strain"].data_ptr()
        it.stress_out = r["stress"].data_ptr() if want_stress else None
        it.eff_stress = _dp(r["eff_stress"])
        it.iterations = r["iterations"].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        it.rel_residual = _dp(r["rel_residual"])
        it.mean_strain = _dp(r["mean_strain"])
        if len(rv) > 2 and rv[2] is not None:
            S = np.ascontiguousarray(np.broadcast_to(np.asarray(rv[2], dtype=np.float64).reshape(-1, 6), (nc, 6)))
            keep.append(S)
            it.macro_stress = _dp(S)
    nbytes = lib.rve_batch_workspace_bytes(items, len(rves), ctypes.byref(opt))
    if nbytes == 0:
        raise RveError(RVE_EINVAL, "rve_batch_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, dev)
    cur = torch.cuda.current_stream(dev)
    ss = _solver_stream(torch, dev)
    ss.wait_stream(cur)
    st = lib.solve_rve_batch(items, len(rves), ctypes.byref(opt), ctypes.c_void_p(ws.data_ptr()),
                             ctypes.c_size_t(ws.numel()), ctypes.c_void_p(ss.cuda_stream))
    cur.wait_stream(ss)
    for i, r in enumerate(results):
        r["status"] = int(items[i].status)
    del keep
    if check and st < 0:
        raise RveError(st, "solve_rve_batch")
    return dict(results=results, status=int(st))


def apply(x, phi=None, C_solid=None, *, C_void=None, mode: int = APPLY_OPERATOR, L=(1.0, 1.0, 1.0),
          scheme: int = ROTATED, nyquist: int = NYQ_NATURAL, stress_mask: int = 0, workspace: Workspace | None = None):
    """rve_apply on fields x (torch [nc,6,n0,n1,n2], float32 -> FP32 kernels, float64 -> FP64 kernels)."""
    torch = _torch()
    lib = load_library()
    if not (x.is_cuda and x.dim() == 5 and x.shape[1] == 6 and x.is_contiguous()):
        raise ValueError("x must be a contiguous CUDA tensor of shape (n_cases, 6, n0, n1, n2)")
    prec = FP32_MIXED if x.dtype == torch.float32 else FP64
    if x.dtype not in (torch.float32, torch.float64):
        raise ValueError("x must be float32 or float64")
    n = tuple(x.shape[2:])
    nc = x.shape[0]
    g = make_grid(n, L)
    C = _stiffness(C_solid if C_solid is not None else np.eye(6), C_void)
    y = torch.empty_like(x)
    nbytes = lib.rve_apply_workspace_bytes(ctypes.byref(g), nc, prec)
    if nbytes == 0:
        raise RveError(RVE_EUNSUPPORTED_SIZE if not all(supported_length(v) for v in n) else RVE_EINVAL,
                       "rve_apply_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, x.device)
    phip = ctypes.c_void_p(phi.data_ptr()) if phi is not None else None
    st = lib.rve_apply(ctypes.byref(g), phip, _dp(C), nc, prec, scheme, nyquist, int(stress_mask), mode,
                       ctypes.c_void_p(x.data_ptr()),
                       ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                       _stream_ptr(torch, x.device))
    if st != RVE_OK:
        raise RveError(st, "rve_apply")
    return y
