"""Lattice phase maps on the GPU: binding of include/rve_geometry.h.

Argument marshalling only: the distances, the Voigt maps, the phase-field FFTs, the coarse average
and the threshold all run in librve.so's kernels (sections "Voigt approaches", "Phase-field
smoothening", "Combined smoothening").  The strut list is uploaded once per call; maps come back as
torch tensors on the device, in FP64 and, for the solver, FP32.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import RVE_OK, RveError, Workspace, _stream_ptr, _torch, load_library

PV, VFG, VA = 0, 1, 2
MAX_STRUTS = 256
MAX_FINE = 1024

GEOMETRY_ABI_SYMBOLS = ("rve_phase_map", "rve_phase_field_workspace_bytes", "rve_phase_field")

_bound = None
_ws = Workspace()


def geolib():
    """librve.so with the rve_phase_* signatures declared."""
    global _bound
    lib = load_library()
    if _bound is lib:
        return lib
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.rve_phase_map.argtypes = [ip, dp, vp, i32, i32, i32, dbl, vp, vp, vp]
    lib.rve_phase_map.restype = ctypes.c_int
    lib.rve_phase_field_workspace_bytes.argtypes = [ip, i32]
    lib.rve_phase_field_workspace_bytes.restype = ctypes.c_size_t
    lib.rve_phase_field.argtypes = [ip, dp, vp, i32, i32, dbl, dbl, dbl, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.rve_phase_field.restype = ctypes.c_int
    _bound = lib
    return lib


def _n3(n):
    if isinstance(n, int):
        n = (n, n, n)
    n = tuple(int(v) for v in n)
    return n, (ctypes.c_int32 * 3)(*n)


def _L3(L):
    return (ctypes.c_double * 3)(*[float(v) for v in L])


def _struts(torch, struts, device):
    s = np.ascontiguousarray(np.asarray(struts, dtype=np.float64).reshape(-1, 7))
    return torch.from_numpy(s).to(device), s.shape[0]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def field_workspace_bytes(n, ratio: int) -> int:
    _, c = _n3(n)
    return int(geolib().rve_phase_field_workspace_bytes(c, int(ratio)))


def phase_map(n, struts, kind: int = VA, *, sub: int = 1, ell: float | None = None, L=(1.0, 1.0, 1.0),
              device="cuda:0", want_f32: bool = False):
    """PV / VFG (sub^3 points per voxel) / VA (width ell, default one voxel) map of the strut lattice.
    Returns the FP64 map, and the FP32 copy the solver reads when want_f32."""
    torch = _torch()
    n, c = _n3(n)
    if ell is None:
        ell = float(L[0]) / n[0]
    st, ns = _struts(torch, struts, device)
    phi = torch.empty(n, dtype=torch.float64, device=device)
    p32 = torch.empty(n, dtype=torch.float32, device=device) if want_f32 else None
    rc = geolib().rve_phase_map(c, _L3(L), _ptr(st), ns, int(kind), int(sub), float(ell), _ptr(phi), _ptr(p32),
                                _stream_ptr(torch, device))
    if rc != RVE_OK:
        raise RveError(rc, "rve_phase_map")
    return (phi, p32) if want_f32 else phi


def phase_field(n, struts, ratio: int, *, ell: float | None = None, eps: float = 1.0, threshold: float = 0.05,
                source=None, L=(1.0, 1.0, 1.0), device="cuda:0", want_f32: bool = False,
                workspace: Workspace | None = None):
    """Phase-field smoothening on the grid ratio * n (ell defaults to half a coarse voxel); with a
    coarse `source` map (a device tensor, e.g. the VA map) it is the combined smoothening.
    Returns (phi, phi before the threshold[, FP32 phi])."""
    torch = _torch()
    n, c = _n3(n)
    if ell is None:
        ell = 0.5 * float(L[0]) / n[0]
    st, ns = (None, 0) if source is not None else _struts(torch, struts, device)
    src = None
    if source is not None:
        src = source.to(device=device, dtype=torch.float64).contiguous()
        assert tuple(src.shape) == n
    nb = field_workspace_bytes(n, ratio)
    if nb == 0:
        raise RveError(-2, "rve_phase_field_workspace_bytes")
    ws = (workspace or _ws).get(nb, torch.device(device))
    phi = torch.empty(n, dtype=torch.float64, device=device)
    raw = torch.empty(n, dtype=torch.float64, device=device)
    p32 = torch.empty(n, dtype=torch.float32, device=device) if want_f32 else None
    rc = geolib().rve_phase_field(c, _L3(L), _ptr(st), ns, int(ratio), float(ell), float(eps), float(threshold),
                                  _ptr(src), _ptr(phi), _ptr(p32), _ptr(raw), _ptr(ws), ws.numel(),
                                  _stream_ptr(torch, device))
    if rc != RVE_OK:
        raise RveError(rc, "rve_phase_field")
    return (phi, raw, p32) if want_f32 else (phi, raw)
