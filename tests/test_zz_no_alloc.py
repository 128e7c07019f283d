"""solve_rve_noalloc (static device scratch, no allocation) against solve_rve, through the C ABI.

Two calls in a row on the same GPU, the second on a smaller grid with fewer load cases, so the second
call runs in scratch that still holds the first call's contents.  Each result must match the
workspace-taking entry point's result on the same inputs: same iteration counts, effective stresses
within 1e-12 relative and strain fields within 1e-6 relative of their maximum (the two entry points
launch the same kernels; only the launch mechanism differs: direct launches with the direction update
inline, against captured graphs with it on a second stream).
"""
import ctypes

import numpy as np
import pytest

import lattice_inputs as li

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C1 = li.isotropic_mandel(1.0, 0.3)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _call(lib, rve, entry, phi, E, tol, precision, stream):
    n = tuple(phi.shape)
    nc = E.shape[0]
    g = rve.make_grid(n)
    opt = rve.default_options(tol=tol, precision=precision)
    C = np.ascontiguousarray(np.stack([np.zeros((6, 6)), C1]).reshape(72))
    E = np.ascontiguousarray(E, dtype=np.float64)
    fdt = torch.float32 if precision == rve.FP32_MIXED else torch.float64
    strain = torch.empty((nc, 6) + n, dtype=fdt, device="cuda")
    stress = torch.empty((nc, 6) + n, dtype=fdt, device="cuda")
    eff = np.zeros((nc, 6))
    its = np.zeros(nc, dtype=np.int32)
    res = np.zeros(nc)
    ip = its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    torch.cuda.synchronize()
    if entry == "noalloc":
        st = lib.solve_rve_noalloc(ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()), _dp(C), _dp(E), nc,
                                   ctypes.byref(opt), None, ctypes.c_void_p(strain.data_ptr()),
                                   ctypes.c_void_p(stress.data_ptr()), _dp(eff), ip, _dp(res),
                                   ctypes.c_void_p(stream.cuda_stream))
    else:
        nbytes = lib.rve_workspace_bytes(ctypes.byref(g), nc, ctypes.byref(opt))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        st = lib.solve_rve(ctypes.byref(g), ctypes.c_void_p(phi.data_ptr()), _dp(C), _dp(E), nc, ctypes.byref(opt),
                           None, ctypes.c_void_p(strain.data_ptr()), ctypes.c_void_p(stress.data_ptr()), _dp(eff),
                           ip, _dp(res), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nbytes),
                           ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    return st, strain.cpu().numpy(), stress.cpu().numpy(), eff, its, res


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_solve_rve_two_calls(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00733_amd as rve
    lib = rve.load_library()
    stream = torch.cuda.Stream()
    cases = [((32, 32, 32), 0.10, np.eye(6)[[0, 3]]),     # first call: two load cases
             ((16, 24, 20), 0.15, np.eye(6)[[1]])]        # second call: smaller grid, one case
    for n, rho, E in cases:
        phi, _ = li.octet_phase_map(n, rho)
        d = torch.as_tensor(phi, device="cuda")
        print(f"noalloc vs solve_rve: grid {n}, {E.shape[0]} case(s), precision {precision}", flush=True)
        a = _call(lib, rve, "noalloc", d, E, 1e-7, precision, stream)
        b = _call(lib, rve, "solve_rve", d, E, 1e-7, precision, stream)
        assert a[0] == 0 and b[0] == 0, (a[0], b[0])
        assert np.array_equal(a[4], b[4])                 # iterations
        assert _rel(a[3], b[3]) < 1e-12                   # <sigma>
        assert _rel(a[1], b[1]) < 1e-6                    # strain fluctuation
        assert _rel(a[2], b[2]) < 1e-6                    # stress
        assert np.all(a[5] <= 1e-7)


def test_noalloc_rejects_oversized_solve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_00733_amd as rve
    lib = rve.load_library()
    n = (64, 64, 64)
    E = np.eye(6)  # six cases at 64^3 need about 730 MiB, beyond the 128 MiB scratch
    g = rve.make_grid(n)
    opt = rve.default_options()
    assert lib.rve_workspace_bytes(ctypes.byref(g), 6, ctypes.byref(opt)) > lib.rve_noalloc_scratch_bytes()
    d = torch.full(n, 0.5, dtype=torch.float32, device="cuda")
    out = torch.empty((6, 6) + n, dtype=torch.float32, device="cuda")
    eff, its, res = np.zeros((6, 6)), np.zeros(6, dtype=np.int32), np.zeros(6)
    C = np.ascontiguousarray(np.stack([np.zeros((6, 6)), C1]).reshape(72))
    E = np.ascontiguousarray(E)
    st = lib.solve_rve_noalloc(ctypes.byref(g), ctypes.c_void_p(d.data_ptr()), _dp(C), _dp(E), 6, ctypes.byref(opt),
                               None, ctypes.c_void_p(out.data_ptr()), None, _dp(eff),
                               its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(res), None)
    assert st == rve.RVE_ENOMEM
    assert b"static scratch" in lib.rve_last_error()
