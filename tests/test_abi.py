"""C ABI checks that need no GPU: the library loads, exports every function include/rve.h declares,
and host-side validation returns the documented status codes."""
import os
import re

import numpy as np
import pytest

import lattice_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rve():
    import paper_2110_00733_amd as rve
    if not os.path.exists(rve.LIB_PATH):
        pytest.skip("librve.so not built")
    return rve


def _declared():
    txt = open(os.path.join(ROOT, "include", "rve.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"sizeof"})


def test_library_exports_every_declared_symbol():
    rve = _rve()
    lib = rve.load_library()
    names = _declared()
    assert "solve_rve" in names and "rve_apply" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(rve.ABI_SYMBOLS) == names


def test_supported_lengths():
    rve = _rve()
    for n in (2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256):
        assert rve.supported_length(n), n
    for n in (0, 1, 7, 11, 13, 17, 1024):
        assert not rve.supported_length(n), n


def test_validation_codes():
    rve = _rve()
    C = li.isotropic_mandel(1.0, 0.3)
    E = np.eye(6)
    assert rve.validate(32, C, E) == rve.RVE_OK
    assert rve.validate((32, 7, 32), C, E) == rve.RVE_EUNSUPPORTED_SIZE
    assert rve.validate((32, 0, 32), C, E) == rve.RVE_EINVAL
    assert rve.validate(32, C, E, L=(1.0, -1.0, 1.0)) == rve.RVE_EINVAL
    Ebad = E.copy()
    Ebad[2, 2] = np.inf
    assert rve.validate(32, C, Ebad) == rve.RVE_ENONFINITE
    Cns = C.copy()
    Cns[0, 1] += 0.1
    assert rve.validate(32, Cns, E) == rve.RVE_EINVAL
    Cnan = C.copy()
    Cnan[3, 3] = np.nan
    assert rve.validate(32, Cnan, E) == rve.RVE_ENONFINITE
    for kw in ({"tol": 0.0}, {"tol": float("nan")}, {"max_iter": 0}, {"precision": 2}, {"nyquist": 3},
               {"scheme": 5}, {"max_refine": 0}, {"check_every": 0}, {"inner_floor": 1.0}, {"inner_safety": 0.0}):
        assert rve.validate(32, C, E, rve.default_options(**kw)) == rve.RVE_EINVAL, kw
    assert rve.status_string(rve.RVE_ENOMEM) == "RVE_ENOMEM"


def test_workspace_sizes_scale():
    rve = _rve()
    w1 = rve.workspace_bytes(64, 1)
    w6 = rve.workspace_bytes(64, 6)
    assert w1 > 0 and 5.5 * w1 < w6 < 6.5 * w1
    assert rve.workspace_bytes((64, 7, 64), 1) == 0
    f64 = rve.workspace_bytes(64, 1, rve.default_options(precision=rve.FP64))
    assert f64 > 0
    # 256^3, one FP32-mixed load case: well inside one GPU's HBM
    assert rve.workspace_bytes(256, 1) < 8 * 2 ** 30


def test_solve_without_gpu_raises_not_falls_back():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    rve = _rve()
    with pytest.raises(RuntimeError):
        rve.solve(torch.zeros(4, 4, 4), np.eye(6), np.eye(6))
