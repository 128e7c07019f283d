"""GPU parity of the lattice phase maps (include/rve_geometry.h) against the FP64 CPU oracle
(oracle.geometry): sections "Voigt approaches", "Phase-field smoothening", "Combined smoothening".

Bars: the plain-voxel and Voigt fine-grid maps count inside/outside decisions and match bit for bit;
the VA map is one division and a clip of the same distance, equal to 1e-15.  The phase-field maps
go through FP64 FFTs on both sides (different factorisations and summation orders): the averages
before the threshold agree to 1e-12 absolute; after the threshold they agree wherever the oracle's
value is more than 1e-10 away from the threshold, and near it either side's choice is accepted.
"""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import geometry as og

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _geo():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_00733_amd import geometry
    return geometry


def _random_struts(seed, count, rmax=0.08):
    u = li.uniforms(seed, count * 7)
    S = np.zeros((count, 7))
    S[:, 0:3] = u[:3 * count].reshape(count, 3) * 1.4 - 0.2
    S[:, 3:6] = S[:, 0:3] + 0.6 * (u[3 * count:6 * count].reshape(count, 3) - 0.5)
    S[:, 6] = rmax * (0.2 + 0.8 * u[6 * count:])
    S[0, 3:6] = S[0, 0:3]  # a sphere: zero-length axis
    return S


LATTICES = {
    "octet": li.octet_struts(0.061),
    "random40": _random_struts(11, 40),
}
GRIDS = [((20, 24, 18), (1.0, 1.2, 0.9)), ((9, 7, 5), (1.0, 1.0, 1.0)), ((1, 16, 3), (0.5, 1.0, 2.0))]


@pytest.mark.parametrize("lat", sorted(LATTICES))
@pytest.mark.parametrize("grid", range(len(GRIDS)))
def test_voigt_maps_vs_oracle(lat, grid):
    geo = _geo()
    S = LATTICES[lat]
    n, L = GRIDS[grid]
    pv, pv32 = geo.phase_map(n, S, geo.PV, L=L, want_f32=True)
    np.testing.assert_array_equal(pv.cpu().numpy(), og.phase_pv(n, S, L))
    np.testing.assert_array_equal(pv32.cpu().numpy(), og.phase_pv(n, S, L).astype(np.float32))
    for sub in (1, 2, 5):
        vfg = geo.phase_map(n, S, geo.VFG, sub=sub, L=L).cpu().numpy()
        np.testing.assert_array_equal(vfg, og.phase_vfg(n, S, sub, L))
    for ell in (L[0] / n[0], 0.037):
        va = geo.phase_map(n, S, geo.VA, ell=ell, L=L).cpu().numpy()
        np.testing.assert_allclose(va, og.phase_va(n, S, L, ell), rtol=0, atol=1e-15)


def _check_thresholded(phi, raw, o_phi, o_raw, thr):
    np.testing.assert_allclose(raw, o_raw, rtol=0, atol=1e-12)
    near = np.abs(o_raw - thr) <= 1e-10
    np.testing.assert_array_equal(phi[~near] == 0, o_phi[~near] == 0)   # the threshold decisions
    np.testing.assert_allclose(phi[~near], o_phi[~near], rtol=0, atol=1e-12)
    assert np.all((phi[near] == 0) | (phi[near] == raw[near]))


FIELD_CASES = [
    # coarse grid, cell, ratio, eps: ragged fine lengths (odd axis 2, odd row count, odd ratio^2)
    ((12, 10, 16), (1.0, 1.3, 0.8), 3, 1.0),
    ((9, 5, 5), (1.0, 1.0, 1.0), 3, 0.5),
    ((8, 6, 10), (1.0, 1.0, 1.0), 1, 1.0),
    ((6, 8, 4), (1.0, 1.0, 1.0), 5, 1.0),
    ((16, 16, 16), (1.0, 1.0, 1.0), 4, 1.0),
]


@pytest.mark.parametrize("case", range(len(FIELD_CASES)))
def test_phase_field_vs_oracle(case):
    geo = _geo()
    n, L, ratio, eps = FIELD_CASES[case]
    S = li.octet_struts(0.07)
    phi, raw = geo.phase_field(n, S, ratio, eps=eps, L=L)
    o_phi, o_raw = og.phase_field(n, S, ratio, L=L, eps=eps)
    _check_thresholded(phi.cpu().numpy(), raw.cpu().numpy(), o_phi, o_raw, 0.05)
    # periodicity keeps the mean: the PFS density is that of VFG with the fine grid's points
    vfg = geo.phase_map(n, S, geo.VFG, sub=ratio, L=L)
    assert abs(raw.mean().item() - vfg.mean().item()) < 1e-13


@pytest.mark.parametrize("case", [0, 1, 4])
def test_combined_smoothening_vs_oracle(case):
    geo = _geo()
    n, L, ratio, eps = FIELD_CASES[case]
    S = li.octet_struts(0.07)
    va = geo.phase_map(n, S, geo.VA, L=L)
    phi, raw = geo.phase_field(n, S, ratio, eps=eps, L=L, source=va)
    o_va = og.phase_va(n, S, L)
    o_phi, o_raw = og.phase_field(n, S, ratio, L=L, eps=eps, source=o_va)
    _check_thresholded(phi.cpu().numpy(), raw.cpu().numpy(), o_phi, o_raw, 0.05)
    assert abs(raw.mean().item() - va.mean().item()) < 1e-13


def test_phase_field_options_and_outputs():
    """ell = 0 leaves omega unchanged (the coarse average of the fine indicator, i.e. VFG); a
    threshold above 1 empties the map; the FP32 output is the rounded FP64 one."""
    geo = _geo()
    n, S = (10, 12, 8), li.octet_struts(0.08)
    phi, raw = geo.phase_field(n, S, 2, ell=0.0, threshold=-1.0)
    vfg = geo.phase_map(n, S, geo.VFG, sub=2)
    np.testing.assert_allclose(raw.cpu().numpy(), vfg.cpu().numpy(), rtol=0, atol=1e-14)
    np.testing.assert_array_equal(phi.cpu().numpy(), raw.cpu().numpy())
    phi, raw, p32 = geo.phase_field(n, S, 2, threshold=1.5, want_f32=True)
    assert phi.abs().max().item() == 0.0 and p32.abs().max().item() == 0.0 and raw.max().item() > 0.5
    phi, raw, p32 = geo.phase_field(n, S, 2, want_f32=True)
    np.testing.assert_array_equal(p32.cpu().numpy(), phi.cpu().numpy().astype(np.float32))


def test_errors_are_reported_before_launch():
    geo = _geo()
    import paper_2110_00733_amd as rve
    S = li.octet_struts(0.05)
    with pytest.raises(rve.RveError) as e:
        geo.phase_field((7, 8, 8), S, 1)          # fine length 7 is not 5-smooth
    assert e.value.status == rve.RVE_EUNSUPPORTED_SIZE
    with pytest.raises(rve.RveError) as e:
        geo.phase_field((8, 8, 8), S, 135)        # 1080 > the longest fine axis
    assert e.value.status == rve.RVE_EUNSUPPORTED_SIZE
    with pytest.raises(rve.RveError) as e:
        geo.phase_map((8, 8, 8), S, geo.VA, ell=-1.0)
    assert e.value.status == rve.RVE_EINVAL
    with pytest.raises(rve.RveError) as e:
        geo.phase_map((8, 8, 8), S, geo.VFG, sub=0)
    assert e.value.status == rve.RVE_EINVAL
    with pytest.raises(rve.RveError) as e:
        geo.phase_field((8, 8, 8), S, 2, eps=0.0)
    assert e.value.status == rve.RVE_EINVAL
    small = rve.Workspace()
    small.get(256, torch.device("cuda:0"))
    lib = geo.geolib()
    import ctypes
    n = (ctypes.c_int32 * 3)(8, 8, 8)
    L = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    out = torch.empty((8, 8, 8), dtype=torch.float64, device="cuda:0")
    st = torch.from_numpy(S).cuda()
    rc = lib.rve_phase_field(n, L, ctypes.c_void_p(st.data_ptr()), 24, 2, 0.05, 1.0, 0.05, None,
                             ctypes.c_void_p(out.data_ptr()), None, None, ctypes.c_void_p(small.buf.data_ptr()),
                             small.buf.numel(), None)
    assert rc == rve.RVE_ENOMEM


def test_density_study_size_vs_oracle():
    """The density-study configuration at its full size: 54^3 coarse voxels, fine grid 540^3
    (ratio 10), octet at about 10 % density; every coarse voxel of PFS compared with the oracle."""
    geo = _geo()
    n, ratio = 54, 10
    S = li.octet_struts(0.0466)
    phi, raw = geo.phase_field(n, S, ratio)
    o_phi, o_raw = og.phase_field(n, S, ratio)
    _check_thresholded(phi.cpu().numpy(), raw.cpu().numpy(), o_phi, o_raw, 0.05)


def test_profiler_times_each_phase_field_pass():
    """With the library's event timing on, one phase-field call records one launch of each of its five
    passes and a phase map one launch of its kernel; nothing else is counted."""
    geo = _geo()
    import paper_2110_00733_amd as rve
    S = li.octet_struts(0.06)
    rve.profile_reset()
    rve.profile_enable(True)
    try:
        geo.phase_field((12, 12, 12), S, 4)
        geo.phase_map((12, 12, 12), S, geo.VA)
    finally:
        rve.profile_enable(False)
    prof = rve.profile_read()
    for k in ("G1_source_fft_axis2", "G2_fft_axis1", "G3_fft_axis0_helmholtz", "G4_ifft_axis1",
              "G5_ifft_axis2_coarsen", "M_phase_map"):
        assert prof[k][1] == 1 and prof[k][0] > 0, k
    assert all(v == (0.0, 0) for k, v in prof.items() if k[0] not in "GM")


def test_density_study_keeps_the_paper_relations():
    """Section "Analysis of the surface smoothening approaches": before the threshold the phase field
    keeps the density of its source (PFS that of VFG with the same fine grid, CS that of VA); the
    threshold only removes material."""
    _geo()
    from paper_2110_00733_amd import density_study as ds
    out = ds.run(0.1, grids=((24, 4), (36, 3)), radius=0.0466, log=lambda *a: None)
    assert out["radius"] == 0.0466 and len(out["rows"]) == 2
    for row in out["rows"]:
        assert abs(row["PFS_before_threshold"] - row["VFG"]) < 1e-13
        assert abs(row["CS_before_threshold"] - row["VA"]) < 1e-13
        assert row["PFS"] <= row["PFS_before_threshold"] + 1e-15 and row["CS"] <= row["CS_before_threshold"] + 1e-15
