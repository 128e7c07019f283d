"""CPU pins of the surface-smoothening oracle (sections "Voigt approaches", "Phase-field smoothening",
"Combined smoothening", "Analysis of the surface smoothening approaches")."""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import geometry as og

SQ2 = np.sqrt(2.0)


def _brute_distance(p, struts, samples=20001):
    """Distance to the union of capsules by sampling every strut axis densely, over all 27 periodic
    images of the unit cell (no nearest-image assumption)."""
    t = np.linspace(0.0, 1.0, samples)
    shifts = np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T
    best = np.inf
    for s in np.asarray(struts).reshape(-1, 7):
        seg = s[0:3][None, :] + t[:, None] * (s[3:6] - s[0:3])[None, :]
        for sh in shifts:
            best = min(best, np.sqrt(((seg + sh - p) ** 2).sum(1)).min() - s[6])
    return best


def test_octet_site_distances_closed_form():
    """FCC node: inside every strut end, D = -r.  Octahedral site (cube centre): the nearest strut axes
    (face centre to face centre) pass at 1/(2 sqrt 2).  Tetrahedral site (1/4,1/4,1/4): 1/4."""
    r = 0.05
    S = li.octet_struts(r)
    pts = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5], [0.25, 0.25, 0.25], [0.5, 0.0, 0.5], [0.75, 0.25, 0.75]])
    D = og.signed_distance(pts, S)
    np.testing.assert_allclose(D, [-r, 1 / (2 * SQ2) - r, 0.25 - r, -r, 0.25 - r], atol=1e-15)


def test_segment_distance_matches_brute_force():
    """Random points near random struts: the exact segment distance lies within half a sample spacing
    below the dense-sampling distance over all periodic images."""
    u = li.uniforms(4242, 40 * 7 + 40 * 3)
    S = np.zeros((40, 7))
    S[:, 0:3] = u[:120].reshape(40, 3)
    S[:, 3:6] = S[:, 0:3] + 0.5 * (u[120:240].reshape(40, 3) - 0.5)
    S[:, 6] = 0.02
    P = S[:, 0:3] + 0.5 * (S[:, 3:6] - S[:, 0:3]) + 0.3 * (u[280:400].reshape(40, 3) - 0.5)
    for s, p in zip(S, P):
        d = og.signed_distance(p[None, :], s[None, :])[0]
        b = _brute_distance(p, s)
        spacing = np.linalg.norm(s[3:6] - s[0:3]) / 20000
        assert d <= b + 1e-12 and b - d <= 0.5 * spacing + 1e-12


def test_octet_distance_map_against_points_and_symmetry():
    """The C distance map equals the point formula at the voxel centres, and the octet's cubic symmetry
    (axis permutations, mirror x -> 1 - x) leaves it unchanged."""
    r = 0.045
    S = li.octet_struts(r)
    n = 12
    D = og.distance_map(n, S)
    x = og.voxel_centres(n)
    pts = np.stack(np.meshgrid(*x, indexing="ij"), axis=-1).reshape(-1, 3)
    np.testing.assert_allclose(D.reshape(-1), og.signed_distance(pts, S), atol=1e-15)
    np.testing.assert_allclose(D, D.transpose(1, 2, 0), atol=1e-14)
    np.testing.assert_allclose(D, D.transpose(0, 2, 1), atol=1e-14)
    np.testing.assert_allclose(D, D[::-1, :, :], atol=1e-14)
    for p in pts[::97]:
        assert abs(og.signed_distance(p[None, :], S)[0] - _brute_distance(p, S, 4001)) < 1e-4


def test_pv_vfg_relations():
    """VFG with one sub-point is PV; VFG with S sub-points is the PV map of the grid S*n averaged over
    each voxel (the same points), and its density tends to the capsule union's volume."""
    S = li.octet_struts(0.06)
    n = 10
    np.testing.assert_array_equal(og.phase_vfg(n, S, 1), og.phase_pv(n, S))
    np.testing.assert_array_equal(og.phase_vfg(n, S, 3), og.coarsen(og.phase_pv(3 * n, S), 3))


def _cylinder(r):
    """One strut spanning the cell along axis 0: with the nearest image of its midpoint it is the
    periodic infinite cylinder of radius r around the line (x, 1/2, 1/2), volume fraction pi r^2."""
    return np.array([[0.0, 0.5, 0.5, 1.0, 0.5, 0.5, r]])


def test_cylinder_volume_fractions():
    r = 0.2
    exact = np.pi * r * r
    S = _cylinder(r)
    errs_va, errs_vfg = [], []
    for n in (16, 32, 64):
        errs_va.append(abs(og.relative_density(og.phase_va(n, S)) - exact))
        errs_vfg.append(abs(og.relative_density(og.phase_vfg(n, S, 8)) - exact))
    assert errs_va[-1] < 1e-3 * exact and errs_va[-1] < errs_va[0]
    assert errs_vfg[-1] < 2e-3 * exact
    # every voxel fraction of VA is within [0, 1] and 1 on the axis, 0 far away
    phi = og.phase_va(32, S)
    assert phi.min() == 0.0 and phi.max() == 1.0 and phi[:, 16, 16].min() == 1.0 and phi[:, 0, 0].max() == 0.0


def test_va_is_exact_voxel_fraction_at_a_planar_interface():
    """eq. phaselin at a plane: for a slab |x_0 - c| <= w with each voxel crossed by at most one face,
    phi(D) is exactly the fraction of the voxel inside the slab, so the density is exactly 2w."""
    n = 40
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    for c, w in ((0.5, 0.2137), (0.31, 0.1234), (0.77, 0.3)):
        d = x - c
        d = d - np.floor(d + 0.5)
        D = np.abs(d) - w
        phi = og.va_from_distance(D, h)
        lo, hi = x - h / 2, x + h / 2
        exact = np.zeros(n)
        for sh in (-1.0, 0.0, 1.0):
            exact += np.clip(np.minimum(hi, c + w + sh) - np.maximum(lo, c - w + sh), 0, None) / h
        np.testing.assert_allclose(phi, exact, atol=1e-12)
        assert abs(phi.mean() - 2 * w) < 1e-12


@pytest.mark.parametrize("eps", [1.0, 0.4])
def test_helmholtz_fourier_modes_are_eigenfunctions(eps):
    """eq. phase3: a Fourier mode of wave vector k is scaled by 1 / (1 + (ell^2/eps) |2 pi k / L|^2)."""
    m = (12, 10, 16)
    L = (1.0, 1.3, 0.8)
    ell = 0.07
    x = og.voxel_centres(m, L)
    X = np.meshgrid(*x, indexing="ij")
    for k in ((1, 0, 0), (2, -3, 5), (0, 0, 8), (6, 5, 1)):
        arg = sum(2 * np.pi * k[p] * X[p] / L[p] for p in range(3))
        xi2 = sum((2 * np.pi * k[p] / L[p]) ** 2 for p in range(3))
        for f in (np.cos(arg), np.sin(arg)):
            if np.abs(f).max() < 1e-8:
                continue
            np.testing.assert_allclose(og.helmholtz_smooth(f, L, ell, eps), f / (1 + ell * ell / eps * xi2),
                                       atol=1e-13)


def test_helmholtz_periodic_slab_closed_form():
    """A slab |x - 1/2| < w in a periodic unit cell: phi - (ell^2/eps) phi'' = omega has
    phi = 1 - A cosh(u/l) inside and B cosh((1/2 - u)/l) outside (u = |x - 1/2|, l = ell/sqrt eps),
    with value and slope continuous at u = w.  The spectral solution of the sampled slab converges to it;
    the slab faces sit on voxel faces."""
    m = 2048
    w = 0.25
    ell, eps = 0.02, 1.0
    x = (np.arange(m) + 0.5) / m
    omega = (np.abs(x - 0.5) < w).astype(np.float64)
    phi = og.helmholtz_smooth(omega.reshape(m, 1, 1), (1.0, 1.0, 1.0), ell, eps).reshape(m)
    l = ell / np.sqrt(eps)
    a, b = w / l, (0.5 - w) / l
    A = 1.0 / (np.cosh(a) + np.sinh(a) * np.cosh(b) / np.sinh(b))
    B = A * np.sinh(a) / np.sinh(b)
    u = np.abs(x - 0.5)
    exact = np.where(u < w, 1 - A * np.cosh(u / l), B * np.cosh((0.5 - u) / l))
    assert np.abs(phi - exact).max() < 2e-3
    assert abs(phi.mean() - 2 * w) < 1e-14


def test_phase_field_keeps_density_and_thresholds():
    """Periodicity makes the phase-field step keep the mean (the paper: PFS has the density of VFG with
    the same fine grid, CS that of VA); values below the 5 % threshold become zero, the rest are kept."""
    S = li.octet_struts(0.05)
    n, ratio = 12, 3
    phi, raw = og.phase_field(n, S, ratio)
    vfg = og.phase_vfg(n, S, ratio)
    assert abs(raw.mean() - vfg.mean()) < 1e-14
    np.testing.assert_array_equal(phi, np.where(raw < 0.05, 0.0, raw))
    assert (raw < 0.05).any() and (raw >= 0.05).any()
    va = og.phase_va(n, S)
    phi_cs, raw_cs = og.phase_field(n, S, ratio, source=va)
    assert abs(raw_cs.mean() - va.mean()) < 1e-14
    # smoothing spreads material: the support grows and the maximum drops
    assert (raw_cs > 1e-3).sum() > (va > 0).sum() and raw_cs.max() < va.max()


def test_coarsen_and_upsample():
    f = li.random_field((6, 4, 8), 77)
    np.testing.assert_allclose(og.coarsen(og.upsample(f, 3), 3), f, atol=1e-15)
    g = li.random_field((12, 8, 4), 78)
    assert abs(og.coarsen(g, 2).mean() - g.mean()) < 1e-15
