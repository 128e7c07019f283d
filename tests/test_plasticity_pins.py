"""CPU pins of the nonlinear oracle (oracle.plasticity): J2 perfect plasticity, eqs. Slin, galnonlin,
galrlin, galrnewton (sections "Non linear extension", "Validation for non linear material response")."""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import plasticity as pl
from tests import bruteforce as bf

E, NU, SY = 1700.0, 0.4, 70.0  # MPa: the paper's PA12 and yield stress
ALL_BUT_11 = 0b111110           # uniaxial stress along 11: the other five components stress-free


def _random_strains(seed, count, scale):
    return (li.random_field((6, count), seed, scale))


def test_return_map_elastic_below_yield_and_on_the_yield_surface_above():
    K, mu = pl.bulk_shear(E, NU)
    eps = _random_strains(1, 400, 0.08)
    eps_p = _random_strains(2, 400, 0.01)
    eps_p -= pl.ONE[:, None] * (eps_p[0] + eps_p[1] + eps_p[2]) / 3.0  # plastic strain is deviatoric
    phi = 0.2 + 0.8 * li.uniforms(3, 400)
    sig, Ct, dep, plastic = pl.return_map(eps, eps_p, phi, E, NU, SY)
    ee = eps - eps_p
    Ce = K * np.outer(pl.ONE, pl.ONE) + 2 * mu * pl.I_DEV
    assert plastic.any() and (~plastic).any()
    el = ~plastic
    np.testing.assert_allclose(sig[:, el], phi[el] * (Ce @ ee[:, el]), rtol=1e-13, atol=1e-10)
    np.testing.assert_allclose(Ct[el], phi[el, None, None] * Ce, rtol=1e-14)
    s = sig / phi
    tr = s[0] + s[1] + s[2]
    dev = s - pl.ONE[:, None] * tr / 3.0
    q = np.sqrt(1.5) * np.sqrt(np.sum(dev * dev, axis=0))
    np.testing.assert_allclose(q[plastic], SY, rtol=1e-12)
    assert np.all(q[el] <= SY)
    # volumetric response untouched; the plastic increment is deviatoric and along the stress deviator
    np.testing.assert_allclose(tr, 3 * K * (ee[0] + ee[1] + ee[2]), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(dep[0] + dep[1] + dep[2], 0.0, atol=1e-15)
    cos = np.sum(dep * dev, axis=0) / (np.linalg.norm(dep, axis=0) * np.linalg.norm(dev, axis=0) + 1e-300)
    np.testing.assert_allclose(cos[plastic], 1.0, atol=1e-12)
    # the return lands where the elastic law of the updated plastic strain gives the stress
    np.testing.assert_allclose(s[:, plastic], Ce @ (ee - dep)[:, plastic], rtol=1e-11, atol=1e-8)


def test_consistent_tangent_is_the_derivative_of_the_return_map():
    eps = _random_strains(4, 60, 0.06)
    eps_p = _random_strains(5, 60, 0.005)
    eps_p -= pl.ONE[:, None] * (eps_p[0] + eps_p[1] + eps_p[2]) / 3.0
    phi = 0.3 + 0.7 * li.uniforms(6, 60)
    _, Ct, _, plastic = pl.return_map(eps, eps_p, phi, E, NU, SY)
    assert plastic.sum() > 10
    h = 1e-7
    fd = np.zeros_like(Ct)
    for b in range(6):
        e1 = eps.copy()
        e2 = eps.copy()
        e1[b] += h
        e2[b] -= h
        s1 = pl.return_map(e1, eps_p, phi, E, NU, SY)[0]
        s2 = pl.return_map(e2, eps_p, phi, E, NU, SY)[0]
        fd[:, :, b] = ((s1 - s2) / (2 * h)).T
    np.testing.assert_allclose(Ct, fd, rtol=0, atol=2e-5 * E)
    # symmetric, and singular along the flow direction on the yield surface
    np.testing.assert_allclose(Ct, np.swapaxes(Ct, 1, 2), atol=1e-9)
    ev = np.linalg.eigvalsh(Ct[plastic])
    assert np.all(np.abs(ev).min(axis=1) < 1e-9 * E)


@pytest.mark.parametrize("phi0", [1.0, 0.6])
def test_homogeneous_cell_uniaxial_stress_closed_form(phi0):
    """A homogeneous cell under uniaxial stress (the other components stress-free) has no fluctuation:
    sigma_11 = phi E eps_11 up to the yield strain, then phi sigma_y (no hardening); the lateral strain
    is -nu eps_11 elastically, then nu sy/E - (eps_11 + sy/E)/2 (incompressible plastic flow)."""
    n = (2, 3, 2)
    phi = np.full(n, phi0)
    Ef = np.array([-0.1, 0, 0, 0, 0, 0])
    out = pl.solve_j2(n, phi, E, NU, SY, Ef, increments=20, stress_mask=ALL_BUT_11, Sbar_final=np.zeros(6),
                      newton_tol=1e-10, lin_tol=1e-12)
    assert out["status"] == 0
    ey = SY / E
    for k, h in enumerate(out["history"]):
        e11 = -0.1 * (k + 1) / 20
        s11 = phi0 * max(E * e11, -SY)
        lat = -NU * e11 if e11 >= -ey else NU * ey - (e11 + ey) / 2
        np.testing.assert_allclose(h["stress_mean"], [s11, 0, 0, 0, 0, 0], atol=1e-9 * SY)
        np.testing.assert_allclose(h["strain_mean"], [e11, lat, lat, 0, 0, 0], atol=1e-10)
        assert h["newton"] <= 4
    np.testing.assert_allclose(out["eps"] - out["eps"].mean(axis=(1, 2, 3), keepdims=True), 0.0, atol=1e-13)


def _dense_j2(n, phi, Ef, increments, stress_mask=0, newton=60):
    """Brute force of the same incremental problem: the strain is Ebar + Z y with Z the compatible
    zero-mean stencil strains (and uniform strains on the stress-controlled components); Newton with
    the dense Jacobian Z^T C_t Z (least squares: voids make it singular) on Z^T (sigma - Sbar) = 0.
    No FFT, no MINRES.  Returns the stress field after each increment."""
    n = tuple(n)
    N = int(np.prod(n))
    KL = [a for a in range(6) if (stress_mask >> a) & 1]
    Q = bf.compatible_basis(n)
    M = np.zeros((6 * N, len(KL)))
    for j, a in enumerate(KL):
        M[a * N:(a + 1) * N, j] = 1.0
    Z = np.concatenate([Q, M], axis=1)
    y = np.zeros(Z.shape[1])
    eps_p = np.zeros((6, N))
    out = []
    for inc in range(1, increments + 1):
        Eb = np.array([0.0 if a in KL else Ef[a] * inc / increments for a in range(6)])
        for _ in range(newton):
            eps = (np.repeat(Eb[:, None], N, axis=1).reshape(-1) + Z @ y).reshape(6, N)
            sig, Ct, dep, _ = pl.return_map(eps, eps_p, phi.reshape(-1), E, NU, SY)
            R = Z.T @ sig.reshape(-1)
            K6 = np.zeros((6, N, 6, N))
            idx = np.arange(N)
            for a in range(6):
                for b in range(6):
                    K6[a, idx, b, idx] = Ct[:, a, b]
            J = Z.T @ K6.reshape(6 * N, 6 * N) @ Z
            dy = np.linalg.lstsq(J, -R, rcond=1e-13)[0]
            y = y + dy
            if np.abs(dy).max() < 1e-14:
                break
        eps = (np.repeat(Eb[:, None], N, axis=1).reshape(-1) + Z @ y).reshape(6, N)
        sig, _, dep, _ = pl.return_map(eps, eps_p, phi.reshape(-1), E, NU, SY)
        eps_p = eps_p + dep
        out.append(sig.reshape((6,) + n))
    return out


@pytest.mark.parametrize("mask", [0, ALL_BUT_11])
def test_heterogeneous_cell_matches_dense_newton(mask):
    """A 4x3x3 cell with a void column and graded solid fractions, compressed past first yield: the
    oracle's FFT/MINRES Newton solve and the dense brute force give the same (unique) stress fields
    after every increment."""
    n = (4, 3, 3)
    phi = 0.4 + 0.6 * li.uniforms(21, 36).reshape(n)
    phi[1, 1, :] = 0.0
    Ef = np.array([-0.06, 0.01, 0, 0, 0, 0.02])
    out = pl.solve_j2(n, phi, E, NU, SY, Ef, increments=3, stress_mask=mask, Sbar_final=np.zeros(6),
                      newton_tol=1e-11, lin_tol=1e-13, max_newton=60)
    ref = _dense_j2(n, phi, Ef, 3, stress_mask=mask)
    assert out["status"] == 0
    assert np.any(out["eps_p"] != 0)
    for k in range(3):
        np.testing.assert_allclose(out["history"][k]["stress_mean"], ref[k].reshape(6, -1).mean(axis=1),
                                   rtol=0, atol=1e-8 * SY)
    np.testing.assert_allclose(out["sigma"], ref[-1], rtol=0, atol=1e-7 * SY)
