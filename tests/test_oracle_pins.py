"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test targets a distinct way the oracle could be wrong:
  - DFT/FFT: naive DFT vs closed forms (delta, pure tones, Parseval); FFT vs naive DFT.
  - Frequencies/projection (eqs. freq, galop, freqrot): the oracle's projection must be exactly the
    orthogonal projector onto the real-space 8-corner stencil strains (dense SVD, no FFT); invariants.
  - Operator + stiffness: plane-wave eigenvalues 2mu, 2mu, lambda+2mu of Ghat C on a homogeneous solid.
  - Solve (eq. gallin with MINRES): dense minimum-norm solve on tiny grids with voids; laminate closed
    forms along every axis (incl. a void layer and anisotropic grids); homogeneous medium; Krylov
    minimisation property of each MINRES iterate; symmetry/cubic/Voigt/Hill-Mandel of C_eff.
  - Paper behaviour: continuous frequencies + CG do not converge with voids, rotated + MINRES do.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import bruteforce as bf

C1 = li.isotropic_mandel(1.0, 0.3)
LAM, MU = 0.5769230769230769, 0.3846153846153846


# ------------------------------------------------------------------ transforms
def test_naive_dft_closed_forms():
    n = 12
    d = np.zeros(n, complex)
    d[0] = 1
    assert np.allclose(oracle.dft(d), np.ones(n), atol=1e-15)
    for k in (1, 5, 7):
        tone = np.exp(2j * np.pi * k * np.arange(n) / n)  # exp(+i...) -> forward DFT = n delta_k
        y = oracle.dft(tone, -1)
        ref = np.zeros(n, complex)
        ref[k] = n
        assert np.abs(y - ref).max() < 1e-12
    x = np.random.default_rng(0).standard_normal(n) + 0j
    assert np.isclose(np.sum(np.abs(oracle.dft(x)) ** 2), n * np.sum(np.abs(x) ** 2), rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 9, 12, 15, 16, 24, 25, 32, 48, 96, 7, 14])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_naive_dft(n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = oracle.fft(x, sign)
    ref = oracle.dft(x, sign)
    assert np.abs(y - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_fft3_separable_and_roundtrip():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))
    f = oracle.fft3(a, -1)
    ref = a.copy()
    for ax in range(3):
        ref = np.apply_along_axis(lambda v: oracle.dft(v, -1), ax, ref)
    assert np.abs(f - ref).max() < 1e-12
    back = oracle.fft3(f, +1)
    assert np.abs(back - a).max() < 1e-13


# ------------------------------------------------------------------ projection
GRIDS = [(4, 4, 4), (4, 6, 8), (5, 3, 4), (6, 5, 4)]


@pytest.mark.parametrize("n", GRIDS)
def test_projection_is_orthogonal_projector_onto_stencil_strains(n):
    L = (1.0, 1.3, 0.7)
    rng = np.random.default_rng(sum(n))
    B = bf.stencil_B(n, L)
    Q = bf.compatible_basis(n, L)
    # compatible fields are fixed
    eps = (B @ rng.standard_normal(B.shape[1])).reshape((6,) + n)
    assert np.abs(oracle.project(n, eps, L=L) - eps).max() < 1e-12 * np.abs(eps).max()
    # an arbitrary field is mapped into range(B) and the remainder is orthogonal to range(B)
    s = rng.standard_normal((6,) + n)
    ps = oracle.project(n, s, L=L).reshape(-1)
    assert np.abs(ps - Q @ (Q.T @ ps)).max() < 1e-12
    assert np.abs(B.T @ (s.reshape(-1) - ps)).max() < 1e-11


@pytest.mark.parametrize("n,m", [((8, 8, 8), (1, 2, 3)), ((8, 6, 4), (4, 1, 0)), ((8, 6, 4), (4, 3, 1)),
                                 ((5, 3, 4), (2, 1, 3)), ((8, 8, 8), (0, 0, 4)), ((6, 6, 6), (0, 0, 0))])
def test_projection_matrix_invariants(n, m):
    G = oracle.projection_matrix(n, m)
    assert np.abs(G.imag).max() < 1e-14
    G = G.real
    assert np.abs(G - G.T).max() < 1e-14          # major symmetry in Mandel form
    assert np.abs(G @ G - G).max() < 1e-13          # idempotent
    nyq = sum(1 for p in range(3) if n[p] % 2 == 0 and 2 * m[p] == n[p])
    vanishes = (tuple(m) == (0, 0, 0)) or nyq >= 2
    assert np.isclose(np.trace(G), 0.0 if vanishes else 3.0, atol=1e-13)


def test_projection_nyquist_modes():
    n = (8, 6, 4)
    # a single Nyquist index keeps a rank-3 projector under the natural reading, zero under zero-all
    G = oracle.projection_matrix(n, (4, 1, 1)).real
    assert np.isclose(np.trace(G), 3.0)
    Gz = oracle.projection_matrix(n, (4, 1, 1), nyquist=oracle.NYQ_ZERO_ALL).real
    assert np.abs(Gz).max() == 0.0
    # two Nyquist indices: the modified frequency itself vanishes
    assert np.abs(oracle.modified_frequency(n, (4, 3, 1))).max() == 0.0


def test_plane_wave_eigenvalues_homogeneous():
    """Ghat C restricted to compatible fields at one frequency has eigenvalues 2mu, 2mu, lambda+2mu."""
    n = (8, 8, 8)
    m = (1, 2, 3)
    G = oracle.projection_matrix(n, m).real
    ev = np.sort(np.linalg.eigvals(G @ C1 @ G).real)
    assert np.allclose(ev, [0, 0, 0, 2 * MU, 2 * MU, LAM + 2 * MU], atol=1e-12)
    # same through the full field operator: a real plane wave in the compatible space is an eigvector
    w = np.linalg.eigh(G @ C1 @ G)[1][:, -1]  # lambda + 2 mu mode
    x = np.indices(n)
    phase = 2 * np.pi * sum(m[p] * x[p] / n[p] for p in range(3))
    # the compatible mode for +k and -k share G (real, even), so cos(phase) * w is compatible
    f = w.reshape(6, 1, 1, 1) * np.cos(phase)[None]
    Af = oracle.apply(n, np.ones(n), C1, f)
    assert np.abs(Af - (LAM + 2 * MU) * f).max() < 1e-12


# ------------------------------------------------------------------ solves
@pytest.mark.parametrize("n,seed", [((4, 4, 4), 5), ((4, 6, 8), 6), ((5, 3, 4), 7)])
def test_minres_matches_dense_min_norm_solution(n, seed):
    phi = li.random_phi(n, seed, 0.4).astype(np.float64)
    E = np.array([1.0, 0.2, -0.3, 0.1, 0.05, -0.2])
    L = (1.0, 0.8, 1.2)
    e, s, sm = bf.min_norm_solution(n, phi, C1, E, L=L)
    r = oracle.solve(n, phi, C1, E, tol=1e-13, maxit=3000, L=L)
    assert r["status"] == 0 and r["true_residual"] < 1e-11
    assert np.abs(r["sigma_mean"] - sm).max() < 1e-12 * np.abs(sm).max()
    assert np.abs(r["sigma"] - s).max() < 1e-11 * np.abs(s).max()
    # zero-start MINRES on the consistent singular system returns the minimum-norm fluctuation,
    # including the (non-unique) strains of empty voxels
    assert np.abs(r["eps"] - e).max() < 1e-9 * np.abs(e).max()


def _random_spd_mandel(seed, scale):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((6, 6))
    return scale * (a @ a.T / 6 + np.eye(6))


@pytest.mark.parametrize("n,seed", [((4, 4, 4), 15), ((4, 6, 8), 16), ((5, 3, 4), 17)])
def test_operator_with_soft_phase_matches_dense(n, seed):
    """A(x) = Ghat : C(x) : x with C(x) = phi C1 + (1 - phi) C0 (section "Voigt approaches") for an
    anisotropic soft phase C0: against the dense projector onto the stencil strains (SVD, no FFT) applied
    to the dense block stiffness."""
    L = (1.0, 0.8, 1.2)
    phi = li.random_phi(n, seed, 0.4).astype(np.float64)
    C0 = _random_spd_mandel(seed, 0.05)
    Cs = _random_spd_mandel(seed + 100, 1.0)
    Q = bf.compatible_basis(n, L)
    K = bf.stiffness_matrix(phi, Cs, C0)
    x = li.random_field((6,) + n, seed + 1)
    ref = Q @ (Q.T @ (K @ x.reshape(-1)))
    got = oracle.apply(n, phi, Cs, x, C0=C0, L=L).reshape(-1)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # the soft-phase term is really there: dropping it changes the result at first order
    no_c0 = oracle.apply(n, phi, Cs, x, L=L).reshape(-1)
    assert np.abs(no_c0 - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("n,seed", [((4, 4, 4), 25), ((4, 6, 8), 26), ((5, 3, 4), 27)])
def test_minres_with_soft_phase_matches_dense_solution(n, seed):
    """With a soft instead of an empty phase the energy is positive definite on the compatible fields,
    so the solution is unique: the oracle's MINRES solve against the dense solve, strain, stress and
    average stress (all six components, anisotropic phases)."""
    L = (1.0, 0.8, 1.2)
    phi = li.random_phi(n, seed, 0.4).astype(np.float64)
    C0 = _random_spd_mandel(seed, 0.05)
    Cs = _random_spd_mandel(seed + 100, 1.0)
    E = np.array([0.4, -0.2, 0.1, 0.3, -0.15, 0.05])
    e, s, sm = bf.min_norm_solution(n, phi, Cs, E, C0=C0, L=L)
    r = oracle.solve(n, phi, Cs, E, tol=1e-13, maxit=3000, C0=C0, L=L)
    assert r["status"] == 0 and r["true_residual"] < 1e-11
    assert np.abs(r["sigma_mean"] - sm).max() < 1e-12 * np.abs(sm).max()
    assert np.abs(r["sigma"] - s).max() < 1e-11 * np.abs(s).max()
    assert np.abs(r["eps"] - e).max() < 1e-10 * np.abs(e).max()


@pytest.mark.parametrize("n,axis,prof,c", [((8, 4, 4), 0, [1, 1, 1, 1, .25, .25, .25, .25], 0.1),
                                           ((5, 6, 3), 1, [1, 0.5, 0, 0.75, 1, 1], 0.02),
                                           ((4, 4, 8), 2, [0.3, 1, 0, 0.8, 1, 0.6, 0.1, 0.9], 0.3)])
def test_laminate_with_soft_phase_closed_form(n, axis, prof, c):
    """Soft phase C0 = c C1: the Voigt stiffness is (phi + (1 - phi) c) C1, a laminate of the solid
    with the layer profile psi = phi + (1 - phi) c, whose closed form (Voigt in-plane, Reuss across)
    fixes C_eff; a void layer becomes a layer of stiffness c C1."""
    phi = li.laminate_phi(n, axis, prof)
    Ce, _ = oracle.effective_stiffness(n, phi, C1, tol=1e-13, maxit=500, C0=c * C1)
    psi = np.asarray(prof, dtype=np.float32).astype(np.float64)
    psi = psi + (1.0 - psi) * c
    ref = bf.laminate_closed_form(psi, axis, 1.0, 0.3)
    assert np.abs(Ce - ref).max() < 1e-11


# ------------------------------------------------------------------ mixed macroscopic control
def test_zero_frequency_projection_mixed_control():
    """eq. (galop) at xi = 0: the identity on the stress-controlled components, zero on the others."""
    for comps in ([], [1, 2, 3, 4, 5], [0, 3], [5]):
        mask = oracle.mask_of(comps)
        G = oracle.projection_matrix((6, 4, 5), (0, 0, 0), stress_mask=mask)
        assert np.array_equal(G, np.diag([1.0 if a in comps else 0.0 for a in range(6)]).astype(complex))
        # every other frequency is unchanged by the mask
        assert np.array_equal(oracle.projection_matrix((6, 4, 5), (1, 2, 3), stress_mask=mask),
                              oracle.projection_matrix((6, 4, 5), (1, 2, 3)))


@pytest.mark.parametrize("n,seed,comps,soft", [((4, 4, 4), 31, [1, 2, 3, 4, 5], True),
                                               ((4, 6, 8), 32, [0, 3], True),
                                               ((5, 3, 4), 33, [2, 4, 5], False),
                                               ((4, 4, 4), 34, [1, 2, 3, 4, 5], False)])
def test_mixed_control_matches_dense_minimisation(n, seed, comps, soft):
    """Mixed control (eq. galop at xi = 0, eq. gallin with the macroscopic stress) against the dense
    minimisation of the energy minus the work of the prescribed stress over compatible fluctuations and
    uniform stress-controlled strains; with a soft phase (unique) and with empty voxels (min-norm)."""
    L = (1.0, 0.8, 1.2)
    phi = li.random_phi(n, seed, 0.5 if soft else 0.3).astype(np.float64)
    C0 = 0.05 * C1 if soft else None
    E = np.array([0.4, -0.2, 0.1, 0.3, -0.15, 0.05])
    S = np.array([0.02, -0.01, 0.03, 0.015, -0.02, 0.01])
    mask = oracle.mask_of(comps)
    fl, sig, sm, em = bf.mixed_solution(n, phi, C1, E, comps, S, C0=C0, L=L)
    r = oracle.solve(n, phi, C1, E, tol=1e-13, maxit=4000, C0=C0, L=L, stress_mask=mask, Sbar=S)
    assert r["status"] == 0 and r["true_residual"] < 1e-11
    assert np.abs(r["sigma_mean"] - sm).max() < 1e-11 * np.abs(sm).max()
    assert np.abs(r["sigma_mean"][comps] - S[comps]).max() < 1e-11 * np.abs(sm).max()
    assert np.abs(r["strain_mean"] - em).max() < 1e-10 * np.abs(em).max()
    assert np.abs(r["sigma"] - sig).max() < 1e-10 * np.abs(sig).max()
    assert np.abs(r["eps"] - fl).max() < 1e-9 * np.abs(fl).max()


def test_mixed_control_consistent_with_effective_stiffness():
    """The macroscopic state of a mixed solve satisfies <sigma> = C_eff <eps> with C_eff from six
    strain-controlled solves; uniaxial stress gives E = 1/S_00 and nu = -S_10/S_00, S = C_eff^-1 (the
    uniaxial-stress modulus and Poisson ratio the paper reports)."""
    n = (6, 5, 4)
    phi = li.random_phi(n, 35, 0.5).astype(np.float64)
    C0 = 0.02 * C1
    Ce, _ = oracle.effective_stiffness(n, phi, C1, tol=1e-13, maxit=4000, C0=C0)
    Sc = np.linalg.inv(Ce)
    r = oracle.solve(n, phi, C1, li.uniaxial_strain(1.0), tol=1e-13, maxit=4000, C0=C0,
                     stress_mask=oracle.mask_of([1, 2, 3, 4, 5]))
    assert r["status"] == 0
    E_mod = r["sigma_mean"][0] / r["strain_mean"][0]
    nu = -r["strain_mean"][1] / r["strain_mean"][0]
    assert abs(E_mod - 1.0 / Sc[0, 0]) < 1e-10 * E_mod
    assert abs(nu + Sc[1, 0] / Sc[0, 0]) < 1e-9
    # a general mixed state: two strain-controlled, four stress-controlled components
    comps = [1, 2, 4, 5]
    E = np.array([1e-3, 0, 0, 4e-4, 0, 0])
    S = np.array([0, 2e-5, -1e-5, 0, 3e-6, -2e-6])
    r = oracle.solve(n, phi, C1, E, tol=1e-13, maxit=4000, C0=C0, stress_mask=oracle.mask_of(comps), Sbar=S)
    assert np.abs(r["sigma_mean"] - Ce @ r["strain_mean"]).max() < 1e-10 * np.abs(r["sigma_mean"]).max()
    assert np.abs(r["sigma_mean"][comps] - S[comps]).max() < 1e-12
    assert np.abs(r["strain_mean"][[0, 3]] - E[[0, 3]]).max() < 1e-15


@pytest.mark.parametrize("n,axis,prof", [((8, 4, 4), 0, [1, 1, 1, 1, .25, .25, .25, .25]),
                                         ((4, 6, 4), 1, [0.3, 1, 0.2, 0.8, 1, 0.6]),
                                         ((4, 4, 5), 2, [0.5, 1, 0.15, 0.9, 0.7])])
@pytest.mark.parametrize("load_axis", [0, 1, 2])
def test_laminate_uniaxial_stress_closed_form(n, axis, prof, load_axis):
    """Uniaxial stress on a laminate along and across its layers: E = 1 / (C_lam^-1)_pp and
    nu = -(C_lam^-1)_qp / (C_lam^-1)_pp from the laminate closed form (Voigt in-plane, Reuss across)."""
    phi = li.laminate_phi(n, axis, prof)
    ref = bf.laminate_closed_form(np.asarray(prof, dtype=np.float32), axis, 1.0, 0.3)
    Sc = np.linalg.inv(ref)
    comps = [a for a in range(6) if a != load_axis]
    E = np.zeros(6)
    E[load_axis] = 1e-3
    r = oracle.solve(n, phi, C1, E, tol=1e-13, maxit=500, stress_mask=oracle.mask_of(comps))
    assert r["status"] == 0
    E_mod = r["sigma_mean"][load_axis] / r["strain_mean"][load_axis]
    assert abs(E_mod - 1.0 / Sc[load_axis, load_axis]) < 1e-10
    q = (load_axis + 1) % 3
    nu = -r["strain_mean"][q] / r["strain_mean"][load_axis]
    assert abs(nu + Sc[q, load_axis] / Sc[load_axis, load_axis]) < 1e-9


def _laminate_cases():
    rng = np.random.default_rng(11)
    prof_rand = rng.uniform(0.1, 1.0, 8)
    return [
        ((8, 4, 4), 0, [1, 1, 1, 1, .25, .25, .25, .25]),
        ((4, 8, 4), 1, list(prof_rand)),          # has Nyquist content along the axis
        ((4, 4, 8), 2, list(prof_rand)),
        ((5, 6, 3), 1, [1, 0.5, 0, 0.75, 1, 1]),   # a void layer, odd lengths
        ((6, 4, 5), 2, [0.3, 1, 0, 0.8, 1]),
    ]


@pytest.mark.parametrize("n,axis,prof", _laminate_cases())
def test_laminate_closed_form(n, axis, prof):
    phi = li.laminate_phi(n, axis, prof)
    Ce, infos = oracle.effective_stiffness(n, phi, C1, tol=1e-13, maxit=500)
    ref = bf.laminate_closed_form(np.asarray(prof, dtype=np.float32), axis, 1.0, 0.3)
    assert np.abs(Ce - ref).max() < 1e-11


def test_laminate_nyquist_reading_matters():
    """Zeroing every Nyquist frequency (the literal alternative) breaks the exact laminate result
    when the layer profile has a Nyquist component; the natural reading keeps it exact."""
    n, axis = (4, 8, 4), 1
    prof = [1.0, 0.2, 1.0, 0.2, 1.0, 0.2, 0.6, 0.2]
    phi = li.laminate_phi(n, axis, prof)
    ref = bf.laminate_closed_form(np.asarray(prof, dtype=np.float32), axis, 1.0, 0.3)
    Cn, _ = oracle.effective_stiffness(n, phi, C1, tol=1e-13, cases=[1], maxit=500)
    Cz, _ = oracle.effective_stiffness(n, phi, C1, tol=1e-13, cases=[1], maxit=500, nyquist=oracle.NYQ_ZERO_ALL)
    assert abs(Cn[1, 1] - ref[1, 1]) < 1e-11
    assert abs(Cz[1, 1] - ref[1, 1]) > 1e-3


def test_homogeneous_medium_exact():
    n = (6, 4, 5)
    c = 0.7
    E = np.array([0.3, -0.1, 0.2, 0.05, 0.0, 0.1])
    r = oracle.solve(n, np.full(n, c), C1, E, tol=1e-10)
    # b = -A(E) vanishes up to the rounding of the transforms of a constant field
    assert r["bnorm"] < 1e-13 * np.sqrt(np.prod(n))
    assert np.abs(r["eps"]).max() < 1e-13
    assert np.abs(r["sigma_mean"] - c * C1 @ E).max() < 1e-14
    # a projected random warm start converges back to the uniform stress
    x0 = li.random_field((6,) + n, 42)
    r2 = oracle.solve(n, np.full(n, c), C1, E, tol=1e-12, x0=x0, maxit=300)
    assert np.abs(r2["sigma"] - (c * C1 @ E)[:, None, None, None]).max() < 1e-9


def test_minres_iterates_minimise_residual_over_krylov_space():
    """Each MINRES iterate x_j is argmin ||b - A x|| over the Krylov space K_j(A, b) (zero start)."""
    n = (3, 4, 3)
    N = int(np.prod(n))
    phi = li.random_phi(n, 21, 0.3).astype(np.float64)
    E = np.array([1.0, 0.0, 0.0, 0.3, 0.0, 0.0])
    cols = []
    for k in range(6 * N):
        e = np.zeros(6 * N)
        e[k] = 1
        cols.append(oracle.apply(n, phi, C1, e.reshape((6,) + n)).reshape(-1))
    A = np.array(cols).T
    b = -A @ np.repeat(E, N)
    K = []
    q = b / np.linalg.norm(b)
    for j in range(1, 11):
        K.append(q)
        Qm = np.array(K).T
        y = np.linalg.lstsq(A @ Qm, b, rcond=None)[0]
        xj = Qm @ y
        r = oracle.solve(n, phi, C1, E, tol=1e-300, maxit=j)
        assert r["iterations"] == j
        assert np.abs(r["eps"].reshape(-1) - xj).max() < 1e-9 * np.abs(xj).max()
        res_min = np.linalg.norm(b - A @ xj) / np.linalg.norm(b)
        assert np.isclose(r["rel_residual"], res_min, rtol=1e-8, atol=1e-14)
        # next orthonormal Krylov vector (modified Gram-Schmidt)
        w = A @ K[-1]
        for u in K:
            w -= (u @ w) * u
        q = w / np.linalg.norm(w)


def test_octet_effective_stiffness_properties():
    """Ideal octet at 16^3: C_eff symmetric, cubic, below the Voigt bound; Hill-Mandel orthogonality."""
    n = (16, 16, 16)
    phi, _ = li.octet_phase_map(n, 0.10)
    phi = phi.astype(np.float64)
    Ce = np.zeros((6, 6))
    sig = {}
    eps = {}
    for J in range(6):
        E = np.zeros(6)
        E[J] = 1.0
        r = oracle.solve(n, phi, C1, E, tol=1e-11, maxit=2000)
        assert r["status"] == 0
        Ce[:, J] = r["sigma_mean"]
        sig[J], eps[J] = r["sigma"], r["eps"]
    s = np.abs(Ce).max()
    assert np.abs(Ce - Ce.T).max() < 1e-9 * s
    assert np.allclose(np.diag(Ce)[:3], Ce[0, 0], rtol=1e-9)
    assert np.allclose([Ce[0, 1], Ce[0, 2], Ce[1, 2]], Ce[0, 1], rtol=1e-9)
    assert np.allclose(np.diag(Ce)[3:], Ce[3, 3], rtol=1e-9)
    mask = np.ones((6, 6), bool)
    mask[:3, :3] = False
    mask[[3, 4, 5], [3, 4, 5]] = False
    assert np.abs(Ce[mask]).max() < 1e-9 * s
    assert np.linalg.eigvalsh(phi.mean() * C1 - Ce).min() > -1e-12   # Voigt upper bound
    assert np.linalg.eigvalsh(Ce).min() > 0
    for I in (0, 3):
        for J in (0, 1, 3):
            hm = np.mean(np.sum(sig[J] * eps[I], axis=0))  # <sigma_J : eps~_I> = 0
            assert abs(hm) < 1e-9 * s


def test_paper_behaviour_cg_continuous_fails_minres_rotated_converges():
    """With empty voxels, continuous frequencies + CG stall while rotated frequencies + MINRES converge
    (closing paragraph of the Galerkin section); with rotated frequencies CG also converges and MINRES
    saves only a modest fraction of the iterations (section on numerical performance)."""
    n = (32, 32, 32)
    phi, _ = li.octet_phase_map(n, 0.10)
    E = li.uniaxial_strain(1.0)
    good = oracle.solve(n, phi, C1, E, tol=1e-6, maxit=600, want_sigma=False)
    cg_rot = oracle.solve(n, phi, C1, E, tol=1e-6, maxit=600, solver=oracle.CG, want_sigma=False)
    bad = oracle.solve(n, phi, C1, E, tol=1e-6, maxit=600, scheme=oracle.CONTINUOUS,
                       nyquist=oracle.NYQ_ZERO_ALL, solver=oracle.CG, want_sigma=False)
    assert good["status"] == 0 and good["iterations"] < 250
    assert cg_rot["status"] == 0 and good["iterations"] <= cg_rot["iterations"] < 1.3 * good["iterations"]
    assert bad["status"] == 1 and bad["true_residual"] > 1e-4
