"""FP64 CPU oracle of the nonlinear Galerkin-FFT solve with J2 perfect plasticity.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the solver package.

Paper sections followed: "Non linear extension" of the Galerkin method (eqs. Slin, galnonlin,
galrlin, galrnewton) and "Validation for non linear material response" (von Mises J2 plasticity,
perfectly plastic, load ramp in increments, Newton tolerance on the strain correction).

Material (Mandel vectors; 1 = (1,1,1,0,0,0); dev e = e - tr(e)/3 1; |.| the Euclidean norm of the
Mandel vector, which is the Frobenius norm of the tensor): isotropic elasticity with bulk modulus K
and shear modulus mu, yield stress sigma_y, no hardening, associated flow.  Radial return from the
plastic strain eps_p of the last accepted increment:
    trial deviatoric stress s = 2 mu dev(eps - eps_p), q = sqrt(3/2) |s|;
    q <= sigma_y:  sigma = K tr(eps - eps_p) 1 + s,            tangent C_e = K 1x1 + 2 mu I_dev;
    q  > sigma_y:  theta = sigma_y / q,  n = s / |s|,
                   sigma = K tr(eps - eps_p) 1 + theta s,       plastic strain increment (1 - theta) dev(eps - eps_p),
                   consistent tangent K 1x1 + 2 mu theta (I_dev - n x n).
A voxel with solid fraction phi carries phi times that stress and tangent (the Voigt rule of section
"Voigt approaches" applied to the pristine material's response, as the phase map weighs the stress
in section "Phase-field smoothening").

Newton scheme per increment (t -> t + dt), with the macroscopic strain on the strain-controlled and the
macroscopic stress on the stress-controlled Mandel components ramped linearly over the increments:
    eps^0 = eps^t + (Ebar^{t+dt} - Ebar^t)                                  (first guess)
    iteration i: sigma^{i-1}, C^{i-1} from the return map at eps^{i-1};
                 b_i = -G(sigma^{i-1} - Sbar^{t+dt})                         (eq. galnonlin, right side)
                 MINRES on A_i(d) = G(C^{i-1} : d) = b_i from d = 0, stopped when
                 |A_i d - b_i| <= lin_tol |b_0|                             (eq. galrlin; b_0 = the
                 increment's first right-hand side)
                 eps^i = eps^{i-1} + d
                 accepted when |d|_inf / |eps^i - eps^t|_inf <= newton_tol   (eq. galrnewton)
G is the projection of eq. galop (oracle.project), A_i the operator with the per-voxel tangent
(or_apply_field / or_minres_field).  Readings: the infinity norms run over all Mandel components of
all voxels; a right-hand side already below lin_tol |b_0| gives d = 0 without a MINRES run.
Accumulated equivalent plastic strain (section "Validation for non linear material response"): the
sum over increments of |delta eps_p|.

Pins (tests/test_oracle_pins.py): return map below/at yield, the consistent tangent against central
differences of the return map, the homogeneous cell's uniaxial-stress closed form, and a dense
brute-force Newton solve on the compatible strain basis of a tiny heterogeneous cell.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import ROTATED, NYQ_NATURAL, _dp, _fields_in, _load, _n3, mandel_to_tensor, project, tensor_to_mandel

ONE = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
I_DEV = np.eye(6) - np.outer(ONE, ONE) / 3.0


def bulk_shear(E: float, nu: float):
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def return_map(eps, eps_p, phi, E: float, nu: float, sy: float):
    """Radial return at every voxel.  eps, eps_p: Mandel [6, N...]; phi: [N...].
    Returns (sigma [6, ...], tangent [..., 6, 6] (Mandel), plastic strain increment [6, ...],
    plastic mask [...])."""
    K, mu = bulk_shear(E, nu)
    ee = np.asarray(eps, dtype=np.float64) - np.asarray(eps_p, dtype=np.float64)
    shape = ee.shape[1:]
    ee = ee.reshape(6, -1)
    ph = np.asarray(phi, dtype=np.float64).reshape(-1)
    tr = ee[0] + ee[1] + ee[2]
    dev = ee - ONE[:, None] * tr / 3.0
    s = 2.0 * mu * dev
    snorm = np.sqrt(np.sum(s * s, axis=0))
    q = np.sqrt(1.5) * snorm
    plastic = q > sy
    theta = np.where(plastic, sy / np.where(plastic, q, 1.0), 1.0)
    sig = K * tr * ONE[:, None] + theta * s
    dep = np.where(plastic, 1.0 - theta, 0.0) * dev
    n = np.where(plastic, s / np.where(plastic, snorm, 1.0), 0.0)
    Ce = K * np.outer(ONE, ONE) + 2.0 * mu * I_DEV
    Ct = np.broadcast_to(Ce, (ee.shape[1], 6, 6)).copy()
    pl = np.nonzero(plastic)[0]
    Ct[pl] = K * np.outer(ONE, ONE) + 2.0 * mu * theta[pl, None, None] * (I_DEV[None] - np.einsum("ai,bi->iab", n[:, pl], n[:, pl]))
    sig = sig * ph
    Ct = Ct * ph[:, None, None]
    return (sig.reshape((6,) + shape), Ct.reshape(shape + (6, 6)), dep.reshape((6,) + shape),
            plastic.reshape(shape))


def apply_tangent(n, Ct, x, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL, stress_mask=0):
    """A_i(x) = Re F^{-1}{ G : F{ C^{i-1}(x) : x } } for a Mandel field x (eq. galnonlin, left side)."""
    n = _n3(n)
    N = int(np.prod(n))
    C = np.ascontiguousarray(np.asarray(Ct, dtype=np.float64).reshape(N, 36))
    xt = _fields_in(x, N)
    y = np.empty_like(xt)
    _load().or_apply_field((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), scheme, nyquist,
                           int(stress_mask), _dp(C), _dp(xt), _dp(y))
    return tensor_to_mandel(y).reshape((6,) + n)


def minres_tangent(n, Ct, b, tol: float, maxit: int, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL,
                   stress_mask=0):
    """MINRES on A_i(d) = b from d = 0, stopped at |phibar| < tol |b|.  Returns (d, iterations, status)."""
    n = _n3(n)
    N = int(np.prod(n))
    C = np.ascontiguousarray(np.asarray(Ct, dtype=np.float64).reshape(N, 36))
    bt = _fields_in(b, N)
    x = np.zeros_like(bt)
    info = np.zeros(8)
    _load().or_minres_field((ctypes.c_int * 3)(*n), _dp(np.asarray(L, dtype=np.float64)), scheme, nyquist,
                            int(stress_mask), _dp(C), _dp(bt), float(tol), int(maxit), _dp(x), _dp(info))
    return tensor_to_mandel(x).reshape((6,) + n), int(info[0]), int(info[1])


def solve_j2(n, phi, E: float, nu: float, sy: float, Ebar_final, increments: int = 20, stress_mask: int = 0,
             Sbar_final=None, newton_tol: float = 5e-3, lin_tol: float = 1e-6, max_newton: int = 25,
             maxit: int = 5000, L=(1.0, 1.0, 1.0), scheme=ROTATED, nyquist=NYQ_NATURAL) -> dict:
    """Load ramp in `increments` equal steps to Ebar_final (strain-controlled components) and
    Sbar_final (stress-controlled components, the bits of stress_mask), Newton scheme of the module
    docstring.  Returns dict(eps, sigma, eps_p, ep_acc (fields), history: list of per-increment dicts
    (strain_mean, stress_mean, newton, minres, r_newton), status)."""
    n = _n3(n)
    N = int(np.prod(n))
    phi = np.asarray(phi, dtype=np.float64).reshape(n)
    kl = np.array([(int(stress_mask) >> a) & 1 for a in range(6)], dtype=bool)
    Ef = np.where(kl, 0.0, np.asarray(Ebar_final, dtype=np.float64).reshape(6))
    Sf = np.zeros(6) if Sbar_final is None else np.where(kl, np.asarray(Sbar_final, np.float64).reshape(6), 0.0)
    eps = np.zeros((6,) + n)
    eps_p = np.zeros((6,) + n)
    ep_acc = np.zeros(n)
    Et = np.zeros(6)
    history = []
    status = 0
    kw = dict(L=L, scheme=scheme, nyquist=nyquist, stress_mask=stress_mask)
    for inc in range(1, increments + 1):
        Eb = Ef * inc / increments
        Sb = Sf * inc / increments
        eps_t = eps.copy()
        eps = eps_t + (Eb - Et).reshape((6,) + (1,) * 3)
        b0 = None
        newton = minres_its = 0
        r_newton = np.inf
        for it in range(1, max_newton + 1):
            sig, Ct, _, _ = return_map(eps, eps_p, phi, E, nu, sy)
            b = -project(n, sig - Sb.reshape((6,) + (1,) * 3), **kw)
            bn = float(np.sqrt(np.sum(b * b)))
            if b0 is None:
                b0 = bn
            if bn <= lin_tol * b0 or bn == 0.0:
                d = np.zeros_like(eps)
            else:
                d, its, st = minres_tangent(n, Ct, b, lin_tol * b0 / bn, maxit, **kw)
                minres_its += its
            eps = eps + d
            newton = it
            den = np.abs(eps - eps_t).max()
            r_newton = np.abs(d).max() / den if den > 0 else 0.0
            if r_newton <= newton_tol:
                break
        if r_newton > newton_tol:
            status = 1
        sig, _, dep, _ = return_map(eps, eps_p, phi, E, nu, sy)
        eps_p = eps_p + dep
        ep_acc = ep_acc + np.sqrt(np.sum(dep * dep, axis=0))
        Et = Eb
        history.append(dict(strain_mean=eps.reshape(6, -1).mean(axis=1), stress_mean=sig.reshape(6, -1).mean(axis=1),
                            newton=newton, minres=minres_its, r_newton=float(r_newton)))
    return dict(eps=eps, sigma=sig, eps_p=eps_p, ep_acc=ep_acc, history=history, status=status)
