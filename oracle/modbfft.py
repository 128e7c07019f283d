"""FP64 CPU oracle of the modified displacement-based FFT solver (MoDBFFT).

TEST INFRASTRUCTURE ONLY: imported by the tests and the CPU-baseline leg of the benchmark, never by
the solver package.  numpy's real FFT is the one library step.

Paper section "Modified displacement based FFT for infinite contrast (MoDBFFT)": eqs. strongnew,
modbfft, diffops, prec, avstiff, precf, modbfftf, modbfftfrhs, modbfftresres.  Strain control: the
unknown is the Fourier transform u_hat of the periodic, zero-mean displacement fluctuation, solved from
    K(u) = -div[ C(x) : grad^s u ] - chi(x) div( alpha grad^s u ) = div( C(x) : Ebar )
with standard Fourier derivatives (grad -> i xi, xi = 2 pi k / L), C(x) = phi(x) C_m and the void
indicator chi, by conjugate gradients preconditioned with M_hat = [xi . Cbar . xi]^{-1},
Cbar = <C(x)>, stopped on |K u - b| / |b| (eq. modbfftresres; b the right-hand side).

Readings (the text is silent or garbled):
  * Sign: the paper's equation is multiplied by -1 so that the operator's stiffness part is positive
    (-div C grad^s); with grad -> i xi its symbol is xi . C . xi.
  * Voxel fractions: chi(x) = 1 - phi(x), so that (1 - chi) C_m = phi C_m is the Voigt stiffness; for
    plain voxels (phi in {0, 1}) this is the paper's indicator.
  * Nyquist: for an even length the frequency of index N/2 is taken as zero (a derivative of a real
    field must stay real there); modes whose whole frequency vector is zero (the mean and the Nyquist
    corners) carry no unknown, u_hat = 0 there, and their equations are dropped (eq. precf defines the
    preconditioner at the non-zero frequencies only; under strain control nothing replaces them, and the
    alpha term's mean, which is not a divergence, is left free).
  * alpha: 1e-4 times the solid's Young's modulus (the paper's choice) unless given.
  * An empty cell (<phi> = 0) has Cbar = 0; it is solved without the preconditioner.
  * Inner products and norms are those of the real fields (Parseval: the half spectrum weighted by 1
    on the k2 = 0 and Nyquist planes, 2 elsewhere).
Symmetric tensors are 3x3 here; Mandel vectors only at the interface.

Pins (tests/test_modbfft_pins.py): the operator on Fourier modes against the acoustic tensor
(solid) and the alpha term (void); one preconditioned CG step solves a homogeneous cell; a dense
brute force of the same operator built from explicit DFT matrices (no FFT) on a tiny cell.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)
_MI = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def mandel_to_tensor4(Cm):
    """Mandel 6x6 -> C[i, j, k, l] (minor and major symmetric)."""
    Cm = np.asarray(Cm, dtype=np.float64).reshape(6, 6)
    C = np.zeros((3, 3, 3, 3))
    for A, (i, j) in enumerate(_MI):
        for B, (k, l) in enumerate(_MI):
            v = Cm[A, B] / ((1.0 if A < 3 else SQ2) * (1.0 if B < 3 else SQ2))
            for a, b in ((i, j), (j, i)):
                for c, d in ((k, l), (l, k)):
                    C[a, b, c, d] = v
    return C


def tensor_to_mandel(t):
    """(3, 3, ...) symmetric -> (6, ...)."""
    return np.stack([t[i, j] * (1.0 if A < 3 else SQ2) for A, (i, j) in enumerate(_MI)])


def mandel_to_tensor(v):
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros((3, 3) + v.shape[1:])
    for A, (i, j) in enumerate(_MI):
        s = v[A] / (1.0 if A < 3 else SQ2)
        t[i, j] = s
        t[j, i] = s
    return t


def frequencies(n, L=(1.0, 1.0, 1.0)):
    """xi_p on the half spectrum grid (n0, n1, n2//2 + 1), zero at the Nyquist index of even lengths."""
    n = tuple(int(v) for v in n)
    ks = []
    for p in range(3):
        k = np.fft.fftfreq(n[p], d=1.0 / n[p]) if p < 2 else np.fft.rfftfreq(n[p], d=1.0 / n[p])
        if n[p] % 2 == 0:
            k = np.where(np.abs(k) == n[p] // 2, 0.0, k)
        ks.append(2.0 * np.pi * k / L[p])
    X0, X1, X2 = np.meshgrid(*ks, indexing="ij")
    return np.stack([X0, X1, X2])


def weights(n):
    """Parseval weights of the half spectrum along axis 2."""
    K = n[2] // 2 + 1
    w = np.full(K, 2.0)
    w[0] = 1.0
    if n[2] % 2 == 0:
        w[-1] = 1.0
    return w


def dot(a, b, n):
    """Real inner product of the fields whose half spectra are a, b (3 components): <a, b> * N."""
    return float(np.sum(weights(n) * np.real(np.conj(a) * b)))


class Problem:
    def __init__(self, n, phi, C_solid, alpha=None, L=(1.0, 1.0, 1.0)):
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        self.phi = np.asarray(phi, dtype=np.float64).reshape(self.n)
        self.Cm = np.asarray(C_solid, dtype=np.float64).reshape(6, 6)
        self.C4 = mandel_to_tensor4(self.Cm)
        if alpha is None:
            S = np.linalg.inv(self.Cm)
            alpha = 1e-4 / S[0, 0]  # 1e-4 E of the solid (E = 1 / S_1111)
        self.alpha = float(alpha)
        self.xi = frequencies(self.n, self.L)
        self.active = np.any(self.xi != 0, axis=0)  # modes that carry an unknown
        Cbar = self.phi.mean() * self.C4
        A = np.einsum("j...,ijkl,l...->...ik", self.xi, Cbar, self.xi)
        A[~self.active] = np.eye(3)
        if self.phi.mean() > 0:
            self.Minv = np.linalg.inv(A)  # preconditioner [xi . Cbar . xi]^-1 per mode (eq. precf)
        else:  # an empty cell has Cbar = 0: no preconditioner
            self.Minv = np.broadcast_to(np.eye(3), A.shape).copy()
        self.Minv[~self.active] = 0.0

    # real fields <-> half spectra
    def fwd(self, f):
        return np.fft.rfftn(f, axes=(-3, -2, -1))

    def inv(self, F):
        return np.fft.irfftn(F, s=self.n, axes=(-3, -2, -1))

    def strain_hat(self, u_hat):
        """grad^s u: eps_hat_ij = (i/2)(xi_i u_j + xi_j u_i)."""
        xi = self.xi
        return 0.5j * (np.einsum("i...,j...->ij...", xi, u_hat) + np.einsum("j...,i...->ij...", xi, u_hat))

    def apply(self, u_hat):
        """K(u) (eq. modbfftf, sign reading above), half spectrum in and out."""
        eps = self.inv(self.strain_hat(u_hat))
        sig = self.phi * np.einsum("ijkl,kl...->ij...", self.C4, eps)
        t1 = -1j * np.einsum("j...,ij...->i...", self.xi, self.fwd(sig))  # -div sigma
        g_hat = self.alpha * np.einsum("j...,ij...->i...", self.xi, -1j * self.strain_hat(u_hat))  # -div(alpha eps)
        t2 = self.fwd((1.0 - self.phi) * self.inv(g_hat))
        out = t1 + t2
        out[:, ~self.active] = 0.0
        return out

    def rhs(self, Ebar):
        """b = div(C(x) : Ebar) (eq. modbfftfrhs, strain control), half spectrum."""
        E = mandel_to_tensor(np.asarray(Ebar, dtype=np.float64).reshape(6))
        sig = self.phi * np.einsum("ijkl,kl->ij", self.C4, E)[:, :, None, None, None] * np.ones(self.n)
        b = 1j * np.einsum("j...,ij...->i...", self.xi, self.fwd(sig))
        b[:, ~self.active] = 0.0
        return b

    def precondition(self, r):
        return np.einsum("...ik,k...->i...", self.Minv, r)

    def fields(self, u_hat, Ebar):
        """Total strain and stress (Mandel [6, *n]) and <sigma>."""
        E = mandel_to_tensor(np.asarray(Ebar, dtype=np.float64).reshape(6))
        eps = self.inv(self.strain_hat(u_hat)) + E[:, :, None, None, None]
        sig = self.phi * np.einsum("ijkl,kl...->ij...", self.C4, eps)
        s = tensor_to_mandel(sig)
        return tensor_to_mandel(eps), s, s.reshape(6, -1).mean(axis=1)


def solve(n, phi, C_solid, Ebar, tol=1e-6, maxit=5000, alpha=None, L=(1.0, 1.0, 1.0), precondition=True) -> dict:
    """Preconditioned conjugate gradients on K u = b from u = 0 (Hestenes-Stiefel with the
    preconditioner of eq. precf), stopped when |r| <= tol |b|.  Returns dict(u_hat, strain, stress,
    sigma_mean, iterations, rel_residual, history, status, alpha)."""
    P = Problem(n, phi, C_solid, alpha, L)
    b = P.rhs(Ebar)
    bn = np.sqrt(dot(b, b, P.n))
    x = np.zeros_like(b)
    r = b.copy()
    hist = []
    status = 0
    it = 0
    if bn > 0:
        z = P.precondition(r) if precondition else r.copy()
        p = z.copy()
        rz = dot(r, z, P.n)
        while True:
            rn = np.sqrt(dot(r, r, P.n))
            if rn <= tol * bn:
                break
            if it >= maxit:
                status = 1
                break
            q = P.apply(p)
            a = rz / dot(p, q, P.n)
            x = x + a * p
            r = r - a * q
            it += 1
            hist.append(np.sqrt(dot(r, r, P.n)) / bn)
            z = P.precondition(r) if precondition else r.copy()
            rz_new = dot(r, z, P.n)
            p = z + (rz_new / rz) * p
            rz = rz_new
    eps, sig, smean = P.fields(x, Ebar)
    rel = np.sqrt(dot(r, r, P.n)) / bn if bn > 0 else 0.0
    return dict(u_hat=x, strain=eps, stress=sig, sigma_mean=smean, iterations=it, rel_residual=float(rel),
                history=np.array(hist), status=status, alpha=P.alpha)
