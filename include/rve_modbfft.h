/*
 * rve_modbfft.h - C ABI of the modified displacement-based FFT solver (MoDBFFT) on gfx950.
 *
 * Paper: "Adaptation and validation of FFT methods for homogenization of lattice based materials",
 * section "Modified displacement based FFT for infinite contrast (MoDBFFT)" (eqs. strongnew, modbfft,
 * diffops, prec, avstiff, precf, modbfftf, modbfftfrhs, modbfftresres).
 *
 * Strain control.  Unknown: the half spectrum u_hat of the periodic displacement fluctuation (3
 * components), solved from
 *     K(u) = -div[ phi(x) C_m : grad^s u ] - (1 - phi(x)) div( alpha grad^s u ) = div( phi(x) C_m : Ebar )
 * with standard Fourier derivatives (grad -> i xi, xi_p = 2 pi k_p / L_p, zero at the Nyquist index of
 * an even length), the equations of the modes with xi = 0 dropped and u_hat = 0 there, by conjugate
 * gradients preconditioned with [xi . Cbar . xi]^{-1} (Cbar = <phi> C_m; no preconditioner when the
 * cell is empty), from u = 0, until |K u - b| <= tol |b| (eq. modbfftresres).  Readings: the paper's
 * equation times -1; chi = 1 - phi (the void indicator for plain voxels); alpha = 1e-4 E of the solid
 * by default.  Every step is FP64.
 *
 * One operator application is six streaming passes over nine components (the six Mandel components
 * of the solid's stress s = C_m eps and the three of g = -div(alpha eps)): expand u_hat -> (s_hat,
 * g_hat); inverse FFT along axis 0, axis 1; along axis 2 the inverse (complex-to-real), the pointwise
 * sigma = phi s and h = (1 - phi) g, and the forward transform in one pass; forward FFT along axis 1,
 * axis 0; then K_hat = -i xi . sigma_hat + h_hat (contract).  Lengths: 5-smooth, at most 1024
 * per axis and 768 along axis 2.
 * Conventions of rve.h: fields [6][n0][n1][n2] (Mandel), device/host as marked, the caller owns every
 * buffer, host validation before any device work, the stream is synchronised before returning.
 */
#ifndef RVE_MODBFFT_H
#define RVE_MODBFFT_H

#include <stddef.h>
#include <stdint.h>

#include "rve.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Passes timed when rve_modbfft_stats.pass_ms is requested (HIP events around every launch). */
enum {
  RVE_MODBFFT_EXPAND = 0,
  RVE_MODBFFT_IFFT_AXIS0,
  RVE_MODBFFT_IFFT_AXIS1,
  RVE_MODBFFT_AXIS2_STRESS,
  RVE_MODBFFT_FFT_AXIS1,
  RVE_MODBFFT_FFT_AXIS0,
  RVE_MODBFFT_CONTRACT,
  RVE_MODBFFT_CG_UPDATE,
  RVE_MODBFFT_NPASS
};

typedef struct {
  int32_t timed;                      /* in: 1 = time every pass (slower: one launch at a time) */
  int32_t iterations;                 /* out: CG iterations */
  double rel_residual;                /* out: |K u - b| / |b| of the CG recurrence at exit */
  double alpha;                       /* out: the alpha used */
  double pass_ms[RVE_MODBFFT_NPASS];  /* out (timed): milliseconds summed over the solve */
  int64_t pass_launches[RVE_MODBFFT_NPASS];
} rve_modbfft_stats;

/* Device workspace bytes for the grid (0 for an unsupported grid). */
size_t rve_modbfft_workspace_bytes(const rve_grid* grid);

/* The solve.  grid: host.  voxel_fraction_field: device float [N] in [0, 1].  C_solid: host Mandel 6x6
 * (row-major, symmetric, positive definite).  macro_strain: host Mandel [6].  alpha: > 0, or <= 0 for
 * 1e-4 / (C_solid^-1)_{00} (1e-4 E for an isotropic solid).  tol in (0, 1), max_iter >= 1.
 * strain_out, stress_out: device FP64 [6][N] or NULL (total strain Ebar + grad^s u, stress
 * phi C_m : strain).  eff_stress: host [6], <stress>.  stats: host, may be NULL.
 * Returns RVE_OK, RVE_NOT_CONVERGED (max_iter reached; outputs from the last iterate),
 * RVE_ENONFINITE, RVE_EINVAL, RVE_EUNSUPPORTED_SIZE, RVE_ENOMEM, RVE_EDEVICE. */
rve_status solve_rve_modbfft(const rve_grid* grid, const float* voxel_fraction_field, const double* C_solid,
                             const double* macro_strain, double alpha, double tol, int32_t max_iter,
                             double* strain_out, double* stress_out, double* eff_stress, rve_modbfft_stats* stats,
                             void* workspace, size_t workspace_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RVE_MODBFFT_H */
