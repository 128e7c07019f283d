/*
 * rve_j2.h - C ABI of the nonlinear Galerkin-FFT solve with J2 perfect plasticity (gfx950).
 *
 * Paper: "Adaptation and validation of FFT methods for homogenization of lattice based materials",
 * section "Non linear extension" of the Galerkin method (eqs. Slin, galnonlin, galrlin, galrnewton)
 * and section "Validation for non linear material response" (von Mises plasticity without hardening,
 * a load ramp in equal increments, Newton iterations per increment).
 *
 * Material: the solid is isotropic elastic (Young's modulus, Poisson's ratio) and perfectly plastic
 * with von Mises yield stress sigma_y and associated flow; a voxel of solid fraction phi carries phi
 * times the solid's stress and consistent tangent (Voigt rule; C_void = 0).  Radial return from the
 * plastic strain of the last accepted increment (Mandel vectors, 1 = (1,1,1,0,0,0)):
 *     s = 2 mu dev(eps - eps_p), q = sqrt(3/2) |s|;  q <= sigma_y: elastic;
 *     else theta = sigma_y / q, sigma = K tr(eps - eps_p) 1 + theta s, plastic increment
 *     (1 - theta) dev(eps - eps_p), tangent K 1(x)1 + 2 mu theta (I_dev - n (x) n), n = s / |s|.
 *
 * Newton scheme per increment, macroscopic strain (strain-controlled components) and stress (the
 * components in rve_options.stress_mask) ramped linearly to their final values:
 *     eps^0 = eps^t + (Ebar^{t+dt} - Ebar^t);
 *     iteration i: b_i = -G(sigma(eps^{i-1}) - Sbar^{t+dt}) (eq. galnonlin), MINRES on
 *     G(C^{i-1} : d) = b_i from d = 0 until |A_i d - b_i| <= lin_tol |b_0| (eq. galrlin, b_0 the
 *     increment's first right-hand side; no MINRES run when |b_i| is already below), eps^i = eps^{i-1} + d;
 *     accepted when |d|_inf / |eps^i - eps^t|_inf <= newton_tol (eq. galrnewton; maxima over all
 *     Mandel components of all voxels).
 * G is the projection of eq. galop with the rotated frequencies of eq. freqrot (as solve_rve).  The
 * MINRES runs are those of solve_rve (FP32 sweeps with FP64 refinement, or FP64), with the tangent
 * fused into the stiffness pass.
 * Conventions of rve.h: fields component-major [6][n0][n1][n2], device/host pointers as marked, the
 * caller owns every buffer, host validation before any device work.
 */
#ifndef RVE_J2_H
#define RVE_J2_H

#include <stddef.h>
#include <stdint.h>

#include "rve.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double young;         /* > 0 */
  double poisson;       /* in (-1, 0.5) */
  double yield_stress;  /* > 0 */
} rve_j2_material;

typedef struct {
  int32_t increments;   /* >= 1 equal steps of the load ramp */
  int32_t max_newton;   /* >= 1 Newton iterations per increment */
  double newton_tol;    /* > 0, on |d|_inf / |eps^i - eps^t|_inf (paper: 5e-3) */
  double lin_tol;       /* > 0, on |A_i d - b_i| / |b_0| */
} rve_j2_options;

/* One accepted increment (or the last Newton iterate of an increment that did not converge). */
typedef struct {
  double strain_mean[6];  /* <eps> (Mandel): the applied strain plus the stress-controlled components' */
  double stress_mean[6];  /* <sigma> (Mandel) */
  double r_newton;        /* eq. galrnewton at the last Newton iteration */
  int32_t newton;         /* Newton iterations */
  int32_t minres;         /* MINRES iterations over those Newton iterations */
  int32_t status;         /* 0 converged; 1 Newton not converged within max_newton */
  int32_t pad;
} rve_j2_increment;

/* Device workspace of solve_rve_j2 for one load path on the grid (precision from opt). */
size_t rve_j2_workspace_bytes(const rve_grid* grid, const rve_options* opt);

/* The nonlinear solve.  grid: as solve_rve.  voxel_fraction_field: device float [N] in [0, 1].
 * material, jopt: host.  macro_strain_final: host [6], the final macroscopic strain (its
 * stress-controlled components are ignored); macro_stress_final: host [6] or NULL (zero), the final
 * macroscopic stress on the components of opt->stress_mask.  opt: as solve_rve (precision, scheme,
 * nyquist, stress_mask, max_iter per MINRES solve, check_every, inner_floor, inner_safety; opt->tol
 * is not used).  Outputs (device FP64 [6][N], each may be NULL): total strain, stress, plastic strain
 * at the end of the ramp; ep_acc_out (device FP64 [N] or NULL): accumulated equivalent plastic strain,
 * the sum over increments of |delta eps_p|.  history: host, jopt->increments entries.
 * workspace: device, rve_j2_workspace_bytes(grid, opt) bytes.  Returns RVE_OK, RVE_NOT_CONVERGED when
 * some increment's Newton iterations did not reach newton_tol (the ramp goes on from its last
 * iterate), or an error of solve_rve. */
rve_status solve_rve_j2(const rve_grid* grid, const float* voxel_fraction_field, const rve_j2_material* material,
                        const double* macro_strain_final, const double* macro_stress_final, const rve_options* opt,
                        const rve_j2_options* jopt, double* strain_out, double* stress_out,
                        double* plastic_strain_out, double* ep_acc_out, rve_j2_increment* history, void* workspace,
                        size_t workspace_bytes, void* hip_stream);

/* The return map alone at n_voxels voxels (device FP64 [6][n_voxels] strain and plastic strain,
 * device float phi): stress (device FP64 [6][n_voxels], may be NULL) and the tangent's data
 * (device FP64 [7][n_voxels], may be NULL): a = 2 mu (1 - theta) and m = sqrt(2 mu theta) n, zero
 * when elastic, so that C_t = phi (C_e - a I_dev - m (x) m).  Asynchronous on the stream. */
rve_status rve_j2_return_map(int64_t n_voxels, const float* voxel_fraction_field, const rve_j2_material* material,
                             const double* strain, const double* plastic_strain, double* stress, double* tangent,
                             void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RVE_J2_H */
