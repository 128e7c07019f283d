/*
 * rve_geometry.h - C ABI of the lattice phase maps (gfx950): the surface-smoothening approaches that
 * turn a strut lattice into the voxel field phi of C(x) = phi(x) C_solid (Voigt rule).
 *
 * Paper: "Adaptation and validation of FFT methods for homogenization of lattice based materials",
 * sections "Voigt approaches" (plain voxels, Voigt fine grid, Voigt analytic: eq. phaselin),
 * "Phase-field smoothening" (eqs. phase, phase2, phase3), "Combined smoothening", and
 * "Analysis of the surface smoothening approaches" (relative density = voxel mean of phi).
 *
 * Geometry.  The solid is the union of capsules: for each strut, the points within `radius` of its
 * axis segment a-b.  Endpoints are fractions of the cell lengths L (they may lie outside [0, 1]: the
 * cell is periodic), the radius is in length units.  The signed distance of a point x is
 *     D(x) = min over struts of ( |x - nearest point of the segment| - radius ),
 * negative inside the solid; each strut is measured at its periodic image nearest to the strut
 * midpoint (exact while the point is within half a cell minus half the strut length of it).
 * Voxel centres of an n-grid: x_p = (i_p + 1/2) L_p / n_p.
 *
 * Readings of the paper used here:
 *   - eq. phaselin: phi = clip(1/2 - D/ell, 0, 1) (D < 0 inside), which is the exact solid fraction of
 *     a voxel of width ell cut by a plane; ell = one voxel length in the paper.
 *   - eq. phase3: phi_hat(xi) = omega_hat(xi) / (1 + (ell^2/eps) |xi|^2) with the continuous
 *     frequency xi = 2 pi k / L of eq. freq (the minimiser of eq. phase; the printed minus sign would
 *     make the multiplier singular for a real xi).
 *   - the fine grid of the phase-field step has `ratio` fine voxels per coarse voxel and axis; its
 *     voxel centres are the sub-grid points of the Voigt fine-grid map with sub = ratio.
 *   - combined smoothening: the fine-grid source is a given coarse map (normally the VA map),
 *     constant over each coarse voxel.
 *
 * Conventions: maps are [n0][n1][n2] with axis 2 contiguous; "device" pointers are HIP device memory
 * of the current device, "host" pointers host memory; the caller owns every buffer; calls are
 * asynchronous on the given HIP stream (NULL = default stream), except that argument validation
 * happens on the host before any HIP call and a rejected call touches no device state.  Status
 * codes are those of rve.h (rve_last_error() describes a RVE_EDEVICE failure).
 */
#ifndef RVE_GEOMETRY_H
#define RVE_GEOMETRY_H

#include <stddef.h>
#include <stdint.h>

#include "rve.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One strut: axis from a to b (fractions of the cell lengths), capsule radius (length units). */
typedef struct {
  double a[3];
  double b[3];
  double radius;
} rve_strut;

enum { RVE_MAP_PV = 0, RVE_MAP_VFG = 1, RVE_MAP_VA = 2 };

/* Largest number of struts per call, and the largest fine-grid length per axis of rve_phase_field. */
enum { RVE_GEOMETRY_MAX_STRUTS = 256, RVE_GEOMETRY_MAX_FINE = 1024 };

/* Phase map of a strut lattice on the n-grid (section "Voigt approaches"):
 *   RVE_MAP_PV  : 1 where D(voxel centre) <= 0, else 0 (plain voxelization);
 *   RVE_MAP_VFG : fraction of the sub^3 sub-voxel centres with D <= 0 (Voigt fine grid);
 *   RVE_MAP_VA  : clip(1/2 - D(voxel centre)/ell, 0, 1) (Voigt analytic, eq. phaselin).
 * n: host, 3 lengths >= 1 with n0*n1*n2 < 2^31.  L: host, 3 cell lengths > 0.
 * struts: device, n_struts (1..RVE_GEOMETRY_MAX_STRUTS) entries.  sub: 1..64 (VFG only; else ignored).
 * ell: VA width > 0 (length units; ignored otherwise).
 * phi (device, double) and phi_f32 (device, float, the solver's input type): outputs of n0*n1*n2
 * values each; either may be NULL, not both.
 * Errors: RVE_EINVAL for a NULL pointer, an unknown kind, or a size, L, sub or ell out of range (the
 * struts live on the device and are not checked on the host: a negative radius is an empty capsule);
 * RVE_EDEVICE for a HIP failure. */
rve_status rve_phase_map(const int32_t n[3], const double L[3], const rve_strut* struts, int32_t n_struts,
                         int32_t kind, int32_t sub, double ell, double* phi, float* phi_f32, void* hip_stream);

/* Device workspace bytes of rve_phase_field for the coarse grid n and the fine-grid ratio
 * (the half spectrum of the fine grid in FP64 plus small per-axis tables); 0 for invalid sizes. */
size_t rve_phase_field_workspace_bytes(const int32_t n[3], int32_t ratio);

/* Phase-field smoothening (eqs. phase, phase3) on the fine grid m = ratio * n, averaged over each
 * coarse voxel and thresholded:
 *   omega(fine voxel) = 1 if D(fine voxel centre) <= 0 else 0            when source == NULL (PFS),
 *                     = source[coarse voxel containing it]               otherwise (combined
 *                       smoothening when source is the VA map of the same grid);
 *   phi_fine          = F^-1{ F{omega} / (1 + (ell^2/eps) |2 pi k / L|^2) }  (FP64 real FFTs);
 *   raw(coarse voxel) = mean of phi_fine over its ratio^3 fine voxels;
 *   phi               = raw where raw >= threshold, else 0 (the paper uses 0.05).
 * n, L: host, as in rve_phase_map; every fine length ratio * n_p must be 5-smooth (a product of
 * 2, 3, 5) and at most RVE_GEOMETRY_MAX_FINE.  ratio >= 1.  ell >= 0 (paper: half a coarse voxel),
 * eps > 0 (paper: 1), threshold finite.  struts: device (read only when source == NULL).
 * source: device coarse map of n0*n1*n2 doubles, or NULL.
 * phi (device double), phi_f32 (device float), phi_raw (device double, before the threshold):
 * outputs of n0*n1*n2 values; any may be NULL, not all.
 * workspace: device, at least rve_phase_field_workspace_bytes(n, ratio) bytes, 256-byte aligned;
 * its contents on entry do not matter.  Errors: RVE_EINVAL (pointers, values),
 * RVE_EUNSUPPORTED_SIZE (a fine length that is not 5-smooth or too long), RVE_ENOMEM (workspace too
 * small), RVE_EDEVICE. */
rve_status rve_phase_field(const int32_t n[3], const double L[3], const rve_strut* struts, int32_t n_struts,
                           int32_t ratio, double ell, double eps, double threshold, const double* source,
                           double* phi, float* phi_f32, double* phi_raw, void* workspace, size_t workspace_bytes,
                           void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RVE_GEOMETRY_H */
