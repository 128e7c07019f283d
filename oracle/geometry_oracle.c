/*
 * FP64 CPU oracle: signed distance of a strut lattice at voxel centres (test infrastructure only).
 *
 * The surface-smoothening maps of the sections "Voigt approaches" and "Phase-field smoothening"
 * start from the lattice geometry: the solid is the union of capsules (cylinders of radius r with
 * spherical ends) around the strut axis segments, and D(x) = min over struts of (distance from x to
 * the axis segment - r), negative inside the solid.  Each strut is measured at its periodic image
 * nearest to the strut midpoint.  Plain loops, OpenMP over the first grid axis.
 */
#include <math.h>

/* distance from point p to the segment of strut s = (a[3], b[3], r), endpoints in cell fractions */
static double seg_dist(const double *s, const double L[3], const double p[3]) {
  double mid[3], half[3], dx[3], hh = 0.0, dh = 0.0;
  for (int q = 0; q < 3; ++q) {
    double a = s[q] * L[q], b = s[3 + q] * L[q];
    mid[q] = 0.5 * (a + b);
    half[q] = 0.5 * (b - a);
    dx[q] = p[q] - mid[q];
    dx[q] -= L[q] * floor(dx[q] / L[q] + 0.5);
    hh += half[q] * half[q];
    dh += dx[q] * half[q];
  }
  double t = hh > 0.0 ? dh / hh : 0.0;
  if (t < -1.0) t = -1.0;
  if (t > 1.0) t = 1.0;
  double e2 = 0.0;
  for (int q = 0; q < 3; ++q) {
    double e = dx[q] - t * half[q];
    e2 += e * e;
  }
  return sqrt(e2);
}

/* D at the voxel centres of the grid sub*n: x_q = (j + 1/2) * L_q / (sub n_q); out is
 * [sub n0][sub n1][sub n2], last axis fastest.  struts: ns rows of 7 doubles (a, b, r). */
void og_distance_map(const int n[3], const double L[3], int sub, const double *struts, int ns, double *out) {
  const long m0 = (long)sub * n[0], m1 = (long)sub * n[1], m2 = (long)sub * n[2];
  const double h0 = L[0] / (double)m0, h1 = L[1] / (double)m1, h2 = L[2] / (double)m2;
#pragma omp parallel for schedule(static)
  for (long i0 = 0; i0 < m0; ++i0)
    for (long i1 = 0; i1 < m1; ++i1)
      for (long i2 = 0; i2 < m2; ++i2) {
        double p[3] = {((double)i0 + 0.5) * h0, ((double)i1 + 0.5) * h1, ((double)i2 + 0.5) * h2};
        double D = INFINITY;
        for (int k = 0; k < ns; ++k) {
          double d = seg_dist(struts + 7 * k, L, p) - struts[7 * k + 6];
          if (d < D) D = d;
        }
        out[(i0 * m1 + i1) * m2 + i2] = D;
      }
}
