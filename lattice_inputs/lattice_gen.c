/*
 * Seeded synthetic inputs for lattice homogenization: octet-truss phase maps.
 *
 * This module only builds INPUTS (voxel solid-fraction maps phi in [0,1]). It holds none of the
 * homogenization arithmetic, so both the FP64 CPU oracle and the GPU solver can consume its output.
 *
 * Geometry (Sec. "Lattice geometry and simulation parameters"): octet truss = all nearest-neighbour
 * bonds of the FCC lattice, 24 struts per cubic cell, each strut a capsule (cylinder with spherical
 * ends) of radius r.  Voxel fractions follow the Voigt fine-grid approach (Sec. "Voigt approaches"):
 * phi = fraction of S^3 sub-voxel centre points inside the solid.  PV (plain voxelization) is S=1.
 *
 * Manufacturing defects (not in the paper; a synthetic stand-in for the tomography volume of the
 * section "Application to a real 3D tomography"): a smooth random roughness field perturbs the strut
 * signed distance, and spherical pores with lognormal radii are carved out of the solid.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood 2014) -> 53-bit uniforms; Box-Muller normals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ RNG */
static inline uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline double sm64_uniform(uint64_t *s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }
static inline double sm64_normal(uint64_t *s) {
  /* Box-Muller, first variate only (keeps the stream position simple to reproduce) */
  double u1 = sm64_uniform(s), u2 = sm64_uniform(s);
  if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

uint64_t lg_splitmix64(uint64_t seed, int64_t n, double *out) {
  uint64_t s = seed;
  for (int64_t i = 0; i < n; ++i) out[i] = sm64_uniform(&s);
  return s;
}

/* ------------------------------------------------------------------ octet struts */
/* FCC basis (4 atoms) x 6 bond directions = 24 struts of length 1/sqrt(2) in the unit cell. */
static const double kBasis[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
static const double kDir[6][3] = {{0.5, 0.5, 0},  {0.5, -0.5, 0}, {0.5, 0, 0.5},
                                  {0.5, 0, -0.5}, {0, 0.5, 0.5},  {0, 0.5, -0.5}};

typedef struct { double mid[3], half[3], inv_len2; } strut_t;

static void octet_struts(strut_t *s) {
  int k = 0;
  for (int b = 0; b < 4; ++b)
    for (int d = 0; d < 6; ++d, ++k) {
      double l2 = 0;
      for (int p = 0; p < 3; ++p) {
        s[k].half[p] = 0.5 * kDir[d][p];
        s[k].mid[p] = kBasis[b][p] + s[k].half[p];
        l2 += s[k].half[p] * s[k].half[p];
      }
      s[k].inv_len2 = 1.0 / l2;
    }
}

static inline double wrap_half(double d) { return d - floor(d + 0.5); }

/* distance from x (unit-cell coordinates) to the capsule axis of strut s, minimum periodic image
 * taken with respect to the strut midpoint (exact whenever the distance is below ~0.3 cell) */
static inline double strut_dist(const strut_t *s, const double x[3]) {
  double dx[3], t = 0;
  for (int p = 0; p < 3; ++p) {
    dx[p] = wrap_half(x[p] - s->mid[p]);
    t += dx[p] * s->half[p];
  }
  t *= s->inv_len2;
  if (t > 1) t = 1;
  if (t < -1) t = -1;
  double d2 = 0;
  for (int p = 0; p < 3; ++p) {
    double e = dx[p] - t * s->half[p];
    d2 += e * e;
  }
  return sqrt(d2);
}

static inline double octet_dist(const strut_t *s, const double x[3]) {
  double d = 1e30;
  for (int k = 0; k < 24; ++k) {
    double e = strut_dist(s + k, x);
    if (e < d) d = e;
  }
  return d;
}

/* Distances above this bound are never inside the solid for any radius or roughness used here. */
#define FAR_BOUND 0.2

/* For every voxel: the centre distance; voxels whose centre distance exceeds FAR_BOUND + half
 * diagonal have all their sub-points farther than FAR_BOUND. */
static double half_diag(const int n[3]) {
  double h2 = 0;
  for (int p = 0; p < 3; ++p) h2 += 0.25 / ((double)n[p] * n[p]);
  return sqrt(h2);
}

/* ------------------------------------------------------------------ roughness field */
/* eta: per-voxel iid U(-1,1) noise (voxel order, axis 2 fastest) -> periodic separable Gaussian
 * filter (std sigma voxels, radius 4 sigma) -> zero mean -> scaled so that max|eta| = amp (voxels). */
int lg_roughness(const int n[3], double sigma, double amp, uint64_t seed, float *eta_out) {
  int64_t N = (int64_t)n[0] * n[1] * n[2];
  double *a = (double *)malloc(sizeof(double) * N), *b = (double *)malloc(sizeof(double) * N);
  if (!a || !b) { free(a); free(b); return -1; }
  uint64_t s = seed;
  for (int64_t i = 0; i < N; ++i) a[i] = 2.0 * sm64_uniform(&s) - 1.0;
  int R = (int)ceil(4.0 * sigma);
  double *w = (double *)malloc(sizeof(double) * (2 * R + 1));
  double ws = 0;
  for (int i = -R; i <= R; ++i) { w[i + R] = exp(-0.5 * i * i / (sigma * sigma)); ws += w[i + R]; }
  for (int i = 0; i <= 2 * R; ++i) w[i] /= ws;
  int64_t st[3] = {(int64_t)n[1] * n[2], n[2], 1};
  for (int ax = 0; ax < 3; ++ax) {
    double *src = (ax % 2 == 0) ? a : b, *dst = (ax % 2 == 0) ? b : a;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      int64_t c = (i / st[ax]) % n[ax];
      int64_t base = i - c * st[ax];
      double acc = 0;
      for (int k = -R; k <= R; ++k) {
        int64_t cc = ((c + k) % n[ax] + n[ax]) % n[ax];
        acc += w[k + R] * src[base + cc * st[ax]];
      }
      dst[i] = acc;
    }
  }
  double *f = b; /* three passes: a->b, b->a, a->b */
  double mean = 0;
  for (int64_t i = 0; i < N; ++i) mean += f[i];
  mean /= (double)N;
  double mx = 0;
  for (int64_t i = 0; i < N; ++i) { f[i] -= mean; if (fabs(f[i]) > mx) mx = fabs(f[i]); }
  double sc = (mx > 0) ? amp / mx : 0;
  for (int64_t i = 0; i < N; ++i) eta_out[i] = (float)(f[i] * sc);
  free(a); free(b); free(w);
  return 0;
}

/* periodic trilinear interpolation of a voxel-centred field at unit-cell point x */
static inline double interp3(const float *f, const int n[3], const double x[3]) {
  int i0[3], i1[3];
  double t[3];
  for (int p = 0; p < 3; ++p) {
    double u = x[p] * n[p] - 0.5;
    double fl = floor(u);
    t[p] = u - fl;
    int ii = (int)fl;
    i0[p] = ((ii % n[p]) + n[p]) % n[p];
    i1[p] = (i0[p] + 1) % n[p];
  }
  double acc = 0;
  for (int c = 0; c < 8; ++c) {
    int a = (c >> 2) & 1, b = (c >> 1) & 1, d = c & 1;
    double wgt = (a ? t[0] : 1 - t[0]) * (b ? t[1] : 1 - t[1]) * (d ? t[2] : 1 - t[2]);
    int64_t idx = ((int64_t)(a ? i1[0] : i0[0]) * n[1] + (b ? i1[1] : i0[1])) * n[2] + (d ? i1[2] : i0[2]);
    acc += wgt * f[idx];
  }
  return acc;
}

/* ------------------------------------------------------------------ pores */
typedef struct { double c[3], R; } pore_t;

static inline int in_pore(const pore_t *pr, int np, const double x[3]) {
  for (int k = 0; k < np; ++k) {
    double d2 = 0;
    for (int p = 0; p < 3; ++p) { double e = wrap_half(x[p] - pr[k].c[p]); d2 += e * e; }
    if (d2 < pr[k].R * pr[k].R) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------ radius by quantile */
/* Radius r such that exactly round(rho * N * S^3) sub-points of the ideal octet have distance < r,
 * i.e. mean(phi) = rho up to 1/(N S^3).  Two histogram passes + an exact selection in one bin. */
static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

#define NBINS (1 << 20)

double lg_octet_radius(const int n[3], int S, double rho) {
  strut_t st[24];
  octet_struts(st);
  int64_t N = (int64_t)n[0] * n[1] * n[2];
  int64_t total = N * (int64_t)S * S * S;
  int64_t target = (int64_t)llround(rho * (double)total);
  if (target <= 0) return 0.0;
  double hd = half_diag(n);
  uint64_t *hist = (uint64_t *)calloc(NBINS, sizeof(uint64_t));
  const double scale = NBINS / FAR_BOUND;
#pragma omp parallel
  {
    uint64_t *lh = (uint64_t *)calloc(NBINS, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 64)
    for (int64_t v = 0; v < N; ++v) {
      int i0 = (int)(v / ((int64_t)n[1] * n[2])), i1 = (int)((v / n[2]) % n[1]), i2 = (int)(v % n[2]);
      double xc[3] = {(i0 + 0.5) / n[0], (i1 + 0.5) / n[1], (i2 + 0.5) / n[2]};
      if (octet_dist(st, xc) - hd >= FAR_BOUND) continue;
      for (int a = 0; a < S; ++a)
        for (int b = 0; b < S; ++b)
          for (int c = 0; c < S; ++c) {
            double x[3] = {(i0 + (a + 0.5) / S) / n[0], (i1 + (b + 0.5) / S) / n[1], (i2 + (c + 0.5) / S) / n[2]};
            double d = octet_dist(st, x);
            if (d < FAR_BOUND) lh[(int64_t)(d * scale)]++;
          }
    }
#pragma omp critical
    for (int i = 0; i < NBINS; ++i) hist[i] += lh[i];
    free(lh);
  }
  int64_t acc = 0;
  int bin = -1;
  int64_t before = 0;
  for (int i = 0; i < NBINS; ++i) {
    if (acc + (int64_t)hist[i] >= target) { bin = i; before = acc; break; }
    acc += hist[i];
  }
  if (bin < 0) { free(hist); return -1.0; }
  int64_t cnt = hist[bin];
  double lo = bin / scale, hi = (bin + 1) / scale;
  double *vals = (double *)malloc(sizeof(double) * (cnt + 1));
  int64_t m = 0;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t v = 0; v < N; ++v) {
    int i0 = (int)(v / ((int64_t)n[1] * n[2])), i1 = (int)((v / n[2]) % n[1]), i2 = (int)(v % n[2]);
    double xc[3] = {(i0 + 0.5) / n[0], (i1 + 0.5) / n[1], (i2 + 0.5) / n[2]};
    double dc = octet_dist(st, xc);
    if (dc - hd >= hi || dc + hd < lo) continue;
    for (int a = 0; a < S; ++a)
      for (int b = 0; b < S; ++b)
        for (int c = 0; c < S; ++c) {
          double x[3] = {(i0 + (a + 0.5) / S) / n[0], (i1 + (b + 0.5) / S) / n[1], (i2 + (c + 0.5) / S) / n[2]};
          double d = octet_dist(st, x);
          if (d < FAR_BOUND && (int64_t)(d * scale) == bin) {
            int64_t k;
#pragma omp atomic capture
            k = m++;
            if (k < cnt) vals[k] = d;
          }
        }
  }
  int64_t mm = (m < cnt ? m : cnt);
  qsort(vals, (size_t)mm, sizeof(double), cmp_double);
  /* k-th smallest overall (1-based target) is vals[target - before - 1].  The symmetric geometry
   * produces large groups of equal distances, so exactly `target` points may not be separable:
   * take whichever side of the tie group at d_k lands closer to the target count. */
  int64_t j = target - before - 1;
  double dk = vals[j];
  /* symmetric points can differ by a few ulps: treat relative differences below 1e-12 as ties so
   * that r always falls in a real gap and mirror-image points are classified alike */
  const double tie = 1e-12 * dk;
  int64_t lo_i = j, hi_i = j;
  while (lo_i > 0 && dk - vals[lo_i - 1] <= tie) lo_i--;
  while (hi_i + 1 < mm && vals[hi_i + 1] - dk <= tie) hi_i++;
  int64_t c_lo = before + lo_i;     /* # points strictly below the tie group */
  int64_t c_hi = before + hi_i + 1; /* # points up to and including the tie group */
  double r;
  if (llabs(c_lo - target) <= llabs(c_hi - target)) {
    r = (lo_i > 0) ? 0.5 * (vals[lo_i - 1] + vals[lo_i]) : lo;
  } else {
    r = (hi_i + 1 < mm) ? 0.5 * (vals[hi_i] + vals[hi_i + 1]) : hi;
  }
  free(vals);
  free(hist);
  return r;
}

/* ------------------------------------------------------------------ phase map */
/* phi[v] = (# sub-points with  dist(x) - r + rough_h * eta(x) < 0  and not in a pore) / S^3.
 * eta may be NULL (no roughness); pores may be empty. */
void lg_octet_phi(const int n[3], int S, double r, const float *eta, double rough_h, const double *pores,
                  int n_pores, float *phi) {
  strut_t st[24];
  octet_struts(st);
  int64_t N = (int64_t)n[0] * n[1] * n[2];
  double hd = half_diag(n);
  double eta_max = 0;
  if (eta)
    for (int64_t i = 0; i < N; ++i) if (fabs(eta[i]) > eta_max) eta_max = fabs(eta[i]);
  double margin = hd + eta_max * rough_h;
  pore_t *pr = (pore_t *)malloc(sizeof(pore_t) * (n_pores > 0 ? n_pores : 1));
  for (int k = 0; k < n_pores; ++k) {
    for (int p = 0; p < 3; ++p) pr[k].c[p] = pores[4 * k + p];
    pr[k].R = pores[4 * k + 3];
  }
  const int S3 = S * S * S;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t v = 0; v < N; ++v) {
    int i0 = (int)(v / ((int64_t)n[1] * n[2])), i1 = (int)((v / n[2]) % n[1]), i2 = (int)(v % n[2]);
    double xc[3] = {(i0 + 0.5) / n[0], (i1 + 0.5) / n[1], (i2 + 0.5) / n[2]};
    double dc = octet_dist(st, xc);
    if (dc - margin >= r) { phi[v] = 0.0f; continue; }
    int inside = 0;
    for (int a = 0; a < S; ++a)
      for (int b = 0; b < S; ++b)
        for (int c = 0; c < S; ++c) {
          double x[3] = {(i0 + (a + 0.5) / S) / n[0], (i1 + (b + 0.5) / S) / n[1], (i2 + (c + 0.5) / S) / n[2]};
          double sdf = octet_dist(st, x) - r;
          if (eta) sdf += rough_h * interp3(eta, n, x);
          if (sdf < 0 && !(n_pores > 0 && in_pore(pr, n_pores, x))) inside++;
        }
    phi[v] = (float)((double)inside / S3);
  }
  free(pr);
}

/* Pores: centres uniform in the cell (seeded), radius R = median * exp(s * Z), Z ~ N(0,1),
 * accepted when the perturbed signed distance at the centre is <= -R/2 (centre well inside the
 * solid); draws continue until n_pores are accepted or max_draws is hit.  Returns # accepted.
 * out: [n_pores][4] = (cx, cy, cz, R) in unit-cell units. */
int lg_place_pores(const int n[3], double r, const float *eta, double rough_h, int n_pores, double median,
                   double s_log, uint64_t seed, int max_draws, double *out) {
  strut_t st[24];
  octet_struts(st);
  uint64_t s = seed;
  int acc = 0;
  for (int d = 0; d < max_draws && acc < n_pores; ++d) {
    double c[3] = {sm64_uniform(&s), sm64_uniform(&s), sm64_uniform(&s)};
    double R = median * exp(s_log * sm64_normal(&s));
    double sdf = octet_dist(st, c) - r;
    if (eta) sdf += rough_h * interp3(eta, n, c);
    if (sdf <= -0.5 * R) {
      out[4 * acc + 0] = c[0]; out[4 * acc + 1] = c[1]; out[4 * acc + 2] = c[2]; out[4 * acc + 3] = R;
      acc++;
    }
  }
  return acc;
}

int lg_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
