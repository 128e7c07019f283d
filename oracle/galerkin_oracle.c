/*
 * FP64 CPU oracle for the Galerkin-FFT homogenization of lattices with empty phases.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or constant with the GPU
 * solver: it is a plain, slow, literal transcription of the method's equations.
 *
 * What it computes (section "Galerkin-FFT with discrete differences and mixed loading control"):
 *   - voxel grid and frequencies of eq. (freq); rotated forward-difference modified frequencies of
 *     eq. (freqrot), with the product read over a dummy axis index;
 *   - the projection of eq. (galop) under mixed macroscopic control: at xi = 0 the symmetric identity
 *     on the stress-controlled components and zero on the strain-controlled ones (pure strain control:
 *     zero), zero where the modified frequency vanishes, and [I^s_ijkl xi_j xi_l]^{-1} xi_j xi_l
 *     (symmetrised over ij and kl) elsewhere;
 *   - the linear operator of eq. (linearOp) with the Voigt stiffness C = phi C_solid (+ (1-phi) C_void)
 *     of section "Voigt approaches", and the right-hand side b of eq. (gallin) with the macroscopic
 *     strain on the strain-controlled and the macroscopic stress on the stress-controlled components;
 *   - MINRES (Paige & Saunders 1975: Lanczos tridiagonalisation + Givens QR of the extended
 *     tridiagonal matrix), stopped on the residual of eq. (galres);
 *   - conjugate gradients, only to reproduce the paper's statement that CG fails with voids and
 *     continuous frequencies.
 * Tensors are stored as the six independent Cartesian components (00,11,22,12,02,01); the L2 norm is
 * the Frobenius norm of the full 3x3 tensor summed over voxels.
 * FFT: textbook recursive mixed-radix Cooley-Tukey (smallest prime factor first) with an O(n^2)
 * DFT for prime lengths; forward unnormalised, inverse scaled by 1/N.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

/* ================================================================== 1-D transforms */

void or_dft_naive(const cplx *x, cplx *y, int n, int sign) {
  for (int k = 0; k < n; ++k) {
    cplx acc = 0;
    for (int j = 0; j < n; ++j) {
      /* reduce j*k mod n before forming the angle, so the table of angles stays exact */
      long jk = ((long)j * k) % n;
      double a = sign * 2.0 * M_PI * (double)jk / (double)n;
      acc += x[j] * (cos(a) + I * sin(a));
    }
    y[k] = acc;
  }
}

static int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

/* out[k] = sum_j in[j*stride] w_n^{jk}, w_n = exp(sign 2 pi i / n); out contiguous, length n. */
static void fft_rec(const cplx *in, int stride, cplx *out, int n, int sign, cplx *tmp) {
  if (n == 1) { out[0] = in[0]; return; }
  int p = smallest_factor(n);
  if (p == n) {
    /* prime length: direct DFT of the strided input */
    for (int k = 0; k < n; ++k) {
      cplx acc = 0;
      for (int j = 0; j < n; ++j) {
        long jk = ((long)j * k) % n;
        double a = sign * 2.0 * M_PI * (double)jk / (double)n;
        acc += in[(long)j * stride] * (cos(a) + I * sin(a));
      }
      out[k] = acc;
    }
    return;
  }
  int m = n / p;
  /* decimation in time: p interleaved sub-sequences, each transformed into its own block of out */
  for (int r = 0; r < p; ++r) fft_rec(in + (long)r * stride, stride * p, out + (long)r * m, m, sign, tmp + n);
  /* combine: X[k + q m] = sum_r w_n^{r (k + q m)} Y_r[k] */
  cplx *t = tmp;
  for (int k = 0; k < m; ++k) {
    for (int r = 0; r < p; ++r) {
      double a = sign * 2.0 * M_PI * (double)((long)r * k % n) / (double)n;
      t[r] = out[(long)r * m + k] * (cos(a) + I * sin(a));
    }
    for (int q = 0; q < p; ++q) {
      cplx acc = 0;
      for (int r = 0; r < p; ++r) {
        double a = sign * 2.0 * M_PI * (double)((long)r * q % p) / (double)p;
        acc += t[r] * (cos(a) + I * sin(a));
      }
      out[k + (long)q * m] = acc;
    }
  }
}

/* scratch needed by fft_rec for length n: sum of lengths down the recursion, bounded by 2n + 64 */
void or_fft(const cplx *x, cplx *y, int n, int sign) {
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (2 * (size_t)n + 64));
  fft_rec(x, 1, y, n, sign, tmp);
  free(tmp);
}

/* In-place 3-D transform of a complex array of shape n[0] x n[1] x n[2] (axis 2 contiguous).
 * sign = -1: forward, unnormalised.  sign = +1: inverse, scaled by 1/N. */
void or_fft3(cplx *a, const int n[3], int sign) {
  long N = (long)n[0] * n[1] * n[2];
  long stride[3] = {(long)n[1] * n[2], n[2], 1};
  for (int ax = 0; ax < 3; ++ax) {
    int len = n[ax];
    if (len == 1) continue;
    long lines = N / len;
#pragma omp parallel
    {
      cplx *buf = (cplx *)malloc(sizeof(cplx) * len);
      cplx *res = (cplx *)malloc(sizeof(cplx) * len);
      cplx *tmp = (cplx *)malloc(sizeof(cplx) * (2 * (size_t)len + 64));
#pragma omp for schedule(static)
      for (long l = 0; l < lines; ++l) {
        /* line l: all indices with the axis coordinate = 0 enumerated in row-major order of the rest */
        long outer = l / stride[ax], inner = l % stride[ax];
        long base = outer * stride[ax] * len + inner;
        for (int j = 0; j < len; ++j) buf[j] = a[base + (long)j * stride[ax]];
        fft_rec(buf, 1, res, len, sign, tmp);
        for (int j = 0; j < len; ++j) a[base + (long)j * stride[ax]] = res[j];
      }
      free(buf); free(res); free(tmp);
    }
  }
  if (sign > 0) {
    double s = 1.0 / (double)N;
    for (long i = 0; i < N; ++i) a[i] *= s;
  }
}

/* ================================================================== grid, frequencies */

typedef struct {
  int n[3];
  double L[3];
  int scheme;  /* 0: rotated forward differences (eq. freqrot), 1: continuous (eq. freq) */
  int nyquist; /* 0: natural (projection vanishes only where xi = 0), 1: zero at every Nyquist index */
  int stress_mask; /* mixed macroscopic control: bit a set = component a (00,11,22,12,02,01) is
                      stress-controlled (the set KL of eq. galop), else strain-controlled (kl) */
} or_grid;

/* signed frequency index for storage index m of an axis of length N: m for m <= (N-1)/2, else m - N;
 * the paper's centred index n_p - N_p/2 reordered, q = 2 pi k / N in [-pi, pi) */
static int signed_k(int m, int N) { return (m <= (N - 1) / 2) ? m : m - N; }
static int is_nyquist(int m, int N) { return (N % 2 == 0) && (2 * m == N); }

/* eq. (freqrot): xi'_p = i 2 (N_p/L_p) tan(q_p/2) prod_{m=1..3} (1 + e^{i q_m})/2, the product taken
 * over a dummy axis index m.  With (1 + e^{iq})/2 = e^{iq/2} cos(q/2), the factor tan(q_p/2) times
 * the m = p term equals sin(q_p/2) e^{i q_p/2}, which stays finite at q_p = -pi.  The half-angle
 * cosine at a Nyquist index is an exact zero (integer test). */
static void modified_frequency(const or_grid *g, const int m[3], cplx xi[3]) {
  double q[3], c[3], s[3];
  for (int p = 0; p < 3; ++p) {
    int k = signed_k(m[p], g->n[p]);
    q[p] = 2.0 * M_PI * (double)k / (double)g->n[p];
    c[p] = is_nyquist(m[p], g->n[p]) ? 0.0 : cos(0.5 * q[p]);
    s[p] = sin(0.5 * q[p]);
  }
  if (g->scheme == 1) {
    /* eq. (freq): xi_p = i q_p N_p / L_p */
    for (int p = 0; p < 3; ++p) xi[p] = I * q[p] * (double)g->n[p] / g->L[p];
    return;
  }
  for (int p = 0; p < 3; ++p) {
    double h = g->L[p] / (double)g->n[p];
    cplx f = s[p] * cexp(I * 0.5 * q[p]);
    for (int mm = 0; mm < 3; ++mm)
      if (mm != p) f *= cexp(I * 0.5 * q[mm]) * c[mm];
    xi[p] = I * (2.0 / h) * f;
  }
}

/* ================================================================== projection (eq. galop) */

static const int kI6[6] = {0, 1, 2, 1, 0, 0};
static const int kJ6[6] = {0, 1, 2, 2, 2, 1};

static inline double Isym(int i, int j, int k, int l) {
  return 0.5 * ((i == k) * (j == l) + (i == l) * (j == k));
}

static int is_zero_frequency(const int m[3]) { return m[0] == 0 && m[1] == 0 && m[2] == 0; }

/* eq. (galop) at xi = 0: the symmetric identity on the stress-controlled components KL, zero on the
 * strain-controlled ones kl (a component pair ij and its transpose ji are one component). */
static void zero_frequency_projection(const or_grid *g, const cplx S[3][3], cplx out[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i][j] = 0;
  for (int a = 0; a < 6; ++a)
    if (g->stress_mask & (1 << a)) {
      int i = kI6[a], j = kJ6[a];
      out[i][j] = S[i][j];
      out[j][i] = S[j][i];
    }
}

/* is the projection identically zero at storage frequency m (m != 0)? */
static int projection_vanishes(const or_grid *g, const int m[3], const cplx xi[3]) {
  if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 1; /* xi = 0, strain-controlled components */
  int nyq = 0;
  for (int p = 0; p < 3; ++p) nyq += is_nyquist(m[p], g->n[p]);
  if (g->nyquist == 1 && nyq > 0) return 1;
  if (xi[0] == 0 && xi[1] == 0 && xi[2] == 0) return 1;
  return 0;
}

/* out = Ghat(xi) : S for a complex symmetric tensor S (3x3).  Ghat_ijkl = sym (K^{-1})_ik xi_j xi_l,
 * K_ik = I^s_ijkl xi_j xi_l. */
static void apply_projection(const cplx xi[3], const cplx S[3][3], cplx out[3][3]) {
  cplx K[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      cplx acc = 0;
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) acc += Isym(i, j, k, l) * xi[j] * xi[l];
      K[i][k] = acc;
    }
  /* inverse of the 3x3 matrix by cofactors */
  cplx Ki[3][3];
  cplx det = K[0][0] * (K[1][1] * K[2][2] - K[1][2] * K[2][1]) - K[0][1] * (K[1][0] * K[2][2] - K[1][2] * K[2][0]) +
             K[0][2] * (K[1][0] * K[2][1] - K[1][1] * K[2][0]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
      Ki[i][j] = (K[i1][j1] * K[i2][j2] - K[i1][j2] * K[i2][j1]) / det;
    }
  /* G_ijkl S_kl with G_ijkl = 1/4 (N_ik xi_j xi_l + N_jk xi_i xi_l + N_il xi_j xi_k + N_jl xi_i xi_k) */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          cplx G = 0.25 * (Ki[i][k] * xi[j] * xi[l] + Ki[j][k] * xi[i] * xi[l] + Ki[i][l] * xi[j] * xi[k] +
                           Ki[j][l] * xi[i] * xi[k]);
          acc += G * S[k][l];
        }
      out[i][j] = acc;
    }
}

/* Ghat(m) as a 6x6 matrix acting on the six independent components of S (S_kl = S_lk), i.e.
 * out_ij = sum_kl G_ijkl S_kl written for (ij),(kl) in the order 00,11,22,12,02,01.  Real/imag parts. */
void or_projection_matrix(const or_grid *g, const int m[3], double *Gre, double *Gim) {
  cplx xi[3];
  modified_frequency(g, m, xi);
  int zero = projection_vanishes(g, m, xi);
  for (int b = 0; b < 6; ++b) {
    cplx S[3][3] = {{0}};
    S[kI6[b]][kJ6[b]] = 1.0;
    S[kJ6[b]][kI6[b]] = 1.0;
    cplx out[3][3] = {{0}};
    if (is_zero_frequency(m))
      zero_frequency_projection(g, S, out);
    else if (!zero)
      apply_projection(xi, S, out);
    for (int a = 0; a < 6; ++a) {
      Gre[a * 6 + b] = creal(out[kI6[a]][kJ6[a]]);
      Gim[a * 6 + b] = cimag(out[kI6[a]][kJ6[a]]);
    }
  }
}

void or_modified_frequency(const or_grid *g, const int m[3], double *xre, double *xim) {
  cplx xi[3];
  modified_frequency(g, m, xi);
  for (int p = 0; p < 3; ++p) { xre[p] = creal(xi[p]); xim[p] = cimag(xi[p]); }
}

/* ================================================================== fields and operator */
/* real tensor fields: [6][N] doubles, component order 00,11,22,12,02,01 */

typedef struct {
  or_grid g;
  const double *phi; /* [N] */
  double C1[3][3][3][3], C0[3][3][3][3];
  const double *Cfield; /* NULL, or a Mandel 6x6 stiffness per voxel [N][36] (replaces phi, C1, C0) */
  long N;
  cplx *work; /* [6][N] */
} or_problem;

static double frob_dot(const double *x, const double *y, long N) {
  double acc = 0;
  for (int a = 0; a < 6; ++a) {
    double w = (a < 3) ? 1.0 : 2.0; /* off-diagonal components appear twice in the 3x3 tensor */
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long v = 0; v < N; ++v) s += x[a * N + v] * y[a * N + v];
    acc += w * s;
  }
  return acc;
}

/* sigma = C(x) : eps at every voxel, C(x) = phi C1 + (1 - phi) C0 (Voigt rule), or the voxel's own
 * Mandel stiffness (the tangent of eq. Slin) when P->Cfield is set */
static void stiffness(const or_problem *P, const double *eps, double *sig_re_out, cplx *sig_c_out) {
  long N = P->N;
  if (P->Cfield) {
#pragma omp parallel for schedule(static)
    for (long v = 0; v < N; ++v) {
      const double *Cm = P->Cfield + 36 * v;
      double em[6];
      for (int b = 0; b < 6; ++b) em[b] = eps[b * N + v] * (b < 3 ? 1.0 : sqrt(2.0));
      for (int a = 0; a < 6; ++a) {
        double acc = 0;
        for (int b = 0; b < 6; ++b) acc += Cm[6 * a + b] * em[b];
        acc /= (a < 3 ? 1.0 : sqrt(2.0));
        if (sig_re_out) sig_re_out[a * N + v] = acc;
        if (sig_c_out) sig_c_out[a * N + v] = acc;
      }
    }
    return;
  }
#pragma omp parallel for schedule(static)
  for (long v = 0; v < N; ++v) {
    double e[3][3];
    for (int a = 0; a < 6; ++a) { e[kI6[a]][kJ6[a]] = eps[a * N + v]; e[kJ6[a]][kI6[a]] = eps[a * N + v]; }
    double f = P->phi[v];
    for (int a = 0; a < 6; ++a) {
      int i = kI6[a], j = kJ6[a];
      double acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += (f * P->C1[i][j][k][l] + (1.0 - f) * P->C0[i][j][k][l]) * e[k][l];
      if (sig_re_out) sig_re_out[a * N + v] = acc;
      if (sig_c_out) sig_c_out[a * N + v] = acc;
    }
  }
}

/* y = Re F^{-1}{ Ghat : F{ field } } for a real tensor field given in P->work (complex, overwritten) */
static void project_work(const or_problem *P, double *y) {
  long N = P->N;
  const int *n = P->g.n;
  for (int a = 0; a < 6; ++a) or_fft3(P->work + a * N, n, -1);
#pragma omp parallel for schedule(static)
  for (long v = 0; v < N; ++v) {
    int m[3] = {(int)(v / ((long)n[1] * n[2])), (int)((v / n[2]) % n[1]), (int)(v % n[2])};
    cplx xi[3];
    modified_frequency(&P->g, m, xi);
    cplx S[3][3], out[3][3];
    for (int a = 0; a < 6; ++a) { S[kI6[a]][kJ6[a]] = P->work[a * N + v]; S[kJ6[a]][kI6[a]] = P->work[a * N + v]; }
    if (is_zero_frequency(m)) {
      zero_frequency_projection(&P->g, S, out);
    } else if (projection_vanishes(&P->g, m, xi)) {
      memset(out, 0, sizeof(out));
    } else {
      apply_projection(xi, S, out);
    }
    for (int a = 0; a < 6; ++a) P->work[a * N + v] = out[kI6[a]][kJ6[a]];
  }
  for (int a = 0; a < 6; ++a) or_fft3(P->work + a * N, n, +1);
  for (long i = 0; i < 6 * N; ++i) y[i] = creal(P->work[i]);
}

/* eq. (linearOp): y = A(x) = F^{-1}{ Ghat : F{ C : x } } */
static void apply_A(const or_problem *P, const double *x, double *y) {
  stiffness(P, x, NULL, P->work);
  project_work(P, y);
}

/* ================================================================== public problem setup */

static void mandel_to_tensor4(const double *Cm, double C[3][3][3][3]) {
  /* C_mandel[A][B] = w_A w_B C_{ijkl}, w = 1 (normal) or sqrt(2) (shear), Mandel order
   * 11,22,33,23,13,12 == 00,11,22,12,02,01 here */
  for (int A = 0; A < 6; ++A)
    for (int B = 0; B < 6; ++B) {
      double wa = (A < 3) ? 1.0 : sqrt(2.0), wb = (B < 3) ? 1.0 : sqrt(2.0);
      double v = Cm[A * 6 + B] / (wa * wb);
      int i = kI6[A], j = kJ6[A], k = kI6[B], l = kJ6[B];
      C[i][j][k][l] = v; C[j][i][k][l] = v; C[i][j][l][k] = v; C[j][i][l][k] = v;
    }
}

static void setup(or_problem *P, const int n[3], const double L[3], int scheme, int nyquist, int stress_mask,
                  const double *phi, const double *C1m, const double *C0m) {
  memset(P, 0, sizeof(*P));
  for (int p = 0; p < 3; ++p) { P->g.n[p] = n[p]; P->g.L[p] = L[p]; }
  P->g.scheme = scheme;
  P->g.nyquist = nyquist;
  P->g.stress_mask = stress_mask;
  P->phi = phi;
  P->N = (long)n[0] * n[1] * n[2];
  mandel_to_tensor4(C1m, P->C1);
  mandel_to_tensor4(C0m, P->C0);
  P->work = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)P->N);
}

static void teardown(or_problem *P) { free(P->work); }

/* y = A(x), tensor components */
void or_apply(const int n[3], const double L[3], int scheme, int nyquist, int stress_mask, const double *phi,
              const double *C1m, const double *C0m, const double *x, double *y) {
  or_problem P;
  setup(&P, n, L, scheme, nyquist, stress_mask, phi, C1m, C0m);
  apply_A(&P, x, y);
  teardown(&P);
}

/* y = Re F^{-1} Ghat F x (projection onto compatible fields) */
void or_project(const int n[3], const double L[3], int scheme, int nyquist, int stress_mask, const double *x,
                double *y) {
  or_problem P;
  double one = 1.0, Z[36] = {0};
  long N = (long)n[0] * n[1] * n[2];
  double *phi1 = (double *)malloc(sizeof(double) * N);
  for (long v = 0; v < N; ++v) phi1[v] = one;
  setup(&P, n, L, scheme, nyquist, stress_mask, phi1, Z, Z);
  for (long i = 0; i < 6 * N; ++i) P.work[i] = x[i];
  project_work(&P, y);
  teardown(&P);
  free(phi1);
}

/* ================================================================== Krylov solvers */

typedef struct {
  int iterations;       /* operator applications inside the loop */
  int status;           /* 0 converged, 1 max_iter, 2 breakdown, 3 non-finite */
  double rel_residual;  /* recurrence estimate |phi_bar|/||b|| (MINRES) or ||r||/||b|| (CG) at exit */
  double true_residual; /* ||b - A x|| / ||b|| recomputed from x */
  double bnorm;
  double loop_seconds;  /* wall time of the iteration loop alone (MINRES) */
} or_result;

/* MINRES vectors, each 6N doubles */
typedef struct {
  double *r, *v, *v_old, *p, *d1, *d2;
} minres_vecs;

static void minres_vecs_alloc(minres_vecs *w, long M) {
  w->r = (double *)malloc(sizeof(double) * M);
  w->v = (double *)malloc(sizeof(double) * M);
  w->v_old = (double *)malloc(sizeof(double) * M);
  w->p = (double *)malloc(sizeof(double) * M);
  w->d1 = (double *)malloc(sizeof(double) * M);
  w->d2 = (double *)malloc(sizeof(double) * M);
}
static void minres_vecs_free(minres_vecs *w) {
  free(w->r); free(w->v); free(w->v_old); free(w->p); free(w->d1); free(w->d2);
}

/* MINRES for A x = b (A symmetric), x holds the start on entry and the iterate on exit.
 * Lanczos: beta_{k+1} v_{k+1} = A v_k - alpha_k v_k - beta_k v_{k-1};
 * QR of the (k+1) x k tridiagonal T_k by Givens rotations; search directions d = V R^{-1}.
 * w: the vectors, or NULL to allocate them for this call. */
static void minres_impl(const or_problem *P, const double *b, double *x, double tol, int maxit, double *hist,
                        or_result *res, int zero_start, int final_residual, minres_vecs *w);
static void minres(const or_problem *P, const double *b, double *x, double tol, int maxit, double *hist,
                   or_result *res) {
  minres_impl(P, b, x, tol, maxit, hist, res, 0, 1, NULL);
}
static void minres_impl(const or_problem *P, const double *b, double *x, double tol, int maxit, double *hist,
                        or_result *res, int zero_start, int final_residual, minres_vecs *w) {
  long M = 6 * P->N;
  minres_vecs own;
  if (!w) {
    minres_vecs_alloc(&own, M);
    w = &own;
  }
  double *r = w->r, *v = w->v, *v_old = w->v_old, *p = w->p, *d1 = w->d1, *d2 = w->d2;
  memset(v_old, 0, sizeof(double) * M);
  memset(d1, 0, sizeof(double) * M);
  memset(d2, 0, sizeof(double) * M);
  res->loop_seconds = 0.0;
  double bnorm = sqrt(frob_dot(b, b, P->N));
  res->bnorm = bnorm;
  res->status = 0;
  if (zero_start) {
    for (long i = 0; i < M; ++i) r[i] = b[i]; /* x = 0 */
  } else {
    apply_A(P, x, r);
    for (long i = 0; i < M; ++i) r[i] = b[i] - r[i];
  }
  double beta = sqrt(frob_dot(r, r, P->N));
  res->iterations = 0;
  if (bnorm == 0.0 || beta == 0.0) {
    res->rel_residual = 0.0;
    goto done;
  }
  for (long i = 0; i < M; ++i) v[i] = r[i] / beta;
  double phibar = beta;
  double c_km2 = 1, s_km2 = 0, c_km1 = 1, s_km1 = 0; /* rotations G_{k-2}, G_{k-1} */
  res->rel_residual = phibar / bnorm;
  double t_loop = omp_get_wtime();
  for (int k = 1; k <= maxit; ++k) {
    /* Lanczos step */
    apply_A(P, v, p);
    for (long i = 0; i < M; ++i) p[i] -= beta * v_old[i];
    double alpha = frob_dot(v, p, P->N);
    for (long i = 0; i < M; ++i) p[i] -= alpha * v[i];
    double beta_next = sqrt(frob_dot(p, p, P->N));
    /* new column (beta, alpha, beta_next) of T, rows k-1, k, k+1: rotate by G_{k-2}, G_{k-1} */
    double eps_k = s_km2 * beta;
    double dtil = c_km2 * beta;
    double delta_k = c_km1 * dtil + s_km1 * alpha;
    double gtil = -s_km1 * dtil + c_km1 * alpha;
    double gamma_k = sqrt(gtil * gtil + beta_next * beta_next);
    res->iterations = k;
    if (!(isfinite(alpha) && isfinite(beta_next))) { res->status = 3; break; }
    if (gamma_k == 0.0) { res->status = 2; break; }
    double c_k = gtil / gamma_k, s_k = beta_next / gamma_k;
    double tau = c_k * phibar;
    phibar = -s_k * phibar;
    /* d_k = (v_k - delta_k d_{k-1} - eps_k d_{k-2}) / gamma_k ; x += tau d_k */
    for (long i = 0; i < M; ++i) {
      double dk = (v[i] - delta_k * d1[i] - eps_k * d2[i]) / gamma_k;
      d2[i] = d1[i];
      d1[i] = dk;
      x[i] += tau * dk;
    }
    res->rel_residual = fabs(phibar) / bnorm;
    if (hist) hist[k - 1] = res->rel_residual;
    c_km2 = c_km1; s_km2 = s_km1; c_km1 = c_k; s_km1 = s_k;
    if (res->rel_residual < tol) break;
    if (beta_next == 0.0) break; /* invariant Krylov space: the iterate is exact */
    for (long i = 0; i < M; ++i) { v_old[i] = v[i]; v[i] = p[i] / beta_next; }
    beta = beta_next;
  }
  res->loop_seconds = omp_get_wtime() - t_loop;
  if (res->status == 0 && !(res->rel_residual < tol)) res->status = 1;
done:
  res->true_residual = -1.0;
  if (final_residual) {
    apply_A(P, x, r);
    for (long i = 0; i < M; ++i) r[i] = b[i] - r[i];
    res->true_residual = (bnorm > 0) ? sqrt(frob_dot(r, r, P->N)) / bnorm : 0.0;
  }
  if (w == &own) minres_vecs_free(&own);
}

/* Operator and MINRES with a stiffness per voxel (the tangent C^{i-1}(x) of eq. galnonlin).
 * Cfield: [N][36] Mandel matrices.  or_apply_field: y = A_i(x).  or_minres_field: A_i x = b from
 * x = 0, stopped when |phibar| < tol ||b||; info = (iterations, status, rel_residual, true_residual,
 * ||b||).  Tensor components in and out, as or_apply. */
void or_apply_field(const int n[3], const double L[3], int scheme, int nyquist, int stress_mask, const double *Cfield,
                    const double *x, double *y) {
  or_problem P;
  double Z[36] = {0};
  setup(&P, n, L, scheme, nyquist, stress_mask, NULL, Z, Z);
  P.Cfield = Cfield;
  apply_A(&P, x, y);
  teardown(&P);
}

void or_minres_field(const int n[3], const double L[3], int scheme, int nyquist, int stress_mask,
                     const double *Cfield, const double *b, double tol, int maxit, double *x, double *info) {
  or_problem P;
  double Z[36] = {0};
  setup(&P, n, L, scheme, nyquist, stress_mask, NULL, Z, Z);
  P.Cfield = Cfield;
  memset(x, 0, sizeof(double) * 6 * P.N);
  or_result res;
  minres(&P, b, x, tol, maxit, NULL, &res);
  info[0] = res.iterations;
  info[1] = res.status;
  info[2] = res.rel_residual;
  info[3] = res.true_residual;
  info[4] = res.bnorm;
  teardown(&P);
}

/* Conjugate gradients (Hestenes & Stiefel) on the same system, for the behavioural comparison. */
static void cg(const or_problem *P, const double *b, double *x, double tol, int maxit, double *hist, or_result *res) {
  long M = 6 * P->N;
  double *r = (double *)malloc(sizeof(double) * M), *p = (double *)malloc(sizeof(double) * M);
  double *q = (double *)malloc(sizeof(double) * M);
  double bnorm = sqrt(frob_dot(b, b, P->N));
  res->bnorm = bnorm;
  res->status = 1;
  apply_A(P, x, r);
  for (long i = 0; i < M; ++i) { r[i] = b[i] - r[i]; p[i] = r[i]; }
  double rr = frob_dot(r, r, P->N);
  res->iterations = 0;
  res->rel_residual = (bnorm > 0) ? sqrt(rr) / bnorm : 0;
  if (bnorm == 0 || rr == 0) { res->status = 0; goto done; }
  for (int k = 1; k <= maxit; ++k) {
    apply_A(P, p, q);
    double pq = frob_dot(p, q, P->N);
    res->iterations = k;
    if (pq == 0.0 || !isfinite(pq)) { res->status = 2; break; }
    double a = rr / pq;
    for (long i = 0; i < M; ++i) { x[i] += a * p[i]; r[i] -= a * q[i]; }
    double rr2 = frob_dot(r, r, P->N);
    res->rel_residual = sqrt(rr2) / bnorm;
    if (hist) hist[k - 1] = res->rel_residual;
    if (res->rel_residual < tol) { res->status = 0; break; }
    double bt = rr2 / rr;
    rr = rr2;
    for (long i = 0; i < M; ++i) p[i] = r[i] + bt * p[i];
  }
done:
  apply_A(P, x, r);
  for (long i = 0; i < M; ++i) r[i] = b[i] - r[i];
  res->true_residual = (bnorm > 0) ? sqrt(frob_dot(r, r, P->N)) / bnorm : 0.0;
  free(r); free(p); free(q);
}

/* ================================================================== the homogenization solve */

/* Solve A(eps) = b, b = -F^{-1}{ Ghat : F{ C : Ebar - Sbar } } (eq. gallin), for the fluctuation eps.
 * Mixed macroscopic control (eq. galop): components whose bit is set in stress_mask are
 * stress-controlled, with the macroscopic stress Sbar; the others are strain-controlled, with the
 * macroscopic strain Ebar.  Ebar's stress-controlled components and Sbar's strain-controlled ones are
 * not used (set to zero here).  The fluctuation's mean over the stress-controlled components is the
 * macroscopic strain they take; over the strain-controlled ones it is zero.
 * Ebar, Sbar: tensor components (6); Sbar may be NULL (zero).  x0: NULL for a zero start, else a start
 * that is first projected onto the admissible fields.  Outputs: eps [6][N], sigma [6][N] (may be
 * NULL), sigma_mean [6], residual history (may be NULL, length maxit).  solver: 0 MINRES, 1 CG. */
void or_solve(const int n[3], const double L[3], int scheme, int nyquist, int stress_mask, const double *phi,
              const double *C1m, const double *C0m, const double *Ebar, const double *Sbar, double tol, int maxit,
              int solver, const double *x0, double *eps, double *sigma, double *sigma_mean, double *hist,
              double *info) {
  or_problem P;
  setup(&P, n, L, scheme, nyquist, stress_mask, phi, C1m, C0m);
  long N = P.N, M = 6 * N;
  double *b = (double *)malloc(sizeof(double) * M), *E = (double *)malloc(sizeof(double) * M);
  double Es[6], Ss[6];
  for (int a = 0; a < 6; ++a) {
    int kl = !(stress_mask & (1 << a));
    Es[a] = kl ? Ebar[a] : 0.0;
    Ss[a] = (!kl && Sbar) ? Sbar[a] : 0.0;
  }
  for (int a = 0; a < 6; ++a)
    for (long v = 0; v < N; ++v) E[a * N + v] = Es[a];
  /* the field C : Ebar - Sbar, transformed and projected */
  stiffness(&P, E, NULL, P.work);
  for (int a = 0; a < 6; ++a)
    for (long v = 0; v < N; ++v) P.work[a * N + v] -= Ss[a];
  project_work(&P, b);
  for (long i = 0; i < M; ++i) b[i] = -b[i];
  if (x0) {
    for (long i = 0; i < M; ++i) P.work[i] = x0[i];
    project_work(&P, eps);
  } else {
    memset(eps, 0, sizeof(double) * M);
  }
  or_result res;
  if (solver == 0)
    minres(&P, b, eps, tol, maxit, hist, &res);
  else
    cg(&P, b, eps, tol, maxit, hist, &res);
  /* total strain, stress, volume average of stress */
  for (long i = 0; i < M; ++i) E[i] += eps[i];
  double *sig = sigma ? sigma : b;
  stiffness(&P, E, sig, NULL);
  for (int a = 0; a < 6; ++a) {
    double s = 0;
    for (long v = 0; v < N; ++v) s += sig[a * N + v];
    sigma_mean[a] = s / (double)N;
  }
  info[0] = res.iterations;
  info[1] = res.status;
  info[2] = res.rel_residual;
  info[3] = res.true_residual;
  info[4] = res.bnorm;
  free(b); free(E);
  teardown(&P);
}

/* Timing sample for the CPU baseline: MINRES iterations of A x = b on the given problem, b a seeded
 * pseudo-random tensor field (the cost of an iteration does not depend on b), zero start.  Every
 * vector is allocated and first touched, and `warmup` iterations run, before the timed run of `iters`
 * iterations; only its iteration loop is timed.  Returns those wall seconds. */
double or_time_minres(const int n[3], const double L[3], const double *phi, const double *C1m, const double *C0m,
                      int iters, int warmup) {
  or_problem P;
  setup(&P, n, L, 0, 0, 0, phi, C1m, C0m);
  long M = 6 * P.N;
  double *b = (double *)malloc(sizeof(double) * M), *x = (double *)malloc(sizeof(double) * M);
  uint64_t st = 0x9E3779B97F4A7C15ULL;
  for (long i = 0; i < M; ++i) {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17; /* xorshift64 */
    b[i] = (double)(st >> 11) * 0x1.0p-53 - 0.5;
  }
  minres_vecs w;
  minres_vecs_alloc(&w, M);
  /* first touch of every buffer the loop uses, with the threads that later use them */
  double *bufs[7] = {w.r, w.v, w.v_old, w.p, w.d1, w.d2, x};
  for (int k = 0; k < 7; ++k) {
    double *a = bufs[k];
#pragma omp parallel for schedule(static)
    for (long i = 0; i < M; ++i) a[i] = 0.0;
  }
#pragma omp parallel for schedule(static)
  for (long i = 0; i < M; ++i) P.work[i] = 0.0;
  or_result res;
  if (warmup > 0) minres_impl(&P, b, x, 0.0, warmup, NULL, &res, 1, 0, &w);
  memset(x, 0, sizeof(double) * M);
  minres_impl(&P, b, x, 0.0, iters, NULL, &res, 1, 0, &w);
  minres_vecs_free(&w);
  free(b); free(x);
  teardown(&P);
  return res.loop_seconds;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
