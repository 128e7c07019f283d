// MoDBFFT on gfx950 (section "Modified displacement based FFT for infinite contrast"): the operator
// K(u) = -div(phi C_m grad^s u) - (1 - phi) div(alpha grad^s u) on the half spectrum of the
// displacement fluctuation, and conjugate gradients preconditioned with [xi . Cbar . xi]^{-1}.
//
// Half spectra are [c][n0][n1][K] FP64 complex (K = n2/2 + 1, k2 contiguous), S = n0 n1 K elements per
// component.  One application of K:
//   expand      u_hat (3) -> s_hat = C_m eps_hat (6, Mandel; C_m is uniform) and
//               g_hat = -i alpha xi . eps_hat (3)                                      pointwise
//   ifft axis 0, ifft axis 1 of the 9 components                      k_strided / k_strided_c2c
//   axis 2      per row and component pair (one complex transform): complex-to-real inverse,
//               sigma = phi s / N or h = (1 - phi) g / N, forward real-to-complex k_row_pair / k_row_stress
//   fft axis 1, fft axis 0 of the 9 components
//   contract    K_hat = -i xi . sigma_hat + h_hat, zero at the modes with xi = 0, and the CG partial
//               of <p, K p>                                                            k_contract
// Inner products are those of the real fields: half-spectrum terms weighted by 1 on the k2 = 0 and
// Nyquist planes and by 2 elsewhere.  Reductions are per-block partials summed in a fixed order by one
// block, so a solve is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rve.h"
#include "rve_lds_fft.h"
#include "rve_modbfft.h"
#include "rve_registry.h"

namespace rve {
void set_last_error(const char* text);
}

namespace rvm {

using namespace rvfft;

constexpr int kBlocks = 2048;  // blocks of the pointwise kernels (and their partials)
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr int kMaxRow = 768;   // longest axis 2 (five complex rows of it in a 64 KiB tile)
constexpr int kRowSlots = (kMaxRow + kThreads - 1) / kThreads;

// pencils per block of the register-stage strided transforms: whole waves where possible, at most
// 256 threads and 64 KiB of LDS, no more than the pencils there are (runs of R adjacent pencils keep
// the loads and stores coalesced; one-wave blocks of 5 pencils at 216 = 18 * 12 took 0.53 ms per
// pass against 0.37-0.42 ms with 16)
static int register_pencils(int na, int nb, long long pencils) {
  const long long per = (long long)(na * (nb + 1) + 1) * (long long)sizeof(C);
  int any = 1, full = 0;
  for (int r = 1; r <= 64 && r * nb <= 256 && r * per <= 65536; ++r) {
    any = r;
    if ((r * nb) % 64 == 0) full = r;
  }
  const int r = full ? full : any;
  return (int)std::max<long long>(1, std::min<long long>(r, pencils));
}

struct MGrid {
  int n0, n1, n2, K;
  long long S, nvox;
  double tpl[3];  // 2 pi / L_p
  double alpha;
};

// Mandel index a <-> symmetric pair (i, j): 00, 11, 22, 12, 02, 01 (resolved at compile time in the
// unrolled loops, so the 3x3 arrays they index stay in registers)
__host__ __device__ constexpr int kMi(int a) { return a < 3 ? a : (a == 3 ? 1 : 0); }
__host__ __device__ constexpr int kMj(int a) { return a < 3 ? a : (a == 5 ? 1 : 2); }

__device__ __forceinline__ double freq_full(int i, int n, double tpl) {
  const int k = (2 * i < n) ? i : i - n;
  if ((n & 1) == 0 && 2 * i == n) return 0.0;
  return tpl * (double)k;
}
__device__ __forceinline__ double freq_half(int k, int n, double tpl) {
  if ((n & 1) == 0 && 2 * k == n) return 0.0;
  return tpl * (double)k;
}

// frequency vector of spectral element e; returns false for a mode with xi = 0
__device__ __forceinline__ bool freq_of(const MGrid& g, long long e, double xi[3], int* k2out) {
  const int k2 = (int)(e % g.K);
  const long long r = e / g.K;
  const int i1 = (int)(r % g.n1), i0 = (int)(r / g.n1);
  xi[0] = freq_full(i0, g.n0, g.tpl[0]);
  xi[1] = freq_full(i1, g.n1, g.tpl[1]);
  xi[2] = freq_half(k2, g.n2, g.tpl[2]);
  if (k2out) *k2out = k2;
  return xi[0] != 0.0 || xi[1] != 0.0 || xi[2] != 0.0;
}

__device__ __forceinline__ double weight_of(const MGrid& g, int k2) {
  return (k2 == 0 || ((g.n2 & 1) == 0 && 2 * k2 == g.n2)) ? 1.0 : 2.0;
}

__device__ __forceinline__ C mul_i(C z) { return mk<double>(-z.im, z.re); }
__device__ __forceinline__ C scale(C z, double s) { return mk<double>(z.re * s, z.im * s); }
__device__ __forceinline__ C add(C a, C b) { return mk<double>(a.re + b.re, a.im + b.im); }

__device__ double block_reduce(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

struct Stiff {
  double Cm[36];   // Mandel stiffness of the solid
  double E[6];     // macroscopic strain (Mandel)
};

// ------------------------------------------------------------------ expand
// eps_hat = Mandel of (i/2)(xi_i u_j + xi_j u_i).  ncomp == 6: W[0..6) = eps_hat (for the fields).
// ncomp == 9 (the operator): W[0..6) = s_hat = C_m eps_hat, the solid's stress of the strain, formed in
// Fourier space since C_m is uniform (sigma = phi s is then a product per component in real space), and
// W[6..9) = g_hat = -i alpha xi_j eps_hat_ij.
__global__ __launch_bounds__(kThreads) void k_expand(const C* __restrict__ u, C* __restrict__ W, MGrid g, Stiff st,
                                                     int ncomp) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.S; e += (long long)gridDim.x * blockDim.x) {
    double xi[3];
    if (!freq_of(g, e, xi, nullptr)) {
      for (int c = 0; c < ncomp; ++c) W[c * g.S + e] = mk<double>(0.0, 0.0);
      continue;
    }
    const C u0 = u[e], u1 = u[g.S + e], u2 = u[2 * g.S + e];
    const C uv[3] = {u0, u1, u2};
    C et[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        et[i][j] = mul_i(scale(add(scale(uv[j], xi[i]), scale(uv[i], xi[j])), 0.5));
    C em[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) em[a] = scale(et[kMi(a)][kMj(a)], a < 3 ? 1.0 : kSqrt2);
    if (ncomp == 9) {
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        C sa = mk<double>(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < 6; ++b) sa = add(sa, scale(em[b], st.Cm[6 * a + b]));
        W[a * g.S + e] = sa;
      }
    } else {
#pragma unroll
      for (int a = 0; a < 6; ++a) W[a * g.S + e] = em[a];
    }
    if (ncomp == 9) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        C s = mk<double>(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 3; ++j) s = add(s, scale(et[i][j], xi[j]));
        W[(6 + i) * g.S + e] = scale(mul_i(s), -g.alpha);
      }
    }
  }
}

// ------------------------------------------------------------------ axis 2: inverse, stress, forward
// mode 0 (operator): 9 components in (s = C_m eps and g), sigma = phi s and h = (1 - phi) g out.
// mode 1 (right-hand side): sigma = phi C_m Ebar, 6 out.
// mode 2 (fields): 6 components in, strain = Ebar + eps and stress = phi C_m strain written as real
// fields, per-block partial sums of the stress components.  One row (i0, i1) per block.
__global__ __launch_bounds__(kThreads) void k_row_stress(C* __restrict__ W, const float* __restrict__ phi, MGrid g,
                                                         Stiff st, int mode, FftPlan P, const C* __restrict__ tw,
                                                         const int* __restrict__ rev, double* __restrict__ strain,
                                                         double* __restrict__ stress, double* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  __shared__ double sh[kThreads / 64];
  const long long row = blockIdx.x;  // i0 * n1 + i1
  const int N = g.n2, K = g.K;
  const int nin = mode == 0 ? 9 : (mode == 2 ? 6 : 0);
  const int nout = mode == 0 ? 9 : (mode == 1 ? 6 : 0);
  const int npen = mode == 0 ? 5 : 3;
  const double invN = 1.0 / (double)g.nvox;
  if (nin) {
    for (int idx = threadIdx.x; idx < npen * K; idx += blockDim.x) {
      const int q = idx / K, k = idx - q * K;
      C A = W[(long long)(2 * q) * g.S + row * K + k];
      C B = (2 * q + 1 < nin) ? W[(long long)(2 * q + 1) * g.S + row * K + k] : mk<double>(0.0, 0.0);
      if (k == 0 || 2 * k == N) {  // a real row's DC and Nyquist terms are real
        A.im = 0.0;
        B.im = 0.0;
      }
      buf[rev[k] * npen + q] = mk<double>(A.re - B.im, A.im + B.re);
      if (k > 0 && 2 * k < N) buf[rev[N - k] * npen + q] = mk<double>(A.re + B.im, B.re - A.im);
    }
    __syncthreads();
    lds_fft<1>(buf, npen, P, tw);
  }
  double v[kRowSlots][10];
  double ssum[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < kRowSlots; ++u) {
    const int e = threadIdx.x + u * kThreads;
    if (e < N) {
      double c[10];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (q < npen && nin) {
          const C z = buf[e * npen + q];
          c[2 * q] = z.re * invN;
          c[2 * q + 1] = z.im * invN;
        } else {
          c[2 * q] = 0.0;
          c[2 * q + 1] = 0.0;
        }
      }
      const double ph = (double)phi[row * N + e];
      double eps[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) eps[a] = (mode == 0 ? 0.0 : st.E[a]) + c[a];
      double sig[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        double s = 0.0;
        if (mode == 0) {
          s = c[a];
        } else {
#pragma unroll
          for (int b = 0; b < 6; ++b) s += st.Cm[6 * a + b] * eps[b];
        }
        sig[a] = ph * s;
      }
      if (mode == 2) {
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          if (strain) strain[(long long)a * g.nvox + row * N + e] = eps[a];
          if (stress) stress[(long long)a * g.nvox + row * N + e] = sig[a];
          ssum[a] += sig[a];
        }
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) v[u][a] = sig[a];
#pragma unroll
      for (int a = 6; a < 9; ++a) v[u][a] = mode == 0 ? (1.0 - ph) * c[a] : 0.0;
      v[u][9] = 0.0;
    }
  }
  if (mode == 2) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double s = block_reduce(ssum[a], sh);
      if (threadIdx.x == 0) partials[(long long)a * gridDim.x + blockIdx.x] = s;
    }
    return;
  }
  __syncthreads();  // every thread has read its inverse-transformed values
#pragma unroll
  for (int u = 0; u < kRowSlots; ++u) {
    const int e = threadIdx.x + u * kThreads;
    if (e < N) {
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if (q < npen) buf[rev[e] * npen + q] = mk<double>(v[u][2 * q], v[u][2 * q + 1]);
    }
  }
  __syncthreads();
  lds_fft<-1>(buf, npen, P, tw);
  for (int idx = threadIdx.x; idx < npen * K; idx += blockDim.x) {
    const int q = idx / K, k = idx - q * K;
    const C z = buf[k * npen + q];
    const C zc = buf[((N - k) % N) * npen + q];
    if (2 * q < nout) W[(long long)(2 * q) * g.S + row * K + k] = mk<double>(0.5 * (z.re + zc.re), 0.5 * (z.im - zc.im));
    if (2 * q + 1 < nout)
      W[(long long)(2 * q + 1) * g.S + row * K + k] = mk<double>(0.5 * (z.im + zc.im), -0.5 * (z.re - zc.re));
  }
}

// ------------------------------------------------------------------ contract
// mode 0: out = -i xi . sigma_hat + h_hat, partials of <p, out>;  mode 1: out = +i xi . sigma_hat (b),
// partials of <out, out>.  sigma_hat from the Mandel components W[0..6).
__global__ __launch_bounds__(kThreads) void k_contract(const C* __restrict__ W, C* __restrict__ out,
                                                       const C* __restrict__ p, MGrid g, int mode,
                                                       double* __restrict__ partials) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.S; e += (long long)gridDim.x * blockDim.x) {
    double xi[3];
    int k2;
    C o[3] = {mk<double>(0.0, 0.0), mk<double>(0.0, 0.0), mk<double>(0.0, 0.0)};
    if (freq_of(g, e, xi, &k2)) {
      C s[3][3];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const C m = scale(W[a * g.S + e], a < 3 ? 1.0 : 1.0 / kSqrt2);
        s[kMi(a)][kMj(a)] = m;
        s[kMj(a)][kMi(a)] = m;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        C d = mk<double>(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 3; ++j) d = add(d, scale(s[i][j], xi[j]));
        d = mul_i(d);
        o[i] = mode == 0 ? add(scale(d, -1.0), W[(6 + i) * g.S + e]) : d;
      }
      const double w = weight_of(g, k2);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const C b = mode == 0 ? p[i * g.S + e] : o[i];
        acc += w * (b.re * o[i].re + b.im * o[i].im);
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) out[i * g.S + e] = o[i];
  }
  const double s = block_reduce(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ------------------------------------------------------------------ CG
struct Prec {
  double Cbar[81];  // <phi> C_m as C_ijkl
  int identity;     // empty cell: no preconditioner
};

// z = [xi . Cbar . xi]^{-1} r at one mode (cofactor inverse of the symmetric 3x3 acoustic tensor)
__device__ __forceinline__ void precondition(const Prec& pc, const double xi[3], const C r[3], C z[3]) {
  if (pc.identity) {
    for (int i = 0; i < 3; ++i) z[i] = r[i];
    return;
  }
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int l = 0; l < 3; ++l) s += xi[j] * pc.Cbar[((i * 3 + j) * 3 + k) * 3 + l] * xi[l];
      A[i][k] = s;
    }
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  const double id = 1.0 / det;
  const double I[3][3] = {{c00 * id, (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id, (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id},
                          {c01 * id, (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id, (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id},
                          {c02 * id, (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id, (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id}};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    z[i] = mk<double>(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) z[i] = add(z[i], scale(r[k], I[i][k]));
  }
}

struct CGState {
  double rz, pq, alpha, beta, rr, bb;
};

// one block: dst = sum of n partials (fixed order)
__global__ void k_sum(const double* __restrict__ partials, int n, double* dst) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
  const double s = block_reduce(acc, sh);
  if (threadIdx.x == 0) *dst = s;
}

// alpha = rz / <p, K p>
__global__ void k_cg_alpha(CGState* st, const double* __restrict__ partials, int n) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
  const double s = block_reduce(acc, sh);
  if (threadIdx.x == 0) {
    st->pq = s;
    st->alpha = st->rz / s;
  }
}

// x += alpha p, r -= alpha q; partials of <r, M r> and <r, r>
__global__ __launch_bounds__(kThreads) void k_cg_xr(C* __restrict__ x, C* __restrict__ r, const C* __restrict__ p,
                                                    const C* __restrict__ q, const CGState* __restrict__ st, MGrid g,
                                                    Prec pc, double* __restrict__ partials) {
  __shared__ double sh[kThreads / 64];
  const double a = st->alpha;
  double arz = 0.0, arr = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.S; e += (long long)gridDim.x * blockDim.x) {
    double xi[3];
    int k2;
    const bool act = freq_of(g, e, xi, &k2);
    C rv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const C pv = p[i * g.S + e], qv = q[i * g.S + e];
      C xv = x[i * g.S + e];
      xv = add(xv, scale(pv, a));
      rv[i] = add(r[i * g.S + e], scale(qv, -a));
      x[i * g.S + e] = xv;
      r[i * g.S + e] = rv[i];
    }
    if (act) {
      C z[3];
      precondition(pc, xi, rv, z);
      const double w = weight_of(g, k2);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        arz += w * (rv[i].re * z[i].re + rv[i].im * z[i].im);
        arr += w * (rv[i].re * rv[i].re + rv[i].im * rv[i].im);
      }
    }
  }
  const double s1 = block_reduce(arz, sh);
  const double s2 = block_reduce(arr, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s1;
    partials[gridDim.x + blockIdx.x] = s2;
  }
}

// beta = rz_new / rz, rz = rz_new, rr
__global__ void k_cg_beta(CGState* st, const double* __restrict__ partials, int n) {
  __shared__ double sh[kThreads / 64];
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a1 += partials[i];
    a2 += partials[n + i];
  }
  const double s1 = block_reduce(a1, sh);
  const double s2 = block_reduce(a2, sh);
  if (threadIdx.x == 0) {
    st->beta = s1 / st->rz;
    st->rz = s1;
    st->rr = s2;
  }
}

// p = M r + beta p (beta from the state, or 0 with init); init also gives partials of <r, M r>
__global__ __launch_bounds__(kThreads) void k_cg_p(C* __restrict__ p, const C* __restrict__ r,
                                                   const CGState* __restrict__ st, MGrid g, Prec pc, int init,
                                                   double* __restrict__ partials) {
  __shared__ double sh[kThreads / 64];
  const double b = init ? 0.0 : st->beta;
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.S; e += (long long)gridDim.x * blockDim.x) {
    double xi[3];
    int k2;
    const bool act = freq_of(g, e, xi, &k2);
    C rv[3], z[3] = {mk<double>(0.0, 0.0), mk<double>(0.0, 0.0), mk<double>(0.0, 0.0)};
#pragma unroll
    for (int i = 0; i < 3; ++i) rv[i] = r[i * g.S + e];
    if (act) precondition(pc, xi, rv, z);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const C pv = init ? mk<double>(0.0, 0.0) : p[i * g.S + e];
      p[i * g.S + e] = add(z[i], scale(pv, b));
    }
    if (init && act) {
      const double w = weight_of(g, k2);
#pragma unroll
      for (int i = 0; i < 3; ++i) acc += w * (rv[i].re * z[i].re + rv[i].im * z[i].im);
    }
  }
  if (init) {
    const double s = block_reduce(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

__global__ void k_zero_c(C* x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = mk<double>(0.0, 0.0);
}

__global__ void k_check_phi_m(const float* phi, long long n, double* partials, int* flag) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float v = phi[i];
    if (!(v >= 0.0f && v <= 1.0f)) atomicOr(flag, 1);
    acc += (double)v;
  }
  const double s = block_reduce(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ------------------------------------------------------------------ host side
struct Layout {
  size_t W, x, r, p, q, tab[3], rev[3], part, state, flag, total;
};

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

static bool plan_grid(const rve_grid* grid, FftPlan P[3], MGrid& g) {
  if (!grid) return false;
  for (int p = 0; p < 3; ++p)
    if (grid->n[p] < 1 || !make_plan(grid->n[p], P[p])) return false;
  if (grid->n[2] > kMaxRow) return false;
  g.n0 = grid->n[0];
  g.n1 = grid->n[1];
  g.n2 = grid->n[2];
  g.K = g.n2 / 2 + 1;
  g.S = (long long)g.n0 * g.n1 * g.K;
  g.nvox = (long long)g.n0 * g.n1 * g.n2;
  for (int p = 0; p < 3; ++p) g.tpl[p] = 2.0 * M_PI / grid->L[p];
  return true;
}

static Layout layout(const MGrid& g, const FftPlan P[3]) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o += a256(b);
    return r;
  };
  const size_t comp = (size_t)g.S * sizeof(C);
  L.W = take(9 * comp);
  L.x = take(3 * comp);
  L.r = take(3 * comp);
  L.p = take(3 * comp);
  L.q = take(3 * comp);
  for (int p = 0; p < 3; ++p) {
    L.tab[p] = take((size_t)P[p].n * sizeof(C));
    L.rev[p] = take((size_t)P[p].n * sizeof(int));
  }
  L.part = take((6 * (size_t)std::max<long long>(kBlocks, (long long)g.n0 * g.n1) + 64) * sizeof(double));
  L.state = take(sizeof(CGState));
  L.flag = take(64);
  L.total = o;
  return L;
}

static rve_status fail(hipError_t e, const char* what) {
  char text[256];
  snprintf(text, sizeof(text), "%s (%d) in %s (rve_modbfft.hip)", hipGetErrorString(e), (int)e, what);
  rve::set_last_error(text);
  return RVE_EDEVICE;
}

#define MCHK(x)                                  \
  do {                                           \
    hipError_t e_ = (x);                         \
    if (e_ != hipSuccess) return fail(e_, #x);   \
  } while (0)

struct Timer {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  void begin(int k) {
    if (!on) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    (void)hipEventRecord(a, s);
    ev.push_back({k, {a, b}});
  }
  void end() {
    if (on && !ev.empty()) (void)hipEventRecord(ev.back().second.second, s);
  }
  void collect(rve_modbfft_stats* st) {
    for (auto& e : ev) {
      float ms = 0.f;
      if (hipEventSynchronize(e.second.second) == hipSuccess &&
          hipEventElapsedTime(&ms, e.second.first, e.second.second) == hipSuccess && st) {
        st->pass_ms[e.first] += ms;
        st->pass_launches[e.first] += 1;
      }
      (void)hipEventDestroy(e.second.first);
      (void)hipEventDestroy(e.second.second);
    }
    ev.clear();
  }
};

}  // namespace rvm

extern "C" {

size_t rve_modbfft_workspace_bytes(const rve_grid* grid) {
  using namespace rvm;
  FftPlan P[3];
  MGrid g;
  if (!plan_grid(grid, P, g)) return 0;
  return layout(g, P).total;
}

rve_status solve_rve_modbfft(const rve_grid* grid, const float* phi, const double* C_solid,
                             const double* macro_strain, double alpha, double tol, int32_t max_iter,
                             double* strain_out, double* stress_out, double* eff_stress, rve_modbfft_stats* stats,
                             void* workspace, size_t workspace_bytes, void* hip_stream) {
  using namespace rvm;
  if (!grid || !phi || !C_solid || !macro_strain || !eff_stress || !workspace) return RVE_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!(std::isfinite(grid->L[p]) && grid->L[p] > 0.0)) return RVE_EINVAL;
  if (!(tol > 0.0 && tol < 1.0) || max_iter < 1 || !std::isfinite(alpha)) return RVE_EINVAL;
  for (int i = 0; i < 36; ++i)
    if (!std::isfinite(C_solid[i])) return RVE_ENONFINITE;
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b)
      if (std::fabs(C_solid[6 * a + b] - C_solid[6 * b + a]) > 1e-12 * (std::fabs(C_solid[6 * a + b]) + 1e-300))
        return RVE_EINVAL;
  for (int a = 0; a < 6; ++a)
    if (!std::isfinite(macro_strain[a])) return RVE_ENONFINITE;
  FftPlan P[3];
  MGrid g;
  if (!plan_grid(grid, P, g)) return RVE_EUNSUPPORTED_SIZE;
  if ((long long)g.n0 * g.n1 >= (1LL << 31)) return RVE_EUNSUPPORTED_SIZE;
  const Layout L = layout(g, P);
  if (workspace_bytes < L.total) return RVE_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RVE_EINVAL;
  // alpha: by default 1e-4 / (C^-1)_00 (1e-4 E of an isotropic solid); (C^-1)_00 from Gauss-Jordan
  double a_used = alpha;
  {
    double M[6][12];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 12; ++j) M[i][j] = j < 6 ? C_solid[6 * i + j] : (j - 6 == i ? 1.0 : 0.0);
    for (int c = 0; c < 6; ++c) {
      int piv = c;
      for (int i = c + 1; i < 6; ++i)
        if (std::fabs(M[i][c]) > std::fabs(M[piv][c])) piv = i;
      if (!(std::fabs(M[piv][c]) > 0.0)) return RVE_EINVAL;  // singular stiffness
      for (int j = 0; j < 12; ++j) std::swap(M[c][j], M[piv][j]);
      const double d = M[c][c];
      for (int j = 0; j < 12; ++j) M[c][j] /= d;
      for (int i = 0; i < 6; ++i)
        if (i != c) {
          const double f = M[i][c];
          for (int j = 0; j < 12; ++j) M[i][j] -= f * M[c][j];
        }
    }
    if (!(alpha > 0.0)) {
      if (!(M[0][6] > 0.0)) return RVE_EINVAL;
      a_used = 1e-4 / M[0][6];
    }
  }
  g.alpha = a_used;
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = static_cast<char*>(workspace);
  C* W = reinterpret_cast<C*>(ws + L.W);
  C* x = reinterpret_cast<C*>(ws + L.x);
  C* r = reinterpret_cast<C*>(ws + L.r);
  C* pv = reinterpret_cast<C*>(ws + L.p);
  C* q = reinterpret_cast<C*>(ws + L.q);
  C* tw[3];
  int* rev[3];
  for (int p = 0; p < 3; ++p) {
    tw[p] = reinterpret_cast<C*>(ws + L.tab[p]);
    rev[p] = reinterpret_cast<int*>(ws + L.rev[p]);
  }
  double* part = reinterpret_cast<double*>(ws + L.part);
  CGState* dst = reinterpret_cast<CGState*>(ws + L.state);
  int* flag = reinterpret_cast<int*>(ws + L.flag);
  Timer T;
  T.on = stats && stats->timed;
  T.s = s;
  if (stats) {
    for (int k = 0; k < RVE_MODBFFT_NPASS; ++k) {
      stats->pass_ms[k] = 0.0;
      stats->pass_launches[k] = 0;
    }
    stats->iterations = 0;
    stats->rel_residual = 0.0;
    stats->alpha = a_used;
  }
  // phase map in [0, 1], its mean
  MCHK(hipMemsetAsync(flag, 0, 64, s));
  hipLaunchKernelGGL(k_check_phi_m, dim3(kBlocks), dim3(kThreads), 0, s, phi, g.nvox, part, flag);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, part, kBlocks, part + kBlocks);
  double hsum = 0.0;
  int hflag = 0;
  MCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MCHK(hipMemcpyAsync(&hsum, part + kBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  MCHK(hipStreamSynchronize(s));
  if (hflag) return RVE_EINVAL;
  const double rho = hsum / (double)g.nvox;
  for (int p = 0; p < 3; ++p)
    hipLaunchKernelGGL(k_fft_tables, dim3((P[p].n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, tw[p], rev[p], P[p]);
  // stiffness, macroscopic strain, preconditioner's reference medium
  Stiff st;
  for (int i = 0; i < 36; ++i) st.Cm[i] = C_solid[i];
  for (int a = 0; a < 6; ++a) st.E[a] = macro_strain[a];
  Prec pc;
  pc.identity = rho > 0.0 ? 0 : 1;
  {
    static const int mi[6] = {0, 1, 2, 1, 0, 0}, mj[6] = {0, 1, 2, 2, 2, 1};
    for (int A = 0; A < 6; ++A)
      for (int B = 0; B < 6; ++B) {
        const double v = rho * C_solid[6 * A + B] / ((A < 3 ? 1.0 : kSqrt2) * (B < 3 ? 1.0 : kSqrt2));
        const int i = mi[A], j = mj[A], k = mi[B], l = mj[B];
        const int I[2][2] = {{i, j}, {j, i}}, J[2][2] = {{k, l}, {l, k}};
        for (int u = 0; u < 2; ++u)
          for (int w = 0; w < 2; ++w) pc.Cbar[((I[u][0] * 3 + I[u][1]) * 3 + J[w][0]) * 3 + J[w][1]] = v;
      }
  }
  const int lds_row9 = 5 * g.n2 * (int)sizeof(C), lds_row6 = 3 * g.n2 * (int)sizeof(C);
  const int TW0 = strided_tile(g.n0, (long long)g.n1 * g.K), TW1 = strided_tile(g.n1, g.K);
  const dim3 gr0((unsigned)(((long long)g.n1 * g.K + TW0 - 1) / TW0), 1, 1);
  const dim3 gr1((unsigned)((g.K + TW1 - 1) / TW1), (unsigned)g.n0, 1);
  const size_t lds0 = (size_t)TW0 * g.n0 * sizeof(C), lds1 = (size_t)TW1 * g.n1 * sizeof(C);
  const unsigned rows = (unsigned)((long long)g.n0 * g.n1);
  // lengths with a compiled factorisation take the register-stage kernels, the others the LDS plan
  const rve::LenEntry* reg[2] = {rve::lookup_len(g.n0), rve::lookup_len(g.n1)};
  int RP[2] = {0, 0};
  dim3 grr[2];
  size_t ldsr[2] = {0, 0};
  for (int p = 0; p < 2; ++p) {
    if (!reg[p]) continue;
    const long long pencils = p == 0 ? (long long)g.n1 * g.K : g.K;
    RP[p] = register_pencils(reg[p]->na, reg[p]->nb, pencils);
    grr[p] = dim3((unsigned)((pencils + RP[p] - 1) / RP[p]), p == 0 ? 1u : (unsigned)g.n0, 1);
    ldsr[p] = (size_t)RP[p] * (reg[p]->na * (reg[p]->nb + 1) + 1) * sizeof(C);
  }
  // the operator's row pass: per component pair with register stages where the length is compiled
  const rve::LenEntry* reg2 = rve::lookup_len(g.n2);
  int RW = 0;
  size_t ldsw = 0;
  if (reg2) {
    // one wave per block (64 / NB rows): its barriers are cheap, and eight such blocks fit a CU's LDS
    // at 216 = 18 * 12 (0.66 ms per pass there, against 0.79 ms with 16 rows of 192 threads); the rows
    // are contiguous in every component, so the loads stay coalesced at any row count
    const int rs = std::max(g.n2 + 1, reg2->na * (reg2->nb + 1));
    RW = (int)std::max<long long>(1, std::min<long long>(std::max(1, 64 / reg2->nb), rows));
    ldsw = (size_t)RW * rs * sizeof(C);
  }
  auto row_pass = [&]() {
    T.begin(RVE_MODBFFT_AXIS2_STRESS);
    if (reg2)
      hipLaunchKernelGGL(reg2->d.rowp, dim3((unsigned)((rows + RW - 1) / RW), 1, 5), dim3(RW * reg2->nb), ldsw, s, W,
                         g.S, phi, (long long)rows, g.K, 9, 6, 1.0 / (double)g.nvox, tw[2], RW);
    else
      hipLaunchKernelGGL(k_row_stress, dim3(rows), dim3(kThreads), lds_row9, s, W, phi, g, st, 0, P[2], tw[2], rev[2],
                         (double*)nullptr, (double*)nullptr, part);
    T.end();
  };
  auto strided = [&](int pass, int sign, int axis, int ncomp) {
    if (reg[axis]) {
      dim3 gr = grr[axis];
      gr.z = ncomp;
      const rve::LenKernels<double>& k = reg[axis]->d;
      T.begin(pass);
      hipLaunchKernelGGL(sign < 0 ? k.scf : k.sci, gr, dim3(RP[axis] * reg[axis]->nb), ldsr[axis], s, W, g.S, g.n1,
                         g.K, axis, tw[axis], RP[axis]);
      T.end();
      return;
    }
    dim3 gr = axis == 0 ? gr0 : gr1;
    gr.z = ncomp;
    T.begin(pass);
    if (sign < 0)
      hipLaunchKernelGGL(k_strided_c2c<-1>, gr, dim3(kThreads), axis == 0 ? lds0 : lds1, s, W, g.S, g.n0, g.n1, g.K,
                         axis, P[axis], tw[axis], rev[axis], axis == 0 ? TW0 : TW1);
    else
      hipLaunchKernelGGL(k_strided_c2c<1>, gr, dim3(kThreads), axis == 0 ? lds0 : lds1, s, W, g.S, g.n0, g.n1, g.K,
                         axis, P[axis], tw[axis], rev[axis], axis == 0 ? TW0 : TW1);
    T.end();
  };
  // b = div(phi C_m Ebar): stress of the macroscopic strain, forward transform, +i xi . sigma_hat
  T.begin(RVE_MODBFFT_AXIS2_STRESS);
  hipLaunchKernelGGL(k_row_stress, dim3(rows), dim3(kThreads), lds_row6, s, W, phi, g, st, 1, P[2], tw[2], rev[2],
                     (double*)nullptr, (double*)nullptr, part);
  T.end();
  strided(RVE_MODBFFT_FFT_AXIS1, -1, 1, 6);
  strided(RVE_MODBFFT_FFT_AXIS0, -1, 0, 6);
  T.begin(RVE_MODBFFT_CONTRACT);
  hipLaunchKernelGGL(k_contract, dim3(kBlocks), dim3(kThreads), 0, s, W, r, (const C*)nullptr, g, 1, part);
  T.end();
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, part, kBlocks, &dst->bb);
  hipLaunchKernelGGL(k_zero_c, dim3(kBlocks), dim3(kThreads), 0, s, x, 3 * g.S);
  hipLaunchKernelGGL(k_cg_p, dim3(kBlocks), dim3(kThreads), 0, s, pv, r, dst, g, pc, 1, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, part, kBlocks, &dst->rz);
  MCHK(hipGetLastError());
  CGState h;
  MCHK(hipMemcpyAsync(&h, dst, sizeof(h), hipMemcpyDeviceToHost, s));
  MCHK(hipStreamSynchronize(s));
  if (!std::isfinite(h.bb) || !std::isfinite(h.rz)) return RVE_ENONFINITE;
  double bnorm = std::sqrt(h.bb);
  {
    // a right-hand side at the rounding level of the transforms of a uniform stress (a homogeneous
    // cell) counts as zero: the exact answer is u = 0
    double cmax = 0.0, emax = 0.0, ximax = 0.0;
    for (int i = 0; i < 36; ++i) cmax = std::max(cmax, std::fabs(C_solid[i]));
    for (int a = 0; a < 6; ++a) emax = std::max(emax, std::fabs(macro_strain[a]));
    for (int p = 0; p < 3; ++p) ximax = std::max(ximax, g.tpl[p] * (double)(grid->n[p] / 2));
    if (bnorm <= 1e-13 * cmax * emax * ximax * (double)g.nvox) bnorm = 0.0;
  }
  double rn = bnorm;
  int it = 0;
  rve_status status = RVE_OK;
  while (bnorm > 0.0 && rn > tol * bnorm) {
    if (it >= max_iter) {
      status = RVE_NOT_CONVERGED;
      break;
    }
    // q = K p
    T.begin(RVE_MODBFFT_EXPAND);
    hipLaunchKernelGGL(k_expand, dim3(kBlocks), dim3(kThreads), 0, s, (const C*)pv, W, g, st, 9);
    T.end();
    strided(RVE_MODBFFT_IFFT_AXIS0, 1, 0, 9);
    strided(RVE_MODBFFT_IFFT_AXIS1, 1, 1, 9);
    row_pass();
    strided(RVE_MODBFFT_FFT_AXIS1, -1, 1, 9);
    strided(RVE_MODBFFT_FFT_AXIS0, -1, 0, 9);
    T.begin(RVE_MODBFFT_CONTRACT);
    hipLaunchKernelGGL(k_contract, dim3(kBlocks), dim3(kThreads), 0, s, W, q, (const C*)pv, g, 0, part);
    T.end();
    T.begin(RVE_MODBFFT_CG_UPDATE);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, dst, part, kBlocks);
    hipLaunchKernelGGL(k_cg_xr, dim3(kBlocks), dim3(kThreads), 0, s, x, r, (const C*)pv, (const C*)q, dst, g, pc, part);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kThreads), 0, s, dst, part, kBlocks);
    hipLaunchKernelGGL(k_cg_p, dim3(kBlocks), dim3(kThreads), 0, s, pv, (const C*)r, dst, g, pc, 0, part);
    T.end();
    MCHK(hipGetLastError());
    MCHK(hipMemcpyAsync(&h, dst, sizeof(h), hipMemcpyDeviceToHost, s));
    MCHK(hipStreamSynchronize(s));
    ++it;
    if (!std::isfinite(h.rr) || !std::isfinite(h.alpha)) return RVE_ENONFINITE;
    rn = std::sqrt(h.rr);
    if (T.on) T.collect(stats);
  }
  // fields and <sigma>
  hipLaunchKernelGGL(k_expand, dim3(kBlocks), dim3(kThreads), 0, s, (const C*)x, W, g, st, 6);
  strided(RVE_MODBFFT_IFFT_AXIS0, 1, 0, 6);
  strided(RVE_MODBFFT_IFFT_AXIS1, 1, 1, 6);
  hipLaunchKernelGGL(k_row_stress, dim3(rows), dim3(kThreads), lds_row6, s, W, phi, g, st, 2, P[2], tw[2], rev[2],
                     strain_out, stress_out, part);
  for (int a = 0; a < 6; ++a)
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, part + (long long)a * rows, (int)rows, part + 6LL * rows + a);
  MCHK(hipGetLastError());
  double hs[6];
  MCHK(hipMemcpyAsync(hs, part + 6LL * rows, sizeof(hs), hipMemcpyDeviceToHost, s));
  MCHK(hipStreamSynchronize(s));
  if (T.on) T.collect(stats);
  for (int a = 0; a < 6; ++a) eff_stress[a] = hs[a] / (double)g.nvox;
  if (stats) {
    stats->iterations = it;
    stats->rel_residual = bnorm > 0.0 ? rn / bnorm : 0.0;
  }
  return status;
}

}  // extern "C"
