// Lattice phase maps on gfx950: plain voxels, Voigt fine grid, Voigt analytic (eq. phaselin) and the
// phase-field smoothening of eqs. phase / phase3 (sections "Voigt approaches", "Phase-field
// smoothening", "Combined smoothening").
//
// The phase-field step is one FFT-diagonal Helmholtz solve on the fine grid m = ratio * n, run as
// five streaming passes over an FP64 half spectrum [m0][m1][m2/2+1] (natural order, k2 contiguous):
//   G1 k_source_r2c   the source omega is generated in registers (solid indicator from the strut
//                     distances, or the coarse map) and transformed along axis 2, two real rows packed
//                     into one complex transform and separated after it; the fine map is never stored
//   G2 k_axis_c2c     complex FFT along axis 1 (tiles of adjacent k2 columns: coalesced rows)
//   G3 k_axis_c2c     FFT along axis 0, multiply by 1 / (1 + (ell^2/eps)|xi|^2) / (m0 m1 m2), inverse
//                     FFT along axis 0, all in one LDS tile
//   G4 k_axis_c2c     inverse FFT along axis 1
//   G5 k_c2r_coarsen  complex-to-real inverse along axis 2 for the ratio^2 fine rows of one coarse
//                     row, summed in registers over the rows and in LDS over ratio consecutive voxels:
//                     the coarse average and the threshold are written directly
// Every 1-D transform runs in LDS with a runtime mixed-radix plan (radices 4, 2, 3, 5): decimation
// in time, in place, with the input scattered to digit-reversed positions when it is loaded and the
// output in natural order; one barrier per stage.  Any 5-smooth length up to 1024 uses the same
// code, so no length needs its own kernel instance.  The distance arithmetic is compiled without
// contraction into fused multiply-adds, which keeps the inside/outside decisions and the Voigt
// maps identical to a plain IEEE evaluation of the same formulas.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "rve.h"
#include "rve_device.h"
#include "rve_geometry.h"
#include "rve_lds_fft.h"

namespace rve {
void set_last_error(const char* text);
void geo_prof_begin(int g, hipStream_t s);
void geo_prof_end(hipStream_t s);
void geo_prof_flush();
}

namespace rvg {

using rve::cmul;
using rve::cx;
using rve::DFT;
using rve::mk;
using C = cx<double>;
using namespace rvfft;

// a strut ready for the distance: midpoint and half axis in length units, |half|^2, radius
struct StrutPrep {
  double mid[3], half[3], hh, r;
};

struct Cell {
  double L[3];
  double h[3];  // voxel lengths of the grid the points are taken on
};

__device__ __forceinline__ void prep_strut(const rve_strut& s, const double L[3], StrutPrep& p) {
#pragma clang fp contract(off)
  double hh = 0.0;
  for (int q = 0; q < 3; ++q) {
    const double a = s.a[q] * L[q], b = s.b[q] * L[q];
    p.mid[q] = 0.5 * (a + b);
    p.half[q] = 0.5 * (b - a);
    hh += p.half[q] * p.half[q];
  }
  p.hh = hh;
  p.r = s.radius;
}

// distance from point x to the strut axis segment (its periodic image nearest to the midpoint)
__device__ __forceinline__ double axis_distance(const StrutPrep& s, const double L[3], const double x[3]) {
#pragma clang fp contract(off)
  double dx[3], dh = 0.0;
  for (int q = 0; q < 3; ++q) {
    dx[q] = x[q] - s.mid[q];
    dx[q] -= L[q] * floor(dx[q] / L[q] + 0.5);
    dh += dx[q] * s.half[q];
  }
  double t = s.hh > 0.0 ? dh / s.hh : 0.0;
  t = t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t);
  double e2 = 0.0;
  for (int q = 0; q < 3; ++q) {
    const double e = dx[q] - t * s.half[q];
    e2 += e * e;
  }
  return sqrt(e2);
}

__device__ __forceinline__ double signed_distance(const StrutPrep* sp, int ns, const double L[3], const double x[3]) {
  double D = INFINITY;
  for (int k = 0; k < ns; ++k) {
    const double d = axis_distance(sp[k], L, x) - sp[k].r;
    if (d < D) D = d;
  }
  return D;
}

// D(x) <= 0: the first strut that contains the point decides
__device__ __forceinline__ bool inside(const StrutPrep* sp, int ns, const double L[3], const double x[3]) {
  for (int k = 0; k < ns; ++k)
    if (axis_distance(sp[k], L, x) - sp[k].r <= 0.0) return true;
  return false;
}

__device__ __forceinline__ void load_struts(const rve_strut* __restrict__ struts, int ns, const double L[3],
                                            StrutPrep* sp) {
  for (int k = threadIdx.x; k < ns; k += blockDim.x) {
    rve_strut s = struts[k];
    prep_strut(s, L, sp[k]);
  }
}

// Candidate struts of a set of rows along axis 2: only x_2 varies along a row, and the nearest-image
// offsets to a strut midpoint in x_0 and x_1 are those of the row, so the distance of every point of
// the row to the strut axis is at least the in-plane distance from (dx_0, dx_1) to the axis projected
// onto the (x_0, x_1) plane.  A strut whose bound minus its radius exceeds `cut` (plus a margin far above
// rounding) cannot decide an inside test (cut = 0) or lower a distance below cut (VA: cut = ell/2).
// row(j, &x0, &x1) gives the rows' coordinates; all threads of the block call this (barriers inside).
template <typename RowFn>
__device__ int block_candidates(const StrutPrep* sp, int ns, const Cell& cell, int nrows, RowFn row, double cut,
                                int* cand, int* wave_cnt) {
#pragma clang fp contract(off)
  bool keep = false;
  const int k = threadIdx.x;
  if (k < ns) {
    const StrutPrep& q = sp[k];
    const double h0 = q.half[0], h1 = q.half[1];
    const double hh2 = h0 * h0 + h1 * h1;
    const double margin = 1e-9 * (cell.L[0] + cell.L[1] + cell.L[2]);
    for (int j = 0; j < nrows && !keep; ++j) {
      double x0, x1;
      row(j, &x0, &x1);
      double d0 = x0 - q.mid[0], d1 = x1 - q.mid[1];
      d0 -= cell.L[0] * floor(d0 / cell.L[0] + 0.5);
      d1 -= cell.L[1] * floor(d1 / cell.L[1] + 0.5);
      double t = hh2 > 0.0 ? (d0 * h0 + d1 * h1) / hh2 : 0.0;
      t = t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t);
      const double e0 = d0 - t * h0, e1 = d1 - t * h1;
      if (sqrt(e0 * e0 + e1 * e1) - q.r <= cut + margin) keep = true;
    }
  }
  const unsigned long long bal = __ballot(keep);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wave_cnt[wv] = __popcll(bal);
  __syncthreads();
  int off = 0, n = 0;
  for (int u = 0; u < (int)(blockDim.x >> 6); ++u) {
    if (u < wv) off += wave_cnt[u];
    n += wave_cnt[u];
  }
  if (keep) cand[off + __popcll(bal & ((1ull << lane) - 1ull))] = k;
  __syncthreads();
  return n;
}

// ------------------------------------------------------------------ Voigt maps on the coarse grid
// A block takes blockDim consecutive voxels at a time; their struts are culled over the rows (and, for
// VFG, the sub-rows) they span, when those are few enough for the test to be cheap.
__global__ __launch_bounds__(kThreads) void k_phase_map(const rve_strut* __restrict__ struts, int ns, Cell cell,
                                                        int n0, int n1, int n2, int kind, int sub, double ell,
                                                        double* __restrict__ phi, float* __restrict__ phi32) {
#pragma clang fp contract(off)
  __shared__ StrutPrep sp[RVE_GEOMETRY_MAX_STRUTS];
  __shared__ int cand[RVE_GEOMETRY_MAX_STRUTS];
  __shared__ int wave_cnt[kThreads / 64];
  load_struts(struts, ns, cell.L, sp);
  __syncthreads();
  const long long nv = (long long)n0 * n1 * n2;
  const double cut = kind == RVE_MAP_VA ? 0.5 * ell : 0.0;
  const int sub2 = sub * sub;
  for (long long v0 = (long long)blockIdx.x * blockDim.x; v0 < nv; v0 += (long long)gridDim.x * blockDim.x) {
    const long long ra = v0 / n2, rb = std::min(nv - 1, v0 + (long long)blockDim.x - 1) / n2;
    const long long nrows = (rb - ra + 1) * sub2;
    int nc = ns;
    const int* list = nullptr;
    if (nrows <= 1024) {
      nc = block_candidates(sp, ns, cell, (int)nrows,
                            [&](int j, double* x0, double* x1) {
                              const long long r = ra + j / sub2;
                              const int s = j % sub2;
                              const int i1 = (int)(r % n1), i0 = (int)(r / n1);
                              *x0 = ((double)(i0 * sub + s / sub) + 0.5) * cell.h[0];
                              *x1 = ((double)(i1 * sub + s % sub) + 0.5) * cell.h[1];
                            },
                            cut, cand, wave_cnt);
      list = cand;
    }
    const long long v = v0 + threadIdx.x;
    if (v < nv) {
      const int i2 = (int)(v % n2);
      const long long r = v / n2;
      const int i1 = (int)(r % n1), i0 = (int)(r / n1);
      auto strut = [&](int c) -> const StrutPrep& { return sp[list ? list[c] : c]; };
      auto is_in = [&](const double x[3]) {
        for (int c = 0; c < nc; ++c)
          if (axis_distance(strut(c), cell.L, x) - strut(c).r <= 0.0) return true;
        return false;
      };
      double val;
      if (kind == RVE_MAP_VFG) {
        int cnt = 0;
        for (int s0 = 0; s0 < sub; ++s0)
          for (int s1 = 0; s1 < sub; ++s1)
            for (int s2 = 0; s2 < sub; ++s2) {
              const double x[3] = {((double)(i0 * sub + s0) + 0.5) * cell.h[0], ((double)(i1 * sub + s1) + 0.5) * cell.h[1],
                                   ((double)(i2 * sub + s2) + 0.5) * cell.h[2]};
              cnt += is_in(x) ? 1 : 0;
            }
        val = (double)cnt / (double)(sub * sub * sub);
      } else {
        const double x[3] = {((double)i0 + 0.5) * cell.h[0], ((double)i1 + 0.5) * cell.h[1], ((double)i2 + 0.5) * cell.h[2]};
        if (kind == RVE_MAP_PV) {
          val = is_in(x) ? 1.0 : 0.0;
        } else {
          double D = INFINITY;
          for (int c = 0; c < nc; ++c) {
            const double d = axis_distance(strut(c), cell.L, x) - strut(c).r;
            if (d < D) D = d;
          }
          val = 0.5 - D / ell;
          val = val < 0.0 ? 0.0 : (val > 1.0 ? 1.0 : val);
        }
      }
      if (phi) phi[v] = val;
      if (phi32) phi32[v] = (float)val;
    }
    __syncthreads();  // the candidate list is rebuilt for the next chunk
  }
}

struct Fine {
  int m0, m1, m2, K;  // fine grid, K = m2/2 + 1
  int ratio, n0, n1, n2;
};

// ------------------------------------------------------------------ G1: source + R2C along axis 2
__global__ __launch_bounds__(kThreads) void k_source_r2c(const rve_strut* __restrict__ struts, int ns, Cell cell,
                                                         const double* __restrict__ source, Fine f, FftPlan P,
                                                         const C* __restrict__ tw, const int* __restrict__ rev, int TP,
                                                         C* __restrict__ spec) {
  extern __shared__ unsigned char smem_raw[];
  StrutPrep* sp = reinterpret_cast<StrutPrep*>(smem_raw);
  C* buf = reinterpret_cast<C*>(smem_raw + (source ? 0 : sizeof(StrutPrep) * ns));
  __shared__ int cand[RVE_GEOMETRY_MAX_STRUTS];
  __shared__ int wave_cnt[kThreads / 64];
  if (!source) load_struts(struts, ns, cell.L, sp);
  __syncthreads();
  const long long rows = (long long)f.m0 * f.m1;
  const long long row0 = (long long)blockIdx.x * 2 * TP;
  const int N = f.m2, K = f.K;
  int ncand = 0;
  if (!source) {
    // Candidate struts of this block's rows.  Along a row only x_2 varies and the nearest-image
    // offsets dx_0, dx_1 to a strut midpoint are fixed, so the distance of every point of the row to
    // the strut axis is at least the in-plane distance from (dx_0, dx_1) to the axis projected onto
    // the (x_0, x_1) plane; a strut whose bound exceeds its radius (with a margin far above rounding)
    // contains no point of the row and cannot change an inside/outside decision.
    bool keep = false;
    const int k = threadIdx.x;
    if (k < ns) {
#pragma clang fp contract(off)
      const StrutPrep& q = sp[k];
      const double h0 = q.half[0], h1 = q.half[1];
      const double hh2 = h0 * h0 + h1 * h1;
      const double margin = 1e-9 * (cell.L[0] + cell.L[1] + cell.L[2]);
      for (int j = 0; j < 2 * TP && !keep; ++j) {
        const long long row = row0 + j;
        if (row >= rows) break;
        const int i0 = (int)(row / f.m1), i1 = (int)(row % f.m1);
        double d0 = ((double)i0 + 0.5) * cell.h[0] - q.mid[0];
        double d1 = ((double)i1 + 0.5) * cell.h[1] - q.mid[1];
        d0 -= cell.L[0] * floor(d0 / cell.L[0] + 0.5);
        d1 -= cell.L[1] * floor(d1 / cell.L[1] + 0.5);
        double t = hh2 > 0.0 ? (d0 * h0 + d1 * h1) / hh2 : 0.0;
        t = t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t);
        const double e0 = d0 - t * h0, e1 = d1 - t * h1;
        if (sqrt(e0 * e0 + e1 * e1) - q.r <= margin) keep = true;
      }
    }
    const unsigned long long bal = __ballot(keep);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wave_cnt[wv] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int u = 0; u < kThreads / 64; ++u) {
      if (u < wv) off += wave_cnt[u];
      ncand += wave_cnt[u];
    }
    if (keep) cand[off + __popcll(bal & ((1ull << lane) - 1ull))] = k;
    __syncthreads();
  }
  auto omega = [&](long long row, int e) -> double {
    const int i0 = (int)(row / f.m1), i1 = (int)(row % f.m1);
    if (source) return source[((long long)(i0 / f.ratio) * f.n1 + i1 / f.ratio) * f.n2 + e / f.ratio];
    const double x[3] = {((double)i0 + 0.5) * cell.h[0], ((double)i1 + 0.5) * cell.h[1], ((double)e + 0.5) * cell.h[2]};
    for (int c = 0; c < ncand; ++c) {
      const StrutPrep& q = sp[cand[c]];
      if (axis_distance(q, cell.L, x) - q.r <= 0.0) return 1.0;
    }
    return 0.0;
  };
  for (int idx = threadIdx.x; idx < TP * N; idx += blockDim.x) {
    const int w = idx / N, e = idx - w * N;
    const long long ra = row0 + 2 * w, rb = ra + 1;
    const double va = ra < rows ? omega(ra, e) : 0.0;
    const double vb = rb < rows ? omega(rb, e) : 0.0;
    buf[rev[e] * TP + w] = mk<double>(va, vb);
  }
  __syncthreads();
  lds_fft<-1>(buf, TP, P, tw);
  // Z = FFT(a + i b): A_k = (Z_k + conj Z_{N-k}) / 2, B_k = (Z_k - conj Z_{N-k}) / (2 i)
  for (int idx = threadIdx.x; idx < TP * K; idx += blockDim.x) {
    const int w = idx / K, k = idx - w * K;
    const long long ra = row0 + 2 * w, rb = ra + 1;
    const C z = buf[k * TP + w];
    const C zc = buf[((N - k) % N) * TP + w];
    if (ra < rows) spec[ra * K + k] = mk<double>(0.5 * (z.re + zc.re), 0.5 * (z.im - zc.im));
    if (rb < rows) spec[rb * K + k] = mk<double>(0.5 * (z.im + zc.im), -0.5 * (z.re - zc.re));
  }
}

// ------------------------------------------------------------------ G2/G3/G4: strided axes
struct Helm {
  double c;      // ell^2 / eps
  double scale;  // 1 / (m0 m1 m2)
  double two_pi_over_L[3];
};

__device__ __forceinline__ double signed_freq(int k, int m) { return (double)(2 * k < m ? k : k - m); }

// axis 1 (pencils (i0, k2), stride K) or axis 0 (pencils q = i1*K + k2, stride m1*K); TW adjacent
// pencils per block.  HELM (axis 0 only): forward, multiply, inverse in one pass.
template <int S, bool HELM>
__global__ __launch_bounds__(kThreads) void k_axis_c2c(C* __restrict__ spec, Fine f, int axis, FftPlan P,
                                                       const C* __restrict__ tw, const int* __restrict__ rev, int TW,
                                                       Helm hm) {
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int N = P.n;
  long long base;
  long long es;
  int valid;
  if (axis == 1) {
    const int k0 = blockIdx.x * TW;
    base = (long long)blockIdx.y * f.m1 * f.K + k0;
    es = f.K;
    valid = min(TW, f.K - k0);
  } else {
    const long long q0 = (long long)blockIdx.x * TW;
    const long long plane = (long long)f.m1 * f.K;
    base = q0;
    es = plane;
    valid = (int)min((long long)TW, plane - q0);
  }
  for (int idx = threadIdx.x; idx < TW * N; idx += blockDim.x) {
    const int e = idx / TW, w = idx - e * TW;
    buf[rev[e] * TW + w] = w < valid ? spec[base + e * es + w] : mk<double>(0.0, 0.0);
  }
  __syncthreads();
  lds_fft<S>(buf, TW, P, tw);
  if (HELM) {
    C v[kStridedSlots];
    const long long q0 = (long long)blockIdx.x * TW;
#pragma unroll
    for (int u = 0; u < kStridedSlots; ++u) {
      const int idx = threadIdx.x + u * kThreads;
      if (idx < TW * N) {
        const int e = idx / TW, w = idx - e * TW;
        const long long q = q0 + w;
        const int i1 = (int)(q / f.K), k2 = (int)(q - (long long)i1 * f.K);
        const double x0 = hm.two_pi_over_L[0] * signed_freq(e, f.m0);
        const double x1 = hm.two_pi_over_L[1] * signed_freq(i1, f.m1);
        const double x2 = hm.two_pi_over_L[2] * (double)k2;
        const double g = hm.scale / (1.0 + hm.c * (x0 * x0 + x1 * x1 + x2 * x2));
        const C z = buf[e * TW + w];
        v[u] = mk<double>(z.re * g, z.im * g);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kStridedSlots; ++u) {
      const int idx = threadIdx.x + u * kThreads;
      if (idx < TW * N) {
        const int e = idx / TW, w = idx - e * TW;
        buf[rev[e] * TW + w] = v[u];
      }
    }
    __syncthreads();
    lds_fft<1>(buf, TW, P, tw);
  }
  for (int idx = threadIdx.x; idx < TW * N; idx += blockDim.x) {
    const int e = idx / TW, w = idx - e * TW;
    if (w < valid) spec[base + e * es + w] = buf[e * TW + w];
  }
}

// ------------------------------------------------------------------ G5: C2R along axis 2 + coarse average
__global__ __launch_bounds__(kThreads) void k_c2r_coarsen(const C* __restrict__ spec, Fine f, FftPlan P,
                                                          const C* __restrict__ tw, const int* __restrict__ rev, int TP,
                                                          double thr, double* __restrict__ phi,
                                                          float* __restrict__ phi32, double* __restrict__ raw) {
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int c1 = blockIdx.x, c0 = blockIdx.y;
  const int r = f.ratio, rr = r * r, npairs = (rr + 1) / 2;
  const int N = f.m2, K = f.K;
  auto row_of = [&](int j) -> long long {  // j-th fine row of this coarse row
    return (long long)(c0 * r + j / r) * f.m1 + (c1 * r + j % r);
  };
  double acc[kRowSlots];
#pragma unroll
  for (int u = 0; u < kRowSlots; ++u) acc[u] = 0.0;
  for (int p0 = 0; p0 < npairs; p0 += TP) {
    const int np = min(TP, npairs - p0);
    for (int idx = threadIdx.x; idx < TP * K; idx += blockDim.x) {
      const int w = idx / K, k = idx - w * K;
      C A = mk<double>(0.0, 0.0), B = mk<double>(0.0, 0.0);
      if (w < np) {
        const int ja = 2 * (p0 + w), jb = ja + 1;
        A = spec[row_of(ja) * K + k];
        if (jb < rr) B = spec[row_of(jb) * K + k];
      }
      if (k == 0 || 2 * k == N) {  // a real row's DC and Nyquist terms are real
        A.im = 0.0;
        B.im = 0.0;
      }
      buf[rev[k] * TP + w] = mk<double>(A.re - B.im, A.im + B.re);                    // A_k + i B_k
      if (k > 0 && 2 * k < N) buf[rev[N - k] * TP + w] = mk<double>(A.re + B.im, B.re - A.im);  // conj A + i conj B
    }
    __syncthreads();
    lds_fft<1>(buf, TP, P, tw);
#pragma unroll
    for (int u = 0; u < kRowSlots; ++u) {
      const int idx = threadIdx.x + u * kThreads;
      if (idx < TP * N) {
        const int w = idx / N, e = idx - w * N;
        if (w < np) {
          const C z = buf[e * TP + w];
          acc[u] += z.re + z.im;  // row a + row b (zero when the pair has one row)
        }
      }
    }
    __syncthreads();
  }
  double* red = reinterpret_cast<double*>(smem_raw);
#pragma unroll
  for (int u = 0; u < kRowSlots; ++u) {
    const int idx = threadIdx.x + u * kThreads;
    if (idx < TP * N) red[idx] = acc[u];
  }
  __syncthreads();
  const double inv = 1.0 / ((double)r * r * r);
  for (int c2 = threadIdx.x; c2 < f.n2; c2 += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < TP; ++w)
      for (int t = 0; t < r; ++t) s += red[w * N + c2 * r + t];
    const double v = s * inv;
    const long long o = ((long long)c0 * f.n1 + c1) * f.n2 + c2;
    const double vt = v < thr ? 0.0 : v;
    if (raw) raw[o] = v;
    if (phi) phi[o] = vt;
    if (phi32) phi32[o] = (float)vt;
  }
}

// ------------------------------------------------------------------ host side
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static bool finite3(const double* L) {
  for (int p = 0; p < 3; ++p)
    if (!std::isfinite(L[p]) || !(L[p] > 0.0)) return false;
  return true;
}

static rve_status hip_fail(hipError_t e, const char* what) {
  char text[256];
  snprintf(text, sizeof(text), "%s (%d) in %s (rve_geometry.hip)", hipGetErrorString(e), (int)e, what);
  rve::set_last_error(text);
  return RVE_EDEVICE;
}

struct FieldLayout {
  Fine f;
  FftPlan P[3];
  size_t spec_off, tab_off[3], rev_off[3], total;
};

static rve_status field_layout(const int32_t n[3], int32_t ratio, FieldLayout& lay) {
  if (!n || ratio < 1) return RVE_EINVAL;
  long long m[3];
  for (int p = 0; p < 3; ++p) {
    if (n[p] < 1) return RVE_EINVAL;
    m[p] = (long long)ratio * n[p];
    if (m[p] > RVE_GEOMETRY_MAX_FINE) return RVE_EUNSUPPORTED_SIZE;
    if (!make_plan((int)m[p], lay.P[p])) return RVE_EUNSUPPORTED_SIZE;
  }
  if ((long long)n[0] * n[1] * n[2] >= (1LL << 31)) return RVE_EINVAL;
  Fine& f = lay.f;
  f.m0 = (int)m[0];
  f.m1 = (int)m[1];
  f.m2 = (int)m[2];
  f.K = f.m2 / 2 + 1;
  f.ratio = ratio;
  f.n0 = n[0];
  f.n1 = n[1];
  f.n2 = n[2];
  size_t off = 0;
  lay.spec_off = off;
  off += align256((size_t)f.m0 * f.m1 * f.K * sizeof(C));
  for (int p = 0; p < 3; ++p) {
    lay.tab_off[p] = off;
    off += align256((size_t)m[p] * sizeof(C));
    lay.rev_off[p] = off;
    off += align256((size_t)m[p] * sizeof(int));
  }
  lay.total = off;
  return RVE_OK;
}

}  // namespace rvg

extern "C" {

rve_status rve_phase_map(const int32_t n[3], const double L[3], const rve_strut* struts, int32_t n_struts,
                         int32_t kind, int32_t sub, double ell, double* phi, float* phi_f32, void* hip_stream) {
  using namespace rvg;
  if (!n || !L || !struts || (!phi && !phi_f32)) return RVE_EINVAL;
  if (n_struts < 1 || n_struts > RVE_GEOMETRY_MAX_STRUTS) return RVE_EINVAL;
  if (kind != RVE_MAP_PV && kind != RVE_MAP_VFG && kind != RVE_MAP_VA) return RVE_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (n[p] < 1) return RVE_EINVAL;
  if ((long long)n[0] * n[1] * n[2] >= (1LL << 31)) return RVE_EINVAL;
  if (!finite3(L)) return RVE_EINVAL;
  if (kind == RVE_MAP_VFG && (sub < 1 || sub > 64)) return RVE_EINVAL;
  if (kind != RVE_MAP_VFG) sub = 1;
  if (kind == RVE_MAP_VA && !(std::isfinite(ell) && ell > 0.0)) return RVE_EINVAL;
  Cell cell;
  for (int p = 0; p < 3; ++p) {
    cell.L[p] = L[p];
    cell.h[p] = L[p] / (double)((long long)sub * n[p]);
  }
  const long long nv = (long long)n[0] * n[1] * n[2];
  const int blocks = (int)std::min<long long>((nv + kThreads - 1) / kThreads, 1LL << 20);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  rve::geo_prof_begin(5, s);
  hipLaunchKernelGGL(k_phase_map, dim3(blocks), dim3(kThreads), 0, s, struts, n_struts, cell, n[0], n[1], n[2], kind,
                     sub, ell, phi, phi_f32);
  rve::geo_prof_end(s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_phase_map launch");
  rve::geo_prof_flush();
  return RVE_OK;
}

size_t rve_phase_field_workspace_bytes(const int32_t n[3], int32_t ratio) {
  rvg::FieldLayout lay;
  if (rvg::field_layout(n, ratio, lay) != RVE_OK) return 0;
  return lay.total;
}

rve_status rve_phase_field(const int32_t n[3], const double L[3], const rve_strut* struts, int32_t n_struts,
                           int32_t ratio, double ell, double eps, double threshold, const double* source,
                           double* phi, float* phi_f32, double* phi_raw, void* workspace, size_t workspace_bytes,
                           void* hip_stream) {
  using namespace rvg;
  if (!n || !L || !workspace || (!phi && !phi_f32 && !phi_raw)) return RVE_EINVAL;
  if (!source && (!struts || n_struts < 1 || n_struts > RVE_GEOMETRY_MAX_STRUTS)) return RVE_EINVAL;
  if (!finite3(L)) return RVE_EINVAL;
  if (!(std::isfinite(ell) && ell >= 0.0) || !(std::isfinite(eps) && eps > 0.0) || !std::isfinite(threshold))
    return RVE_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RVE_EINVAL;
  FieldLayout lay;
  const rve_status st = field_layout(n, ratio, lay);
  if (st != RVE_OK) return st;
  if (workspace_bytes < lay.total) return RVE_ENOMEM;
  const Fine& f = lay.f;
  char* ws = static_cast<char*>(workspace);
  C* spec = reinterpret_cast<C*>(ws + lay.spec_off);
  C* tw[3];
  int* rev[3];
  for (int p = 0; p < 3; ++p) {
    tw[p] = reinterpret_cast<C*>(ws + lay.tab_off[p]);
    rev[p] = reinterpret_cast<int*>(ws + lay.rev_off[p]);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e;
  for (int p = 0; p < 3; ++p)
    hipLaunchKernelGGL(k_fft_tables, dim3((lay.P[p].n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, tw[p], rev[p],
                       lay.P[p]);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_fft_tables launch");

  Cell cell;
  for (int p = 0; p < 3; ++p) cell.L[p] = L[p];
  cell.h[0] = L[0] / (double)f.m0;
  cell.h[1] = L[1] / (double)f.m1;
  cell.h[2] = L[2] / (double)f.m2;
  const int ns = source ? 0 : n_struts;

  // G1: two real rows per complex pencil, TP pencils per block
  const long long rows = (long long)f.m0 * f.m1;
  int TP1 = std::max(1, std::min(kRowTile / f.m2, (int)std::min<long long>((rows + 1) / 2, 64)));
  const long long g1 = (rows + 2LL * TP1 - 1) / (2LL * TP1);
  const size_t lds1 = (size_t)ns * sizeof(StrutPrep) + (size_t)TP1 * f.m2 * sizeof(C);
  rve::geo_prof_begin(0, s);
  hipLaunchKernelGGL(k_source_r2c, dim3((unsigned)g1), dim3(kThreads), lds1, s, struts, ns, cell, source, f, lay.P[2],
                     tw[2], rev[2], TP1, spec);
  rve::geo_prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_source_r2c launch");

  // G2: axis 1 forward
  const int TWa1 = std::max(1, std::min(kStridedTile / f.m1, std::min(f.K, 64)));
  const size_t lds_a1 = (size_t)TWa1 * f.m1 * sizeof(C);
  const dim3 grid_a1((f.K + TWa1 - 1) / TWa1, f.m0);
  Helm hm;
  hm.c = ell * ell / eps;
  hm.scale = 1.0 / ((double)f.m0 * f.m1 * f.m2);
  for (int p = 0; p < 3; ++p) hm.two_pi_over_L[p] = 2.0 * M_PI / L[p];
  rve::geo_prof_begin(1, s);
  hipLaunchKernelGGL((k_axis_c2c<-1, false>), grid_a1, dim3(kThreads), lds_a1, s, spec, f, 1, lay.P[1], tw[1], rev[1],
                     TWa1, hm);
  rve::geo_prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_axis_c2c axis 1 launch");

  // G3: axis 0 forward, Helmholtz multiplier, inverse
  const long long plane = (long long)f.m1 * f.K;
  const int TWa0 = std::max(1, std::min(kStridedTile / f.m0, (int)std::min<long long>(plane, 64)));
  const size_t lds_a0 = (size_t)TWa0 * f.m0 * sizeof(C);
  rve::geo_prof_begin(2, s);
  hipLaunchKernelGGL((k_axis_c2c<-1, true>), dim3((unsigned)((plane + TWa0 - 1) / TWa0)), dim3(kThreads), lds_a0, s,
                     spec, f, 0, lay.P[0], tw[0], rev[0], TWa0, hm);
  rve::geo_prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_axis_c2c axis 0 launch");

  // G4: axis 1 inverse
  rve::geo_prof_begin(3, s);
  hipLaunchKernelGGL((k_axis_c2c<1, false>), grid_a1, dim3(kThreads), lds_a1, s, spec, f, 1, lay.P[1], tw[1], rev[1],
                     TWa1, hm);
  rve::geo_prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_axis_c2c axis 1 inverse launch");

  // G5: inverse along axis 2 over the ratio^2 fine rows of each coarse row, averaged and thresholded
  const int npairs = (ratio * ratio + 1) / 2;
  const int TP5 = std::max(1, std::min(kRowTile / f.m2, npairs));
  const size_t lds5 = (size_t)TP5 * f.m2 * sizeof(C);
  rve::geo_prof_begin(4, s);
  hipLaunchKernelGGL(k_c2r_coarsen, dim3(f.n1, f.n0), dim3(kThreads), lds5, s, spec, f, lay.P[2], tw[2], rev[2], TP5,
                     threshold, phi, phi_f32, phi_raw);
  rve::geo_prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_c2r_coarsen launch");
  rve::geo_prof_flush();
  return RVE_OK;
}

}  // extern "C"
