// Mixed-radix FFTs in LDS for any 5-smooth length up to 1024 (FP64), shared by the phase-field and
// MoDBFFT kernels.  A runtime plan lists the radices (4, 2, 3, 5); a transform of npen pencils stored
// element-major in LDS (element e of pencil w at buf[e * npen + w]) runs as decimation in time, in place,
// with the input at digit-reversed positions (the table `rev`) and the output in natural order, one
// barrier per stage.  Twiddles exp(-2 pi i k / N) come from a table built on the device.
#pragma once
#include <hip/hip_runtime.h>

#include "rve_device.h"

namespace rvfft {

using rve::cmul;
using rve::cx;
using rve::DFT;
using rve::mk;
using C = cx<double>;

constexpr int kThreads = 256;
constexpr int kMaxStages = 10;
constexpr int kMaxLen = 1024;  // longest transform (LDS tiles and register slots are sized for it)
constexpr int kStridedTile = 4096;  // complex elements of a strided-axis LDS tile (64 KiB)
constexpr int kRowTile = 2048;      // complex elements of a row-pass LDS tile (32 KiB)
constexpr int kStridedSlots = kStridedTile / kThreads;
constexpr int kRowSlots = kRowTile / kThreads;

struct FftPlan {
  int n, stages;
  int radix[kMaxStages];
};

// ------------------------------------------------------------------ LDS transforms
// twiddles exp(-2 pi i k / N) and the digit-reversed position of every input index
static __global__ void k_fft_tables(C* __restrict__ tw, int* __restrict__ rev, FftPlan P) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P.n; k += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)k / (double)P.n, &s, &c);
    tw[k] = mk<double>(c, -s);
    // input index k = sum_q p_q r_q (r_q = N / (R_1...R_q)) goes to sum_q p_q (R_1...R_{q-1})
    int pos = 0, rem = k, lp = 1, rq = P.n;
    for (int q = 0; q < P.stages; ++q) {
      rq /= P.radix[q];
      const int p = rem / rq;
      rem -= p * rq;
      pos += p * lp;
      lp *= P.radix[q];
    }
    rev[k] = pos;
  }
}

template <int R, int S>
__device__ __forceinline__ void butterfly(C* buf, int base, int L, int tw_stride, int w, const C* __restrict__ tw,
                                          int step) {
  C a[R];
#pragma unroll
  for (int p = 0; p < R; ++p) a[p] = buf[(base + p * L) * tw_stride + w];
#pragma unroll
  for (int p = 1; p < R; ++p) {
    C t = tw[p * step];
    if (S > 0) t.im = -t.im;
    a[p] = cmul(a[p], t);
  }
  DFT<R, S, double>::run(a);
#pragma unroll
  for (int m = 0; m < R; ++m) buf[(base + m * L) * tw_stride + w] = a[m];
}

// In-place transform of npen pencils stored element-major (element e of pencil w at buf[e*npen + w]),
// input at digit-reversed positions, output in natural order; S = -1 forward, +1 inverse
// (unnormalised).  Every stage ends with a barrier; the caller orders the loads before it.
template <int S>
__device__ void lds_fft(C* buf, int npen, const FftPlan& P, const C* __restrict__ tw) {
  int L = 1;
  for (int q = 0; q < P.stages; ++q) {
    const int R = P.radix[q];
    const int Lq = L * R, r = P.n / Lq, nb = P.n / R;
    for (int idx = threadIdx.x; idx < nb * npen; idx += blockDim.x) {
      const int w = idx % npen, b = idx / npen;
      const int j = b % L, base = (b / L) * Lq + j;
      switch (R) {
        case 4: butterfly<4, S>(buf, base, L, npen, w, tw, j * r); break;
        case 2: butterfly<2, S>(buf, base, L, npen, w, tw, j * r); break;
        case 3: butterfly<3, S>(buf, base, L, npen, w, tw, j * r); break;
        default: butterfly<5, S>(buf, base, L, npen, w, tw, j * r); break;
      }
    }
    __syncthreads();
    L = Lq;
  }
}

// Complex FFT along a strided axis, in place, for ncomp components (blockIdx.z; cstride elements
// apart): pencils of P.n elements `es` apart; a block takes TW pencils that are adjacent in memory
// (tile_base(blockIdx) + w, w < valid), so every load and store row is contiguous.
// axis 1 of a [n0][n1][K] array: base = blockIdx.y * n1 * K + blockIdx.x * TW, es = K, limit K;
// axis 0: base = blockIdx.x * TW, es = n1 * K, limit n1 * K.
template <int S>
__global__ __launch_bounds__(kThreads) void k_strided_c2c(C* __restrict__ data, long long cstride, int n0, int n1, int K,
                                                          int axis, FftPlan P, const C* __restrict__ tw,
                                                          const int* __restrict__ rev, int TW) {
  extern __shared__ unsigned char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  C* d = data + (long long)blockIdx.z * cstride;
  const int N = P.n;
  long long base, es;
  int valid;
  if (axis == 1) {
    const int k0 = blockIdx.x * TW;
    base = (long long)blockIdx.y * n1 * K + k0;
    es = K;
    valid = min(TW, K - k0);
  } else {
    const long long q0 = (long long)blockIdx.x * TW;
    const long long plane = (long long)n1 * K;
    base = q0;
    es = plane;
    valid = (int)min((long long)TW, plane - q0);
  }
  for (int idx = threadIdx.x; idx < TW * N; idx += blockDim.x) {
    const int e = idx / TW, w = idx - e * TW;
    buf[rev[e] * TW + w] = w < valid ? d[base + e * es + w] : mk<double>(0.0, 0.0);
  }
  __syncthreads();
  lds_fft<S>(buf, TW, P, tw);
  for (int idx = threadIdx.x; idx < TW * N; idx += blockDim.x) {
    const int e = idx / TW, w = idx - e * TW;
    if (w < valid) d[base + e * es + w] = buf[e * TW + w];
  }
}

// ------------------------------------------------------------------ host side
inline bool make_plan(int n, FftPlan& P) {
  if (n < 1 || n > kMaxLen) return false;
  P.n = n;
  P.stages = 0;
  int m = n;
  const int order[4] = {4, 2, 3, 5};
  for (int oi = 0; oi < 4; ++oi) {
    const int R = order[oi];
    while (m % R == 0 && m > 1) {
      if (P.stages == kMaxStages) return false;
      P.radix[P.stages++] = R;
      m /= R;
    }
  }
  for (int q = P.stages; q < kMaxStages; ++q) P.radix[q] = 1;
  return m == 1;
}


// pencils per block of the strided passes: as many as a 64 KiB tile holds, at most 64
inline int strided_tile(int n, long long limit) {
  long long t = kStridedTile / n;
  if (t > 64) t = 64;
  if (t > limit) t = limit;
  return t < 1 ? 1 : (int)t;
}

}  // namespace rvfft
