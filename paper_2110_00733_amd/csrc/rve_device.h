// Device building blocks for the gfx950 Galerkin-FFT path: complex arithmetic, compile-time
// twiddles, register-resident small DFTs (radix 2, 3, 4, 5, 8, 16 and products), wave64 reductions.
//
// Transform convention: forward X_k = sum_j x_j exp(-2 pi i jk/N) (unnormalised), inverse with
// exp(+2 pi i jk/N); the 1/N of the inverse 3-D transform is folded into the projection step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rve {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
// Streaming load: the nontemporal hint lets the caches evict the line first.  Used where a pass reads
// an operand for the last time and its lanes cover whole cache lines (a row's lanes read 128 bytes
// together); with four-byte lanes, half a line per row and instruction, the hint slowed the passes.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ cx<T> ld_stream(const cx<T>* p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return mk<T>(v.x, v.y);
}
// Streaming store: the line goes to HBM while the writer runs instead of being written back from the
// caches while the next pass streams its own operands.
template <typename T>
__device__ __forceinline__ void st_stream(cx<T>* p, cx<T> z) {
  using V = T __attribute__((ext_vector_type(2)));
  V v;
  v.x = z.re;
  v.y = z.im;
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}
// Streaming only in FP64 (eight-byte lanes, whole lines), an ordinary load in FP32 (four-byte lanes):
// for the field loads of the axis-2 passes.
template <typename T>
__device__ __forceinline__ T ld_stream_wide(const T* p) {
  if constexpr (sizeof(T) == 8)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T>
__device__ __forceinline__ cx<T> scl(cx<T> a, T s) { return mk<T>(a.re * s, a.im * s); }
// multiply by S*i (S = +-1)
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  return (S > 0) ? mk<T>(-a.im, a.re) : mk<T>(a.im, -a.re);
}

// ------------------------------------------------------------------ compile-time trigonometry
// exp(2 pi i a / b) from a reduced angle in [-pi/4, pi/4] and Taylor series (constexpr, ~1 ulp).
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ce_sin_small(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos_small(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
struct CS {
  double c, s;
};
// (cos, sin) of 2 pi a / b
constexpr CS ce_expi(long a, long b) {
  a %= b;
  if (a < 0) a += b;
  long k = (8 * a + b) / (2 * b);  // round(4a/b): quadrant
  long num = 4 * a - k * b;        // angle = pi num / (2b) in [-pi/4, pi/4]
  double phi = kPi * (double)num / (2.0 * (double)b);
  double c = ce_cos_small(phi), s = ce_sin_small(phi);
  switch (k & 3) {
    case 0: return CS{c, s};
    case 1: return CS{-s, c};
    case 2: return CS{-c, -s};
    default: return CS{s, -c};
  }
}

// twiddle exp(S 2 pi i a / b) as a complex constant
template <typename T, int S>
__device__ __forceinline__ cx<T> ctw(long a, long b) {
  CS t = ce_expi(a, b);
  return mk<T>((T)t.c, (T)(S * t.s));
}

// ------------------------------------------------------------------ small DFTs in registers
// x[0..R) in place, X_k = sum_j x_j exp(S 2 pi i jk/R), output in natural order.
template <int R, int S, typename T>
struct DFT;

template <int S, typename T>
struct DFT<1, S, T> {
  __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int S, typename T>
struct DFT<2, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};

template <int S, typename T>
struct DFT<3, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    const T h = (T)0.86602540378443864676372317075294;  // sin(2 pi/3)
    cx<T> a = x[0], b = x[1], c = x[2];
    cx<T> t1 = b + c;
    cx<T> t2 = a - scl(t1, (T)0.5);
    cx<T> t3 = mul_si<S>(scl(b - c, h));
    x[0] = a + t1;
    x[1] = t2 + t3;
    x[2] = t2 - t3;
  }
};

template <int S, typename T>
struct DFT<4, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a = x[0], b = x[1], c = x[2], d = x[3];
    cx<T> s0 = a + c, d0 = a - c, s1 = b + d, d1 = mul_si<S>(b - d);
    x[0] = s0 + s1;
    x[1] = d0 + d1;
    x[2] = s0 - s1;
    x[3] = d0 - d1;
  }
};

template <int S, typename T>
struct DFT<5, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    const T c1 = (T)0.30901699437494742410229341718282;   // cos(2pi/5)
    const T c2 = (T)-0.80901699437494742410229341718282;  // cos(4pi/5)
    const T s1 = (T)0.95105651629515357211643933337938;   // sin(2pi/5)
    const T s2 = (T)0.58778525229247312916870595463907;   // sin(4pi/5)
    cx<T> a0 = x[0];
    cx<T> p1 = x[1] + x[4], m1 = x[1] - x[4], p2 = x[2] + x[3], m2 = x[2] - x[3];
    cx<T> r1 = a0 + scl(p1, c1) + scl(p2, c2);
    cx<T> r2 = a0 + scl(p1, c2) + scl(p2, c1);
    cx<T> i1 = mul_si<S>(scl(m1, s1) + scl(m2, s2));
    cx<T> i2 = mul_si<S>(scl(m1, s2) - scl(m2, s1));
    x[0] = a0 + p1 + p2;
    x[1] = r1 + i1;
    x[4] = r1 - i1;
    x[2] = r2 + i2;
    x[3] = r2 - i2;
  }
};

// Composite R = P * M (P the first factor): decimation in time with constant twiddles.
template <int R>
struct FirstFactor {
  static constexpr int value = (R % 4 == 0 && R > 4 && R != 8 && R != 16) ? 4
                               : (R % 2 == 0 && R > 2 && R != 4 && R != 8 && R != 16) ? 2
                               : (R % 3 == 0 && R > 3) ? 3
                               : (R % 5 == 0 && R > 5) ? 5
                                                       : R;
};

template <int R, int S, typename T>
struct DFT {
  static constexpr int P = FirstFactor<R>::value;
  static constexpr int M = R / P;
  static_assert(P * M == R && P < R, "unsupported radix");
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> y[R];
    // sub-sequences x[r + P j], j < M
#pragma unroll
    for (int r = 0; r < P; ++r) {
      cx<T> s[M];
#pragma unroll
      for (int j = 0; j < M; ++j) s[j] = x[r + P * j];
      DFT<M, S, T>::run(s);
#pragma unroll
      for (int k = 0; k < M; ++k) y[r * M + k] = (r == 0 || k == 0) ? s[k] : cmul(s[k], ctw<T, S>(r * k, R));
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
      cx<T> t[P];
#pragma unroll
      for (int r = 0; r < P; ++r) t[r] = y[r * M + k];
      DFT<P, S, T>::run(t);
#pragma unroll
      for (int q = 0; q < P; ++q) x[k + M * q] = t[q];
    }
  }
};

// radix 8 and 16 as split-by-2 over radix 4 / radix 8 with constant twiddles
template <int S, typename T>
struct DFT<8, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    const T r = (T)0.70710678118654752440084436210485;
    cx<T> e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
    DFT<4, S, T>::run(e);
    DFT<4, S, T>::run(o);
    cx<T> o1 = mk<T>(r * (o[1].re - S * o[1].im), r * (o[1].im + S * o[1].re));  // * (1 + S i)/sqrt2
    cx<T> o2 = mul_si<S>(o[2]);
    cx<T> o3 = mk<T>(r * (-o[3].re - S * o[3].im), r * (-o[3].im + S * o[3].re));  // * (-1 + S i)/sqrt2
    x[0] = e[0] + o[0];
    x[4] = e[0] - o[0];
    x[1] = e[1] + o1;
    x[5] = e[1] - o1;
    x[2] = e[2] + o2;
    x[6] = e[2] - o2;
    x[3] = e[3] + o3;
    x[7] = e[3] - o3;
  }
};

template <int S, typename T>
struct DFT<16, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> e[8], o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      e[j] = x[2 * j];
      o[j] = x[2 * j + 1];
    }
    DFT<8, S, T>::run(e);
    DFT<8, S, T>::run(o);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cx<T> t = (k == 0) ? o[0] : cmul(o[k], ctw<T, S>(k, 16));
      x[k] = e[k] + t;
      x[k + 8] = e[k] - t;
    }
  }
};

// ------------------------------------------------------------------ barriers
// Workgroup barrier that orders LDS traffic only: waits for this wave's LDS operations, then
// s_barrier.  Outstanding global loads stay in flight across it (a full __syncthreads() fence would
// also drain them), which lets the pass kernels prefetch the next component during an exchange.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum in a fixed order (wave shuffles, then wave 0 adds the per-wave values in order).
// All threads must call it; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh /* >= 16 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

}  // namespace rve
