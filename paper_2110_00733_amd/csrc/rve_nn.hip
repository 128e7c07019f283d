// Learned warm start: kernels of a small 3-D convolutional encoder-decoder for gfx950 (BF16
// weights and activations, FP32 accumulation on MFMA), behind the C ABI in rve_nn.h.
//
// Activations are channels-last, x[b][z][y][x][c], addressed with a channel stride and a channel
// offset so that a layer can read or write one channel slice of a concatenation buffer.
// Convolution weights are W[tap][n][k] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1) for 3x3x3, tap 0 for
// 1x1x1; n output channel, k input channel).  Padding is periodic, as the cell is.
//
// MFMA operand layout of v_mfma_f32_16x16x16bf16_1k (wave64): lane l supplies A[l%16][4(l/16)+e]
// and B[4(l/16)+e][l%16] (e = 0..3) and receives D[4(l/16)+j][l%16] (j = 0..3).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "../../include/rve_nn.h"

namespace rvenn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// FP32 -> BF16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Vol {
  int B, D, H, W;
  __device__ __forceinline__ int nvox() const { return B * D * H * W; }
};
struct Coord {
  int b, z, y, x;
};
__device__ __forceinline__ Coord decompose(const Vol& v, int idx) {
  Coord c;
  c.x = idx % v.W;
  idx /= v.W;
  c.y = idx % v.H;
  idx /= v.H;
  c.z = idx % v.D;
  c.b = idx / v.D;
  return c;
}
// advance a coordinate by `step` voxels in linear order (step >= 0)
__device__ __forceinline__ void advance(const Vol& v, Coord& c, int step) {
  c.x += step;
  while (c.x >= v.W) {
    c.x -= v.W;
    ++c.y;
  }
  while (c.y >= v.H) {
    c.y -= v.H;
    ++c.z;
  }
  while (c.z >= v.D) {
    c.z -= v.D;
    ++c.b;
  }
}
__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
// linear index of the periodic neighbour at offset (dz, dy, dx), |d| <= 1
__device__ __forceinline__ int neighbor(const Vol& v, const Coord& c, int dz, int dy, int dx) {
  return ((c.b * v.D + wrapi(c.z + dz, v.D)) * v.H + wrapi(c.y + dy, v.H)) * v.W + wrapi(c.x + dx, v.W);
}

// ---------------------------------------------------------------------------- convolution
// y[v][n] = act(sum_tap sum_k x[v + off(tap)][k] W[tap][n][k] + bias[n]), optionally multiplied by
// (mask[v][n] > 0).  Grid: ceil(nvox / 64) blocks of 4 waves; a wave computes 16 voxels x 16 NT
// output channels, one MFMA per (tap, 16-channel k step, 16-channel n tile).
template <int NT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, int cin, int xs, int xo,
                                                  const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                                  int cout, void* __restrict__ y, int ys, int yo, int y_f32, int relu,
                                                  const uint16_t* __restrict__ mask, int ms, int mo, Vol vol,
                                                  int ksize) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nv = vol.nvox();
  const int v0 = blockIdx.x * 64 + wave * 16;
  const int row = lane & 15, kq = lane >> 4;
  const int va = v0 + row;  // voxel of this lane's A row
  const bool va_ok = va < nv;
  const Coord ca = decompose(vol, va_ok ? va : 0);
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int taps = ksize == 3 ? 27 : 1;
  const int ksteps = cin / 16;
  for (int tap = 0; tap < taps; ++tap) {
    const int dz = ksize == 3 ? tap / 9 - 1 : 0, dy = ksize == 3 ? (tap / 3) % 3 - 1 : 0,
              dx = ksize == 3 ? tap % 3 - 1 : 0;
    const long long nb = neighbor(vol, ca, dz, dy, dx);
    const uint16_t* xa = x + nb * xs + xo + 4 * kq;
    const uint16_t* wb = w + ((long long)tap * cout + row) * cin + 4 * kq;
    for (int ks = 0; ks < ksteps; ++ks) {
      bf16x4 a = (bf16x4){0, 0, 0, 0};
      if (va_ok) a = __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2*>(xa + ks * 16));
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x4 b =
            __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2*>(wb + (long long)t * 16 * cin + ks * 16));
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // lane holds D[4kq + j][row]: voxel v0 + 4kq + j, channel 16t + row
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const long long vo = v0 + 4 * kq + j;
    if (vo >= nv) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = 16 * t + row;
      float val = acc[t][j] + (bias ? bias[n] : 0.f);
      if (relu) val = fmaxf(val, 0.f);
      if (mask && !(bf2f(mask[vo * ms + mo + n]) > 0.f)) val = 0.f;
      if (y_f32)
        reinterpret_cast<float*>(y)[vo * ys + yo + n] = val;
      else
        reinterpret_cast<uint16_t*>(y)[vo * ys + yo + n] = f2bf(val);
    }
  }
}

// Weight and bias gradient, per chunk of voxels:
//   partial[chunk][tap][n][k] = sum_v dy[v][n] x[v + off(tap)][k],  partial[chunk][taps*cout*cin + n] = sum_v dy[v][n]
// Grid (n_chunks, ceil(tiles / 4)), tiles = (cout/16)(cin/16); a wave owns one (n, k) 16x16 tile for
// all taps (one accumulator per tap), so dy is read once per voxel for every tap.
template <int TAPS>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t* __restrict__ x, int cin, int xs, int xo,
                                                    const uint16_t* __restrict__ dy, int cout, int ds, int dof,
                                                    float* __restrict__ partial, int chunk, Vol vol) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntn = cout / 16, ntk = cin / 16;
  const int tile = blockIdx.y * 4 + wave;
  if (tile >= ntn * ntk) return;
  const int tn = tile / ntk, tk = tile % ntk;
  const int nv = vol.nvox();
  const int c0 = blockIdx.x * chunk, c1 = std::min(nv, c0 + chunk);
  const int row = lane & 15, kq = lane >> 4;
  f32x4 acc[TAPS];
#pragma unroll
  for (int t = 0; t < TAPS; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  // A = dy^T (M = n, K = voxel): A[row][4kq + i] = dy[v + 4kq + i][16 tn + row]
  // B = x_tap (K = voxel, N = k): B[4kq + i][row] = x[v + 4kq + i + off(tap)][16 tk + row]
  Coord cc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cc[i] = decompose(vol, std::min(c0 + 4 * kq + i, nv - 1));
  for (int v = c0; v < c1; v += 16) {
    short av[4];
    bool ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int vv = v + 4 * kq + i;
      ok[i] = vv < c1;
      av[i] = ok[i] ? (short)dy[(long long)vv * ds + dof + 16 * tn + row] : (short)0;
      bsum += bf2f((uint16_t)av[i]);
    }
    const bf16x4 a = (bf16x4){av[0], av[1], av[2], av[3]};
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      const int dz = TAPS == 27 ? t / 9 - 1 : 0, dyy = TAPS == 27 ? (t / 3) % 3 - 1 : 0, dx = TAPS == 27 ? t % 3 - 1 : 0;
      short bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long nb = neighbor(vol, cc[i], dz, dyy, dx);
        bv[i] = ok[i] ? (short)x[nb * xs + xo + 16 * tk + row] : (short)0;
      }
      const bf16x4 b = (bf16x4){bv[0], bv[1], bv[2], bv[3]};
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) advance(vol, cc[i], 16);
  }
  // D[4kq + j][row] = dW[n = 16 tn + 4kq + j][k = 16 tk + row]
  const long long per_chunk = (long long)TAPS * cout * cin + cout;
  float* out = partial + (long long)blockIdx.x * per_chunk;
#pragma unroll
  for (int t = 0; t < TAPS; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[((long long)t * cout + 16 * tn + 4 * kq + j) * cin + 16 * tk + row] = acc[t][j];
  // bias: lanes row, row+16, row+32, row+48 hold partial sums of channel 16 tn + row
  bsum += __shfl_xor(bsum, 16, 64);
  bsum += __shfl_xor(bsum, 32, 64);
  if (tk == 0 && kq == 0) out[(long long)TAPS * cout * cin + 16 * tn + row] = bsum;
}

// dw[i] = sum_c partial[c][i] (fixed order), the trailing cout entries go to db
__global__ void k_sum_chunks(const float* __restrict__ partial, int nchunks, long long nw, int nb,
                             float* __restrict__ dw, float* __restrict__ db) {
  const long long n = nw + nb;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partial[(long long)c * n + i];
    if (i < nw)
      dw[i] = s;
    else if (db)
      db[i - nw] = s;
  }
}

// weights of the data gradient: wd[t][k][n] = w[taps-1-t][n][k] (offset negated, in/out swapped)
__global__ void k_flip_weights(const uint16_t* __restrict__ w, uint16_t* __restrict__ wd, int cin, int cout,
                               int taps) {
  const long long n_all = (long long)taps * cin * cout;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_all; i += (long long)gridDim.x * blockDim.x) {
    const int tp = (int)(i / ((long long)cin * cout));
    const int k = (int)((i / cout) % cin);
    const int n = (int)(i % cout);
    wd[i] = w[((long long)(taps - 1 - tp) * cout + n) * cin + k];
  }
}

// ---------------------------------------------------------------------------- resampling
// 2x average pooling (vin = fine dims)
__global__ void k_pool2(const uint16_t* __restrict__ x, int c, int xs, int xo, uint16_t* __restrict__ y, int ys,
                        int yo, Vol vin) {
  const Vol vo{vin.B, vin.D / 2, vin.H / 2, vin.W / 2};
  const long long n = (long long)vo.nvox() * c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const Coord p = decompose(vo, (int)(i / c));
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const long long src =
          ((long long)(p.b * vin.D + 2 * p.z + (o >> 2)) * vin.H + 2 * p.y + ((o >> 1) & 1)) * vin.W + 2 * p.x + (o & 1);
      s += bf2f(x[src * xs + xo + ch]);
    }
    y[(i / c) * ys + yo + ch] = f2bf(0.125f * s);
  }
}
// backward of pool2, accumulated and masked: dx[child] += (mask[child] > 0) dy[parent] / 8 (vin = fine dims)
__global__ void k_pool2_bwd_acc(const uint16_t* __restrict__ dy, int c, int ds, int dof, uint16_t* __restrict__ dx,
                                int xs, int xo, const uint16_t* __restrict__ mask, int ms, int mo, Vol vin) {
  const long long n = (long long)vin.nvox() * c;
  const Vol vc{vin.B, vin.D / 2, vin.H / 2, vin.W / 2};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const long long v = i / c;
    const Coord f = decompose(vin, (int)v);
    const long long par = ((long long)(f.b * vc.D + f.z / 2) * vc.H + f.y / 2) * vc.W + f.x / 2;
    if (bf2f(mask[v * ms + mo + ch]) > 0.f) {
      const float g = bf2f(dx[v * xs + xo + ch]) + 0.125f * bf2f(dy[par * ds + dof + ch]);
      dx[v * xs + xo + ch] = f2bf(g);
    }
  }
}
// 2x nearest upsampling (vin = coarse dims)
__global__ void k_up2(const uint16_t* __restrict__ x, int c, int xs, int xo, uint16_t* __restrict__ y, int ys, int yo,
                      Vol vin) {
  const Vol vo{vin.B, vin.D * 2, vin.H * 2, vin.W * 2};
  const long long n = (long long)vo.nvox() * c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const Coord f = decompose(vo, (int)(i / c));
    const long long par = ((long long)(f.b * vin.D + f.z / 2) * vin.H + f.y / 2) * vin.W + f.x / 2;
    y[(i / c) * ys + yo + ch] = x[par * xs + xo + ch];
  }
}
// backward of up2: dx[parent] = sum of the 8 children (vin = coarse dims)
__global__ void k_up2_bwd(const uint16_t* __restrict__ dy, int c, int ds, int dof, uint16_t* __restrict__ dx, int xs,
                          int xo, Vol vin) {
  const long long n = (long long)vin.nvox() * c;
  const int W2 = vin.W * 2, H2 = vin.H * 2, D2 = vin.D * 2;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i % c);
    const Coord p = decompose(vin, (int)(i / c));
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const long long src =
          ((long long)(p.b * D2 + 2 * p.z + (o >> 2)) * H2 + 2 * p.y + ((o >> 1) & 1)) * W2 + 2 * p.x + (o & 1);
      s += bf2f(dy[src * ds + dof + ch]);
    }
    dx[(i / c) * xs + xo + ch] = f2bf(s);
  }
}

// ---------------------------------------------------------------------------- data, loss, optimiser
// network input, oc channels (a multiple of 16): [phi, extra_0 .. extra_{ne-1}, 0, ...] with the extra
// fields component-major per sample, extra[(s ne + c) nvs + v]
__global__ void k_pack_input(const float* __restrict__ phi, const float* __restrict__ extra, int ne,
                             uint16_t* __restrict__ out, int oc, long long nvs, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long s = i / nvs, v = i % nvs;
    uint16_t* o = out + i * oc;
    o[0] = f2bf(phi[i]);
    for (int c = 0; c < ne; ++c) o[1 + c] = f2bf(extra[(s * ne + c) * nvs + v]);
    for (int c = 1 + ne; c < oc; ++c) o[c] = 0;
  }
}

// Weighted squared error.  pred: f32 [v][ps]; target: f32 [sample][nch][nvs] (component-major, like the
// solver's fields); weight w = wc + wp phi + wi [0 < phi < 1].  dpred (bf16 [v][dps]) = 2 w (pred - target)
// * inv_norm for channels < nch, 0 above; partials[block] = sum w (pred - target)^2 over the block's voxels.
__global__ void k_loss(const float* __restrict__ pred, int ps, const float* __restrict__ target, int nch,
                       const float* __restrict__ phi, float wc, float wp, float wi, long long nvs, int nsamples,
                       uint16_t* __restrict__ dpred, int dps, double* __restrict__ partials, float inv_norm) {
  __shared__ double red[256];
  const long long n = nvs * nsamples;
  double acc = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long s = i / nvs, v = i % nvs;
    const float ph = phi[i];
    const float w = wc + wp * ph + ((ph > 0.f && ph < 1.f) ? wi : 0.f);
    float part = 0.f;
    for (int c = 0; c < dps; ++c) {
      float g = 0.f;
      if (c < nch) {
        const float d = pred[i * ps + c] - target[(s * nch + c) * nvs + v];
        part += d * d;
        g = 2.f * w * d * inv_norm;
      }
      dpred[i * dps + c] = f2bf(g);
    }
    acc += (double)w * part;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Adam on FP32 master weights, refreshing their BF16 copy
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       uint16_t* __restrict__ pbf, long long n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, float wd) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i] + wd * p[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (pbf) pbf[i] = f2bf(pi);
  }
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = f2bf(a[i]);
}

// coarse phi: mean over f^3 blocks of the fine field (one sample, fine dims n0 n1 n2 = f * coarse)
__global__ void k_restrict(const float* __restrict__ fine, int n0, int n1, int n2, int f, float* __restrict__ coarse) {
  const int c0 = n0 / f, c1 = n1 / f, c2 = n2 / f;
  const long long n = (long long)c0 * c1 * c2;
  const float inv = 1.f / (float)(f * f * f);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % c2), y = (int)((i / c2) % c1), z = (int)(i / ((long long)c1 * c2));
    float s = 0.f;
    for (int a = 0; a < f; ++a)
      for (int b = 0; b < f; ++b)
        for (int c = 0; c < f; ++c) s += fine[((long long)(f * z + a) * n1 + f * y + b) * n2 + f * x + c];
    coarse[i] = s * inv;
  }
  (void)c0;
}

// Fine strain field from the coarse prediction: eps[c][v] = sum_J E[J] P(pred[.][6J + c])(v), with P
// periodic trilinear interpolation at the fine voxel centres (coarse centre of cell i at (i + 1/2) f).
__global__ void k_prolong(const float* __restrict__ pred, int ps, int c0, int c1, int c2, int f,
                          const double* __restrict__ E, float* __restrict__ eps) {
  const int n0 = c0 * f, n1 = c1 * f, n2 = c2 * f;
  const long long n = (long long)n0 * n1 * n2;
  float e[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) e[j] = (float)E[j];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % n2), y = (int)((i / n2) % n1), z = (int)(i / ((long long)n1 * n2));
    // position in coarse cell units
    const float pz = ((float)z + 0.5f) / (float)f - 0.5f, py = ((float)y + 0.5f) / (float)f - 0.5f,
                px = ((float)x + 0.5f) / (float)f - 0.5f;
    const float fz = floorf(pz), fy = floorf(py), fx = floorf(px);
    const float tz = pz - fz, ty = py - fy, tx = px - fx;
    const int iz = (int)fz, iy = (int)fy, ix = (int)fx;
    float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int o = 0; o < 8; ++o) {
      const int az = (o >> 2) & 1, ay = (o >> 1) & 1, ax = o & 1;
      const float wgt = (az ? tz : 1.f - tz) * (ay ? ty : 1.f - ty) * (ax ? tx : 1.f - tx);
      const int zz = (iz + az + c0) % c0, yy = (iy + ay + c1) % c1, xx = (ix + ax + c2) % c2;
      const float* p = pred + ((long long)(zz * c1 + yy) * c2 + xx) * ps;
#pragma unroll
      for (int J = 0; J < 6; ++J) {
        if (e[J] == 0.f) continue;
        const float s = wgt * e[J];
#pragma unroll
        for (int c = 0; c < 6; ++c) out[c] += s * p[6 * J + c];
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) eps[(long long)c * n + i] = out[c];
  }
}

}  // namespace rvenn

using namespace rvenn;

namespace {

int grid_for(long long n) { return (int)std::max(1LL, std::min<long long>((n + 255) / 256, 65535LL * 4)); }

bool dims_ok(const int32_t* d) {
  if (!d) return false;
  long long n = 1;
  for (int i = 0; i < 4; ++i) {
    if (d[i] < 1) return false;
    n *= d[i];
  }
  return n < (1LL << 31);
}

// voxels per wgrad chunk: at least 256, enough chunks that chunks x tiles fill the chip
int wgrad_chunk(int cin, int cout, long long nv) {
  const long long tiles = (long long)(cin / 16) * (cout / 16);
  long long ch = (nv * tiles + 4095) / 4096;
  ch = std::max<long long>(256, (ch + 15) / 16 * 16);
  return (int)std::min<long long>(ch, std::max<long long>(256, (nv + 15) / 16 * 16));
}

rve_status launch_status() { return hipGetLastError() == hipSuccess ? RVE_OK : RVE_EDEVICE; }

}  // namespace

extern "C" {

rve_status rve_nn_conv3d(const void* x, int32_t cin, int32_t x_stride, int32_t x_off, const void* w, const float* bias,
                         int32_t cout, void* y, int32_t y_stride, int32_t y_off, int32_t y_f32, int32_t relu,
                         const void* mask, int32_t m_stride, int32_t m_off, const int32_t* dims4, int32_t ksize,
                         void* hip_stream) {
  if (!x || !w || !y || !dims_ok(dims4) || (ksize != 1 && ksize != 3)) return RVE_EINVAL;
  if (cin < 16 || cin % 16 || cout < 16 || cout % 16 || cout > 256) return RVE_EINVAL;
  if (x_off < 0 || y_off < 0 || m_off < 0 || x_stride < x_off + cin || y_stride < y_off + cout ||
      (mask && m_stride < m_off + cout))
    return RVE_EINVAL;
  if (x_stride % 4 || x_off % 4) return RVE_EINVAL;  // 8-byte operand loads
  const Vol v{dims4[0], dims4[1], dims4[2], dims4[3]};
  const long long nv = (long long)v.B * v.D * v.H * v.W;
  const dim3 grid((unsigned)((nv + 63) / 64));
  hipStream_t s = (hipStream_t)hip_stream;
  const uint16_t* xb = (const uint16_t*)x;
  const uint16_t* wb = (const uint16_t*)w;
  const uint16_t* mb = (const uint16_t*)mask;
  switch (cout / 16) {
#define RVE_CONV_CASE(NT_)                                                                                       \
  case NT_:                                                                                                      \
    hipLaunchKernelGGL(k_conv_fwd<NT_>, grid, dim3(256), 0, s, xb, cin, x_stride, x_off, wb, bias, cout, y,      \
                       y_stride, y_off, y_f32, relu, mb, m_stride, m_off, v, ksize);                              \
    break;
    RVE_CONV_CASE(1)
    RVE_CONV_CASE(2)
    RVE_CONV_CASE(3)
    RVE_CONV_CASE(4)
    RVE_CONV_CASE(6)
    RVE_CONV_CASE(8)
    RVE_CONV_CASE(12)
    RVE_CONV_CASE(16)
#undef RVE_CONV_CASE
    default:
      return RVE_EINVAL;
  }
  return launch_status();
}

size_t rve_nn_wgrad_workspace_bytes(int32_t cin, int32_t cout, const int32_t* dims4, int32_t ksize) {
  if (!dims_ok(dims4) || cin < 16 || cout < 16 || (ksize != 1 && ksize != 3)) return 0;
  const long long nv = (long long)dims4[0] * dims4[1] * dims4[2] * dims4[3];
  const int chunk = wgrad_chunk(cin, cout, nv);
  const long long nch = (nv + chunk - 1) / chunk;
  return (size_t)(nch * ((ksize == 3 ? 27LL : 1LL) * cin * cout + cout) * (long long)sizeof(float));
}

rve_status rve_nn_conv3d_wgrad(const void* x, int32_t cin, int32_t x_stride, int32_t x_off, const void* dy,
                               int32_t cout, int32_t dy_stride, int32_t dy_off, float* dw, float* db,
                               const int32_t* dims4, int32_t ksize, void* workspace, size_t workspace_bytes,
                               void* hip_stream) {
  if (!x || !dy || !dw || !dims_ok(dims4) || (ksize != 1 && ksize != 3)) return RVE_EINVAL;
  if (cin < 16 || cin % 16 || cout < 16 || cout % 16) return RVE_EINVAL;
  if (x_off < 0 || dy_off < 0 || x_stride < x_off + cin || dy_stride < dy_off + cout) return RVE_EINVAL;
  if (!workspace || workspace_bytes < rve_nn_wgrad_workspace_bytes(cin, cout, dims4, ksize)) return RVE_ENOMEM;
  const Vol v{dims4[0], dims4[1], dims4[2], dims4[3]};
  const long long nv = (long long)v.B * v.D * v.H * v.W;
  const int chunk = wgrad_chunk(cin, cout, nv);
  const int nch = (int)((nv + chunk - 1) / chunk);
  const int tiles = (cout / 16) * (cin / 16);
  hipStream_t s = (hipStream_t)hip_stream;
  float* part = (float*)workspace;
  const dim3 grid(nch, (tiles + 3) / 4);
  if (ksize == 3)
    hipLaunchKernelGGL(k_conv_wgrad<27>, grid, dim3(256), 0, s, (const uint16_t*)x, cin, x_stride, x_off,
                       (const uint16_t*)dy, cout, dy_stride, dy_off, part, chunk, v);
  else
    hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, s, (const uint16_t*)x, cin, x_stride, x_off,
                       (const uint16_t*)dy, cout, dy_stride, dy_off, part, chunk, v);
  const long long nw = (ksize == 3 ? 27LL : 1LL) * cin * cout;
  hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(nw + cout)), dim3(256), 0, s, part, nch, nw, cout, dw, db);
  return launch_status();
}

rve_status rve_nn_flip_weights(const void* w, void* wd, int32_t cin, int32_t cout, int32_t ksize, void* hip_stream) {
  if (!w || !wd || cin < 1 || cout < 1 || (ksize != 1 && ksize != 3)) return RVE_EINVAL;
  const int taps = ksize == 3 ? 27 : 1;
  const long long n = (long long)taps * cin * cout;
  hipLaunchKernelGGL(k_flip_weights, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, (const uint16_t*)w,
                     (uint16_t*)wd, cin, cout, taps);
  return launch_status();
}

rve_status rve_nn_resample(int32_t op, const void* x, int32_t c, int32_t x_stride, int32_t x_off, void* y,
                           int32_t y_stride, int32_t y_off, const void* mask, int32_t m_stride, int32_t m_off,
                           const int32_t* dims4, void* hip_stream) {
  if (!x || !y || !dims_ok(dims4) || c < 1 || x_off < 0 || y_off < 0 || x_stride < x_off + c || y_stride < y_off + c)
    return RVE_EINVAL;
  const Vol v{dims4[0], dims4[1], dims4[2], dims4[3]};
  const bool fine = (op == RVE_NN_POOL2 || op == RVE_NN_POOL2_BWD_ACC);
  if (fine && (v.D % 2 || v.H % 2 || v.W % 2)) return RVE_EINVAL;
  if (!fine && (long long)v.B * v.D * v.H * v.W * 8 >= (1LL << 31)) return RVE_EINVAL;
  if (op == RVE_NN_POOL2_BWD_ACC && (!mask || m_off < 0 || m_stride < m_off + c)) return RVE_EINVAL;
  const long long nv = (long long)v.B * v.D * v.H * v.W;
  hipStream_t s = (hipStream_t)hip_stream;
  const uint16_t* xb = (const uint16_t*)x;
  uint16_t* yb = (uint16_t*)y;
  switch (op) {
    case RVE_NN_POOL2:
      hipLaunchKernelGGL(k_pool2, dim3(grid_for(nv / 8 * c)), dim3(256), 0, s, xb, c, x_stride, x_off, yb, y_stride,
                         y_off, v);
      break;
    case RVE_NN_POOL2_BWD_ACC:
      hipLaunchKernelGGL(k_pool2_bwd_acc, dim3(grid_for(nv * c)), dim3(256), 0, s, xb, c, x_stride, x_off, yb,
                         y_stride, y_off, (const uint16_t*)mask, m_stride, m_off, v);
      break;
    case RVE_NN_UP2:
      hipLaunchKernelGGL(k_up2, dim3(grid_for(nv * 8 * c)), dim3(256), 0, s, xb, c, x_stride, x_off, yb, y_stride,
                         y_off, v);
      break;
    case RVE_NN_UP2_BWD:
      hipLaunchKernelGGL(k_up2_bwd, dim3(grid_for(nv * c)), dim3(256), 0, s, xb, c, x_stride, x_off, yb, y_stride,
                         y_off, v);
      break;
    default:
      return RVE_EINVAL;
  }
  return launch_status();
}

rve_status rve_nn_pack_input(const float* phi, const float* extra, int32_t n_extra, void* out, int32_t out_channels,
                             int64_t nvox_per_sample, int32_t n_samples, void* hip_stream) {
  if (!phi || !out || nvox_per_sample < 1 || n_samples < 1 || n_extra < 0 || (n_extra > 0 && !extra) ||
      out_channels < 16 || out_channels % 16 || out_channels < 1 + n_extra)
    return RVE_EINVAL;
  const long long n = (long long)nvox_per_sample * n_samples;
  hipLaunchKernelGGL(k_pack_input, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, phi, extra, n_extra,
                     (uint16_t*)out, out_channels, (long long)nvox_per_sample, n);
  return launch_status();
}

rve_status rve_nn_loss(const float* pred, int32_t pred_stride, const float* target, int32_t n_channels,
                       const float* phi, const float* weight3, int64_t nvox_per_sample, int32_t n_samples,
                       float inv_norm, void* dpred, int32_t dpred_stride, double* partials, int32_t n_partials,
                       void* hip_stream) {
  if (!pred || !target || !phi || !weight3 || !dpred || !partials || n_partials < 1 || n_partials > 65535 || n_channels < 1 ||
      pred_stride < n_channels || dpred_stride < n_channels || nvox_per_sample < 1 || n_samples < 1)
    return RVE_EINVAL;
  hipLaunchKernelGGL(k_loss, dim3(n_partials), dim3(256), 0, (hipStream_t)hip_stream, pred, pred_stride, target,
                     n_channels, phi, weight3[0], weight3[1], weight3[2], (long long)nvox_per_sample, n_samples, (uint16_t*)dpred,
                     dpred_stride, partials, inv_norm);
  return launch_status();
}

rve_status rve_nn_adam(float* p, const float* g, float* m, float* v, void* p_bf16, int64_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step, float weight_decay, void* hip_stream) {
  if (!p || !g || !m || !v || n < 1 || step < 1) return RVE_EINVAL;
  const float bc1 = 1.f - std::pow(beta1, (float)step), bc2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, p, g, m, v, (uint16_t*)p_bf16,
                     (long long)n, lr, beta1, beta2, eps, bc1, bc2, weight_decay);
  return launch_status();
}

rve_status rve_nn_to_bf16(const float* a, void* b, int64_t n, void* hip_stream) {
  if (!a || !b || n < 1) return RVE_EINVAL;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, a, (uint16_t*)b,
                     (long long)n);
  return launch_status();
}

rve_status rve_nn_restrict(const float* fine, const int32_t* n3, int32_t factor, float* coarse, void* hip_stream) {
  if (!fine || !coarse || !n3 || factor < 1) return RVE_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (n3[i] < factor || n3[i] % factor) return RVE_EINVAL;
  const long long n = (long long)(n3[0] / factor) * (n3[1] / factor) * (n3[2] / factor);
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, fine, n3[0], n3[1], n3[2],
                     factor, coarse);
  return launch_status();
}

rve_status rve_nn_prolong(const float* pred, int32_t pred_stride, const int32_t* coarse3, int32_t factor,
                          const double* macro_strain_dev, float* eps, void* hip_stream) {
  if (!pred || !eps || !coarse3 || !macro_strain_dev || factor < 1 || pred_stride < 36) return RVE_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (coarse3[i] < 1) return RVE_EINVAL;
  const long long n = (long long)coarse3[0] * coarse3[1] * coarse3[2] * factor * factor * factor;
  if (n >= (1LL << 31)) return RVE_EINVAL;
  hipLaunchKernelGGL(k_prolong, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, pred, pred_stride,
                     coarse3[0], coarse3[1], coarse3[2], factor, macro_strain_dev, eps);
  return launch_status();
}

}  // extern "C"
