// Streaming vector and Krylov scalar kernels of the solver driver (rve_solver.hip): frequency tables,
// fills and linear combinations, FP64 partial sums, the MINRES start / alpha / Givens steps, the U2
// direction + solution update, refinement bookkeeping, post-processing and the phase-map check.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/rve.h"
#include "rve_kernels.h"

namespace rve {

// ============================================================================ small kernels
constexpr int kRedBlocks = 2048;  // blocks per case for streaming vector kernels (and their partials)
constexpr int kThreads = 256;

// Frequency and twiddle tables per axis:
//   tw[m] = exp(-2 pi i m / N)                                 (transform twiddles)
//   rotated scheme:    s[m] = sin(q/2)/h, c[m] = cos(q/2)       (eq. freqrot, real direction)
//   continuous scheme: s[m] = q/h,        c[m] = 1               (eq. freq)
//   q = 2 pi k/N, k = m for m <= (N-1)/2 else m - N; at a Nyquist index c = 0 exactly, and with
//   the zero-all Nyquist reading s = 0 too, so the projection vanishes there.
template <typename T>
__global__ void k_tables(cx<T>* tw, T* s, T* c, int N, double h, int scheme, int nyq_zero_all) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double sn, cs;
  sincospi(-2.0 * (double)m / (double)N, &sn, &cs);
  tw[m] = mk<T>((T)cs, (T)sn);
  const int k = (m <= (N - 1) / 2) ? m : m - N;
  const bool nyq = (N % 2 == 0) && (2 * m == N);
  double sh, ch;
  sincospi((double)k / (double)N, &sh, &ch);  // half angle q/2 = pi k / N
  double sv, cv;
  if (scheme == RVE_SCHEME_CONTINUOUS) {
    sv = 2.0 * kPi * (double)k / (double)N / h;
    cv = 1.0;
  } else {
    sv = sh / h;
    cv = ch;
  }
  if (nyq) {
    cv = 0.0;
    // the continuous scheme always zeroes Nyquist frequencies (otherwise the projection would not
    // be even in k and the real-to-complex symmetry of the spectrum would break)
    if (nyq_zero_all || scheme == RVE_SCHEME_CONTINUOUS) sv = 0.0;
  }
  s[m] = (T)sv;
  c[m] = (T)cv;
}

template <typename T>
__global__ void k_fill_const(T* x, const double* E /* [nc][6] */, long long nvox) {
  const int cs = blockIdx.y;
  T* xc = x + (long long)cs * 6 * nvox;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 6 * nvox; i += (long long)gridDim.x * blockDim.x)
    xc[i] = (T)E[cs * 6 + i / nvox];
}

template <typename T>
__global__ void k_zero(T* x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = (T)0;
}

// out = alpha * a + beta * b (per case), partial sums of out^2
template <typename Ta, typename To>
__global__ void k_lincomb(To* out, const Ta* a, double alpha, const double* b, double beta, long long n6,
                          double* partials) {
  __shared__ double red[16];
  const int cs = blockIdx.y;
  const long long off = (long long)cs * n6;
  double acc = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long long)gridDim.x * blockDim.x) {
    double v = alpha * (double)a[off + i] + (b ? beta * b[off + i] : 0.0);
    To o = (To)v;
    out[off + i] = o;
    acc += (double)o * (double)o;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0 && partials) partials[(long long)cs * gridDim.x + blockIdx.x] = s;
}

// Right-hand side of eq. (gallin) under mixed control: out = -a + sconst[cs][component] (the macroscopic
// stress on the stress-controlled components, zero on the others), per-block partial sums of out^2.
__global__ void k_rhs(double* out, const double* a, const double* sconst, long long nvox, double* partials) {
  __shared__ double red[16];
  const int cs = blockIdx.y;
  const long long n6 = 6 * nvox;
  const long long off = (long long)cs * n6;
  double acc = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long long)gridDim.x * blockDim.x) {
    const double v = -a[off + i] + sconst[cs * 6 + i / nvox];
    out[off + i] = v;
    acc += v * v;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long long)cs * gridDim.x + blockIdx.x] = s;
}

// Per-block partial sums of each component of an FP64 field (its volume average after the fixed-order
// sum of the partials).  Grid (blocks, nc); partials [nc][6][blocks].
__global__ void k_field_sums(const double* x64, long long nvox, double* partials) {
  __shared__ double red[16];
  const int cs = blockIdx.y;
  const long long off = (long long)cs * 6 * nvox;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += x64[off + c * nvox + v];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double s = block_sum(acc[c], red);
    if (threadIdx.x == 0) partials[((long long)cs * 6 + c) * gridDim.x + blockIdx.x] = s;
  }
}

// x64 += (double) d  (per case, only where mask[cs] != 0)
template <typename Td>
__global__ void k_accum(double* x64, const Td* d, long long n6, const int* active) {
  const int cs = blockIdx.y;
  if (active && !active[cs]) return;
  const long long off = (long long)cs * n6;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long long)gridDim.x * blockDim.x)
    x64[off + i] += (double)d[off + i];
}

// deterministic per-case sum of partials[cs][0..np) -> out[cs * ostride]
__global__ void k_sum_partials(const double* partials, int np, double* out, int ostride, int take_sqrt) {
  __shared__ double red[16];
  const int cs = blockIdx.x;
  const double s = sum_partials(partials + (long long)cs * np, np, red);
  if (threadIdx.x == 0) out[(long long)cs * ostride] = take_sqrt ? sqrt(s) : s;
}

// ---------------------------------------------------------------------------- MINRES scalars
// Per-case bookkeeping of the whole solve.
struct CaseInfo {
  double bnorm;       // ||b||
  double rnorm;       // ||b - A x64|| (last true residual)
  int active;         // this case still needs an inner sweep
  int iters;          // MINRES iterations summed over sweeps
  int status;         // worst inner status
  int warm_rejected;  // the warm start was replaced by zero
  double r0;          // ||b - A x0|| of the start (before a rejected warm start is dropped)
};

// Start an inner MINRES on A d = r with u_1 = r (partials hold ||u_1||^2).
__global__ void k_minres_init(MinresState* st, const double* partials, int np, CaseInfo* ci, double tol,
                              double safety, double inner_floor, int max_iter) {
  __shared__ double red[16];
  const int cs = blockIdx.x;
  const double s = sum_partials(partials + (long long)cs * np, np, red);
  if (threadIdx.x == 0) {
    MinresState& S = st[cs];
    const double beta = sqrt(s);
    S.beta = beta;
    S.ib = beta > 0 ? 1.0 / beta : 0.0;
    S.ib_prev = 0.0;
    S.alpha = 0.0;
    S.c1 = S.c2 = 1.0;
    S.s1 = S.s2 = 0.0;
    S.phibar = beta;
    S.tol_abs = fmax(safety * tol * ci[cs].bnorm, inner_floor * beta);
    S.cu_v = S.cu_vp = S.cd_u = S.cd_d1 = S.cd_d2 = S.cx = S.cx_prev = S.cx_pp = 0.0;
    S.xmode = 0;
    S.pending = 0;
    S.iter = 0;
    S.max_iter = max_iter - ci[cs].iters;
    S.status = 0;
    S.finish = (!ci[cs].active || beta <= S.tol_abs || S.max_iter <= 0) ? 1 : 0;
    S.done = 0;
  }
}

// 16-byte vector access for the streaming vector kernels (falls back to scalars when a case's
// field length is not a multiple of the vector width).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

// S2: beta_{k+1} from the P5 partials, Givens step, convergence test; the iteration's U2
// coefficients go to slot `slot` (inactive when the case had already finished).
__global__ void k_minres_givens(MinresState* st, const double* partials, int np, int slot) {
  __shared__ double red[16];
  const int cs = blockIdx.x;
  MinresState& S = st[cs];
  if (S.done) {
    if (threadIdx.x == 0) S.u2[slot].active = 0;
    return;
  }
  const double s = sum_partials(partials + (long long)cs * np, np, red);
  if (threadIdx.x == 0) {
    givens_step(S, s);
    U2Coef& u = S.u2[slot];
    u.cd_u = S.cd_u;
    u.cd_d1 = S.cd_d1;
    u.cd_d2 = S.cd_d2;
    u.cx = S.cx;
    u.cx_prev = S.cx_prev;
    u.cx_pp = S.cx_pp;
    u.xmode = S.xmode;
    u.active = 1;
  }
}

// U2: d_k = cd_u u_k + cd_d1 d_{k-1} + cd_d2 d_{k-2} (written over d_{k-2}); the solution update
// the slot's xmode schedules (x += cx d_k plus the terms deferred from the two previous iterations).
// One 16-byte vector per thread over a grid that covers the field once (a grid-stride loop over a
// fixed grid streamed about 10% slower); every load of the element is issued before its arithmetic.
// All its loads and stores are nontemporal: nothing reads these lines again before the next
// iteration's U2, and U2 runs beside P3, whose output P4 partly finds in the memory-side cache.
// Coefficients come from the slot S2 filled for this iteration (the live state already belongs to
// the next iteration when U2 runs beside it).
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_direction(T* d2, const T* d1, const T* uk, T* x, const MinresState* st,
                                                   long long n6, int slot) {
  const int cs = blockIdx.y;
  const U2Coef& S = st[cs].u2[slot];
  if (!S.active) return;
  const T a = (T)S.cd_u, b = (T)S.cd_d1, c = (T)S.cd_d2, xc = (T)S.cx, xp = (T)S.cx_prev, xpp = (T)S.cx_pp;
  const int mode = S.xmode;  // uniform per block (one case)
  const long long off = (long long)cs * n6;
  constexpr int V = VEC ? Vec16<T>::n : 1;
  using VT = typename Vec16<T>::type;
  const long long nv = n6 / V;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (long long)gridDim.x * blockDim.x) {
    if constexpr (VEC) {
      VT dv = __builtin_nontemporal_load(reinterpret_cast<const VT*>(d2 + off) + i);
      const VT d2v = dv;  // d_{k-2}, for a mode-3 solution update
      const VT uv = __builtin_nontemporal_load(reinterpret_cast<const VT*>(uk + off) + i);
      const VT d1v = __builtin_nontemporal_load(reinterpret_cast<const VT*>(d1 + off) + i);
      VT xv;
      if (mode != 0) xv = __builtin_nontemporal_load(reinterpret_cast<const VT*>(x + off) + i);
      T* de = reinterpret_cast<T*>(&dv);
      const T* ue = reinterpret_cast<const T*>(&uv);
      const T* d1e = reinterpret_cast<const T*>(&d1v);
      const T* d2e = reinterpret_cast<const T*>(&d2v);
#pragma unroll
      for (int e = 0; e < V; ++e) de[e] = a * ue[e] + b * d1e[e] + c * de[e];
      __builtin_nontemporal_store(dv, reinterpret_cast<VT*>(d2 + off) + i);
      if (mode != 0) {
        T* xe = reinterpret_cast<T*>(&xv);
#pragma unroll
        for (int e = 0; e < V; ++e)
          xe[e] += (mode == 3 ? xpp * d2e[e] : (T)0) + (mode >= 2 ? xp * d1e[e] : (T)0) + xc * de[e];
        __builtin_nontemporal_store(xv, reinterpret_cast<VT*>(x + off) + i);
      }
    } else {
      const T d1s = d1[off + i];
      const T d2s = d2[off + i];
      const T d = a * uk[off + i] + b * d1s + c * d2s;
      d2[off + i] = d;
      if (mode != 0) x[off + i] += (mode == 3 ? xpp * d2s : (T)0) + (mode >= 2 ? xp * d1s : (T)0) + xc * d;
    }
  }
}

// Inner sweep bookkeeping: add iterations, record status.
__global__ void k_sweep_done(const MinresState* st, CaseInfo* ci, int nc) {
  const int cs = blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= nc || !ci[cs].active) return;
  ci[cs].iters += st[cs].iter;
  if (st[cs].status != 0 && st[cs].status != RVE_NOT_CONVERGED) ci[cs].status = st[cs].status;
  if (st[cs].status == RVE_NOT_CONVERGED) ci[cs].status = RVE_NOT_CONVERGED;
}

// After a true-residual evaluation: rnorm from the summed partial; decide whether another sweep runs.
// A case that had already stopped keeps its residual and stays stopped (its iterate did not change, and
// the recomputed residual could only differ by rounding), so every case's result is independent of how
// many sweeps the other cases of the solve need.
__global__ void k_residual_update(CaseInfo* ci, const double* sums, int nc, double tol, int max_iter) {
  const int cs = blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= nc || !ci[cs].active) return;
  ci[cs].rnorm = sqrt(sums[cs]);
  const bool conv = ci[cs].bnorm == 0.0 || ci[cs].rnorm <= tol * ci[cs].bnorm;
  const bool bad = ci[cs].status == RVE_ENONFINITE || ci[cs].status == RVE_BREAKDOWN;
  ci[cs].active = (!conv && !bad && ci[cs].iters < max_iter) ? 1 : 0;
}

// keep = x for the cases that did not run the sweep (their re-projection is not used).  Grid (blocks, nc).
__global__ void k_keep_inactive(double* keep, const double* x, const CaseInfo* ci, long long n6) {
  const int cs = blockIdx.y;
  if (ci[cs].active) return;
  const long long off = (long long)cs * n6;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long long)gridDim.x * blockDim.x)
    keep[off + i] = x[off + i];
}

// A warm start that does not reduce the residual below ||b|| is dropped: x = 0, r = b (the zero
// start, bit for bit).  A case whose right-hand side counts as zero (bnorm = 0: homogeneous cell,
// all-empty cell, zero macro strain) has the exact answer eps = 0, whatever the start: it takes the
// zero start too, without being recorded as a rejection.  Grid (blocks, nc).
__global__ void k_warm_fallback(double* x64, double* r64, const double* b64, CaseInfo* ci, long long n6) {
  const int cs = blockIdx.y;
  if (!(ci[cs].bnorm == 0.0 || ci[cs].rnorm >= ci[cs].bnorm)) return;
  const long long off = (long long)cs * n6;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n6; i += (long long)gridDim.x * blockDim.x) {
    x64[off + i] = 0.0;
    r64[off + i] = b64[off + i];
  }
}
// after k_warm_fallback: record the rejection, the residual is now ||b||
__global__ void k_residual_update_fallback(CaseInfo* ci, int nc) {
  const int cs = blockIdx.x * blockDim.x + threadIdx.x;
  if (cs >= nc) return;
  if (ci[cs].bnorm == 0.0) {  // zero start taken by k_warm_fallback; nothing to solve
    ci[cs].r0 = 0.0;
    ci[cs].rnorm = 0.0;
    return;
  }
  ci[cs].r0 = ci[cs].rnorm;
  if (ci[cs].rnorm < ci[cs].bnorm) return;
  ci[cs].warm_rejected = 1;
  ci[cs].rnorm = ci[cs].bnorm;
}

// Post-processing: sigma = C(x) (Ebar + eps) in FP64, write strain/stress in the output type,
// per-block partial sums of each stress component.
template <typename To>
__global__ void k_post(const double* x64, const float* phi, Material<double> mat, const double* E, To* strain_out,
                       To* stress_out, long long nvox, double* partials /* [nc][6][blocks] */) {
  __shared__ double red[16];
  const int cs = blockIdx.y;
  const long long off = (long long)cs * 6 * nvox;
  const float* phic = phi + (long long)cs * mat.phi_stride;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
    double e[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double f = x64[off + c * nvox + v];
      if (strain_out) strain_out[off + c * nvox + v] = (To)f;
      e[c] = E[cs * 6 + c] + f;
    }
    const double ph = phic[v];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double s = 0, s0 = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        s += mat.Cd[a * 6 + b] * e[b];
        s0 += mat.C0[a * 6 + b] * e[b];
      }
      const double sig = ph * s + s0;
      acc[a] += sig;
      if (stress_out) stress_out[off + a * nvox + v] = (To)sig;
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const double s = block_sum(acc[a], red);
    if (threadIdx.x == 0) partials[((long long)cs * 6 + a) * gridDim.x + blockIdx.x] = s;
  }
}

// phi validity: counts of non-finite and out-of-range entries
__global__ void k_check_phi(const float* phi, long long n, int* bad) {
  int nb = 0, nr = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float v = phi[i];
    if (!isfinite(v)) nb++;
    else if (v < 0.0f || v > 1.0f) nr++;
  }
  if (nb) atomicAdd(&bad[0], nb);
  if (nr) atomicAdd(&bad[1], nr);
}

// ---------------------------------------------------------------------------- J2 plasticity (eq. Slin)
// Isotropic elastic, perfectly plastic (von Mises) solid of bulk modulus K, shear modulus mu2/2 and
// yield stress sy; a voxel carries phi times the solid's stress and tangent.
struct J2Mat {
  double K, mu2, sy;
};
struct Vec6 {
  double v[6];
};

// Radial return at every voxel from the plastic strain eps_p of the last accepted increment:
// s = mu2 dev(eps - eps_p), q = sqrt(3/2)|s|; elastic when q <= sy, else the deviator is scaled by
// theta = sy/q and (1 - theta) dev(eps - eps_p) is the plastic strain increment.  Writes sigma and the
// tangent data of P1 (a = mu2 (1 - theta), m = sqrt(mu2 theta) s/|s|; zero when elastic) in FP64 and
// FP32 ([7][nvox]; each may be null).  accept: eps_p += increment, ep_acc += |increment|.
__global__ void k_j2_return(const double* __restrict__ eps, double* eps_p, const float* __restrict__ phi, J2Mat jm,
                            long long nvox, double* __restrict__ sig, double* __restrict__ tan64,
                            float* __restrict__ tan32, int accept, double* __restrict__ ep_acc) {
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long long)gridDim.x * blockDim.x) {
    double ee[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) ee[a] = eps[a * nvox + v] - eps_p[a * nvox + v];
    const double tr = ee[0] + ee[1] + ee[2];
    double dev[6], s[6], s2 = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      dev[a] = a < 3 ? ee[a] - tr / 3.0 : ee[a];
      s[a] = jm.mu2 * dev[a];
      s2 += s[a] * s[a];
    }
    const double sn = sqrt(s2);
    const double q = sqrt(1.5) * sn;
    const bool plastic = q > jm.sy;
    const double theta = plastic ? jm.sy / q : 1.0;
    const double ph = (double)phi[v];
    if (sig) {
#pragma unroll
      for (int a = 0; a < 6; ++a) sig[a * nvox + v] = ((a < 3 ? jm.K * tr : 0.0) + theta * s[a]) * ph;
    }
    const double ta = plastic ? jm.mu2 * (1.0 - theta) : 0.0;
    const double mf = plastic ? sqrt(jm.mu2 * theta) / sn : 0.0;
    if (tan64) {
      tan64[v] = ta;
#pragma unroll
      for (int a = 0; a < 6; ++a) tan64[(1 + a) * nvox + v] = mf * s[a];
    }
    if (tan32) {
      tan32[v] = (float)ta;
#pragma unroll
      for (int a = 0; a < 6; ++a) tan32[(1 + a) * nvox + v] = (float)(mf * s[a]);
    }
    if (accept && plastic) {
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double d = (1.0 - theta) * dev[a];
        eps_p[a * nvox + v] += d;
        d2 += d * d;
      }
      ep_acc[v] += sqrt(d2);
    }
  }
}

// x += c (a uniform Mandel vector) at every voxel
__global__ void k_add_uniform(double* x, Vec6 c, long long nvox) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 6 * nvox; i += (long long)gridDim.x * blockDim.x)
    x[i] += c.v[i / nvox];
}

// per-block maxima of |d| and |e - et| over n values: partials[2 b], partials[2 b + 1]
__global__ void k_absmax2(const double* __restrict__ d, const double* __restrict__ e, const double* __restrict__ et,
                          long long n, double* partials) {
  __shared__ double red[2][kThreads / 64];
  double m1 = 0.0, m2 = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    m1 = fmax(m1, fabs(d[i]));
    m2 = fmax(m2, fabs(e[i] - et[i]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m1 = fmax(m1, __shfl_xor(m1, o));
    m2 = fmax(m2, __shfl_xor(m2, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m1;
    red[1][threadIdx.x >> 6] = m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      m1 = fmax(m1, red[0][w]);
      m2 = fmax(m2, red[1][w]);
    }
    partials[2 * blockIdx.x] = m1;
    partials[2 * blockIdx.x + 1] = m2;
  }
}

}  // namespace rve
