// HIP pass kernels of the Galerkin operator A(e) = F^{-1}{ Ghat : F{ C(x) : e } } for gfx950.
//
// Data layout (per load case):
//   real fields   [6][N0][N1][N2]        Mandel components (11,22,33,sqrt2*23,sqrt2*13,sqrt2*12), axis 2 contiguous
//   half spectrum [K2][6][N0][N1] complex, K2 = N2/2 + 1 (plane-major: axis 1 contiguous)
// One operator application is five passes, each one streaming read + write over HBM:
//   P1 k_fwd_axis2     stiffness sigma = C(x) e (Voigt rule) fused into the real-to-complex FFT along axis 2;
//                      two real components are packed into one complex transform and separated after it;
//                      output written transposed into the plane-major half spectrum
//   P2 k_axis1<-1>     complex FFT along axis 1 (contiguous rows)
//   P3 k_axis0_project FFT along axis 0, per-frequency Galerkin projection (eq. galop with the rotated
//                      modified frequencies of eq. freqrot), inverse FFT along axis 0 - all 6 components of a
//                      pencil meet in registers here
//   P4 k_axis1<+1>     inverse FFT along axis 1
//   P5 k_inv_axis2     complex-to-real inverse FFT along axis 2 back to [6][N0][N1][N2], fused with the
//                      per-block FP64 partial of <A v, v> used by MINRES
// Every 1-D transform of length N = NA*NB runs as two register-resident small DFTs (radix NA, then NB)
// with one LDS exchange between them.  Each thread owns one stage-A column t in [0,NB).
#pragma once
#include "rve_device.h"

namespace rve {

struct GridDims {
  int n0, n1, n2, k2;      // k2 = n2/2 + 1
  long long nvox;          // n0*n1*n2
  long long spec_case;     // 6*k2*n0*n1 complex elements per load case
  int tile, tile_shift;    // n0 tile of P3's spectrum copy (a power of two dividing n0 and NB of axis 0)
};

// The U2 coefficients of one iteration, copied out by S2 into one of two slots (iteration parity):
// U2 runs on a second stream beside the next iteration's operator passes, which change the state.
struct U2Coef {
  double cd_u, cd_d1, cd_d2, cx, cx_prev, cx_pp;
  int xmode;   // as MinresState::xmode
  int active;  // 0: the case had finished before this iteration; U2 does nothing
};

// Per-solve MINRES scalars (FP64), one per load case, resident on the device.
struct MinresState {
  double beta, ib, ib_prev;          // beta_k, 1/beta_k, 1/beta_{k-1} (deferred normalisation of v)
  double alpha;                      // Lanczos diagonal
  double c1, s1, c2, s2;             // Givens rotations G_{k-1}, G_{k-2}
  double phibar;                     // |phibar| = residual norm of the current iterate
  double tol_abs;                    // stop when |phibar| <= tol_abs
  double cu_v, cu_vp;                // Lanczos update coefficients (on raw u_k, u_{k-1})
  double cd_u, cd_d1, cd_d2, cx;     // search-direction / solution update coefficients
  double cx_prev, cx_pp;             // solution coefficients of d_{k-1}, d_{k-2} while deferred
  double sumsq;                      // scratch: last reduced sum
  int iter, max_iter, finish, done, status;
  int xmode;    // U2's solution update: 0 defer, 1 x += cx d_k, 2 x += cx_prev d_{k-1} + cx d_k,
                // 3 x += cx_pp d_{k-2} + cx_prev d_{k-1} + cx d_k
  int pending;  // deferred terms owed to x: 0, 1 (cx_prev d_{k-1}) or 2 (and cx_pp d_{k-2})
  int pad;
  U2Coef u2[2];  // U2's coefficients of the last two iterations (slot = iteration parity in the chunk)
};

// U2 touches x only every third iteration: the updates of two iterations are deferred and added
// together with the third one's, when d_{k-1} and d_{k-2} are still in the buffers U2 reads anyway
// (d_{k-2} is read before its buffer takes d_k); a finishing iteration always settles what is owed.
__device__ __forceinline__ void schedule_x_update(MinresState& S) {
  if (S.pending == 2) {
    S.xmode = 3;
    S.pending = 0;
  } else if (S.finish) {
    S.xmode = S.pending ? 2 : 1;
    S.pending = 0;
  } else if (S.pending == 1) {
    S.xmode = 0;
    S.pending = 2;
    S.cx_pp = S.cx_prev;
    S.cx_prev = S.cx;
  } else {
    S.xmode = 0;
    S.pending = 1;
    S.cx_prev = S.cx;
  }
}

template <typename T>
struct Material {
  T C0[36];  // stiffness of the empty phase (normally zero)
  T Cd[36];  // C_solid - C_void:  C(x) = C0 + phi(x) Cd  (Voigt rule)
  int has_c0;
  int use_phi;  // 0: C(x) = C0 everywhere (phi is not read)
  // isotropic fast path (set when the Mandel matrix is exactly lam 1(x)1 + mu2 I):
  // sigma = lam tr(eps) 1 + mu2 eps, with 1 = (1,1,1,0,0,0)
  int iso_d, iso_0;
  T lam_d, mu2_d, lam_0, mu2_0;
  long long phi_stride;  // voxels between the phase maps of consecutive load cases (0: one map for all)
  // Tangent of an elastic-plastic solid (P1 instance with TAN = true, eq. Slin): per voxel a and m[6]
  // in [7][nvox], C_t(x) = phi(x) (Cd - a I_dev - m (x) m), Cd isotropic and C0 = 0; tan_stride values
  // between consecutive load cases.  nullptr otherwise.
  const T* tan;
  long long tan_stride;
};

// x when A, else y (references of possibly different types, chosen at compile time)
template <bool A, typename X, typename Y>
__device__ __forceinline__ auto& pick(X& x, Y& y) {
  if constexpr (A) return x;
  else return y;
}

// sigma_a = (C e)_a for one voxel, general 6x6 or isotropic form
template <typename T>
__device__ __forceinline__ T stiff_row(const T* C, int iso, T lam, T mu2, int a, const T (&e)[6], T tr) {
  if (iso) return (a < 3 ? lam * tr : (T)0) + mu2 * e[a];
  T sv = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) sv += C[a * 6 + b] * e[b];
  return sv;
}

template <typename T>
struct FreqTables {
  const T* s[3];  // sin(q/2)/h (rotated scheme) per axis and storage index
  const T* c[3];  // cos(q/2), exact 0 at a Nyquist index
  int stress_mask;  // mixed macroscopic control: Mandel components kept by the projection at xi = 0
};

__device__ __forceinline__ long long spec_idx(const GridDims& g, int cs, int k2, int c, int n0, int n1) {
  return ((((long long)cs * g.k2 + k2) * 6 + c) * g.n0 + n0) * (long long)g.n1 + n1;
}
// P3's copy of the spectrum: every (case, k2, component) plane stored in tiles of g.tile consecutive
// n0, [n0 / tile][n1][n0 % tile], so that a pencil along axis 0 reads runs of g.tile values and
// neighbouring pencils (n1, n1 + 1) are adjacent
__device__ __forceinline__ long long spec_t_plane(const GridDims& g, int cs, int k2, int c) {
  return (((long long)cs * g.k2 + k2) * 6 + c) * g.n0 * (long long)g.n1;
}
__device__ __forceinline__ long long spec_t_off(const GridDims& g, int n0, int n1) {
  return (long long)(n0 >> g.tile_shift) * g.n1 * g.tile + (long long)n1 * g.tile + (n0 & (g.tile - 1));
}

// ---------------------------------------------------------------------------- Krylov scalar steps
// (run by single-block kernels after P1 and P5: per-block partials are summed in a fixed order, so the
// reductions are deterministic; device-wide fences inside the streaming kernels would write back the
// whole L2 of every XCD and cost far more than a separate launch)
__device__ __forceinline__ double sum_partials(const double* p, int np, double* red) {
  // eight independent loads in flight per thread (a dependent chain of loads made these single-block
  // steps latency-bound), combined in a fixed order
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int nt = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * nt < np; i += 8 * nt) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[i + u * nt];
  }
  for (; i < np; i += nt) a[0] += p[i];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum(acc, red);
}

// Lanczos diagonal from sum = <u_k, C u_k> * ib_k:  alpha_k = <v_k, A v_k> = <v_k, C v_k> for a compatible
// v_k (Ghat is an orthogonal projector, so <v, Ghat C v> = <Ghat v, C v>).  Coefficients of the three-
// term update u_{k+1} = A v_k - alpha_k v_k - beta_k v_{k-1} on the stored (unscaled) u vectors.
__device__ __forceinline__ void alpha_step(MinresState& S, double sum) {
  const double alpha = S.ib * sum;
  S.alpha = alpha;
  S.cu_v = alpha * S.ib;
  S.cu_vp = S.beta * S.ib_prev;
}

// S1: alpha_k from the P1 partials of case cs; a case whose previous iteration finished is retired
// instead (that iteration's U2 has run by now).  Run by extra blocks of P2 (the pass after P1, which
// reads none of what this writes), so that it needs no launch of its own.  The partials are summed in
// the order a 256-thread block sums them (eight loads in flight per thread; per wave the shuffle
// tree, whose lane 0 adds the upper half onto the lower one at halving distances; the four wave sums
// in turn), whatever the size of the block that runs it, which may be below one wave; vsum holds 256
// doubles of LDS.
__device__ void minres_alpha_block(MinresState* st, const double* partials, int np, int cs, double* vsum) {
  MinresState& S = st[cs];
  if (S.done) return;
  if (S.finish) {
    if (threadIdx.x == 0) S.done = 1;
    return;
  }
  constexpr int VT = 256;
  const double* p = partials + (long long)cs * np;
  for (int v = threadIdx.x; v < VT; v += blockDim.x) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = v;
    for (; i + 7 * VT < np; i += 8 * VT) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += p[i + u * VT];
    }
    for (; i < np; i += VT) a[0] += p[i];
    vsum[v] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    for (int q = threadIdx.x; q < (VT / 64) * off; q += blockDim.x) {
      const int l = (q / off) * 64 + q % off;  // lane q % off of virtual wave q / off
      vsum[l] += vsum[l + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < VT / 64; ++w) sum += vsum[w * 64];
    alpha_step(S, sum);
  }
}

// beta_{k+1} = ||u_{k+1}||; Givens QR step of the extended tridiagonal matrix; residual recurrence
// |phibar|; coefficients of d_k = (v_k - delta_k d_{k-1} - eps_k d_{k-2}) / gamma_k and x += tau d_k.
__device__ __forceinline__ void givens_step(MinresState& S, double sumsq) {
  const double beta_next = sqrt(sumsq);
  const double alpha = S.alpha, beta = S.beta;
  const double eps = S.s2 * beta, dtil = S.c2 * beta;
  const double delta = S.c1 * dtil + S.s1 * alpha;
  const double gtil = -S.s1 * dtil + S.c1 * alpha;
  const double gamma = hypot(gtil, beta_next);
  S.iter += 1;
  if (!(isfinite(alpha) && isfinite(beta_next) && isfinite(gamma))) {
    S.status = -3;  // non-finite scalar
    S.cd_u = S.cd_d1 = S.cd_d2 = S.cx = 0.0;
    S.finish = 1;
    schedule_x_update(S);
    return;
  }
  if (gamma == 0.0) {
    S.status = 2;  // breakdown
    S.cd_u = S.cd_d1 = S.cd_d2 = S.cx = 0.0;
    S.finish = 1;
    schedule_x_update(S);
    return;
  }
  const double c = gtil / gamma, sn = beta_next / gamma;
  const double tau = c * S.phibar;
  S.phibar = -sn * S.phibar;
  S.cd_u = S.ib / gamma;
  S.cd_d1 = -delta / gamma;
  S.cd_d2 = -eps / gamma;
  S.cx = tau;
  S.c2 = S.c1;
  S.s2 = S.s1;
  S.c1 = c;
  S.s1 = sn;
  S.ib_prev = S.ib;
  S.ib = beta_next > 0 ? 1.0 / beta_next : 0.0;
  S.beta = beta_next;
  if (fabs(S.phibar) <= S.tol_abs || beta_next == 0.0) {
    S.finish = 1;
  } else if (S.iter >= S.max_iter) {
    S.status = 1;  // not converged
    S.finish = 1;
  }
  schedule_x_update(S);
}

// ============================================================================ P1
// grid (ceil(N1/W), N0, ncases), block W*NB threads, dyn. LDS W*max(NA*(NB+1), N+1) complex (+ N
// complex in FP32 for the twiddle table)
// With `partials` (MINRES iterations): per-block <x, sigma> partials for the Lanczos alpha.
// Waves per SIMD P1 is compiled for: at 256 = 16 x 16 in FP32 (no tangent) it needs 130 VGPRs, two more
// than four waves allow; capped there it runs four waves per SIMD.
template <typename T, int NA, int NB, bool TAN>
struct P1Waves {
  static constexpr int value = (sizeof(T) == 4 && NA == 16 && NB == 16 && !TAN) ? 4 : 1;
};

template <typename T, int NA, int NB, bool TAN = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P1Waves<T, NA, NB, TAN>::value))) void
k_fwd_axis2(const T* __restrict__ x, const double* __restrict__ xscale_ib,
                                                   int xscale_stride, const float* __restrict__ phi, Material<T> mat,
                                                   cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw, GridDims g,
                                                   int W, const MinresState* __restrict__ st, double* partials) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int cs = blockIdx.z;
  if (st && st[cs].finish) return;
  // FP32: the stage twiddles come from a copy of the table in LDS behind the exchange areas (read
  // before the first transform, after a barrier), which keeps them out of the registers
  constexpr bool TWL = sizeof(T) == 4;
  constexpr int XA = (NA * (NB + 1) > N + 1) ? NA * (NB + 1) : N + 1;
  cx<T>* twl = lds + W * XA;
  if (TWL) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = tw[i];
  }
  // planes in descending n0: P5 (ascending) wrote the high planes last, so part of them is still in
  // the memory-side cache when this pass starts
  const int n0 = g.n0 - 1 - (int)blockIdx.y;
  const int n1_0 = blockIdx.x * W;
  const int tid = threadIdx.x;
  const int t = tid % TT, w = tid / TT;
  const int n1 = n1_0 + w;
  const bool row_ok = n1 < g.n1;
  const T xs = xscale_ib ? (T)xscale_ib[(long long)cs * xscale_stride] : (T)1;
  const long long row = ((long long)n0 * g.n1 + n1) * N;
  const T* xc = x + (long long)cs * 6 * g.nvox;
  const float* phic = phi + (long long)cs * mat.phi_stride;
  __shared__ double red[16];
  double acc = 0.0;

  T sg[6][NA];
  {
    // loads without a branch per element: a row past the grid's end reads the last row and its
    // stresses are scaled by zero (a load under a per-lane condition made the compiler wait for the
    // loads in flight before each address computation); the offsets NB * i are immediates on one base
    // per field
    const long long rowc = row_ok ? row : ((long long)n0 * g.n1 + (g.n1 - 1)) * N;
    const T xso = row_ok ? xs : (T)0;
    T e[6][NA], ph[NA];
    const float* pr = phic + rowc + t;
    const T* xr[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) xr[c] = xc + (long long)c * g.nvox + rowc + t;
    // element-major, so that the stiffness of element i can start once its seven values are in
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      ph[i] = mat.use_phi ? (T)pr[NB * i] : (T)0;
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c][i] = ld_stream_wide(xr[c] + NB * i);
    }
    // element by element, so that e[.][i] is dead once sg[.][i] and its <x, sigma> terms exist
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      T ev[6];
#pragma unroll
      for (int b = 0; b < 6; ++b) ev[b] = e[b][i];
      const T tr = ev[0] + ev[1] + ev[2];
      if constexpr (TAN) {
        // C_t e = phi (Cd e - a dev(e) - (m . e) m), the tangent's data read element by element
        const T* tp = mat.tan + (long long)cs * mat.tan_stride + rowc + t + NB * i;
        T tm[6], md = 0;
        const T ta = tp[0];
#pragma unroll
        for (int b = 0; b < 6; ++b) tm[b] = tp[(long long)(1 + b) * g.nvox];
#pragma unroll
        for (int b = 0; b < 6; ++b) md += tm[b] * ev[b];
        const T tr3 = tr * (T)(1.0 / 3.0);
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const T dv = a < 3 ? ev[a] - tr3 : ev[a];
          const T sv = stiff_row(mat.Cd, mat.iso_d, mat.lam_d, mat.mu2_d, a, ev, tr) - ta * dv - md * tm[a];
          sg[a][i] = ph[i] * sv * xso;
        }
      } else {
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          T sv = 0;
          if (mat.use_phi) sv = ph[i] * stiff_row(mat.Cd, mat.iso_d, mat.lam_d, mat.mu2_d, a, ev, tr);
          if (mat.has_c0) sv += stiff_row(mat.C0, mat.iso_0, mat.lam_0, mat.mu2_0, a, ev, tr);
          sg[a][i] = sv * xso;
        }
      }
      if (partials) {
#pragma unroll
        for (int a = 0; a < 6; ++a) acc += (double)e[a][i] * (double)sg[a][i];
      }
    }
  }
  const int ws = tid % W, m = tid / W, M = blockDim.x / W;
  const int n1s = n1_0 + ws;
  if (TWL) lds_barrier();
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    cx<T> z[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) z[i] = mk<T>(sg[2 * pr][i], sg[2 * pr + 1][i]);
    DFT<NA, -1, T>::run(z);
#pragma unroll
    for (int a = 1; a < NA; ++a) z[a] = cmul(z[a], TWL ? twl[(t * a) % N] : tw[(t * a) % N]);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) lds[(w * NA + a) * (NB + 1) + t] = z[a];
    lds_barrier();
    cx<T> yb[CB][NB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) yb[j][u] = lds[(w * NA + a) * (NB + 1) + u];
        DFT<NB, -1, T>::run(yb[j]);
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int b = 0; b < NB; ++b) lds[w * (N + 1) + a + NA * b] = yb[j][b];
      }
    }
    lds_barrier();
    if (n1s < g.n1) {
      for (int k = m; k < g.k2; k += M) {
        const cx<T> Z = lds[ws * (N + 1) + k];
        const cx<T> Zm = lds[ws * (N + 1) + (N - k) % N];
        const cx<T> A = mk<T>((Z.re + Zm.re) * (T)0.5, (Z.im - Zm.im) * (T)0.5);
        const cx<T> B = mk<T>((Z.im + Zm.im) * (T)0.5, (Zm.re - Z.re) * (T)0.5);
        // streaming stores: slower here, but P2 then reads without this pass's write-backs beside it
        st_stream(spec + spec_idx(g, cs, k, 2 * pr, n0, n1s), A);
        st_stream(spec + spec_idx(g, cs, k, 2 * pr + 1, n0, n1s), B);
      }
    }
  }
  if (partials) {
    const unsigned nb = gridDim.x * gridDim.y;
    const double sblk = block_sum(acc, red);
    if (tid == 0) partials[(long long)cs * nb + blockIdx.y * gridDim.x + blockIdx.x] = sblk;
  }
}

// ============================================================================ P2 / P4
// Rows of N1 complex, one per (case, k2, component, n0); grid (ceil(rows/R)), block R*NB threads,
// dyn. LDS R*(NA*(NB+1)+1) complex (+ N complex in FP32 for the twiddle table).  P2 (S < 0) reads
// rows of spec and writes P3's tiled copy (spec_t_off), P4 (S > 0) reads the tiled copy and writes
// rows of spec.  The side on spec runs with
// the element index fastest across lanes (adjacent along a row), the side on the tiled copy with the
// row index fastest (consecutive n0 at one n1 are adjacent there); the LDS exchange between the two
// transform stages hands the data from one lane order to the other.
template <typename T, int NA, int NB, int S>
__global__ __launch_bounds__(256) void k_axis1(cx<T>* __restrict__ spec, cx<T>* __restrict__ spec_t,
                                               const cx<T>* __restrict__ tw, GridDims g, int R, long long total_rows,
                                               const MinresState* __restrict__ st, MinresState* s1_st,
                                               const double* s1_partials, int s1_np, int s1_blocks) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int RSW = NA * (NB + 1) + 1;  // LDS words (complex) per row: odd, so rows fall on distinct banks
  extern __shared__ unsigned char smem_raw[];
  // MINRES iterations: the first s1_blocks blocks (one per load case) run S1 and nothing else
  if ((int)blockIdx.x < s1_blocks) {
    minres_alpha_block(s1_st, s1_partials, s1_np, (int)blockIdx.x, reinterpret_cast<double*>(smem_raw));
    return;
  }
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  // FP32: the stage twiddles come from a copy of the table in LDS behind the rows' exchange areas,
  // written first so that its loads do not wait behind the row loads
  constexpr bool TWL = sizeof(T) == 4;
  cx<T>* twl = lds + R * RSW;
  if (TWL) {
    for (int i = tid; i < N; i += blockDim.x) twl[i] = tw[i];
  }
  const long long row0 = ((long long)blockIdx.x - s1_blocks) * R;
  const int t_row = tid % TT, w_row = tid / TT;  // element index fastest
  const int w_til = tid % R, t_til = tid / R;    // row index fastest
  const int t1 = (S < 0) ? t_row : t_til, w1 = (S < 0) ? w_row : w_til;  // stage A (input side)
  const int t2 = (S < 0) ? t_til : t_row, w2 = (S < 0) ? w_til : w_row;  // stage B (output side)
  // row row0 + w lies in plane p (case, k2, component) at n0; the block's first row is split once
  // (uniform), the lanes step from it (R may not divide n0)
  const long long p0 = row0 / g.n0;
  const int n00 = (int)(row0 - p0 * g.n0);
  const int planes_per_case = 6 * g.k2;
  auto locate = [&](int w, long long* p, int* n0) {
    int q = n00 + w;
    long long pp = p0;
    while (q >= g.n0) {
      q -= g.n0;
      ++pp;
    }
    *p = pp;
    *n0 = q;
  };
  auto live = [&](long long r, long long p) {  // p < 65535 cases * 6 * k2 fits 32 bits
    return r < total_rows && !(st && st[(int)p / planes_per_case].finish);
  };
  const long long ra = row0 + w1;
  long long pa;
  int n0a;
  locate(w1, &pa, &n0a);
  const bool oka = live(ra, pa);
  // offset of element 0 of the row in the tiled copy (element j at + j * tile)
  // the tiled side addresses from the block's first plane with 32-bit offsets (the block's rows span
  // at most a few planes of n0*N1 <= 2^16 elements), so the loads and stores take a uniform base
  const cx<T>* tblk = spec_t + p0 * g.n0 * (long long)N;
  // loads without a per-lane condition (one made the compiler wait for the loads in flight): a row
  // past the end reads the block's first row, a dead row (finished case) its own, and neither is
  // stored; a wave with no live row loads nothing
  const bool in_range = ra < total_rows;
  const unsigned ta = in_range ? (unsigned)((pa - p0) * g.n0 * N + spec_t_off(g, n0a, 0)) : 0u;
  const long long rac = in_range ? ra : row0;
  cx<T> z[NA];
  if (__ballot(oka) != 0) {
    if (S < 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) z[i] = ld_stream(spec + rac * N + t1 + NB * i);
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) z[i] = ld_stream(tblk + ta + (unsigned)((t1 + NB * i) * g.tile));
    }
  } else {
#pragma unroll
    for (int i = 0; i < NA; ++i) z[i] = mk<T>(0, 0);
  }
  DFT<NA, S, T>::run(z);
  if (TWL) lds_barrier();  // the twiddle table is in place
  const cx<T>* tws = TWL ? twl : tw;
#pragma unroll
  for (int a = 1; a < NA; ++a) z[a] = (S < 0) ? cmul(z[a], tws[(t1 * a) % N]) : cmulc(z[a], tws[(t1 * a) % N]);
#pragma unroll
  for (int a = 0; a < NA; ++a) lds[w1 * RSW + a * (NB + 1) + t1] = z[a];
  lds_barrier();
  const long long rb = row0 + w2;
  long long pb;
  int n0b;
  locate(w2, &pb, &n0b);
  const bool okb = live(rb, pb);
  const unsigned tb = okb ? (unsigned)((pb - p0) * g.n0 * N + spec_t_off(g, n0b, 0)) : 0u;
  cx<T>* tblk_w = spec_t + p0 * g.n0 * (long long)N;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t2 + TT * j;
    if (a < NA) {
      cx<T> yb[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) yb[u] = lds[w2 * RSW + a * (NB + 1) + u];
      DFT<NB, S, T>::run(yb);
      if (okb) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (S > 0)  // streaming stores: P5's gather then runs without P4's write-backs beside it
            st_stream(spec + rb * N + a + NA * b, yb[b]);
          else
            tblk_w[tb + (unsigned)((a + NA * b) * g.tile)] = yb[b];
        }
      }
    }
  }
}

// ============================================================================ strided axes
// Complex FFT along a strided axis of [ncomp][n0][n1][K] arrays (the displacement solver's half
// spectra, K = n2/2 + 1 contiguous), in place, component blockIdx.z (cstride elements apart): axis 1
// (pencils of n1 elements K apart, blockIdx.y = n0) or axis 0 (pencils of n0 elements n1*K apart).
// A block takes R pencils that are adjacent in memory, with the pencil index fastest across lanes, so
// that every load and store instruction covers runs of R consecutive complex values; the transform is
// the same two register stages with one LDS exchange as the Galerkin passes.  S < 0 forward, S > 0
// inverse (unnormalised).  grid (ceil(pencils/R), n0 or 1, ncomp), block R*NB threads, dyn. LDS
// R*(NA*(NB+1)+1) complex.
template <typename T, int NA, int NB, int S>
__global__ __launch_bounds__(256) void k_strided(cx<T>* __restrict__ data, long long cstride, int n1, int K, int axis,
                                                 const cx<T>* __restrict__ tw, int R) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int RSW = NA * (NB + 1) + 1;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int w = tid % R, t = tid / R;
  long long base, es;
  int valid;
  if (axis == 1) {
    const int k0 = blockIdx.x * R;
    base = (long long)blockIdx.y * n1 * K + k0;
    es = K;
    valid = min(R, K - k0);
  } else {
    const long long q0 = (long long)blockIdx.x * R;
    es = (long long)n1 * K;
    base = q0;
    valid = (int)min((long long)R, es - q0);
  }
  const bool ok = w < valid;
  // a lane past the last pencil loads the last one (no per-lane condition on the loads) and stores nothing
  cx<T>* d = data + (long long)blockIdx.z * cstride + base + (ok ? w : valid - 1);
  cx<T> z[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) z[i] = d[(long long)(t + NB * i) * es];
  DFT<NA, S, T>::run(z);
#pragma unroll
  for (int a = 1; a < NA; ++a) z[a] = (S < 0) ? cmul(z[a], tw[(t * a) % N]) : cmulc(z[a], tw[(t * a) % N]);
#pragma unroll
  for (int a = 0; a < NA; ++a) lds[w * RSW + a * (NB + 1) + t] = z[a];
  lds_barrier();
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
      cx<T> yb[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) yb[u] = lds[w * RSW + a * (NB + 1) + u];
      DFT<NB, S, T>::run(yb);
      if (ok) {
#pragma unroll
        for (int b = 0; b < NB; ++b) d[(long long)(a + NA * b) * es] = yb[b];
      }
    }
  }
}

// Rows along axis 2 of the same arrays: per component pair (2 q, 2 q + 1; blockIdx.z = q, the second
// absent when 2 q + 1 = ncomp) the complex-to-real inverse of the two half spectra packed as one
// complex transform, the real fields times scale * phi(x) (components below nphi, an even count) or
// scale * (1 - phi(x)), and the real-to-complex forward transform back in place.  A block takes W
// consecutive rows (contiguous in every component, NB threads per row); per row one LDS area holds in
// turn the Hermitian-extended sequence, the exchange between the register stages and the natural-order
// result.  grid (ceil(rows/W), 1, ceil(ncomp/2)), block W*NB threads, dyn. LDS W*max(N+1, NA*(NB+1))
// complex.
template <typename T, int NA, int NB>
__global__ __launch_bounds__(256) void k_row_pair(cx<T>* __restrict__ data, long long cstride,
                                                  const float* __restrict__ phi, long long rows, int K, int ncomp,
                                                  int nphi, T scale, const cx<T>* __restrict__ tw, int W) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int RS = (N + 1 > NA * (NB + 1)) ? N + 1 : NA * (NB + 1);
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int q = blockIdx.z;
  const bool has1 = 2 * q + 1 < ncomp;
  const bool by_phi = 2 * q < nphi;
  const int tid = threadIdx.x;
  const int t = tid % TT, w = tid / TT;
  const long long r0 = (long long)blockIdx.x * W;
  const int nrow = (int)min((long long)W, rows - r0);
  const bool row_ok = w < nrow;
  cx<T>* A = data + (long long)(2 * q) * cstride + r0 * K;
  cx<T>* B = data + (long long)(has1 ? 2 * q + 1 : 2 * q) * cstride + r0 * K;
  cx<T>* L = lds + w * RS;
  // the pair's half spectra -> a + i b on the full circle (a real row's DC and Nyquist terms are real)
  for (int idx = tid; idx < nrow * K; idx += blockDim.x) {
    const int ww = idx / K, k = idx - ww * K;
    const cx<T> a = A[idx];
    const cx<T> b = has1 ? B[idx] : mk<T>(0, 0);
    cx<T>* sq = lds + ww * RS;
    if (k == 0 || 2 * k == N) {
      sq[k] = mk<T>(a.re, b.re);
    } else {
      sq[k] = mk<T>(a.re - b.im, a.im + b.re);
      sq[N - k] = mk<T>(a.re + b.im, b.re - a.im);
    }
  }
  lds_barrier();
  cx<T> z[NA];
  cx<T> yb[CB][NB];
  // inverse transform: register stage A, exchange, register stage B
#pragma unroll
  for (int i = 0; i < NA; ++i) z[i] = L[t + NB * i];
  DFT<NA, 1, T>::run(z);
#pragma unroll
  for (int a = 1; a < NA; ++a) z[a] = cmulc(z[a], tw[(t * a) % N]);
  lds_barrier();
#pragma unroll
  for (int a = 0; a < NA; ++a) L[a * (NB + 1) + t] = z[a];
  lds_barrier();
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int u = 0; u < NB; ++u) yb[j][u] = L[a * (NB + 1) + u];
      DFT<NB, 1, T>::run(yb[j]);
    }
  }
  lds_barrier();
  // the two real fields times the phase factor, in natural order
  const float* ph = phi + (r0 + (row_ok ? w : 0)) * (long long)N;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int e = a + NA * b;
        const T m = (T)ph[e];  // a row past the end reads row r0 and is not stored
        const T f = (by_phi ? m : (T)1 - m) * scale;
        L[e] = mk<T>(yb[j][b].re * f, yb[j][b].im * f);
      }
    }
  }
  lds_barrier();
  // forward transform
#pragma unroll
  for (int i = 0; i < NA; ++i) z[i] = L[t + NB * i];
  DFT<NA, -1, T>::run(z);
#pragma unroll
  for (int a = 1; a < NA; ++a) z[a] = cmul(z[a], tw[(t * a) % N]);
  lds_barrier();
#pragma unroll
  for (int a = 0; a < NA; ++a) L[a * (NB + 1) + t] = z[a];
  lds_barrier();
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int u = 0; u < NB; ++u) yb[j][u] = L[a * (NB + 1) + u];
      DFT<NB, -1, T>::run(yb[j]);
    }
  }
  lds_barrier();
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int b = 0; b < NB; ++b) L[a + NA * b] = yb[j][b];
    }
  }
  lds_barrier();
  // separate the two half spectra
  for (int idx = tid; idx < nrow * K; idx += blockDim.x) {
    const int ww = idx / K, k = idx - ww * K;
    const cx<T>* sq = lds + ww * RS;
    const cx<T> Z = sq[k], Zm = sq[(N - k) % N];
    A[idx] = mk<T>((Z.re + Zm.re) * (T)0.5, (Z.im - Zm.im) * (T)0.5);
    if (has1) B[idx] = mk<T>((Z.im + Zm.im) * (T)0.5, (Zm.re - Z.re) * (T)0.5);
  }
}

// ============================================================================ P3
// Galerkin projection of one frequency (eq. galop): Ghat S = t (x) n + n (x) t - (n.t) n (x) n with
// n = w/|w| and t = S n, applied to the Mandel components (S0..S5) in place and scaled by f (the 1/N
// of the inverse transform); w = 0 gives 0, except for the components in `keep` (the stress-controlled
// ones under mixed control, passed only at xi = 0), on which Ghat is the identity.
// 1/sqrt: the hardware reciprocal square root (1 ulp) in FP32, the correctly rounded form in FP64
__device__ __forceinline__ float rnorm(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rnorm(double x) { return 1.0 / sqrt(x); }

template <typename T>
__device__ __forceinline__ void project_mandel(cx<T>& D0, cx<T>& D1, cx<T>& D2, cx<T>& D3, cx<T>& D4, cx<T>& D5,
                                               T w0, T w1, T w2, T f, int keep) {
  const T sq2 = (T)1.41421356237309504880168872420970, isq2 = (T)0.70710678118654752440084436210485;
  const T nn = w0 * w0 + w1 * w1 + w2 * w2;
  if (nn > (T)0) {
    const T inv = rnorm(nn);
    const T m0 = w0 * inv, m1 = w1 * inv, m2 = w2 * inv;
    // t = f S n with the Mandel off-diagonals unscaled (S_ij = D_k / sqrt2), q = n . t
    const T fh = f * isq2;
    const cx<T> S00 = scl(D0, f), S11 = scl(D1, f), S22 = scl(D2, f);
    const cx<T> S12 = scl(D3, fh), S02 = scl(D4, fh), S01 = scl(D5, fh);
    const cx<T> t0 = scl(S00, m0) + scl(S01, m1) + scl(S02, m2);
    const cx<T> t1 = scl(S01, m0) + scl(S11, m1) + scl(S12, m2);
    const cx<T> t2 = scl(S02, m0) + scl(S12, m1) + scl(S22, m2);
    const cx<T> q = scl(t0, m0) + scl(t1, m1) + scl(t2, m2);
    D0 = scl(t0, (T)2 * m0) - scl(q, m0 * m0);
    D1 = scl(t1, (T)2 * m1) - scl(q, m1 * m1);
    D2 = scl(t2, (T)2 * m2) - scl(q, m2 * m2);
    D3 = scl(scl(t1, m2) + scl(t2, m1) - scl(q, m1 * m2), sq2);
    D4 = scl(scl(t0, m2) + scl(t2, m0) - scl(q, m0 * m2), sq2);
    D5 = scl(scl(t0, m1) + scl(t1, m0) - scl(q, m0 * m1), sq2);
  } else {
    D0 = (keep & 1) ? scl(D0, f) : mk<T>(0, 0);
    D1 = (keep & 2) ? scl(D1, f) : mk<T>(0, 0);
    D2 = (keep & 4) ? scl(D2, f) : mk<T>(0, 0);
    D3 = (keep & 8) ? scl(D3, f) : mk<T>(0, 0);
    D4 = (keep & 16) ? scl(D4, f) : mk<T>(0, 0);
    D5 = (keep & 32) ? scl(D5, f) : mk<T>(0, 0);
  }
}

// grid (ceil(N1/W), K2, ncases), block W*NB threads, dyn. LDS NA*(NB*W+1) complex
// All six components of the thread's pencil elements are loaded up front (maximum loads in flight)
// and transformed in place in one register array D[c][.]: stage-A layout D[c][i] = x[t + NB i],
// stage-B layout D[c][j*NB + b] = X[a_j + NA b] with a_j = t + NB j.  IDENT replaces the projection
// by the identity (test mode of the stiffness/transform round trip).
template <typename T, int NA, int NB, bool IDENT>
__global__ __launch_bounds__(256) void k_axis0_project(cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw,
                                                       FreqTables<T> ft, GridDims g, int W, T inv_total,
                                                       const MinresState* __restrict__ st) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int E = (NA > CB * NB) ? NA : CB * NB;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int cs = blockIdx.z;
  if (st && st[cs].finish) return;
  // planes in descending k2: P2 (ascending rows) wrote the high planes last, so part of them is still in
  // the memory-side cache, and P4 (ascending again) then starts on the planes written last here
  const int k2 = g.k2 - 1 - (int)blockIdx.y;
  const int tid = threadIdx.x;
  const int t = tid % NB, w = tid / NB;  // a pencil's threads are adjacent lanes
  const int k1 = blockIdx.x * W + w;
  const bool ok = k1 < g.n1;
  const int RS = NB * W + 1;
  const long long pstride = (long long)g.n0 * g.n1;  // component stride inside one k2 plane
  cx<T>* base = spec + spec_t_plane(g, cs, k2, 0) + spec_t_off(g, 0, ok ? k1 : 0);
  const long long toff = spec_t_off(g, t, 0);  // element t + NB i at toff + i NB n1 (tile divides NB)

  cx<T> D[6][E];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int i = 0; i < NA; ++i) D[c][i] = ok ? ld_stream(base + c * pstride + toff + (long long)i * (NB * g.n1)) : mk<T>(0, 0);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    DFT<NA, -1, T>::run(D[c]);
#pragma unroll
    for (int a = 1; a < NA; ++a) D[c][a] = cmul(D[c][a], tw[(t * a) % N]);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) lds[a * RS + w * NB + t] = D[c][a];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) D[c][j * NB + u] = lds[a * RS + w * NB + u];
        DFT<NB, -1, T>::run(&D[c][j * NB]);
      }
    }
  }

  // ---- per-frequency projection
  const int k1c = ok ? k1 : 0;
  const T s1 = ft.s[1][k1c], c1 = ft.c[1][k1c], s2 = ft.s[2][k2], c2 = ft.c[2][k2];
  const T c1c2 = c1 * c2, s1c2 = s1 * c2, c1s2 = c1 * s2;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int e = j * NB + b;
        const int k0 = a + NA * b;
        if (IDENT) {
#pragma unroll
          for (int c = 0; c < 6; ++c) D[c][e] = scl(D[c][e], inv_total);
        } else {
          const T s0 = ft.s[0][k0], c0 = ft.c[0][k0];
          const T w0 = s0 * c1c2, w1 = c0 * s1c2, w2 = c0 * c1s2;
          const int keep = (k0 | k1c | k2) == 0 ? ft.stress_mask : 0;
          project_mandel(D[0][e], D[1][e], D[2][e], D[3][e], D[4][e], D[5][e], w0, w1, w2, inv_total, keep);
        }
      }
    }
  }

  // ---- inverse along axis 0
#pragma unroll
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
        DFT<NB, 1, T>::run(&D[c][j * NB]);
        // D[c][j*NB + u] now holds Z_a[u], u = stage-A column index
        if (a > 0) {
#pragma unroll
          for (int u = 1; u < NB; ++u) D[c][j * NB + u] = cmulc(D[c][j * NB + u], tw[(u * a) % N]);
        }
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) lds[a * RS + w * NB + u] = D[c][j * NB + u];
      }
    }
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) D[c][a] = lds[a * RS + w * NB + t];
    DFT<NA, 1, T>::run(D[c]);
    if (ok) {
#pragma unroll
      for (int i = 0; i < NA; ++i) base[c * pstride + toff + (long long)i * (NB * g.n1)] = D[c][i];
    }
  }
}

// P3 with the six components split over two halves of the block (half h owns components 3h..3h+2),
// halving the registers per thread.  W*NB must be a multiple of the wave size (64) so that the half
// index is uniform per wave and the half-dependent branches are scalar.
// grid (ceil(N1/W), K2, ncases), block 2*W*NB threads, dyn. LDS
// 2*NA*(NB*W+1) complex (one transform exchange area per half, reused for the projection exchange),
// plus NA*NB complex in FP32 for a copy of the twiddle table.
// For the projection, half h takes the entries e of parity h: in three rounds (one component
// slot each) the halves swap the values of the entries the other half projects, so that a thread
// holds all six components of its entries (own ones in D[r][e], the other half's in the slot D[r][e^1]
// it has just sent), and three more rounds return the projected values.
template <typename T, int NA, int NB, bool IDENT>
__global__ __launch_bounds__(512) void k_axis0_project_split(cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw,
                                                             FreqTables<T> ft, GridDims g, int W, T inv_total,
                                                             const MinresState* __restrict__ st) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int E0 = (NA > CB * NB) ? NA : CB * NB;
  constexpr int E = E0 + (E0 & 1);  // even, so that every entry has a parity partner e ^ 1
  static_assert(E <= 2 * NA, "the projection exchange must fit the two transform exchange areas");
  extern __shared__ unsigned char smem_raw[];
  const int cs = blockIdx.z;
  if (st && st[cs].finish) return;
  // planes in descending k2: P2 (ascending rows) wrote the high planes last, so part of them is still in
  // the memory-side cache, and P4 (ascending again) then starts on the planes written last here
  const int k2 = g.k2 - 1 - (int)blockIdx.y;
  const int tid = threadIdx.x;
  const int WNB = W * NB;  // a multiple of 64: each half is whole waves, so h is wave-uniform
  const int q = tid % WNB, h = __builtin_amdgcn_readfirstlane(tid / WNB);
  const int t = q % NB, w = q / NB;  // a pencil's threads are adjacent lanes
  const int k1 = blockIdx.x * W + w;
  const bool ok = k1 < g.n1;
  const int RS = NB * W + 1;
  cx<T>* lds_all = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* lds = lds_all + h * NA * RS;
  const long long pstride = (long long)g.n0 * g.n1;
  cx<T>* base = spec + spec_t_plane(g, cs, k2, 3 * h) + spec_t_off(g, 0, ok ? k1 : 0);
  const long long toff = spec_t_off(g, t, 0);  // element t + NB i at toff + i NB n1 (tile divides NB)

  cx<T> D[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int i = 0; i < NA; ++i) D[c][i] = ok ? ld_stream(base + c * pstride + toff + (long long)i * (NB * g.n1)) : mk<T>(0, 0);
#pragma unroll
    for (int i = NA; i < E; ++i) D[c][i] = mk<T>(0, 0);
  }
  // FP32: the twiddles are read from a copy in LDS (behind the two exchange areas), which keeps them
  // out of the registers; FP64 reloads them from cache
  constexpr bool TWL = sizeof(T) == 4;
  cx<T>* twl = lds_all + 2 * NA * RS;
  if (TWL) {
    for (int i = tid; i < N; i += blockDim.x) twl[i] = tw[i];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    DFT<NA, -1, T>::run(D[c]);
#pragma unroll
    for (int a = 1; a < NA; ++a) D[c][a] = cmul(D[c][a], TWL ? twl[(t * a) % N] : tw[(t * a) % N]);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) lds[a * RS + w * NB + t] = D[c][a];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) D[c][j * NB + u] = lds[a * RS + w * NB + u];
        DFT<NB, -1, T>::run(&D[c][j * NB]);
      }
    }
  }

  const int k1c = ok ? k1 : 0;
  const T s1 = ft.s[1][k1c], c1 = ft.c[1][k1c], s2 = ft.s[2][k2], c2 = ft.c[2][k2];
  const T c1c2 = c1 * c2, s1c2 = s1 * c2, c1s2 = c1 * s2;
  if (IDENT) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) D[c][e] = scl(D[c][e], inv_total);
  } else {
    // entries of one parity are numbered e / 2; the value a half hw sends for entry e of thread q
    // sits at ((e / 2) * 2 + hw) * WNB + q (at most E * WNB <= 2 NA RS slots)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      lds_barrier();
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & 1) != h) lds_all[((e >> 1) * 2 + h) * WNB + q] = D[r][e];  // entries the other half projects
      lds_barrier();
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & 1) == h) D[r][e ^ 1] = lds_all[((e >> 1) * 2 + (1 - h)) * WNB + q];
    }
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int e = j * NB + b;
          if ((e & 1) != h) continue;
          const int k0 = a + NA * b;
          const T s0 = ft.s[0][k0], c0 = ft.c[0][k0];
          const T w0 = s0 * c1c2, w1 = c0 * s1c2, w2 = c0 * c1s2;
          const int keep = (k0 | k1c | k2) == 0 ? ft.stress_mask : 0;
          if (h == 0)
            project_mandel(D[0][e], D[1][e], D[2][e], D[0][e ^ 1], D[1][e ^ 1], D[2][e ^ 1], w0, w1, w2, inv_total,
                           keep);
          else
            project_mandel(D[0][e ^ 1], D[1][e ^ 1], D[2][e ^ 1], D[0][e], D[1][e], D[2][e], w0, w1, w2, inv_total,
                           keep);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      lds_barrier();
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & 1) == h) lds_all[((e >> 1) * 2 + h) * WNB + q] = D[r][e ^ 1];  // the other half's, projected
      lds_barrier();
#pragma unroll
      for (int e = 0; e < E; ++e)
        if ((e & 1) != h) D[r][e] = lds_all[((e >> 1) * 2 + (1 - h)) * WNB + q];
    }
  }

  // ---- inverse along axis 0
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
        DFT<NB, 1, T>::run(&D[c][j * NB]);
        if (a > 0) {
#pragma unroll
          for (int u = 1; u < NB; ++u)
            D[c][j * NB + u] = cmulc(D[c][j * NB + u], TWL ? twl[(u * a) % N] : tw[(u * a) % N]);
        }
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) lds[a * RS + w * NB + u] = D[c][j * NB + u];
      }
    }
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) D[c][a] = lds[a * RS + w * NB + t];
    DFT<NA, 1, T>::run(D[c]);
    if (ok) {
#pragma unroll
      for (int i = 0; i < NA; ++i) base[c * pstride + toff + (long long)i * (NB * g.n1)] = D[c][i];
    }
  }
}

// Projection step of the three-group P3 for group G (a compile-time constant, so that every register
// slot index is one).  Entry e is projected by group e % 3.  The value a non-owner group sends for
// entry e of lane q sits at slot (2 e + k) WNB + q, k = 0 for the group after the owner (mod 3), 1 for
// the one before; after the exchange D[r][3m + j] holds component 2j + r of the group's entry 3m + G
// (j = 0..2), and the projected values go back the same way.  Every group passes the same barriers.
template <typename T, int NA, int NB, int E, int G>
__device__ __forceinline__ void split3_project(cx<T> (&D)[2][E], cx<T>* lds_all, int WNB, int q, int t,
                                               const FreqTables<T>& ft, T c1c2, T s1c2, T c1s2, T inv_total,
                                               int keep0) {
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int GA = (G + 1) % 3, GB = (G + 2) % 3;  // the groups after and before G
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    lds_barrier();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int o = e % 3;
      if (o != G) lds_all[(e * 2 + (G == (o + 1) % 3 ? 0 : 1)) * WNB + q] = D[r][e];
    }
    lds_barrier();
#pragma unroll
    for (int m = 0; m < E / 3; ++m) {
      const int e = 3 * m + G;
      D[r][3 * m + GA] = lds_all[(e * 2 + 0) * WNB + q];
      D[r][3 * m + GB] = lds_all[(e * 2 + 1) * WNB + q];
    }
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int a = t + TT * j;
    if (a < NA) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int e = j * NB + b;
        if (e % 3 != G) continue;
        const int k0 = a + NA * b;
        const T s0 = ft.s[0][k0], c0 = ft.c[0][k0];
        const T w0 = s0 * c1c2, w1 = c0 * s1c2, w2 = c0 * c1s2;
        const int m3 = e - G;
        project_mandel(D[0][m3], D[1][m3], D[0][m3 + 1], D[1][m3 + 1], D[0][m3 + 2], D[1][m3 + 2], w0, w1, w2,
                       inv_total, k0 == 0 ? keep0 : 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    lds_barrier();
#pragma unroll
    for (int m = 0; m < E / 3; ++m) {
      const int e = 3 * m + G;
      lds_all[(e * 2 + 0) * WNB + q] = D[r][3 * m + GA];
      lds_all[(e * 2 + 1) * WNB + q] = D[r][3 * m + GB];
    }
    lds_barrier();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int o = e % 3;
      if (o != G) D[r][e] = lds_all[(e * 2 + (G == (o + 1) % 3 ? 0 : 1)) * WNB + q];
    }
  }
}

// P3 with the six components split over three groups of the block (group g owns components 2g and
// 2g+1): a third of the whole-pencil registers, which keeps the FP64 transform out of scratch.
// Each group is one wave (W*NB = 64).  grid (ceil(N1/W), K2, ncases), block 3*W*NB threads, dyn. LDS
// max(3*NA*(NB*W+1), 2*E*NB*W) complex (one transform exchange area per group, reused for the
// projection exchange).
template <typename T, int NA, int NB, bool IDENT>
__global__ __launch_bounds__(192) void k_axis0_project_split3(cx<T>* __restrict__ spec, const cx<T>* __restrict__ tw,
                                                              FreqTables<T> ft, GridDims g, int W, T inv_total,
                                                              const MinresState* __restrict__ st) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  constexpr int E0 = (NA > CB * NB) ? NA : CB * NB;
  constexpr int E = (E0 + 2) / 3 * 3;  // the host sizes LDS for max(3 NA (NB W + 1), 2 E NB W) complex
  extern __shared__ unsigned char smem_raw[];
  const int cs = blockIdx.z;
  if (st && st[cs].finish) return;
  const int k2 = g.k2 - 1 - (int)blockIdx.y;  // descending, as the other P3 variants
  const int tid = threadIdx.x;
  const int WNB = W * NB;  // 64: the group index is wave-uniform
  const int q = tid % WNB, grp = __builtin_amdgcn_readfirstlane(tid / WNB);
  const int t = q % NB, w = q / NB;
  const int k1 = blockIdx.x * W + w;
  const bool ok = k1 < g.n1;
  const int RS = NB * W + 1;
  cx<T>* lds_all = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* lds = lds_all + grp * NA * RS;
  const long long pstride = (long long)g.n0 * g.n1;
  cx<T>* base = spec + spec_t_plane(g, cs, k2, 2 * grp) + spec_t_off(g, 0, ok ? k1 : 0);
  const long long toff = spec_t_off(g, t, 0);  // element t + NB i at toff + i NB n1 (tile divides NB)

  cx<T> D[2][E];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int i = 0; i < NA; ++i) D[c][i] = ok ? ld_stream(base + c * pstride + toff + (long long)i * (NB * g.n1)) : mk<T>(0, 0);
#pragma unroll
    for (int i = NA; i < E; ++i) D[c][i] = mk<T>(0, 0);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    DFT<NA, -1, T>::run(D[c]);
#pragma unroll
    for (int a = 1; a < NA; ++a) D[c][a] = cmul(D[c][a], tw[(t * a) % N]);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) lds[a * RS + w * NB + t] = D[c][a];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) D[c][j * NB + u] = lds[a * RS + w * NB + u];
        DFT<NB, -1, T>::run(&D[c][j * NB]);
      }
    }
  }

  const int k1c = ok ? k1 : 0;
  const T s1 = ft.s[1][k1c], c1 = ft.c[1][k1c], s2 = ft.s[2][k2], c2 = ft.c[2][k2];
  const T c1c2 = c1 * c2, s1c2 = s1 * c2, c1s2 = c1 * s2;
  if (IDENT) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) D[c][e] = scl(D[c][e], inv_total);
  } else {
    // the stress-controlled components survive the projection only at xi = 0 (k0 = 0 is checked inside)
    const int keep0 = (k1c | k2) == 0 ? ft.stress_mask : 0;
    if (grp == 0)
      split3_project<T, NA, NB, E, 0>(D, lds_all, WNB, q, t, ft, c1c2, s1c2, c1s2, inv_total, keep0);
    else if (grp == 1)
      split3_project<T, NA, NB, E, 1>(D, lds_all, WNB, q, t, ft, c1c2, s1c2, c1s2, inv_total, keep0);
    else
      split3_project<T, NA, NB, E, 2>(D, lds_all, WNB, q, t, ft, c1c2, s1c2, c1s2, inv_total, keep0);
  }

  // ---- inverse along axis 0
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
        DFT<NB, 1, T>::run(&D[c][j * NB]);
        if (a > 0) {
#pragma unroll
          for (int u = 1; u < NB; ++u) D[c][j * NB + u] = cmulc(D[c][j * NB + u], tw[(u * a) % N]);
        }
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
#pragma unroll
        for (int u = 0; u < NB; ++u) lds[a * RS + w * NB + u] = D[c][j * NB + u];
      }
    }
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) D[c][a] = lds[a * RS + w * NB + t];
    DFT<NA, 1, T>::run(D[c]);
    if (ok) {
#pragma unroll
      for (int i = 0; i < NA; ++i) base[c * pstride + toff + (long long)i * (NB * g.n1)] = D[c][i];
    }
  }
}

// ============================================================================ P5
// grid (ceil(N1/W), N0, ncases), block W*NB threads, dyn. LDS W*max(NA*(NB+1), N+1) complex
// Lanczos mode (uk != nullptr, MINRES iterations): the transform output p = A v_k is never stored;
// instead y = u_{k+1} = p - cu_v u_k - cu_vp u_{k-1} is written with per-block ||u_{k+1}||^2 partials.
template <typename T, int NA, int NB>
__global__ __launch_bounds__(256) void k_inv_axis2(const cx<T>* __restrict__ spec, T* __restrict__ y,
                                                   const T* __restrict__ uk, const T* __restrict__ ukm1,
                                                   double* partials, const cx<T>* __restrict__ tw, GridDims g, int W,
                                                   const MinresState* __restrict__ st) {
  constexpr int N = NA * NB;
  constexpr int TT = NB;
  constexpr int CB = (NA + TT - 1) / TT;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  __shared__ double red[16];
  const int cs = blockIdx.z;
  if (st && st[cs].finish) return;
  const int n0 = blockIdx.y;
  const int n1_0 = blockIdx.x * W;
  const int tid = threadIdx.x;
  const int t = tid % TT, w = tid / TT;
  const int n1 = n1_0 + w;
  const bool row_ok = n1 < g.n1;
  const int ws = tid % W, m = tid / W, M = blockDim.x / W;
  const int n1s = n1_0 + ws;
  const long long row = ((long long)n0 * g.n1 + n1) * N;
  T* yc = y + (long long)cs * 6 * g.nvox;
  const bool lz = uk != nullptr;
  const T* uc = lz ? uk + (long long)cs * 6 * g.nvox : nullptr;
  const T* umc = lz ? ukm1 + (long long)cs * 6 * g.nvox : nullptr;
  const T cv = lz ? (T)st[cs].cu_v : (T)0, cvp = lz ? (T)st[cs].cu_vp : (T)0;
  double acc = 0.0;
  // spectrum components this thread gathers, one pair ahead of the transform that uses them
  constexpr int LK = (N / 2 + 1 + TT - 1) / TT;
  cx<T> sp[6][LK];
  auto gather_pair = [&](int p2) {
#pragma unroll
    for (int l = 0; l < LK; ++l) {
      const int k = m + M * l;
#pragma unroll
      for (int c = 2 * p2; c < 2 * p2 + 2; ++c)
        sp[c][l] = (n1s < g.n1 && k < g.k2) ? ld_stream(spec + spec_idx(g, cs, k, c, n0, n1s)) : mk<T>(0, 0);
    }
  };
  // Lanczos operands (combination c u_k + c' u_{k-1}) of a pair, fetched early: one pair ahead in
  // FP32 where the CB*NB*2 extra registers leave the waves per SIMD unchanged (NA >= 15: the kernel
  // holds two waves per SIMD either way, at 200-250 VGPRs), else at the start of the pair (smaller NA
  // would drop from four or three waves per SIMD, larger CB*NB to one; FP64 gains nothing)
  constexpr bool DV_AHEAD = sizeof(T) == 4 && NA >= 15 && CB * NB <= 16;
  T dvs[DV_AHEAD ? 3 : 1][CB][NB][2];
  auto load_dv = [&](int p2) {
    if (lz && row_ok) {
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int a = t + TT * j;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const long long o = row + a + NA * b;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const long long oo = (2 * p2 + h) * g.nvox + o;
            dvs[DV_AHEAD ? p2 : 0][j][b][h] = (CB == 1 || a < NA) ? cv * ld_stream_wide(uc + oo) + cvp * ld_stream_wide(umc + oo) : (T)0;
          }
        }
      }
    }
  };
  if constexpr (DV_AHEAD) load_dv(0);
  gather_pair(0);
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    if (pr < 2) gather_pair(pr + 1);
    T dvl[DV_AHEAD ? 1 : CB][NB][2];
    if constexpr (DV_AHEAD) {
      if (pr < 2) load_dv(pr + 1);
    } else {
      if (lz && row_ok) {
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          const int a = t + TT * j;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const long long o = row + a + NA * b;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const long long oo = (2 * pr + h) * g.nvox + o;
              dvl[j][b][h] = (CB == 1 || a < NA) ? cv * ld_stream_wide(uc + oo) + cvp * ld_stream_wide(umc + oo) : (T)0;
            }
          }
        }
      }
    }
    auto& dv = pick<DV_AHEAD>(dvs[DV_AHEAD ? pr : 0], dvl);
    lds_barrier();
    if (n1s < g.n1) {
#pragma unroll
      for (int l = 0; l < LK; ++l) {
        const int k = m + M * l;
        if (k < g.k2) {
          const cx<T> A = sp[2 * pr][l];
          const cx<T> B = sp[2 * pr + 1][l];
          if (k == 0 || 2 * k == N) {
            lds[ws * (N + 1) + k] = mk<T>(A.re, B.re);
          } else {
            lds[ws * (N + 1) + k] = mk<T>(A.re - B.im, A.im + B.re);
            lds[ws * (N + 1) + N - k] = mk<T>(A.re + B.im, B.re - A.im);
          }
        }
      }
    }
    lds_barrier();
    cx<T> z[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) z[i] = lds[w * (N + 1) + t + NB * i];
    DFT<NA, 1, T>::run(z);
#pragma unroll
    for (int a = 1; a < NA; ++a) z[a] = cmulc(z[a], tw[(t * a) % N]);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < NA; ++a) lds[(w * NA + a) * (NB + 1) + t] = z[a];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int a = t + TT * j;
      if (a < NA) {
        cx<T> yb[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) yb[u] = lds[(w * NA + a) * (NB + 1) + u];
        DFT<NB, 1, T>::run(yb);
        if (row_ok) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const long long o = row + a + NA * b;
            T r0 = yb[b].re, r1 = yb[b].im;
            if (lz) {
              r0 -= dv[j][b][0];
              r1 -= dv[j][b][1];
              acc += (double)r0 * (double)r0 + (double)r1 * (double)r1;
            }
            yc[(2 * pr) * g.nvox + o] = r0;
            yc[(2 * pr + 1) * g.nvox + o] = r1;
          }
        }
      }
    }
  }
  if (lz) {
    const unsigned nb = gridDim.x * gridDim.y;
    const double sblk = block_sum(acc, red);
    if (tid == 0) partials[(long long)cs * nb + blockIdx.y * gridDim.x + blockIdx.x] = sblk;
  }
}

}  // namespace rve
