// Host driver and Krylov kernels of the gfx950 Galerkin-FFT homogenization solver (C ABI in rve.h).
//
// One MINRES iteration is seven launches, no host involvement:
//   P1 stiffness + FFT axis 2, with per-block partials of alpha = <v, C v>
//   P2, P3 (projection), P4 transforms; S1 (alpha from P1's partials) runs in extra blocks of P2
//   P5 inverse FFT axis 2 fused with the Lanczos three-term update and ||u_{k+1}||^2 partials
//   S2 Givens QR step + convergence test (one block);  U2 search direction + solution update, on a
//   second stream beside the next iteration's P3 (see U2Side).
// Vectors carry a deferred normalisation: the Lanczos vector v_k is stored unscaled (u_k) and its
// 1/beta_k is applied inside the consumers (P1 stiffness, P5 update, U2).
// FP32_MIXED: fields and transforms in FP32, Krylov scalars and all inner products in FP64; the
// outer loop recomputes the true residual with FP64 operator kernels and refines (x64 += delta).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/rve.h"
#include "../../include/rve_j2.h"
#include "rve_registry.h"

namespace rve {

// ============================================================================ registry
static std::vector<LenEntry>& registry() {
  static std::vector<LenEntry> r;
  return r;
}
void register_len(const LenEntry& e) { registry().push_back(e); }
// The v-th registered factorisation of length n (v = 0: the default, the first registered).
const LenEntry* find_len(int n, int v) {
  for (const auto& e : registry())
    if (e.n == n && v-- == 0) return &e;
  return nullptr;
}
static int len_variants(int n) {
  int k = 0;
  for (const auto& e : registry()) k += e.n == n;
  return k;
}
void register_group_a();
void register_group_b();
void register_group_c();
void register_group_d();
void register_group_e();
void register_group_f();
void register_group_g();
void register_group_h();
extern "C" int32_t rve_load_tuning(const char* path);
static void ensure_registry() {
  static std::once_flag once;
  std::call_once(once, [] {
    register_group_a();
    register_group_b();
    register_group_c();
    register_group_d();
    register_group_e();
    register_group_f();
    register_group_g();
    register_group_h();
    const char* f = getenv("RVE_TUNE_FILE");
    if (f && f[0]) rve_load_tuning(f);
  });
}
const LenEntry* lookup_len(int n) {
  ensure_registry();
  return find_len(n, 0);
}

// ============================================================================ per-kernel timing
// Optional HIP-event timing of every launch inside the MINRES iteration loop (on the solve stream).
// Events come from a pool created on first enable; pairs are read back at the host's chunk syncs.
namespace prof {
enum Kind { P1 = 0, P2, P3, P4, P5, S1, S2, U2, NKIND };
// kinds 0..NKIND-1 time passes on FP32 fields, NKIND..2 NKIND-1 the same passes on FP64 fields,
// then the phase-map kernels (FP64 only)
constexpr int NGEO = 6;
constexpr int NSLOT = 2 * NKIND + NGEO;
static const char* kNames[NSLOT] = {
    "P1_stiffness_fft_axis2_alpha",     "P2_fft_axis1",     "P3_fft_axis0_projection",
    "P4_ifft_axis1",                    "P5_ifft_axis2_lanczos", "S1_alpha", "S2_givens", "U2_direction_update",
    "P1_stiffness_fft_axis2_alpha_f64", "P2_fft_axis1_f64", "P3_fft_axis0_projection_f64",
    "P4_ifft_axis1_f64",                "P5_ifft_axis2_lanczos_f64", "S1_alpha_f64", "S2_givens_f64",
    "U2_direction_update_f64",          "G1_source_fft_axis2", "G2_fft_axis1", "G3_fft_axis0_helmholtz",
    "G4_ifft_axis1",                    "G5_ifft_axis2_coarsen", "M_phase_map"};
static std::atomic<bool> on{false};
static std::vector<hipEvent_t> pool;
static std::vector<std::pair<int, int>> pending;
static size_t next = 0;
static double ms[NSLOT];
static long long cnt[NSLOT];
static long long dropped = 0;
static std::mutex mu;
static inline void begin_slot(int kind, hipStream_t s);
template <typename T>
static inline void begin(int kind, hipStream_t s) {
  if (!on) return;
  begin_slot(sizeof(T) == 8 ? kind + NKIND : kind, s);
}
static inline void begin_slot(int kind, hipStream_t s) {
  if (!on) return;
  std::lock_guard<std::mutex> lk(mu);
  if (next + 2 > pool.size()) {
    dropped++;
    return;
  }
  hipEventRecord(pool[next], s);
  pending.push_back({kind, (int)next});
  next += 2;
}
static inline void end(hipStream_t s) {
  if (!on) return;
  std::lock_guard<std::mutex> lk(mu);
  if (pending.empty() || (size_t)pending.back().second + 1 != next - 1) return;
  hipEventRecord(pool[pending.back().second + 1], s);
}
static void read_pairs(const std::vector<std::pair<int, int>>& pairs) {
  if (!on) return;
  for (auto& pe : pairs) {
    float t = 0.f;
    if (hipEventSynchronize(pool[pe.second + 1]) == hipSuccess &&
        hipEventElapsedTime(&t, pool[pe.second], pool[pe.second + 1]) == hipSuccess) {
      ms[pe.first] += t;
      cnt[pe.first] += 1;
    }
  }
}
static void flush() {
  if (!on) return;
  std::lock_guard<std::mutex> lk(mu);
  read_pairs(pending);
  pending.clear();
  next = 0;
}
}  // namespace prof

// timing hooks of the phase-map kernels (kinds G1..G5, M in launch order)
void geo_prof_begin(int g, hipStream_t s) { prof::begin_slot(2 * prof::NKIND + g, s); }
void geo_prof_end(hipStream_t s) { prof::end(s); }
void geo_prof_flush() { prof::flush(); }

}  // namespace rve

#include "rve_solver_kernels.h"

namespace rve {

// ============================================================================ plan + workspace
static long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

struct Tiles {
  int W1, W3, R2;       // P1/P5 row tile, P3 pencil tile, P2/P4 rows per block
  int S3 = 2;           // P3 component split: 1 = all six per thread, 2 = three per thread (two block halves),
                        // 3 = two per thread (three one-wave groups)
  int F[3] = {0, 0, 0};  // factorisation (registry variant) of each axis length
};
struct Plan {
  int n[3];
  GridDims g;
  const LenEntry* ax[2][3];     // per precision ([0] FP32, [1] FP64) and axis: the kernels in use
  Tiles t[2];                   // [0] FP32 kernels, [1] FP64 kernels
  long long lds_cap3 = 65536;   // dynamic LDS limit of the P3 kernels (the device's per-block maximum)
};
static const LenEntry* axis(const Plan& pl, int elem, int p) { return pl.ax[elem == 8][p]; }

// Tuned tiles per (grid, precision), filled by rve_autotune / rve_load_tuning.
struct TuneKey {
  int n0, n1, n2, elem;
  bool operator==(const TuneKey& o) const { return n0 == o.n0 && n1 == o.n1 && n2 == o.n2 && elem == o.elem; }
};
static std::vector<std::pair<TuneKey, Tiles>>& tuned() {
  static std::vector<std::pair<TuneKey, Tiles>> t;
  return t;
}
static std::mutex g_tune_mutex;
static bool find_tuned(const TuneKey& k, Tiles* out) {
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  for (auto& e : tuned())
    if (e.first == k) {
      *out = e.second;
      return true;
    }
  return false;
}
static void set_tuned(const TuneKey& k, const Tiles& t) {
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  for (auto& e : tuned())
    if (e.first == k) {
      e.second = t;
      return;
    }
  tuned().push_back({k, t});
}

static int pick_tile(int threads_per_row, int len) {
  int W = std::max(1, std::min(64, 256 / threads_per_row));
  while (W > 1 && W / 2 >= len) W /= 2;  // do not tile far beyond the axis length
  return W;
}

// Largest tile not above the plan's choice with at most 256 threads per block (per half for the
// split P3) and dynamic LDS within 64 KiB (P1/P5, P2/P4) or the device limit (P3).
constexpr long long kLdsCap = 64 * 1024;
static int tile_p1(const Plan& pl, int elem) {
  const int na = axis(pl, elem, 2)->na, nb = axis(pl, elem, 2)->nb;
  int W = pl.t[elem == 8].W1;
  while (W > 1 && (W * nb > 256 || 2LL * elem * W * std::max(na * (nb + 1), pl.g.n2 + 1) > kLdsCap)) W /= 2;
  return W;
}
// P3 may use the device's whole per-block LDS (160 KiB on gfx950): the split kernel's two exchange
// areas need just over 64 KiB for 16 pencils of 256 (the tuner usually takes 4-8 on the tiled copy).
static int tile_p3_for(const Plan& pl, int elem, int sp) {
  const int na = axis(pl, elem, 0)->na, nb = axis(pl, elem, 0)->nb;
  if (sp == 3) return 64 / nb;  // one wave per component group
  int W = pl.t[elem == 8].W3;
  // LDS of the split variants: the exchange areas, and in FP32 the twiddle table of the two-way split
  auto lds_bytes = [&](int w) {
    return sp * 2LL * elem * na * (nb * w + 1) + (sp == 2 && elem == 4 ? 2LL * elem * na * nb : 0);
  };
  while (W > 1 && (W * nb > 256 || lds_bytes(W) > pl.lds_cap3)) W /= 2;
  return W;
}
// LDS (complex elements) of the three-group P3 at tile W: the larger of its three transform exchange
// areas and its projection exchange.
static long long lds_p3_split3(int na, int nb, int W) {
  const int cb = (na + nb - 1) / nb;
  const int e0 = std::max(na, cb * nb), e = (e0 + 2) / 3 * 3;
  return std::max(3LL * na * (nb * W + 1), 2LL * e * nb * W);
}
// The split variants need each block part (W*NB threads) to be whole waves; otherwise whole pencils.
// A three-group request falls back to halves (then whole pencils) where NB does not divide 64 or the
// LDS does not fit.
static int split_p3(const Plan& pl, int elem) {
  const int req = pl.t[elem == 8].S3;
  if (req == 1) return 1;
  const int na = axis(pl, elem, 0)->na, nb = axis(pl, elem, 0)->nb;
  if (req == 3 && 64 % nb == 0 && 2LL * elem * lds_p3_split3(na, nb, 64 / nb) <= pl.lds_cap3) return 3;
  const int W = tile_p3_for(pl, elem, 2);
  return (W * nb) % 64 == 0 ? 2 : 1;
}
static int tile_p3(const Plan& pl, int elem) { return tile_p3_for(pl, elem, split_p3(pl, elem)); }
static int rows_p2(const Plan& pl, int elem) {
  const int na = axis(pl, elem, 1)->na, nb = axis(pl, elem, 1)->nb;
  int R = pl.t[elem == 8].R2;
  while (R > 1 && (R * nb > 256 || 2LL * elem * R * (na * (nb + 1) + 1) > kLdsCap)) R /= 2;
  return R;
}

// Kernel entries of every axis for each precision from the tiles' factorisation choice (an unknown
// variant falls back to the default).
static void select_axes(Plan* pl) {
  for (int e = 0; e < 2; ++e)
    for (int p = 0; p < 3; ++p) {
      const LenEntry* a = find_len(pl->n[p], pl->t[e].F[p]);
      if (!a) {
        pl->t[e].F[p] = 0;
        a = find_len(pl->n[p], 0);
      }
      pl->ax[e][p] = a;
    }
}

static bool make_plan(const rve_grid* grid, Plan* pl) {
  ensure_registry();
  for (int p = 0; p < 3; ++p) {
    pl->n[p] = grid->n[p];
    if (!find_len(grid->n[p])) return false;
  }
  GridDims& g = pl->g;
  g.n0 = pl->n[0];
  g.n1 = pl->n[1];
  g.n2 = pl->n[2];
  g.k2 = g.n2 / 2 + 1;
  g.nvox = (long long)g.n0 * g.n1 * g.n2;
  g.tile = 1;  // set per apply from the axis-0 factorisation in use (apply_op)
  g.tile_shift = 0;
  g.spec_case = 6LL * g.k2 * g.n0 * g.n1;
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      pl->lds_cap3 = std::min<long long>(lds, 160 * 1024);
    else
      (void)hipGetLastError();  // no device (host-only queries): keep 64 KiB
  }
  for (int e = 0; e < 2; ++e) {
    Tiles& t = pl->t[e];
    const LenEntry* a0 = find_len(pl->n[0]);
    const LenEntry* a1 = find_len(pl->n[1]);
    const LenEntry* a2 = find_len(pl->n[2]);
    t.W1 = pick_tile(a2->nb, g.n1);
    t.W3 = pick_tile(a0->nb, g.n1);
    t.R2 = std::max(1, std::min(64, 256 / a1->nb));
    Tiles tt;
    if (find_tuned(TuneKey{g.n0, g.n1, g.n2, e ? 8 : 4}, &tt)) t = tt;
  }
  select_axes(pl);
  return true;
}

template <typename T>
struct Tables {
  cx<T>* tw[3];
  T* s[3];
  T* c[3];
  int stress_mask = 0;  // mixed control: Mandel components the projection keeps at xi = 0
};

// Workspace carve-out.  Sizes depend only on (grid, n_cases, precision).
struct Layout {
  long long off_state, off_info, off_part, off_sums, off_tab32, off_tab64, off_u32[3], off_d32[2], off_x32,
      off_spec32, off_x64, off_b64, off_r64, off_t64, off_spec64, off_u64[3], off_d64[2], off_flag, total;
  int np_p5, np_vec, np_post;
};

static long long tab_bytes(const Plan& pl, int elem) {
  long long b = 0;
  for (int p = 0; p < 3; ++p) b += align_up((long long)pl.n[p] * (2 * elem) + 2LL * pl.n[p] * elem + 64, 256);
  return b;
}

static Layout make_layout(const Plan& pl, int nc, int precision, bool solve) {
  Layout L;
  memset(&L, 0, sizeof(L));
  const GridDims& g = pl.g;
  const long long n6 = 6 * g.nvox * nc;
  L.np_p5 = g.n0 * g.n1;  // P1/P5 blocks at the narrowest possible tile (W = 1): any tuned tile fits
  L.np_vec = kRedBlocks;
  L.np_post = 6 * kRedBlocks;
  const int np_max = std::max(std::max(L.np_p5, L.np_vec), L.np_post);
  long long o = 0;
  auto take = [&](long long bytes) {
    long long r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  L.off_state = take(sizeof(MinresState) * nc);
  L.off_info = take(sizeof(CaseInfo) * nc);
  L.off_part = take(sizeof(double) * (long long)np_max * nc);
  L.off_sums = take(sizeof(double) * 16 * nc);
  L.off_flag = take(64);
  L.off_tab32 = take(tab_bytes(pl, 4));
  L.off_tab64 = take(tab_bytes(pl, 8));
  if (precision == RVE_FP32_MIXED) {
    L.off_spec32 = take(2 * 8 * g.spec_case * nc);  // plane-major half spectrum + P3's tiled copy
    if (solve) {
      for (int i = 0; i < 3; ++i) L.off_u32[i] = take(4 * n6);
      for (int i = 0; i < 2; ++i) L.off_d32[i] = take(4 * n6);
      L.off_x32 = take(4 * n6);
    }
  } else if (solve) {
    for (int i = 0; i < 3; ++i) L.off_u64[i] = take(8 * n6);
    for (int i = 0; i < 2; ++i) L.off_d64[i] = take(8 * n6);
  }
  if (solve || precision == RVE_FP64) L.off_spec64 = take(2 * 16 * g.spec_case * nc);
  if (solve) {
    L.off_x64 = take(8 * n6);
    L.off_b64 = take(8 * n6);
    L.off_r64 = take(8 * n6);
    if (precision == RVE_FP32_MIXED) L.off_t64 = take(8 * n6);
  }
  L.total = o;
  return L;
}

template <typename T>
static Tables<T> tables_at(const Plan& pl, char* base) {
  Tables<T> t;
  for (int p = 0; p < 3; ++p) {
    t.tw[p] = reinterpret_cast<cx<T>*>(base);
    t.s[p] = reinterpret_cast<T*>(base + sizeof(cx<T>) * pl.n[p]);
    t.c[p] = t.s[p] + pl.n[p];
    base += align_up((long long)pl.n[p] * (2 * sizeof(T)) + 2LL * pl.n[p] * sizeof(T) + 64, 256);
  }
  return t;
}

// Text of the last HIP failure seen by this library (for diagnostics; see rve_last_error()).
static thread_local char g_last_error[256] = "";
struct LastInfo {
  double r0_rel = 0.0;
  int warm_rejected = 0;
  double mean_strain[6] = {0, 0, 0, 0, 0, 0};  // total macroscopic strain Ebar + <eps>
};
static thread_local std::vector<LastInfo> g_last_info;  // per case, last solve_rve on this thread
static void note_hip_error(hipError_t e, const char* expr, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (%d) in '%s' at rve_solver.hip:%d", hipGetErrorString(e), (int)e,
           expr, line);
}
void set_last_error(const char* text) { snprintf(g_last_error, sizeof(g_last_error), "%s", text); }
#define HIPCHK(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) {                \
      note_hip_error(e_, #x, __LINE__);    \
      return RVE_EDEVICE;                  \
    }                                      \
  } while (0)

template <typename T>
static rve_status build_tables(const Plan& pl, const rve_grid* grid, char* base, int scheme, int nyq, hipStream_t s) {
  Tables<T> t = tables_at<T>(pl, base);
  for (int p = 0; p < 3; ++p) {
    const double h = grid->L[p] / pl.n[p];
    hipLaunchKernelGGL(k_tables<T>, dim3((pl.n[p] + 255) / 256), dim3(256), 0, s, t.tw[p], t.s[p], t.c[p], pl.n[p], h,
                       scheme, nyq);
  }
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

// Exactly isotropic Mandel stiffness lam 1(x)1 + mu2 I (lam = C01, mu2 = C33, bitwise): the P1 fast path.
static bool isotropic_form(const double* C, double* lam, double* mu2) {
  *lam = C[1];
  *mu2 = C[21];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double want = 0.0;
      if (i < 3 && j < 3) want = (i == j) ? *lam + *mu2 : *lam;
      else if (i == j) want = *mu2;
      if (C[i * 6 + j] != want) return false;
    }
  return true;
}

template <typename T>
static Material<T> make_material(const double* Cvoid, const double* Csolid) {
  Material<T> m;
  memset(&m, 0, sizeof(m));
  bool any = false;
  double Cd[36];
  for (int i = 0; i < 36; ++i) {
    m.C0[i] = (T)Cvoid[i];
    Cd[i] = Csolid[i] - Cvoid[i];
    m.Cd[i] = (T)Cd[i];
    any = any || Cvoid[i] != 0.0;
  }
  m.has_c0 = any ? 1 : 0;
  m.use_phi = 1;
  double lam, mu2;
  if (isotropic_form(Cd, &lam, &mu2)) {
    m.iso_d = 1;
    m.lam_d = (T)lam;
    m.mu2_d = (T)mu2;
  }
  if (isotropic_form(Cvoid, &lam, &mu2)) {
    m.iso_0 = 1;
    m.lam_0 = (T)lam;
    m.mu2_0 = (T)mu2;
  }
  return m;
}

// ---------------------------------------------------------------------------- operator apply
// y = F^{-1}{ Ghat : F{ C(x) : xs * x } } for nc cases.
// Lanczos mode (uk != nullptr): P1 also forms alpha, P5 writes u_{k+1} instead of A x and performs the
// Givens step (see rve_kernels.h); the partials buffer is then required.
template <typename T>
static void apply_op(const Plan& pl, int nc, const T* x, const double* xscale, const float* phi,
                     const Material<T>& mat, const Tables<T>& tb, cx<T>* spec, T* y, const T* uk, const T* ukm1,
                     double* partials, MinresState* st, int identity, hipStream_t s, int u2_slot = 0,
                     hipEvent_t before_p5 = nullptr, hipEvent_t after_p2 = nullptr) {
  constexpr int el = (int)sizeof(T);
  const LenKernels<T>& K0 = axis(pl, el, 0)->k<T>();
  const LenKernels<T>& K1 = axis(pl, el, 1)->k<T>();
  const LenKernels<T>& K2 = axis(pl, el, 2)->k<T>();
  const int na2 = axis(pl, el, 2)->na, nb2 = axis(pl, el, 2)->nb;
  const int na1 = axis(pl, el, 1)->na, nb1 = axis(pl, el, 1)->nb;
  const int na0 = axis(pl, el, 0)->na, nb0 = axis(pl, el, 0)->nb;
  // tile of P3's spectrum copy: the largest power of two (<= 16) dividing both n0 and the threads
  // per pencil, so that a thread's pencil elements t + nb0 i sit at a fixed stride in the copy
  GridDims g = pl.g;
  while (g.tile < 16 && g.n0 % (2 * g.tile) == 0 && nb0 % (2 * g.tile) == 0) {
    g.tile *= 2;
    g.tile_shift++;
  }
  const int N2 = g.n2;
  const int elem = (int)sizeof(T);
  int s1_np = 0;  // P1 blocks (alpha partials per case), summed by S1 inside P2
  // P1
  {
    const int W = tile_p1(pl, elem);
    const size_t lds = sizeof(cx<T>) * (W * std::max(na2 * (nb2 + 1), N2 + 1) + (elem == 4 ? N2 : 0));
    dim3 grid((g.n1 + W - 1) / W, g.n0, nc);
    prof::begin<T>(prof::P1, s);
    hipLaunchKernelGGL(mat.tan ? K2.p1t : K2.p1, grid, dim3(W * nb2), lds, s, x, xscale, (int)(sizeof(MinresState) / sizeof(double)),
                       phi, mat, spec, tb.tw[2], g, W, st, uk ? partials : nullptr);
    prof::end(s);
    s1_np = (int)(grid.x * grid.y);
  }
  // P2 (rows of spec -> P3's tiled copy, the second half of the spectrum buffer)
  const long long rows = (long long)nc * g.k2 * 6 * g.n0;
  cx<T>* spec_t = spec + (long long)nc * g.spec_case;
  {
    const int R = rows_p2(pl, elem);
    // in MINRES iterations P2's first nc blocks run S1 (alpha_k from P1's partials), in 256 doubles of LDS
    const int s1b = uk ? nc : 0;
    const size_t lds = std::max<size_t>(sizeof(cx<T>) * (R * (na1 * (nb1 + 1) + 1) + (elem == 4 ? na1 * nb1 : 0)),
                                        s1b ? 256 * sizeof(double) : 0);
    prof::begin<T>(prof::P2, s);
    hipLaunchKernelGGL(K1.p2f, dim3((unsigned)((rows + R - 1) / R + s1b)), dim3(R * nb1), lds, s, spec, spec_t,
                       tb.tw[1], g, R, rows, st, uk ? st : nullptr, uk ? partials : nullptr, s1_np, s1b);
    prof::end(s);
    if (after_p2) (void)hipEventRecord(after_p2, s);
  }
  // P3
  {
    const int W = tile_p3(pl, elem);
    const int sp = split_p3(pl, elem);
    const size_t lds = sizeof(cx<T>) * (sp == 3 ? lds_p3_split3(na0, nb0, W)
                                                : (long long)sp * na0 * (nb0 * W + 1) +
                                                      (sp == 2 && elem == 4 ? (long long)na0 * nb0 : 0));
    FreqTables<T> ft;
    for (int p = 0; p < 3; ++p) {
      ft.s[p] = tb.s[p];
      ft.c[p] = tb.c[p];
    }
    ft.stress_mask = tb.stress_mask;
    dim3 grid((g.n1 + W - 1) / W, g.k2, nc);
    prof::begin<T>(prof::P3, s);
    const P3Fn<T> fn = sp == 3   ? (identity ? K0.p3t_ident : K0.p3t)
                       : sp == 2 ? (identity ? K0.p3s_ident : K0.p3s)
                                 : (identity ? K0.p3_ident : K0.p3);
    hipLaunchKernelGGL(fn, grid, dim3(sp * W * nb0), lds, s, spec_t, tb.tw[0], ft, g, W, (T)(1.0 / (double)g.nvox),
                       st);
    prof::end(s);
  }
  // P4 (P3's tiled copy -> rows of spec)
  {
    const int R = rows_p2(pl, elem);
    const size_t lds = sizeof(cx<T>) * (R * (na1 * (nb1 + 1) + 1) + (elem == 4 ? na1 * nb1 : 0));
    prof::begin<T>(prof::P4, s);
    hipLaunchKernelGGL(K1.p2i, dim3((unsigned)((rows + R - 1) / R)), dim3(R * nb1), lds, s, spec, spec_t, tb.tw[1], g,
                       R, rows, st, (MinresState*)nullptr, (const double*)nullptr, 0, 0);
    prof::end(s);
  }
  // P5
  {
    const int W = tile_p1(pl, elem);
    const size_t lds = sizeof(cx<T>) * W * std::max(na2 * (nb2 + 1), N2 + 1);
    dim3 grid((g.n1 + W - 1) / W, g.n0, nc);
    // P5 overwrites the field an earlier iteration's U2 (second stream) may still be reading
    if (before_p5) (void)hipStreamWaitEvent(s, before_p5, 0);
    prof::begin<T>(prof::P5, s);
    hipLaunchKernelGGL(K2.p5, grid, dim3(W * nb2), lds, s, spec, y, uk, ukm1, partials, tb.tw[2], g, W, st);
    prof::end(s);
    if (uk) {
      prof::begin<T>(prof::S2, s);
      hipLaunchKernelGGL(k_minres_givens, dim3(nc), dim3(256), 0, s, st, partials, (int)(grid.x * grid.y),
                         u2_slot);
    }
    prof::end(s);
  }
}

// ---------------------------------------------------------------------------- MINRES driver
template <typename T>
struct MinresBufs {
  T* u[3];
  T* d[2];
  T* x;
};

static void vec_grid(int nc, dim3* grid, dim3* block) {
  *grid = dim3(kRedBlocks, nc);
  *block = dim3(kThreads);
}

// U2 of iteration k depends only on S2(k) and on U2(k-1); the next iteration's operator passes do not
// read what it writes.  So it runs on a second stream (default priority) beside them, filling the
// memory bandwidth the latency-bound P3 leaves unused.  Ordering: U2(k) after P2(k+1) (hence after
// S2(k)); P5(k+2) after U2(k) (P5(k+2) overwrites u_k, which U2(k) reads, and S2(k+2) refills U2(k)'s
// coefficient slot); the main stream joins the last U2 at the end of every batch of iterations.
// Inside a captured chunk these events become graph edges.
struct U2Side {
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> after_p2, after_u2;
};

// A captured chunk of MINRES iterations, replayed until every case has finished.  The key holds every
// value baked into the captured launches; a solve with other pointers, sizes or material recaptures.
struct ChunkGraph {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<unsigned char> key;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
};

// Resources kept between solves, one set per (device, solve stream): the U2 side stream and its
// events, the captured chunk graphs ([0] FP32 fields, [1] FP64 fields), and for batches the branch
// streams, fork/join events and the lockstep graph of all solves of the batch.  Repeated calls on the
// same stream find their set again instead of creating new objects.  A set is owned by one solve at a
// time (a second concurrent solve on the same stream gets a set of its own).  Everything is freed by
// rve_release_caches().
constexpr int kBranchStreams = 64;  // parallel branches of a batch graph (one per solve up to this many)
struct StreamCache {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool busy = false;
  U2Side u2;
  ChunkGraph graph[2];
  std::vector<hipStream_t> branch;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  ChunkGraph multi[2];
  void release() {
    graph[0].reset();
    graph[1].reset();
    multi[0].reset();
    multi[1].reset();
    for (hipEvent_t e : u2.after_p2) (void)hipEventDestroy(e);
    for (hipEvent_t e : u2.after_u2) (void)hipEventDestroy(e);
    u2.after_p2.clear();
    u2.after_u2.clear();
    if (u2.s2) (void)hipStreamDestroy(u2.s2);
    u2.s2 = nullptr;
    for (hipStream_t b : branch) (void)hipStreamDestroy(b);
    branch.clear();
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    join.clear();
    if (fork) (void)hipEventDestroy(fork);
    fork = nullptr;
  }
};
static std::mutex g_cache_mu;
static std::vector<StreamCache*> g_caches;

static StreamCache* cache_acquire(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (StreamCache* c : g_caches)
    if (!c->busy && c->dev == dev && c->stream == s) {
      c->busy = true;
      return c;
    }
  StreamCache* c = new StreamCache;
  c->dev = dev;
  c->stream = s;
  c->busy = true;
  g_caches.push_back(c);
  return c;
}
static void cache_release(StreamCache* c) {
  if (!c) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  c->busy = false;
}
struct CacheLease {
  StreamCache* c;
  explicit CacheLease(StreamCache* c_) : c(c_) {}
  ~CacheLease() { cache_release(c); }
};

// How a solve drives its iterations: with a cache set (side stream, captured graphs) or, for the
// entry point that may not create runtime objects, with neither (U2 inline, direct launches).
struct LoopCtx {
  StreamCache* cache = nullptr;  // nullptr: U2 inline on the solve stream, no graph
  bool u2_inline = false;        // batch workers and profiled solves keep U2 on the solve stream
  bool allow_graph = true;
};

static rve_status u2_events(U2Side& U, int count, bool need_stream) {
  if (need_stream && !U.s2) HIPCHK(hipStreamCreateWithFlags(&U.s2, hipStreamNonBlocking));
  while ((int)U.after_p2.size() < count + 1) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b, hipEventDisableTiming));
    U.after_p2.push_back(a);
    U.after_u2.push_back(b);
  }
  return RVE_OK;
}

// Enqueue `count` MINRES iterations starting from buffer phase (ia, ib, ic, id1, id2); returns the
// phase after them.  The buffer roles rotate with period 3 (u) and 2 (d).  U == nullptr: U2 runs on
// the solve stream right after each iteration's S2 (no events).
template <typename T>
static rve_status enqueue_iterations(const Plan& pl, int nc, MinresBufs<T>& B, const float* phi,
                                     const Material<T>& mat, const Tables<T>& tb, cx<T>* spec, MinresState* st,
                                     double* part, int count, int ph[5], hipStream_t s, U2Side* U) {
  const long long n6 = 6 * pl.g.nvox;
  dim3 vg, vb;
  vec_grid(nc, &vg, &vb);
  // 16-byte access needs each case's field to start on a 16-byte boundary
  const bool vec = (n6 * (long long)sizeof(T)) % 16 == 0;
  int& ia = ph[0];
  int& ib = ph[1];
  int& ic = ph[2];
  int& id1 = ph[3];
  int& id2 = ph[4];
  const long long nv = vec ? n6 / Vec16<T>::n : n6;
  const dim3 ug((unsigned)((nv + kThreads - 1) / kThreads), nc);
  auto launch_u2 = [&](hipStream_t on, int jj, int d2, int d1, int uk) {
    prof::begin<T>(prof::U2, on);
    if (vec)
      hipLaunchKernelGGL((k_direction<T, true>), ug, vb, 0, on, B.d[d2], B.d[d1], B.u[uk], B.x, st, n6, jj & 1);
    else
      hipLaunchKernelGGL((k_direction<T, false>), ug, vb, 0, on, B.d[d2], B.d[d1], B.u[uk], B.x, st, n6, jj & 1);
    prof::end(on);
  };
  if (!U) {
    for (int j = 0; j < count; ++j) {
      apply_op<T>(pl, nc, B.u[ib], &st[0].ib, phi, mat, tb, spec, B.u[ic], B.u[ib], B.u[ia], part, st, 0, s, j & 1);
      launch_u2(s, j, id2, id1, ib);
      const int t0 = ia;
      ia = ib;
      ib = ic;
      ic = t0;
      std::swap(id1, id2);
    }
    return RVE_OK;
  }
  hipStream_t s2 = U->s2;
  // U2 of iteration jj on the second stream, after event `ev` of the main stream
  auto u2 = [&](int jj, int d2, int d1, int uk, hipEvent_t ev) -> rve_status {
    HIPCHK(hipStreamWaitEvent(s2, ev, 0));
    launch_u2(s2, jj, d2, d1, uk);
    HIPCHK(hipEventRecord(U->after_u2[jj], s2));
    return RVE_OK;
  };
  int prev[3] = {0, 0, 0};  // (d2, d1, uk) buffer indices of the previous iteration
  for (int j = 0; j < count; ++j) {
    // iteration j's operator; U2(j-1) starts when P2(j) is done and streams beside P3(j), the pass
    // that leaves the most bandwidth unused
    apply_op<T>(pl, nc, B.u[ib], &st[0].ib, phi, mat, tb, spec, B.u[ic], B.u[ib], B.u[ia], part, st, 0, s, j & 1,
                j >= 2 ? U->after_u2[j - 2] : nullptr, j >= 1 ? U->after_p2[j] : nullptr);
    if (j >= 1) {
      const rve_status r2 = u2(j - 1, prev[0], prev[1], prev[2], U->after_p2[j]);
      if (r2 != RVE_OK) return r2;
    }
    prev[0] = id2;
    prev[1] = id1;
    prev[2] = ib;
    const int t0 = ia;
    ia = ib;
    ib = ic;
    ic = t0;
    std::swap(id1, id2);
  }
  if (count > 0) {
    HIPCHK(hipEventRecord(U->after_p2[count], s));  // after the last S2
    const rve_status r2 = u2(count - 1, prev[0], prev[1], prev[2], U->after_p2[count]);
    if (r2 != RVE_OK) return r2;
    HIPCHK(hipStreamWaitEvent(s, U->after_u2[count - 1], 0));
  }
  return RVE_OK;
}

template <typename T>
static std::vector<unsigned char> chunk_key(const Plan& pl, int nc, const MinresBufs<T>& B, const float* phi,
                                            const Material<T>& mat, const Tables<T>& tb, const cx<T>* spec,
                                            const MinresState* st, const double* part, int chunk, bool inl) {
  std::vector<unsigned char> k;
  auto put = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    k.insert(k.end(), c, c + n);
  };
  put(pl.n, sizeof(pl.n));
  put(pl.t, sizeof(pl.t));  // tiles and splits: a retune or a loaded table recaptures
  put(&pl.lds_cap3, sizeof(pl.lds_cap3));
  put(&nc, sizeof(nc));
  put(&B, sizeof(B));
  put(&phi, sizeof(phi));
  put(&mat, sizeof(mat));
  put(&tb, sizeof(tb));
  put(&spec, sizeof(spec));
  put(&st, sizeof(st));
  put(&part, sizeof(part));
  put(&chunk, sizeof(chunk));
  put(&inl, sizeof(inl));  // the captured graph has U2 on a side stream or inline
  return k;
}

static bool graphs_enabled() {
  const char* e = getenv("RVE_DISABLE_GRAPHS");
  return !(e && e[0] == '1');
}

// Runs MINRES iterations until every case has finished or the iteration budget is spent.
// States must be initialised (k_minres_init).  Host polls the finish flags every `check` iterations;
// each chunk of `check` iterations (rounded up to the buffer-rotation period 6) is one hipGraph replay
// when the context allows graphs (capture needs a non-NULL stream; profiled solves launch directly so
// that every launch can be bracketed by events).
template <typename T>
static rve_status minres_loop(const Plan& pl, int nc, MinresBufs<T>& B, const float* phi, const Material<T>& mat,
                              const Tables<T>& tb, cx<T>* spec, MinresState* st, double* part, int max_iter,
                              int check, hipStream_t s, const LoopCtx& ctx) {
  std::vector<MinresState> hs(nc);
  const int chunk = ((check + 5) / 6) * 6;
  const bool inl = ctx.u2_inline || prof::on || ctx.cache == nullptr;
  U2Side* U = nullptr;
  if (ctx.cache) {
    // the side stream (if used) and the events exist before any capture starts
    const rve_status r = u2_events(ctx.cache->u2, std::max(chunk, check), !inl);
    if (r != RVE_OK) return r;
    if (!inl) U = &ctx.cache->u2;
  }
  bool use_graph = ctx.cache && ctx.allow_graph && graphs_enabled() && !prof::on && s != nullptr;
  ChunkGraph* G = use_graph ? &ctx.cache->graph[sizeof(T) == 8 ? 1 : 0] : nullptr;
  if (use_graph) {
    std::vector<unsigned char> key = chunk_key<T>(pl, nc, B, phi, mat, tb, spec, st, part, chunk, inl);
    if (G->exec == nullptr || G->key != key) {
      G->reset();
      int ph[5] = {0, 1, 2, 0, 1};
      bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const rve_status er = enqueue_iterations<T>(pl, nc, B, phi, mat, tb, spec, st, part, chunk, ph, s, U);
        const hipError_t le = hipGetLastError();
        hipGraph_t gr = nullptr;
        ok = hipStreamEndCapture(s, &gr) == hipSuccess && le == hipSuccess && gr != nullptr && er == RVE_OK;
        if (ok) {
          G->graph = gr;
          ok = hipGraphInstantiate(&G->exec, gr, nullptr, nullptr, 0) == hipSuccess;
        } else if (gr) {
          hipGraphDestroy(gr);
        }
      }
      if (ok) {
        G->key = key;
      } else {
        G->reset();
        (void)hipGetLastError();
        use_graph = false;
      }
    }
  }
  int ph[5] = {0, 1, 2, 0, 1};  // u_{k-1}, u_k, p ; d_{k-1}, d_{k-2}
  int it = 0;
  while (it < max_iter) {
    if (use_graph) {
      HIPCHK(hipGraphLaunch(G->exec, s));
      it += chunk;
    } else {
      const int n = std::min(check, max_iter - it);
      const rve_status er = enqueue_iterations<T>(pl, nc, B, phi, mat, tb, spec, st, part, n, ph, s, U);
      if (er != RVE_OK) return er;
      it += n;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hs.data(), st, sizeof(MinresState) * nc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    prof::flush();
    bool all = true;
    for (int c = 0; c < nc; ++c) all = all && hs[c].finish;
    if (all) break;
  }
  return RVE_OK;
}

// ---------------------------------------------------------------------------- one solve, in phases
// The work of a solve_rve call (n_cases load cases on one grid and material), split into the phases a
// heterogeneous batch runs in lockstep over many such solves: setup (phase-map check, tables, right-hand
// side, start), sweeps (an MINRES run from the current FP64 residual, then the refinement bookkeeping)
// and post-processing.  The load cases may each have their own phase map (mat.phi_stride voxels apart).
struct SolveRun {
  const rve_grid* grid = nullptr;
  const float* phi = nullptr;
  const double* C = nullptr;
  const rve_options* opt = nullptr;
  int nc = 0, prec = 0;
  Plan pl;
  Layout L;
  char* ws = nullptr;
  hipStream_t s = nullptr;
  long long n6 = 0, phi_count = 0;
  MinresState* dst = nullptr;
  CaseInfo* dci = nullptr;
  double *part = nullptr, *sums = nullptr, *Ed2 = nullptr;
  int* flag = nullptr;
  double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr, *t64 = nullptr;
  cx<double>* spec64 = nullptr;
  cx<float>* spec32 = nullptr;
  Tables<double> tb64;
  Tables<float> tb32;
  Material<double> mat64, ident64;
  Material<float> mat32;
  MinresBufs<float> B32;
  MinresBufs<double> B64;
  std::vector<double> hE, hS;
  std::vector<CaseInfo> hci;
  dim3 vg, vb;

  template <typename T>
  MinresBufs<T>& bufs() {
    if constexpr (sizeof(T) == 8) return B64;
    else return B32;
  }
  template <typename T>
  const Material<T>& mat() const {
    if constexpr (sizeof(T) == 8) return mat64;
    else return mat32;
  }
  template <typename T>
  const Tables<T>& tables() const {
    if constexpr (sizeof(T) == 8) return tb64;
    else return tb32;
  }
  template <typename T>
  cx<T>* spec() const {
    if constexpr (sizeof(T) == 8) return spec64;
    else return spec32;
  }

  // Carve the workspace and stage the per-case macroscopic loads (host only, no HIP call).
  // macro_stress: [nc][6] or NULL.  phi_stride: voxels between consecutive cases' phase maps (0: shared).
  rve_status init(const rve_grid* grid_, const float* phi_, long long phi_stride, const double* C_,
                  const double* macro_strain, const double* macro_stress, int nc_, const rve_options* opt_,
                  char* ws_, size_t ws_bytes, hipStream_t s_) {
    grid = grid_;
    phi = phi_;
    C = C_;
    opt = opt_;
    nc = nc_;
    prec = opt->precision;
    ws = ws_;
    s = s_;
    if (!make_plan(grid, &pl)) return RVE_EUNSUPPORTED_SIZE;
    L = make_layout(pl, nc, prec, true);
    if ((long long)ws_bytes < L.total) return RVE_ENOMEM;
    const GridDims& g = pl.g;
    n6 = 6 * g.nvox;
    phi_count = phi_stride ? (long long)nc * phi_stride : g.nvox;
    dst = reinterpret_cast<MinresState*>(ws + L.off_state);
    dci = reinterpret_cast<CaseInfo*>(ws + L.off_info);
    part = reinterpret_cast<double*>(ws + L.off_part);
    sums = reinterpret_cast<double*>(ws + L.off_sums);
    flag = reinterpret_cast<int*>(ws + L.off_flag);
    x64 = reinterpret_cast<double*>(ws + L.off_x64);
    b64 = reinterpret_cast<double*>(ws + L.off_b64);
    r64 = reinterpret_cast<double*>(ws + L.off_r64);
    t64 = reinterpret_cast<double*>(ws + L.off_t64);
    spec64 = reinterpret_cast<cx<double>*>(ws + L.off_spec64);
    Ed2 = sums;  // 6 nc doubles of the 16 nc
    mat64 = make_material<double>(C, C + 36);
    mat32 = make_material<float>(C, C + 36);
    mat64.phi_stride = mat32.phi_stride = phi_stride;
    memset(&ident64, 0, sizeof(ident64));  // projection material: C = identity independent of phi
    for (int i = 0; i < 6; ++i) ident64.C0[i * 7] = 1.0;
    ident64.has_c0 = 1;
    ident64.use_phi = 0;
    if (prec == RVE_FP32_MIXED) {
      for (int i = 0; i < 3; ++i) B32.u[i] = reinterpret_cast<float*>(ws + L.off_u32[i]);
      for (int i = 0; i < 2; ++i) B32.d[i] = reinterpret_cast<float*>(ws + L.off_d32[i]);
      B32.x = reinterpret_cast<float*>(ws + L.off_x32);
      spec32 = reinterpret_cast<cx<float>*>(ws + L.off_spec32);
    } else {
      for (int i = 0; i < 3; ++i) B64.u[i] = reinterpret_cast<double*>(ws + L.off_u64[i]);
      for (int i = 0; i < 2; ++i) B64.d[i] = reinterpret_cast<double*>(ws + L.off_d64[i]);
      B64.x = x64;
    }
    // Mixed macroscopic control (eq. galop, eq. gallin): the macroscopic strain acts on the
    // strain-controlled components only, the macroscopic stress on the stress-controlled ones
    hE.assign(6 * nc, 0.0);
    hS.assign(6 * nc, 0.0);
    for (int c = 0; c < nc; ++c)
      for (int a = 0; a < 6; ++a) {
        const bool stress_ctl = (opt->stress_mask >> a) & 1;
        hE[c * 6 + a] = stress_ctl ? 0.0 : macro_strain[c * 6 + a];
        if (stress_ctl && macro_stress) hS[c * 6 + a] = macro_stress[c * 6 + a];
      }
    vec_grid(nc, &vg, &vb);
    return RVE_OK;
  }

  // Phase maps in [0, 1] and finite (device pre-pass; synchronises the stream).
  rve_status check_phi() {
    HIPCHK(hipMemsetAsync(flag, 0, 64, s));
    hipLaunchKernelGGL(k_check_phi, dim3(256), dim3(256), 0, s, phi, phi_count, flag);
    int hflag[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hflag[0]) return RVE_ENONFINITE;
    if (hflag[1]) return RVE_EINVAL;
    return RVE_OK;
  }

  // Tables, right-hand side b = -A(Ebar) + Ghat(0) Sbar with ||b||, and the start x64 (zero or the
  // projected warm start eps0 [nc][6][N] in the solve's field type), r64 = b - A x64.
  rve_status setup_tables() {
    rve_status r = build_tables<double>(pl, grid, ws + L.off_tab64, opt->scheme, opt->nyquist, s);
    if (r != RVE_OK) return r;
    tb64 = tables_at<double>(pl, ws + L.off_tab64);
    tb64.stress_mask = opt->stress_mask;
    if (prec == RVE_FP32_MIXED) {
      r = build_tables<float>(pl, grid, ws + L.off_tab32, opt->scheme, opt->nyquist, s);
      if (r != RVE_OK) return r;
      tb32 = tables_at<float>(pl, ws + L.off_tab32);
      tb32.stress_mask = opt->stress_mask;
    }
    return RVE_OK;
  }

  // A right-hand side the caller has put into b64 (one case): ||b|| (synchronises), x64 = 0,
  // r64 = b64.  Returns ||b|| in *bnorm; the case is inactive when it is zero.
  rve_status start_given_rhs(double* bnorm) {
    const GridDims& g = pl.g;
    (void)g;
    hipLaunchKernelGGL((k_lincomb<double, double>), vg, vb, 0, s, r64, b64, 1.0, (const double*)nullptr, 0.0, n6,
                       part);
    hipLaunchKernelGGL(k_sum_partials, dim3(nc), dim3(kThreads), 0, s, part, kRedBlocks, sums, 1, 1);
    double hb = 0.0;
    HIPCHK(hipMemcpyAsync(&hb, sums, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    hci.assign(nc, CaseInfo{});
    hci[0].bnorm = hb;
    hci[0].rnorm = hb;
    hci[0].r0 = hb;
    hci[0].active = hb > 0.0 ? 1 : 0;
    HIPCHK(hipMemcpyAsync(dci, hci.data(), sizeof(CaseInfo) * nc, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, s, x64, n6 * nc);
    HIPCHK(hipGetLastError());
    *bnorm = hb;
    return RVE_OK;
  }

  rve_status setup(const void* eps0) {
    const GridDims& g = pl.g;
    rve_status r = setup_tables();
    if (r != RVE_OK) return r;
    // macro strains live in the partials buffer's head while b is formed
    double* Ed = part;
    double* Sd = sums + 8 * nc;  // 6 nc doubles of the 16 nc
    HIPCHK(hipMemcpyAsync(Ed, hE.data(), sizeof(double) * 6 * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(Sd, hS.data(), sizeof(double) * 6 * nc, hipMemcpyHostToDevice, s));
    // b = -A(Ebar) + Ghat(0) Sbar  (FP64 operator; a uniform Sbar transforms to xi = 0 only, where the
    // projection keeps its stress-controlled components), and ||b||
    hipLaunchKernelGGL(k_fill_const<double>, vg, vb, 0, s, x64, Ed, g.nvox);
    apply_op<double>(pl, nc, x64, nullptr, phi, mat64, tb64, spec64, r64, nullptr, nullptr, nullptr, nullptr, 0, s);
    hipLaunchKernelGGL(k_rhs, vg, vb, 0, s, b64, r64, Sd, g.nvox, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(nc), dim3(kThreads), 0, s, part, kRedBlocks, sums, 1, 1);
    hci.assign(nc, CaseInfo{});
    std::vector<double> hb(nc);
    HIPCHK(hipMemcpyAsync(hb.data(), sums, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double cn = 0;
    for (int i = 0; i < 36; ++i) cn = std::max(cn, std::fabs(C[36 + i]));
    for (int c = 0; c < nc; ++c) {
      hci[c].bnorm = hb[c];
      hci[c].rnorm = hb[c];
      hci[c].iters = 0;
      hci[c].status = 0;
      hci[c].warm_rejected = 0;
      hci[c].r0 = hb[c];
      hci[c].active = 1;
      // A right-hand side at the rounding level of the transforms of a constant field counts as zero:
      // the homogeneous case, answered exactly by eps = 0.
      double en = 0, sn = 0;
      for (int i = 0; i < 6; ++i) en = std::max(en, std::fabs(hE[c * 6 + i]));
      for (int i = 0; i < 6; ++i) sn = std::max(sn, std::fabs(hS[c * 6 + i]));
      const double scale = (cn * en + sn) * std::sqrt((double)n6);
      if (hci[c].bnorm <= 1e-13 * scale) {
        hci[c].bnorm = 0.0;
        hci[c].active = 0;
      }
    }
    HIPCHK(hipMemcpyAsync(dci, hci.data(), sizeof(CaseInfo) * nc, hipMemcpyHostToDevice, s));
    // re-upload Ebar (part was overwritten by the norm partials)
    HIPCHK(hipMemcpyAsync(Ed2, hE.data(), sizeof(double) * 6 * nc, hipMemcpyHostToDevice, s));
    if (eps0) {
      // x64 = Ghat eps0 (projection, C = identity); a start that does not lower the residual below
      // ||b|| is dropped (k_warm_fallback)
      if (prec == RVE_FP32_MIXED)
        hipLaunchKernelGGL((k_lincomb<float, double>), vg, vb, 0, s, r64, (const float*)eps0, 1.0,
                           (const double*)nullptr, 0.0, n6, part);
      else
        hipLaunchKernelGGL((k_lincomb<double, double>), vg, vb, 0, s, r64, (const double*)eps0, 1.0,
                           (const double*)nullptr, 0.0, n6, part);
      apply_op<double>(pl, nc, r64, nullptr, phi, ident64, tb64, spec64, x64, nullptr, nullptr, nullptr, nullptr, 0,
                       s);
      apply_op<double>(pl, nc, x64, nullptr, phi, mat64, tb64, spec64, r64, nullptr, nullptr, nullptr, nullptr, 0, s);
      hipLaunchKernelGGL((k_lincomb<double, double>), vg, vb, 0, s, r64, r64, -1.0, b64, 1.0, n6, part);
      hipLaunchKernelGGL(k_sum_partials, dim3(nc), dim3(kThreads), 0, s, part, kRedBlocks, sums + 6 * nc, 1, 0);
      hipLaunchKernelGGL(k_residual_update, dim3((nc + 63) / 64), dim3(64), 0, s, dci, sums + 6 * nc, nc, opt->tol,
                         opt->max_iter);
      hipLaunchKernelGGL(k_warm_fallback, dim3(1024, nc), dim3(256), 0, s, x64, r64, b64, dci, n6);
      hipLaunchKernelGGL(k_residual_update_fallback, dim3((nc + 63) / 64), dim3(64), 0, s, dci, nc);
    } else {
      hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, s, x64, n6 * nc);
      HIPCHK(hipMemcpyAsync(r64, b64, sizeof(double) * n6 * nc, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipGetLastError());
    return RVE_OK;
  }

  // Start an MINRES run on A d = r64 for the cases still active (FP32_MIXED: a sweep, u_1 = fp32(r64);
  // FP64: the one run, on A x = b from x64).  *any: some case of this solve runs (read from the device,
  // which synchronises); with any == nullptr the run is launched without that check (cases that are
  // not active finish at once).
  rve_status sweep_begin(bool* any) {
    if (any) {
      HIPCHK(hipMemcpyAsync(hci.data(), dci, sizeof(CaseInfo) * nc, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      *any = false;
      for (int c = 0; c < nc; ++c) *any = *any || hci[c].active;
    }
    if (prec == RVE_FP32_MIXED) {
      if (any && !*any) return RVE_OK;
      // u_1 = fp32(r64), u_0 = d = x32 = 0
      hipLaunchKernelGGL((k_lincomb<double, float>), vg, vb, 0, s, B32.u[1], r64, 1.0, (const double*)nullptr, 0.0,
                         n6, part);
      hipLaunchKernelGGL(k_minres_init, dim3(nc), dim3(kThreads), 0, s, dst, part, kRedBlocks, dci, opt->tol,
                         opt->inner_safety, opt->inner_floor, opt->max_iter);
      hipLaunchKernelGGL(k_zero<float>, dim3(1024), dim3(256), 0, s, B32.u[0], n6 * nc);
      hipLaunchKernelGGL(k_zero<float>, dim3(1024), dim3(256), 0, s, B32.d[0], n6 * nc);
      hipLaunchKernelGGL(k_zero<float>, dim3(1024), dim3(256), 0, s, B32.d[1], n6 * nc);
      hipLaunchKernelGGL(k_zero<float>, dim3(1024), dim3(256), 0, s, B32.x, n6 * nc);
    } else {
      // FP64: one MINRES on A x = b from the start x64 (r64 = b - A x64); inactive cases finish at once
      hipLaunchKernelGGL((k_lincomb<double, double>), vg, vb, 0, s, B64.u[1], r64, 1.0, (const double*)nullptr, 0.0,
                         n6, part);
      hipLaunchKernelGGL(k_minres_init, dim3(nc), dim3(kThreads), 0, s, dst, part, kRedBlocks, dci, opt->tol, 1.0,
                         1e-300, opt->max_iter);
      hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, s, B64.u[0], n6 * nc);
      hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, s, B64.d[0], n6 * nc);
      hipLaunchKernelGGL(k_zero<double>, dim3(1024), dim3(256), 0, s, B64.d[1], n6 * nc);
    }
    HIPCHK(hipGetLastError());
    return RVE_OK;
  }

  // After an MINRES run: count its iterations, update x64 (FP32_MIXED: x64 += x32, re-projected onto
  // compatible fields), recompute the FP64 residual r64 = b - A x64 and decide which cases go on.
  rve_status sweep_end() {
    hipLaunchKernelGGL(k_sweep_done, dim3((nc + 63) / 64), dim3(64), 0, s, dst, dci, nc);
    if (prec == RVE_FP32_MIXED) {
      hipLaunchKernelGGL(k_accum<float>, vg, vb, 0, s, x64, B32.x, n6, (const int*)nullptr);
      // The exact fluctuation is compatible and has zero mean.  FP32 rounding inside the sweep leaves
      // incompatible components (a mean among them) that the projected residual cannot see but the
      // average stress does: project the FP64 iterate back onto compatible fields.
      apply_op<double>(pl, nc, x64, nullptr, phi, ident64, tb64, spec64, t64, nullptr, nullptr, nullptr, nullptr, 0,
                       s);
      hipLaunchKernelGGL(k_keep_inactive, dim3(1024, nc), dim3(256), 0, s, t64, x64, dci, n6);
      std::swap(x64, t64);
    }
    apply_op<double>(pl, nc, x64, nullptr, phi, mat64, tb64, spec64, r64, nullptr, nullptr, nullptr, nullptr, 0, s);
    hipLaunchKernelGGL((k_lincomb<double, double>), vg, vb, 0, s, r64, r64, -1.0, b64, 1.0, n6, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(nc), dim3(kThreads), 0, s, part, kRedBlocks, sums + 6 * nc, 1, 0);
    hipLaunchKernelGGL(k_residual_update, dim3((nc + 63) / 64), dim3(64), 0, s, dci, sums + 6 * nc, nc, opt->tol,
                       opt->max_iter);
    HIPCHK(hipGetLastError());
    return RVE_OK;
  }

  // Post-processing of cases [c0, c0 + ncs): strain/stress fields into the caller's buffers
  // ([ncs][6][N]), <sigma>, iterations, FP64 residuals, total macroscopic strain; returns the worst
  // status over those cases.  Synchronises.
  rve_status post(int c0, int ncs, void* strain_out, void* stress_out, double* eff_stress, int32_t* iterations,
                  double* rel_residual, double* mean_strain, rve_status* worst) {
    const GridDims& g = pl.g;
    const float* phic = phi + (long long)c0 * mat64.phi_stride;
    const double* xc = x64 + (long long)c0 * n6;
    if (prec == RVE_FP32_MIXED)
      hipLaunchKernelGGL(k_post<float>, dim3(kRedBlocks, ncs), dim3(kThreads), 0, s, xc, phic, mat64, Ed2 + 6 * c0,
                         (float*)strain_out, (float*)stress_out, g.nvox, part);
    else
      hipLaunchKernelGGL(k_post<double>, dim3(kRedBlocks, ncs), dim3(kThreads), 0, s, xc, phic, mat64, Ed2 + 6 * c0,
                         (double*)strain_out, (double*)stress_out, g.nvox, part);
    // r64 is free now: it holds the sums
    hipLaunchKernelGGL(k_sum_partials, dim3(6 * ncs), dim3(kThreads), 0, s, part, kRedBlocks, r64, 1, 0);
    hipLaunchKernelGGL(k_field_sums, dim3(kRedBlocks, ncs), dim3(kThreads), 0, s, xc, g.nvox, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(6 * ncs), dim3(kThreads), 0, s, part, kRedBlocks, r64 + 6 * ncs, 1, 0);
    std::vector<double> hs(12 * ncs);
    HIPCHK(hipMemcpyAsync(hs.data(), r64, sizeof(double) * 12 * ncs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hci.data(), dci, sizeof(CaseInfo) * nc, hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    rve_status worst_err = RVE_OK, worst_warn = RVE_OK;
    for (int k = 0; k < ncs; ++k) {
      const CaseInfo& ci = hci[c0 + k];
      for (int a = 0; a < 6; ++a) eff_stress[k * 6 + a] = hs[k * 6 + a] / (double)g.nvox;
      if (mean_strain)
        for (int a = 0; a < 6; ++a)
          mean_strain[k * 6 + a] = hE[(c0 + k) * 6 + a] + hs[6 * ncs + k * 6 + a] / (double)g.nvox;
      iterations[k] = ci.iters;
      rel_residual[k] = ci.bnorm > 0 ? ci.rnorm / ci.bnorm : 0.0;
      if (ci.status == RVE_ENONFINITE || !std::isfinite(rel_residual[k])) worst_err = RVE_ENONFINITE;
      else if (ci.status == RVE_BREAKDOWN) worst_warn = RVE_BREAKDOWN;
      else if (ci.bnorm > 0 && !(rel_residual[k] <= opt->tol) && worst_warn == RVE_OK) worst_warn = RVE_NOT_CONVERGED;
    }
    *worst = worst_err != RVE_OK ? worst_err : worst_warn;
    return RVE_OK;
  }
};

// MINRES iterations of many solves at once: one captured graph whose parallel branches (fork from the
// solve stream onto the cache's branch streams, join back) each run one solve's chunk of iterations.
// After every replay each solve whose cases have all finished their MINRES run is refined at once
// (FP64 residual, next FP32 sweep started), independently of the others, and rejoins the next replay:
// a chunk always starts from the same buffer phase, so a restarted solve fits the captured graph.  A
// solve that is converged (or out of sweeps or iterations) leaves the graph when the graph is next
// captured, which happens once such solves make up half of it.  U2 runs inline in each branch.
// `count` iterations of every solve in `runs`, each on a branch stream, forked from and joined to `on`.
template <typename T>
static rve_status enqueue_multi(std::vector<SolveRun*>& runs, int count, hipStream_t on, StreamCache* cache) {
  const int nr = (int)runs.size();
  const int nbr = std::min(nr, kBranchStreams);
  HIPCHK(hipEventRecord(cache->fork, on));
  for (int b = 0; b < nbr; ++b) HIPCHK(hipStreamWaitEvent(cache->branch[b], cache->fork, 0));
  for (int r = 0; r < nr; ++r) {
    SolveRun& R = *runs[r];
    int ph[5] = {0, 1, 2, 0, 1};
    const rve_status er = enqueue_iterations<T>(R.pl, R.nc, R.bufs<T>(), R.phi, R.mat<T>(), R.tables<T>(), R.spec<T>(),
                                                R.dst, R.part, count, ph, cache->branch[r % nbr], nullptr);
    if (er != RVE_OK) return er;
  }
  for (int b = 0; b < nbr; ++b) {
    HIPCHK(hipEventRecord(cache->join[b], cache->branch[b]));
    HIPCHK(hipStreamWaitEvent(on, cache->join[b], 0));
  }
  return RVE_OK;
}

template <typename T>
static rve_status capture_multi(std::vector<SolveRun*>& runs, int chunk, hipStream_t s, StreamCache* cache,
                                bool* use_graph) {
  const int nr = (int)runs.size();
  const int nbr = std::min(nr, kBranchStreams);
  while ((int)cache->branch.size() < nbr) {
    hipStream_t b = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    cache->branch.push_back(b);
  }
  if (!cache->fork) HIPCHK(hipEventCreateWithFlags(&cache->fork, hipEventDisableTiming));
  while ((int)cache->join.size() < nbr) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cache->join.push_back(e);
  }
  *use_graph = graphs_enabled() && !prof::on && s != nullptr;
  if (!*use_graph) return RVE_OK;
  ChunkGraph& G = cache->multi[sizeof(T) == 8 ? 1 : 0];
  std::vector<unsigned char> key;
  for (SolveRun* R : runs) {
    const std::vector<unsigned char> k = chunk_key<T>(R->pl, R->nc, R->bufs<T>(), R->phi, R->mat<T>(), R->tables<T>(),
                                                      R->spec<T>(), R->dst, R->part, chunk, true);
    key.insert(key.end(), k.begin(), k.end());
  }
  if (G.exec != nullptr && G.key == key) return RVE_OK;
  G.reset();
  bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const rve_status er = enqueue_multi<T>(runs, chunk, s, cache);
    const hipError_t le = hipGetLastError();
    hipGraph_t gr = nullptr;
    ok = hipStreamEndCapture(s, &gr) == hipSuccess && le == hipSuccess && gr != nullptr && er == RVE_OK;
    if (ok) {
      G.graph = gr;
      ok = hipGraphInstantiate(&G.exec, gr, nullptr, nullptr, 0) == hipSuccess;
    } else if (gr) {
      (void)hipGraphDestroy(gr);
    }
  }
  if (ok) {
    G.key = key;
  } else {
    G.reset();
    (void)hipGetLastError();
    *use_graph = false;
  }
  return RVE_OK;
}

// Drives all solves of a batch from their first sweep (already begun) to the end: replays, per-solve
// refinement as soon as a solve's run ends, graph recapture when half of it has converged.
// started[r]: the first sweep_begin of run r launched an MINRES run (a run with no active case did not).
template <typename T>
static rve_status batch_iterate(std::vector<SolveRun>& runs, const std::vector<char>& started,
                                const rve_options* opt, hipStream_t s, StreamCache* cache) {
  const bool fp32 = opt->precision == RVE_FP32_MIXED;
  const int chunk = ((opt->check_every + 5) / 6) * 6;
  const int nr = (int)runs.size();
  std::vector<int> sweeps(nr, 1);          // runs begun so far
  std::vector<char> done(nr, 0);           // converged, or out of sweeps
  std::vector<SolveRun*> live;
  for (int r = 0; r < nr; ++r) {
    done[r] = started[r] ? 0 : 1;
    if (!done[r]) live.push_back(&runs[r]);
  }
  if (live.empty()) return RVE_OK;
  std::vector<std::vector<MinresState>> hs(nr);
  for (int r = 0; r < nr; ++r) hs[r].resize(runs[r].nc);
  std::vector<char> pending_check(nr, 0);  // a sweep was begun without checking for active cases
  bool use_graph = false;
  rve_status st = capture_multi<T>(live, chunk, s, cache, &use_graph);
  if (st != RVE_OK) return st;
  long long guard = 0;
  const long long guard_max = (long long)opt->max_iter * opt->max_refine / chunk + 2LL * opt->max_refine + 8;
  while (!live.empty()) {
    if (++guard > guard_max) break;  // every case's iteration budget is spent by now
    if (use_graph) {
      HIPCHK(hipGraphLaunch(cache->multi[sizeof(T) == 8 ? 1 : 0].exec, s));
    } else {
      st = enqueue_multi<T>(live, chunk, s, cache);
      if (st != RVE_OK) return st;
    }
    HIPCHK(hipGetLastError());
    for (int r = 0; r < nr; ++r)
      if (!done[r]) {
        HIPCHK(hipMemcpyAsync(hs[r].data(), runs[r].dst, sizeof(MinresState) * runs[r].nc, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(runs[r].hci.data(), runs[r].dci, sizeof(CaseInfo) * runs[r].nc, hipMemcpyDeviceToHost,
                              s));
      }
    HIPCHK(hipStreamSynchronize(s));
    prof::flush();
    int done_in_graph = 0;
    for (int r = 0; r < nr; ++r) {
      if (done[r]) {
        // still has nodes in the graph until the next capture
        for (SolveRun* L : live) done_in_graph += L == &runs[r];
        continue;
      }
      bool all = true;
      for (int c = 0; c < runs[r].nc; ++c) all = all && hs[r][c].finish;
      if (!all) continue;
      if (pending_check[r]) {
        // the sweep just replayed was begun unchecked: with no active case it ran nothing (and the solve
        // ends here, as solve_rve's loop ends on a sweep without active cases)
        bool any = false;
        for (int c = 0; c < runs[r].nc; ++c) any = any || runs[r].hci[c].active;
        pending_check[r] = 0;
        if (!any) {
          done[r] = 1;
          continue;
        }
      }
      st = runs[r].sweep_end();
      if (st != RVE_OK) return st;
      if (fp32 && sweeps[r] < opt->max_refine) {
        st = runs[r].sweep_begin(nullptr);  // its active flags are checked after the next replay
        if (st != RVE_OK) return st;
        sweeps[r]++;
        pending_check[r] = 1;
      } else {
        done[r] = 1;  // counted among the graph's finished solves from the next replay on
      }
    }
    std::vector<SolveRun*> still;
    for (int r = 0; r < nr; ++r)
      if (!done[r]) still.push_back(&runs[r]);
    if (still.empty()) break;
    if (2 * done_in_graph >= (int)live.size() || !use_graph) {
      if (still.size() != live.size()) {
        live.swap(still);
        if (use_graph) {
          st = capture_multi<T>(live, chunk, s, cache, &use_graph);
          if (st != RVE_OK) return st;
        }
      }
    }
  }
  return RVE_OK;
}

}  // namespace rve

using namespace rve;

// ============================================================================ C ABI
static std::mutex g_solve_mutex;  // serialises autotuning

extern "C" {

static rve_status validate_grid(const rve_grid* grid);

void rve_default_options(rve_options* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 5000;
  o->precision = RVE_FP32_MIXED;
  o->max_refine = 24;
  o->nyquist = RVE_NYQ_NATURAL;
  o->scheme = RVE_SCHEME_ROTATED;
  o->check_every = 24;
  o->inner_floor = 3e-2;
  o->inner_safety = 0.9;
  o->stress_mask = 0;
  o->macro_stress = nullptr;
}

int32_t rve_supported_length(int32_t n) {
  ensure_registry();
  return find_len(n) ? 1 : 0;
}

void rve_profile_enable(int32_t on_) {
  std::lock_guard<std::mutex> lk(prof::mu);
  if (on_ && prof::pool.empty()) {
    prof::pool.resize(2048);
    for (auto& e : prof::pool)
      if (hipEventCreate(&e) != hipSuccess) {
        prof::pool.clear();
        return;
      }
  }
  prof::on = on_ != 0 && !prof::pool.empty();
}

void rve_profile_reset(void) {
  std::lock_guard<std::mutex> lk(prof::mu);
  for (int k = 0; k < prof::NSLOT; ++k) {
    prof::ms[k] = 0;
    prof::cnt[k] = 0;
  }
  prof::dropped = 0;
}

int32_t rve_profile_read(double* total_ms, int64_t* launches, int32_t max_kinds) {
  std::lock_guard<std::mutex> lk(prof::mu);
  const int n = std::min<int>(max_kinds, prof::NSLOT);
  for (int k = 0; k < n; ++k) {
    if (total_ms) total_ms[k] = prof::ms[k];
    if (launches) launches[k] = prof::cnt[k];
  }
  return prof::NSLOT;
}

const char* rve_profile_kind_name(int32_t k) { return (k >= 0 && k < prof::NSLOT) ? prof::kNames[k] : ""; }

const char* rve_last_error(void) { return g_last_error; }

int32_t rve_last_mean_strain(double* mean_strain, int32_t max_cases) {
  const int n = (int)g_last_info.size();
  if (mean_strain)
    for (int c = 0; c < std::min(n, (int)max_cases); ++c)
      for (int a = 0; a < 6; ++a) mean_strain[c * 6 + a] = g_last_info[c].mean_strain[a];
  return n;
}

int32_t rve_last_solve_info(double* initial_rel_residual, int32_t* warm_rejected, int32_t max_cases) {
  const int n = (int)g_last_info.size();
  for (int c = 0; c < std::min(n, (int)max_cases); ++c) {
    if (initial_rel_residual) initial_rel_residual[c] = g_last_info[c].r0_rel;
    if (warm_rejected) warm_rejected[c] = g_last_info[c].warm_rejected;
  }
  return n;
}

}  // extern "C"

// ---------------------------------------------------------------------------- autotuner
static bool tile_fits(int threads_per_row, int W) { return W >= 1 && W * threads_per_row <= 256; }

static int write_tuning_file(const char* path) {
  // one JSON object per line: {"n":[a,b,c],"elem":e,"W1":w,"W3":w,"R2":r,"S3":s,"F":[f0,f1,f2]}
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  FILE* f = fopen(path, "w");
  if (!f) return -1;
  for (auto& e : tuned())
    fprintf(f, "{\"n\":[%d,%d,%d],\"elem\":%d,\"W1\":%d,\"W3\":%d,\"R2\":%d,\"S3\":%d,\"F\":[%d,%d,%d]}\n",
            e.first.n0, e.first.n1, e.first.n2, e.first.elem, e.second.W1, e.second.W3, e.second.R2, e.second.S3,
            e.second.F[0], e.second.F[1], e.second.F[2]);
  fclose(f);
  return (int)tuned().size();
}

extern "C" int32_t rve_load_tuning(const char* path) {
  if (!path) return -1;
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  char line[512];
  int n = 0;
  while (fgets(line, sizeof(line), f)) {
    TuneKey k;
    Tiles t;
    if (sscanf(line, " {\"n\":[%d,%d,%d],\"elem\":%d,\"W1\":%d,\"W3\":%d,\"R2\":%d", &k.n0, &k.n1, &k.n2,
               &k.elem, &t.W1, &t.W3, &t.R2) == 7 &&
        (k.elem == 4 || k.elem == 8) && t.W1 >= 1 && t.W3 >= 1 && t.R2 >= 1 && t.W1 <= 256 && t.W3 <= 256 &&
        t.R2 <= 256) {
      const char* sp = strstr(line, "\"S3\":");
      const int s3 = sp ? atoi(sp + 5) : 2;
      t.S3 = (s3 == 1 || s3 == 3) ? s3 : 2;  // absent (older tables): the default
      const char* fp = strstr(line, "\"F\":[");
      int f0 = 0, f1 = 0, f2 = 0;
      if (fp && sscanf(fp, "\"F\":[%d,%d,%d]", &f0, &f1, &f2) == 3 && f0 >= 0 && f1 >= 0 && f2 >= 0 && f0 < 16 &&
          f1 < 16 && f2 < 16) {
        t.F[0] = f0;
        t.F[1] = f1;
        t.F[2] = f2;
      }
      set_tuned(k, t);
      n++;
    }
  }
  fclose(f);
  return n;
}

template <typename T>
static rve_status autotune_impl(Plan& pl, const rve_grid* grid, int nc, const Layout& L, char* ws, hipStream_t s,
                                Tiles* best, double* best_ms) {
  const int elem = (int)sizeof(T);
  const long long n6 = 6 * pl.g.nvox;
  char* tab = ws + (elem == 4 ? L.off_tab32 : L.off_tab64);
  rve_status r = build_tables<T>(pl, grid, tab, RVE_SCHEME_ROTATED, RVE_NYQ_NATURAL, s);
  if (r != RVE_OK) return r;
  Tables<T> tb = tables_at<T>(pl, tab);
  T* x = reinterpret_cast<T*>(ws + (elem == 4 ? L.off_u32[0] : L.off_x64));
  T* y = reinterpret_cast<T*>(ws + (elem == 4 ? L.off_u32[1] : L.off_r64));
  cx<T>* spec = reinterpret_cast<cx<T>*>(ws + (elem == 4 ? L.off_spec32 : L.off_spec64));
  hipLaunchKernelGGL(k_zero<T>, dim3(1024), dim3(256), 0, s, x, n6 * nc);
  Material<T> id;
  memset(&id, 0, sizeof(id));
  for (int i = 0; i < 6; ++i) id.C0[i * 7] = (T)1;
  id.has_c0 = 1;
  id.use_phi = 0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int reps = 10;  // three gave tile choices that flipped between runs
  auto time_apply = [&](double* ms) -> rve_status {
    apply_op<T>(pl, nc, x, nullptr, nullptr, id, tb, spec, y, nullptr, nullptr, nullptr, nullptr, 0, s);
    HIPCHK(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i)
      apply_op<T>(pl, nc, x, nullptr, nullptr, id, tb, spec, y, nullptr, nullptr, nullptr, nullptr, 0, s);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipGetLastError());
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    return RVE_OK;
  };
  Tiles& cur = pl.t[elem == 8];
  double bms = 0;
  r = time_apply(&bms);
  if (r != RVE_OK) return r;
  // factorisation of each axis length first (tiles are clamped to what each one allows)
  for (int p = 0; p < 3; ++p) {
    const int nv = len_variants(pl.n[p]);
    if (nv < 2) continue;
    const int keep = cur.F[p];
    int bestv = keep;
    for (int v = 0; v < nv; ++v) {
      if (v == keep) continue;
      cur.F[p] = v;
      select_axes(&pl);
      double ms = 0;
      r = time_apply(&ms);
      if (r != RVE_OK) {
        cur.F[p] = keep;
        select_axes(&pl);
        return r;
      }
      if (ms < bms) {
        bms = ms;
        bestv = v;
      }
    }
    cur.F[p] = bestv;
    select_axes(&pl);
  }
  // P3 component split (whole / halves / thirds), at the current tiles.  Thirds only for FP64, where
  // they keep the transform out of scratch: in FP32 the plain apply timed here favours them by a hair,
  // but in the MINRES loop, where U2 streams beside P3, the halves are faster (557 vs 576 ms at 256^3).
  {
    const int keep = cur.S3;
    int bestv = keep;
    for (int v = 1; v <= (elem == 8 ? 3 : 2); ++v) {
      if (v == keep) continue;
      cur.S3 = v;
      double ms = 0;
      r = time_apply(&ms);
      if (r != RVE_OK) {
        cur.S3 = keep;
        return r;
      }
      if (ms < bms) {
        bms = ms;
        bestv = v;
      }
    }
    cur.S3 = bestv;
  }
  const int cands[] = {1, 2, 4, 8, 16, 32, 64, 128, 256};
  // coordinate descent over the three tiles (P3 pencils, P2/P4 rows, P1/P5 rows)
  for (int role = 0; role < 3; ++role) {
    const int nb = axis(pl, elem, role == 0 ? 0 : role == 1 ? 1 : 2)->nb;
    int* slot = role == 0 ? &cur.W3 : role == 1 ? &cur.R2 : &cur.W1;
    const int keep = *slot;
    int bestv = keep;
    for (int c : cands) {
      if (c == keep || !tile_fits(nb, c)) continue;
      *slot = c;
      // the LDS cap may reduce the candidate; skip duplicates of what it resolves to
      const int eff = role == 0 ? tile_p3(pl, elem) : role == 1 ? rows_p2(pl, elem) : tile_p1(pl, elem);
      if (eff != c) continue;
      double ms = 0;
      r = time_apply(&ms);
      if (r != RVE_OK) {
        *slot = keep;
        return r;
      }
      if (ms < bms) {
        bms = ms;
        bestv = c;
      }
    }
    *slot = bestv;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *best = cur;
  if (best_ms) *best_ms = bms;
  return RVE_OK;
}

extern "C" {

rve_status rve_autotune(const rve_grid* grid, int32_t n_cases, int32_t precision, void* workspace,
                        size_t workspace_bytes, void* hip_stream, const char* cache_path, double* best_ms) {
  std::lock_guard<std::mutex> solve_lock(g_solve_mutex);
  rve_status st = validate_grid(grid);
  if (st != RVE_OK) return st;
  if (n_cases < 1 || n_cases > 65535 || (precision != RVE_FP32_MIXED && precision != RVE_FP64) || !workspace)
    return RVE_EINVAL;
  Plan pl;
  if (!make_plan(grid, &pl)) return RVE_EUNSUPPORTED_SIZE;
  const Layout L = make_layout(pl, n_cases, precision, true);
  if ((long long)workspace_bytes < L.total) return RVE_ENOMEM;
  hipStream_t s = (hipStream_t)hip_stream;
  Tiles best;
  double ms = 0;
  const int elem = precision == RVE_FP64 ? 8 : 4;
  st = elem == 4 ? autotune_impl<float>(pl, grid, n_cases, L, (char*)workspace, s, &best, &ms)
                 : autotune_impl<double>(pl, grid, n_cases, L, (char*)workspace, s, &best, &ms);
  if (st != RVE_OK) return st;
  set_tuned(TuneKey{pl.g.n0, pl.g.n1, pl.g.n2, elem}, best);
  if (best_ms) *best_ms = ms;
  if (cache_path && write_tuning_file(cache_path) < 0) return RVE_EINVAL;
  return RVE_OK;
}

int32_t rve_tuned_tiles(const rve_grid* grid, int32_t precision, int32_t* tiles7) {
  if (validate_grid(grid) != RVE_OK || !tiles7) return 0;
  Plan pl;
  if (!make_plan(grid, &pl)) return 0;
  const int elem = precision == RVE_FP64 ? 8 : 4;
  const Tiles& t = pl.t[elem == 8];
  tiles7[0] = t.W1;
  tiles7[1] = t.W3;
  tiles7[2] = t.R2;
  tiles7[3] = split_p3(pl, elem);
  for (int p = 0; p < 3; ++p) tiles7[4 + p] = axis(pl, elem, p)->na;
  Tiles tt;
  return find_tuned(TuneKey{pl.g.n0, pl.g.n1, pl.g.n2, precision == RVE_FP64 ? 8 : 4}, &tt) ? 1 : 0;
}

const char* rve_status_string(rve_status s) {
  switch (s) {
    case RVE_OK: return "RVE_OK";
    case RVE_NOT_CONVERGED: return "RVE_NOT_CONVERGED";
    case RVE_BREAKDOWN: return "RVE_BREAKDOWN";
    case RVE_EINVAL: return "RVE_EINVAL";
    case RVE_EUNSUPPORTED_SIZE: return "RVE_EUNSUPPORTED_SIZE";
    case RVE_ENONFINITE: return "RVE_ENONFINITE";
    case RVE_ENOMEM: return "RVE_ENOMEM";
    case RVE_EDEVICE: return "RVE_EDEVICE";
  }
  return "RVE_UNKNOWN";
}

static rve_status validate_grid(const rve_grid* grid) {
  if (!grid) return RVE_EINVAL;
  for (int p = 0; p < 3; ++p) {
    if (grid->n[p] < 1 || !(std::isfinite(grid->L[p]) && grid->L[p] > 0)) return RVE_EINVAL;
  }
  for (int p = 0; p < 3; ++p)
    if (!rve_supported_length(grid->n[p])) return RVE_EUNSUPPORTED_SIZE;
  return RVE_OK;
}

static rve_status validate_stiffness(const double* C) {
  if (!C) return RVE_EINVAL;
  for (int ph = 0; ph < 2; ++ph) {
    const double* M = C + 36 * ph;
    double mx = 0;
    for (int i = 0; i < 36; ++i) {
      if (!std::isfinite(M[i])) return RVE_ENONFINITE;
      mx = std::max(mx, std::fabs(M[i]));
    }
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j)
        if (std::fabs(M[i * 6 + j] - M[j * 6 + i]) > 1e-12 * mx) return RVE_EINVAL;
  }
  return RVE_OK;
}

static rve_status validate_options(const rve_options* o) {
  if (!o) return RVE_EINVAL;
  if (!(std::isfinite(o->tol) && o->tol > 0)) return RVE_EINVAL;
  if (o->max_iter < 1 || o->max_refine < 1 || o->check_every < 1) return RVE_EINVAL;
  if (o->precision != RVE_FP32_MIXED && o->precision != RVE_FP64) return RVE_EINVAL;
  if (o->nyquist != RVE_NYQ_NATURAL && o->nyquist != RVE_NYQ_ZERO_ALL) return RVE_EINVAL;
  if (o->scheme != RVE_SCHEME_ROTATED && o->scheme != RVE_SCHEME_CONTINUOUS) return RVE_EINVAL;
  if (!(o->inner_floor > 0 && o->inner_floor < 1) || !(o->inner_safety > 0 && o->inner_safety <= 1))
    return RVE_EINVAL;
  if (o->stress_mask < 0 || o->stress_mask > 63) return RVE_EINVAL;
  return RVE_OK;
}

rve_status rve_validate(const rve_grid* grid, const double* phase_stiffness, const double* macro_strain,
                        int32_t n_cases, const rve_options* opt) {
  rve_status s = validate_grid(grid);
  if (s != RVE_OK) return s;
  if (n_cases < 1 || n_cases > 65535) return RVE_EINVAL;
  s = validate_options(opt);
  if (s != RVE_OK) return s;
  s = validate_stiffness(phase_stiffness);
  if (s != RVE_OK) return s;
  if (!macro_strain) return RVE_EINVAL;
  for (int i = 0; i < 6 * n_cases; ++i)
    if (!std::isfinite(macro_strain[i])) return RVE_ENONFINITE;
  if (opt->macro_stress)
    for (int i = 0; i < 6 * n_cases; ++i)
      if (!std::isfinite(opt->macro_stress[i])) return RVE_ENONFINITE;
  return RVE_OK;
}

size_t rve_workspace_bytes(const rve_grid* grid, int32_t n_cases, const rve_options* opt) {
  if (validate_grid(grid) != RVE_OK || n_cases < 1 || validate_options(opt) != RVE_OK) return 0;
  Plan pl;
  if (!make_plan(grid, &pl)) return 0;
  return (size_t)make_layout(pl, n_cases, opt->precision, true).total;
}

size_t rve_apply_workspace_bytes(const rve_grid* grid, int32_t n_cases, int32_t precision) {
  if (validate_grid(grid) != RVE_OK || n_cases < 1 || (precision != RVE_FP32_MIXED && precision != RVE_FP64)) return 0;
  Plan pl;
  if (!make_plan(grid, &pl)) return 0;
  return (size_t)make_layout(pl, n_cases, precision, false).total;
}

rve_status rve_apply(const rve_grid* grid, const float* phi, const double* phase_stiffness, int32_t n_cases,
                     int32_t precision, int32_t scheme, int32_t nyquist, int32_t stress_mask, int32_t mode,
                     const void* x, void* y, void* workspace, size_t workspace_bytes, void* hip_stream) {
  rve_status st = validate_grid(grid);
  if (st != RVE_OK) return st;
  if (n_cases < 1 || n_cases > 65535) return RVE_EINVAL;
  if (precision != RVE_FP32_MIXED && precision != RVE_FP64) return RVE_EINVAL;
  if (scheme != RVE_SCHEME_ROTATED && scheme != RVE_SCHEME_CONTINUOUS) return RVE_EINVAL;
  if (nyquist != RVE_NYQ_NATURAL && nyquist != RVE_NYQ_ZERO_ALL) return RVE_EINVAL;
  if (stress_mask < 0 || stress_mask > 63) return RVE_EINVAL;
  if (mode < 0 || mode > 2) return RVE_EINVAL;
  if (!x || !y || !workspace) return RVE_EINVAL;
  if (mode != RVE_APPLY_PROJECTION) {
    if (!phi) return RVE_EINVAL;
    st = validate_stiffness(phase_stiffness);
    if (st != RVE_OK) return st;
  }
  Plan pl;
  if (!make_plan(grid, &pl)) return RVE_EUNSUPPORTED_SIZE;
  const Layout L = make_layout(pl, n_cases, precision, false);
  if ((long long)workspace_bytes < L.total) return RVE_ENOMEM;
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  double ident[72] = {0};
  for (int i = 0; i < 6; ++i) ident[i * 7] = 1.0;  // void phase = identity, solid = identity
  for (int i = 0; i < 6; ++i) ident[36 + i * 7] = 1.0;
  const double* C = (mode == RVE_APPLY_PROJECTION) ? ident : phase_stiffness;
  if (precision == RVE_FP32_MIXED) {
    rve_status r = build_tables<float>(pl, grid, ws + L.off_tab32, scheme, nyquist, s);
    if (r != RVE_OK) return r;
    Tables<float> tb = tables_at<float>(pl, ws + L.off_tab32);
    tb.stress_mask = stress_mask;
    Material<float> mat = make_material<float>(C, C + 36);
    if (mode == RVE_APPLY_PROJECTION) {
      // C = identity independent of phi: C0 = I and phi is not read
      for (int i = 0; i < 36; ++i) mat.Cd[i] = 0.0f;
      mat.has_c0 = 1;
      mat.use_phi = 0;
    }
    apply_op<float>(pl, n_cases, (const float*)x, nullptr, phi, mat, tb, (cx<float>*)(ws + L.off_spec32), (float*)y,
                    nullptr, nullptr, nullptr, nullptr, mode == RVE_APPLY_STIFFNESS_ROUNDTRIP, s);
  } else {
    rve_status r = build_tables<double>(pl, grid, ws + L.off_tab64, scheme, nyquist, s);
    if (r != RVE_OK) return r;
    Tables<double> tb = tables_at<double>(pl, ws + L.off_tab64);
    tb.stress_mask = stress_mask;
    Material<double> mat = make_material<double>(C, C + 36);
    if (mode == RVE_APPLY_PROJECTION) {
      for (int i = 0; i < 36; ++i) mat.Cd[i] = 0.0;
      mat.has_c0 = 1;
      mat.use_phi = 0;
    }
    apply_op<double>(pl, n_cases, (const double*)x, nullptr, phi, mat, tb, (cx<double>*)(ws + L.off_spec64),
                     (double*)y, nullptr, nullptr, nullptr, nullptr, mode == RVE_APPLY_STIFFNESS_ROUNDTRIP, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return RVE_OK;
}

// How solve_impl drives the MINRES iterations.
enum SolveMode {
  kSolveDefault = 0,  // per-stream cache: U2 on a side stream, captured iteration chunks
  kSolveBatch = 1,    // batch worker: per-stream cache, U2 inline on the worker's stream
  kSolveNoAlloc = 2   // no runtime objects at all: U2 inline, direct launches, caller-provided workspace
};

static rve_status solve_impl(const rve_grid* grid, const float* phi, const double* phase_stiffness,
                             const double* macro_strain, int32_t n_cases, const rve_options* opt, const void* eps0,
                             void* strain_out, void* stress_out, double* eff_stress, int32_t* iterations,
                             double* rel_residual, void* workspace, size_t workspace_bytes, void* hip_stream,
                             SolveMode mode) {
  rve_status st = rve_validate(grid, phase_stiffness, macro_strain, n_cases, opt);
  if (st != RVE_OK) return st;
  if (!phi || !strain_out || !eff_stress || !iterations || !rel_residual || !workspace) return RVE_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  SolveRun R;
  st = R.init(grid, phi, 0, phase_stiffness, macro_strain, opt->macro_stress, n_cases, opt, (char*)workspace,
              workspace_bytes, s);
  if (st != RVE_OK) return st;
  StreamCache* cache = mode == kSolveNoAlloc ? nullptr : cache_acquire(s);
  CacheLease lease(cache);
  LoopCtx ctx;
  ctx.cache = cache;
  ctx.u2_inline = mode != kSolveDefault;
  ctx.allow_graph = mode != kSolveNoAlloc;
  st = R.check_phi();
  if (st != RVE_OK) return st;
  st = R.setup(eps0);
  if (st != RVE_OK) return st;
  const bool fp32 = opt->precision == RVE_FP32_MIXED;
  const int sweeps = fp32 ? opt->max_refine : 1;  // FP64: one MINRES run
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    bool any = false;
    st = R.sweep_begin(&any);
    if (st != RVE_OK) return st;
    if (fp32 && !any) break;
    st = fp32 ? minres_loop<float>(R.pl, R.nc, R.B32, phi, R.mat32, R.tb32, R.spec32, R.dst, R.part, opt->max_iter,
                                   opt->check_every, s, ctx)
              : minres_loop<double>(R.pl, R.nc, R.B64, phi, R.mat64, R.tb64, R.spec64, R.dst, R.part, opt->max_iter,
                                    opt->check_every, s, ctx);
    if (st != RVE_OK) return st;
    st = R.sweep_end();
    if (st != RVE_OK) return st;
  }
  std::vector<double> ms(6 * (size_t)n_cases);
  rve_status worst = RVE_OK;
  st = R.post(0, n_cases, strain_out, stress_out, eff_stress, iterations, rel_residual, ms.data(), &worst);
  if (st != RVE_OK) return st;
  g_last_info.assign(n_cases, LastInfo{});
  for (int c = 0; c < n_cases; ++c) {
    g_last_info[c].r0_rel = R.hci[c].bnorm > 0 ? R.hci[c].r0 / R.hci[c].bnorm : 0.0;
    g_last_info[c].warm_rejected = R.hci[c].warm_rejected;
    for (int a = 0; a < 6; ++a) g_last_info[c].mean_strain[a] = ms[c * 6 + a];
  }
  return worst;
}

rve_status solve_rve(const rve_grid* grid, const float* phi, const double* phase_stiffness,
                     const double* macro_strain, int32_t n_cases, const rve_options* opt, const void* eps0,
                     void* strain_out, void* stress_out, double* eff_stress, int32_t* iterations,
                     double* rel_residual, void* workspace, size_t workspace_bytes, void* hip_stream) {
  return solve_impl(grid, phi, phase_stiffness, macro_strain, n_cases, opt, eps0, strain_out, stress_out, eff_stress,
                    iterations, rel_residual, workspace, workspace_bytes, hip_stream, kSolveDefault);
}

// ---------------------------------------------------------------------------- J2 plasticity
// Nonlinear solve of eqs. Slin / galnonlin / galrlin / galrnewton: Newton iterations per increment of a
// linear load ramp, each linearised problem solved by the MINRES machinery of solve_rve on a
// right-hand side formed here, with the elastic-plastic tangent fused into P1 (Material::tan).
static rve_status validate_j2(const rve_j2_material* m, const rve_j2_options* j) {
  if (!m || !j) return RVE_EINVAL;
  if (!(std::isfinite(m->young) && m->young > 0.0)) return RVE_EINVAL;
  if (!(std::isfinite(m->poisson) && m->poisson > -1.0 && m->poisson < 0.5)) return RVE_EINVAL;
  if (!(std::isfinite(m->yield_stress) && m->yield_stress > 0.0)) return RVE_EINVAL;
  if (j->increments < 1 || j->max_newton < 1) return RVE_EINVAL;
  if (!(std::isfinite(j->newton_tol) && j->newton_tol > 0.0) || !(std::isfinite(j->lin_tol) && j->lin_tol > 0.0))
    return RVE_EINVAL;
  return RVE_OK;
}

struct J2Layout {
  long long eps, eps_t, eps_p, sig, rhs, tan64, tan32, ep, red, total;
};

static J2Layout j2_layout(const Plan& pl, int prec) {
  J2Layout J;
  const long long nv = pl.g.nvox;
  long long off = make_layout(pl, 1, prec, true).total;
  auto take = [&](long long bytes) {
    const long long o = off;
    off += align_up(bytes, 256);
    return o;
  };
  J.eps = take(6 * nv * 8);
  J.eps_t = take(6 * nv * 8);
  J.eps_p = take(6 * nv * 8);
  J.sig = take(6 * nv * 8);
  J.rhs = take(6 * nv * 8);
  J.tan64 = take(7 * nv * 8);
  J.tan32 = prec == RVE_FP32_MIXED ? take(7 * nv * 4) : 0;
  J.ep = take(nv * 8);
  J.red = take(2 * kRedBlocks * 8);
  J.total = off;
  return J;
}

size_t rve_j2_workspace_bytes(const rve_grid* grid, const rve_options* opt) {
  if (validate_grid(grid) != RVE_OK || validate_options(opt) != RVE_OK) return 0;
  Plan pl;
  if (!make_plan(grid, &pl)) return 0;
  return (size_t)j2_layout(pl, opt->precision).total;
}

static J2Mat j2_mat(const rve_j2_material* m) {
  J2Mat j;
  j.K = m->young / (3.0 * (1.0 - 2.0 * m->poisson));
  j.mu2 = m->young / (1.0 + m->poisson);
  j.sy = m->yield_stress;
  return j;
}

rve_status rve_j2_return_map(int64_t n_voxels, const float* phi, const rve_j2_material* material, const double* strain,
                             const double* plastic_strain, double* stress, double* tangent, void* hip_stream) {
  if (n_voxels < 1 || !phi || !material || !strain || !plastic_strain || (!stress && !tangent)) return RVE_EINVAL;
  rve_j2_options jo = {1, 1, 1.0, 1.0};
  rve_status st = validate_j2(material, &jo);
  if (st != RVE_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_j2_return, dim3(2048), dim3(kThreads), 0, s, strain, const_cast<double*>(plastic_strain), phi,
                     j2_mat(material), (long long)n_voxels, stress, tangent, (float*)nullptr, 0, (double*)nullptr);
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

rve_status solve_rve_j2(const rve_grid* grid, const float* phi, const rve_j2_material* material,
                        const double* macro_strain_final, const double* macro_stress_final, const rve_options* opt,
                        const rve_j2_options* jopt, double* strain_out, double* stress_out,
                        double* plastic_strain_out, double* ep_acc_out, rve_j2_increment* history, void* workspace,
                        size_t workspace_bytes, void* hip_stream) {
  rve_status st = validate_grid(grid);
  if (st != RVE_OK) return st;
  st = validate_options(opt);
  if (st != RVE_OK) return st;
  st = validate_j2(material, jopt);
  if (st != RVE_OK) return st;
  if (!phi || !macro_strain_final || !history || !workspace) return RVE_EINVAL;
  for (int a = 0; a < 6; ++a) {
    if (!std::isfinite(macro_strain_final[a])) return RVE_ENONFINITE;
    if (macro_stress_final && !std::isfinite(macro_stress_final[a])) return RVE_ENONFINITE;
  }
  Plan pl;
  if (!make_plan(grid, &pl)) return RVE_EUNSUPPORTED_SIZE;
  const J2Layout J = j2_layout(pl, opt->precision);
  if ((long long)workspace_bytes < J.total) return RVE_ENOMEM;
  const J2Mat jm = j2_mat(material);
  // the solid's elastic stiffness (Mandel), empty phase zero
  double C[72];
  memset(C, 0, sizeof(C));
  const double lam = jm.K - jm.mu2 / 3.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[36 + a * 6 + b] = lam;
  for (int a = 0; a < 6; ++a) C[36 + a * 7] += jm.mu2;
  rve_options lo = *opt;  // the MINRES tolerance is set per Newton iteration
  lo.macro_stress = nullptr;
  const double zero6[6] = {0, 0, 0, 0, 0, 0};
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  SolveRun R;
  st = R.init(grid, phi, 0, C, zero6, nullptr, 1, &lo, ws, workspace_bytes, s);
  if (st != RVE_OK) return st;
  StreamCache* cache = cache_acquire(s);
  CacheLease lease(cache);
  LoopCtx ctx;
  ctx.cache = cache;
  ctx.u2_inline = false;
  ctx.allow_graph = true;
  st = R.check_phi();
  if (st != RVE_OK) return st;
  st = R.setup_tables();
  if (st != RVE_OK) return st;
  const long long nv = pl.g.nvox, n6 = 6 * nv;
  double* eps = reinterpret_cast<double*>(ws + J.eps);
  double* eps_t = reinterpret_cast<double*>(ws + J.eps_t);
  double* eps_p = reinterpret_cast<double*>(ws + J.eps_p);
  double* sig = reinterpret_cast<double*>(ws + J.sig);
  double* rhs = reinterpret_cast<double*>(ws + J.rhs);  // -sigma + Sbar before the projection
  double* tan64 = reinterpret_cast<double*>(ws + J.tan64);
  float* tan32 = J.tan32 ? reinterpret_cast<float*>(ws + J.tan32) : nullptr;
  double* ep = reinterpret_cast<double*>(ws + J.ep);
  double* red = reinterpret_cast<double*>(ws + J.red);
  R.mat64.tan = tan64;
  R.mat64.tan_stride = 7 * nv;
  R.mat32.tan = tan32;
  R.mat32.tan_stride = 7 * nv;
  const dim3 vg(kRedBlocks), vb(kThreads);
  hipLaunchKernelGGL(k_zero<double>, vg, vb, 0, s, eps, n6);
  hipLaunchKernelGGL(k_zero<double>, vg, vb, 0, s, eps_p, n6);
  hipLaunchKernelGGL(k_zero<double>, vg, vb, 0, s, ep, nv);
  HIPCHK(hipGetLastError());
  double Ef[6], Sf[6], Et[6] = {0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 6; ++a) {
    const bool sc = (opt->stress_mask >> a) & 1;
    Ef[a] = sc ? 0.0 : macro_strain_final[a];
    Sf[a] = (sc && macro_stress_final) ? macro_stress_final[a] : 0.0;
  }
  double* Sd = R.sums + 8;  // the macroscopic stress of the increment, read by k_rhs
  const bool fp32 = opt->precision == RVE_FP32_MIXED;
  std::vector<double> hred(2 * kRedBlocks), hsum(12);
  rve_status worst = RVE_OK;
  auto field_mean = [&](const double* f, double* out6) -> rve_status {
    hipLaunchKernelGGL(k_field_sums, dim3(kRedBlocks, 1), dim3(kThreads), 0, s, f, nv, R.part);
    hipLaunchKernelGGL(k_sum_partials, dim3(6), dim3(kThreads), 0, s, R.part, kRedBlocks, red, 1, 0);
    HIPCHK(hipMemcpyAsync(out6, red, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < 6; ++a) out6[a] /= (double)nv;
    return RVE_OK;
  };
  for (int inc = 1; inc <= jopt->increments; ++inc) {
    rve_j2_increment& H = history[inc - 1];
    memset(&H, 0, sizeof(H));
    double Eb[6], Sb[6];
    Vec6 dE;
    for (int a = 0; a < 6; ++a) {
      Eb[a] = Ef[a] * inc / jopt->increments;
      Sb[a] = Sf[a] * inc / jopt->increments;
      dE.v[a] = Eb[a] - Et[a];
    }
    HIPCHK(hipMemcpyAsync(eps_t, eps, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_add_uniform, vg, vb, 0, s, eps, dE, nv);
    double b0 = -1.0, r_newton = INFINITY;
    for (int it = 1; it <= jopt->max_newton; ++it) {
      // sigma and tangent at eps^{i-1}; b_i = -G(sigma - Sbar)
      hipLaunchKernelGGL(k_j2_return, vg, vb, 0, s, eps, eps_p, phi, jm, nv, sig, tan64, tan32, 0, (double*)nullptr);
      HIPCHK(hipMemcpyAsync(Sd, Sb, 6 * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_rhs, dim3(kRedBlocks, 1), dim3(kThreads), 0, s, rhs, sig, Sd, nv, R.part);
      apply_op<double>(R.pl, 1, rhs, nullptr, phi, R.ident64, R.tb64, R.spec64, R.b64, nullptr, nullptr, nullptr,
                       nullptr, 0, s);
      HIPCHK(hipGetLastError());
      double bn = 0.0;
      st = R.start_given_rhs(&bn);
      if (st != RVE_OK) return st;
      if (b0 < 0.0) b0 = bn;
      H.newton = it;
      if (bn > jopt->lin_tol * b0 && bn > 0.0) {
        lo.tol = jopt->lin_tol * b0 / bn;
        const int sweeps = fp32 ? lo.max_refine : 1;
        for (int sw = 0; sw < sweeps; ++sw) {
          bool any = false;
          st = R.sweep_begin(&any);
          if (st != RVE_OK) return st;
          if (fp32 && !any) break;
          st = fp32 ? minres_loop<float>(R.pl, 1, R.B32, phi, R.mat32, R.tb32, R.spec32, R.dst, R.part, lo.max_iter,
                                         lo.check_every, s, ctx)
                    : minres_loop<double>(R.pl, 1, R.B64, phi, R.mat64, R.tb64, R.spec64, R.dst, R.part, lo.max_iter,
                                          lo.check_every, s, ctx);
          if (st != RVE_OK) return st;
          st = R.sweep_end();
          if (st != RVE_OK) return st;
        }
        HIPCHK(hipMemcpyAsync(R.hci.data(), R.dci, sizeof(CaseInfo), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        H.minres += R.hci[0].iters;
        if (R.hci[0].status == RVE_ENONFINITE) return RVE_ENONFINITE;
        // eps^i = eps^{i-1} + d
        hipLaunchKernelGGL((k_lincomb<double, double>), dim3(kRedBlocks, 1), vb, 0, s, eps, eps, 1.0, R.x64, 1.0, n6,
                           R.part);
      }
      // eq. galrnewton: |d|_inf / |eps^i - eps^t|_inf (d = x64, zero when no MINRES ran)
      hipLaunchKernelGGL(k_absmax2, vg, vb, 0, s, R.x64, eps, eps_t, n6, red);
      HIPCHK(hipMemcpyAsync(hred.data(), red, 2 * kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double dmax = 0.0, emax = 0.0;
      for (int b = 0; b < kRedBlocks; ++b) {
        dmax = std::max(dmax, hred[2 * b]);
        emax = std::max(emax, hred[2 * b + 1]);
      }
      r_newton = emax > 0.0 ? dmax / emax : 0.0;
      if (r_newton <= jopt->newton_tol) break;
    }
    H.r_newton = r_newton;
    H.status = r_newton <= jopt->newton_tol ? 0 : 1;
    if (H.status) worst = RVE_NOT_CONVERGED;
    // accept: stress at eps^i, plastic strain and its accumulated norm updated
    hipLaunchKernelGGL(k_j2_return, vg, vb, 0, s, eps, eps_p, phi, jm, nv, sig, (double*)nullptr, (float*)nullptr, 1, ep);
    HIPCHK(hipGetLastError());
    st = field_mean(eps, H.strain_mean);
    if (st != RVE_OK) return st;
    st = field_mean(sig, H.stress_mean);
    if (st != RVE_OK) return st;
    for (int a = 0; a < 6; ++a) Et[a] = Eb[a];
  }
  if (strain_out) HIPCHK(hipMemcpyAsync(strain_out, eps, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (stress_out) HIPCHK(hipMemcpyAsync(stress_out, sig, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (plastic_strain_out)
    HIPCHK(hipMemcpyAsync(plastic_strain_out, eps_p, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (ep_acc_out) HIPCHK(hipMemcpyAsync(ep_acc_out, ep, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return worst;
}

// ---------------------------------------------------------------------------- no-allocation entry point
// Static scratch for solve_rve_noalloc: a file-scope device array, one copy per GPU the library runs
// on, held until the process ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in); its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static rve_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RVE_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return RVE_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RVE_OK;
}

size_t rve_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

rve_status solve_rve_noalloc(const rve_grid* grid, const float* phi, const double* phase_stiffness,
                             const double* macro_strain, int32_t n_cases, const rve_options* opt, const void* eps0,
                             void* strain_out, void* stress_out, double* eff_stress, int32_t* iterations,
                             double* rel_residual, void* hip_stream) {
  rve_status st = rve_validate(grid, phase_stiffness, macro_strain, n_cases, opt);
  if (st != RVE_OK) return st;
  if (!phi || !strain_out || !eff_stress || !iterations || !rel_residual) return RVE_EINVAL;
  const size_t need = rve_workspace_bytes(grid, n_cases, opt);
  if (need == 0) return RVE_EINVAL;
  if (need > kNoAllocScratchBytes) {
    snprintf(g_last_error, sizeof(g_last_error),
             "solve_rve_noalloc: this solve needs %zu bytes of workspace, the static scratch holds %zu", need,
             kNoAllocScratchBytes);
    return RVE_ENOMEM;
  }
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != RVE_OK) return st;
  return solve_impl(grid, phi, phase_stiffness, macro_strain, n_cases, opt, eps0, strain_out, stress_out, eff_stress,
                    iterations, rel_residual, ws, kNoAllocScratchBytes, hip_stream, kSolveNoAlloc);
}

int32_t rve_release_caches(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  int32_t freed = 0;
  std::vector<StreamCache*> keep;
  for (StreamCache* c : g_caches) {
    if (c->busy) {
      keep.push_back(c);
      continue;
    }
    int cur = 0;
    const bool switch_dev = c->dev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != c->dev;
    if (switch_dev) (void)hipSetDevice(c->dev);
    c->release();
    if (switch_dev) (void)hipSetDevice(cur);
    delete c;
    freed++;
  }
  g_caches.swap(keep);
  (void)hipGetLastError();
  return freed;
}

int32_t rve_cache_counts(int64_t* counts4) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  int64_t sets = 0, streams = 0, events = 0, graphs = 0;
  for (const StreamCache* c : g_caches) {
    sets++;
    streams += (c->u2.s2 != nullptr) + (int64_t)c->branch.size();
    events += (int64_t)c->u2.after_p2.size() + (int64_t)c->u2.after_u2.size() + (int64_t)c->join.size() +
              (c->fork != nullptr);
    graphs += (c->graph[0].exec != nullptr) + (c->graph[1].exec != nullptr) + (c->multi[0].exec != nullptr) +
              (c->multi[1].exec != nullptr);
  }
  if (counts4) {
    counts4[0] = sets;
    counts4[1] = streams;
    counts4[2] = events;
    counts4[3] = graphs;
  }
  return (int32_t)sets;
}

// ---------------------------------------------------------------------------- heterogeneous batches
// RVEs with the same grid (lengths and cell size) and the same phase stiffness form one group; a group
// is one multi-case solve whose load cases are the cases of all its RVEs, each case with its own copy
// of its RVE's phase map (and warm start) in the group's workspace region.  Groups run their sweeps in
// lockstep, and their MINRES iterations run as the parallel branches of one captured graph.
struct BatchGroup {
  std::vector<int> items;  // item indices
  std::vector<int> c0;     // first case of each item within the group
  int nc = 0;
  long long nvox = 0;
  bool warm = false;
  size_t off_ws = 0, ws_bytes = 0, off_phi = 0, off_eps0 = 0;
};

static bool same_group(const rve_batch_item& a, const rve_batch_item& b) {
  for (int p = 0; p < 3; ++p)
    if (a.grid.n[p] != b.grid.n[p] || a.grid.L[p] != b.grid.L[p]) return false;
  return memcmp(a.phase_stiffness, b.phase_stiffness, sizeof(double) * 72) == 0;
}

// Groups in decreasing work (voxels x cases) and their workspace carve-out; 0 total on a bad item.
static size_t plan_batch(const rve_batch_item* items, int n_items, const rve_options* opt,
                         std::vector<BatchGroup>* groups) {
  groups->clear();
  for (int i = 0; i < n_items; ++i) {
    BatchGroup* gp = nullptr;
    for (auto& g : *groups)
      if (same_group(items[g.items[0]], items[i])) gp = &g;
    if (!gp) {
      groups->push_back(BatchGroup{});
      gp = &groups->back();
    }
    gp->c0.push_back(gp->nc);
    gp->items.push_back(i);
    gp->nc += items[i].n_cases;
    gp->warm = gp->warm || items[i].eps0 != nullptr;
  }
  std::stable_sort(groups->begin(), groups->end(), [&](const BatchGroup& a, const BatchGroup& b) {
    const rve_grid& ga = items[a.items[0]].grid;
    const rve_grid& gb = items[b.items[0]].grid;
    return (double)ga.n[0] * ga.n[1] * ga.n[2] * a.nc > (double)gb.n[0] * gb.n[1] * gb.n[2] * b.nc;
  });
  const size_t elem = opt->precision == RVE_FP64 ? 8 : 4;
  size_t off = 0;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  for (auto& g : *groups) {
    const rve_grid& gr = items[g.items[0]].grid;
    g.nvox = (long long)gr.n[0] * gr.n[1] * gr.n[2];
    const size_t w = rve_workspace_bytes(&gr, g.nc, opt);
    if (w == 0) return 0;
    g.off_ws = off;
    g.ws_bytes = up(w);
    off += g.ws_bytes;
    g.off_phi = off;
    off += up(sizeof(float) * (size_t)g.nvox * g.nc);
    if (g.warm) {
      g.off_eps0 = off;
      off += up(elem * 6 * (size_t)g.nvox * g.nc);
    }
  }
  return off;
}

size_t rve_batch_workspace_bytes(const rve_batch_item* items, int32_t n_items, const rve_options* opt) {
  if (!items || n_items < 1 || !opt) return 0;
  for (int i = 0; i < n_items; ++i)
    if (rve_workspace_bytes(&items[i].grid, items[i].n_cases, opt) == 0 || !items[i].phase_stiffness) return 0;
  std::vector<BatchGroup> groups;
  return plan_batch(items, n_items, opt, &groups);
}

rve_status solve_rve_batch(rve_batch_item* items, int32_t n_items, const rve_options* opt, void* workspace,
                           size_t workspace_bytes, void* hip_stream) {
  if (!items || n_items < 1 || !opt || !workspace) return RVE_EINVAL;
  for (int i = 0; i < n_items; ++i) {
    rve_options o = *opt;
    o.macro_stress = items[i].macro_stress;
    rve_status v = rve_validate(&items[i].grid, items[i].phase_stiffness, items[i].macro_strain, items[i].n_cases, &o);
    if (v != RVE_OK) return v;
    if (!items[i].voxel_fraction_field || !items[i].strain_out || !items[i].eff_stress || !items[i].iterations ||
        !items[i].rel_residual)
      return RVE_EINVAL;
  }
  std::vector<BatchGroup> groups;
  const size_t need = plan_batch(items, n_items, opt, &groups);
  if (need == 0) return RVE_EINVAL;
  if (workspace_bytes < need) return RVE_ENOMEM;
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = (char*)workspace;
  const size_t elem = opt->precision == RVE_FP64 ? 8 : 4;
  const int ng = (int)groups.size();
  // per group: stacked loads, phase maps (and warm starts) per case
  std::vector<std::vector<double>> strains(ng), stresses(ng);
  std::vector<SolveRun> runs(ng);
  for (int gi = 0; gi < ng; ++gi) {
    BatchGroup& G = groups[gi];
    strains[gi].assign(6 * (size_t)G.nc, 0.0);
    stresses[gi].assign(6 * (size_t)G.nc, 0.0);
    bool any_stress = false;
    float* phis = reinterpret_cast<float*>(ws + G.off_phi);
    for (size_t k = 0; k < G.items.size(); ++k) {
      const rve_batch_item& it = items[G.items[k]];
      for (int c = 0; c < it.n_cases; ++c) {
        const int cc = G.c0[k] + c;
        for (int a = 0; a < 6; ++a) {
          strains[gi][cc * 6 + a] = it.macro_strain[c * 6 + a];
          if (it.macro_stress) stresses[gi][cc * 6 + a] = it.macro_stress[c * 6 + a];
        }
        any_stress = any_stress || it.macro_stress != nullptr;
        HIPCHK(hipMemcpyAsync(phis + (size_t)cc * G.nvox, it.voxel_fraction_field, sizeof(float) * G.nvox,
                              hipMemcpyDeviceToDevice, s));
      }
      if (G.warm) {
        char* e0 = ws + G.off_eps0 + elem * 6 * (size_t)G.nvox * G.c0[k];
        const size_t bytes = elem * 6 * (size_t)G.nvox * it.n_cases;
        if (it.eps0)
          HIPCHK(hipMemcpyAsync(e0, it.eps0, bytes, hipMemcpyDeviceToDevice, s));
        else
          HIPCHK(hipMemsetAsync(e0, 0, bytes, s));  // zero start for the items that bring none
      }
    }
    const rve_batch_item& first = items[G.items[0]];
    rve_status st = runs[gi].init(&first.grid, phis, G.nvox, first.phase_stiffness, strains[gi].data(),
                                  any_stress ? stresses[gi].data() : nullptr, G.nc, opt, ws + G.off_ws, G.ws_bytes, s);
    if (st != RVE_OK) return st;
  }
  for (int gi = 0; gi < ng; ++gi) {
    rve_status st = runs[gi].check_phi();
    if (st != RVE_OK) return st;
    st = runs[gi].setup(groups[gi].warm ? (const void*)(ws + groups[gi].off_eps0) : nullptr);
    if (st != RVE_OK) return st;
  }
  StreamCache* cache = cache_acquire(s);
  CacheLease lease(cache);
  const bool fp32 = opt->precision == RVE_FP32_MIXED;
  std::vector<char> started(ng, 0);
  for (int gi = 0; gi < ng; ++gi) {
    bool any = false;
    rve_status st = runs[gi].sweep_begin(&any);
    if (st != RVE_OK) return st;
    started[gi] = (any || !fp32) ? 1 : 0;  // FP64 always starts its one run (inactive cases finish at once)
  }
  {
    rve_status st = fp32 ? batch_iterate<float>(runs, started, opt, s, cache)
                         : batch_iterate<double>(runs, started, opt, s, cache);
    if (st != RVE_OK) return st;
  }
  rve_status worst_err = RVE_OK, worst_warn = RVE_OK;
  for (int gi = 0; gi < ng; ++gi) {
    BatchGroup& G = groups[gi];
    for (size_t k = 0; k < G.items.size(); ++k) {
      rve_batch_item& it = items[G.items[k]];
      rve_status w = RVE_OK;
      rve_status st = runs[gi].post(G.c0[k], it.n_cases, it.strain_out, it.stress_out, it.eff_stress, it.iterations,
                                    it.rel_residual, it.mean_strain, &w);
      if (st != RVE_OK) return st;
      it.status = w;
      if (w < 0 && worst_err == RVE_OK) worst_err = w;
      if (w > 0 && worst_warn == RVE_OK) worst_warn = w;
    }
  }
  return worst_err != RVE_OK ? worst_err : worst_warn;
}

}  // extern "C"
