// Table of the compiled FFT pass kernels, one entry per supported axis length N = NA * NB.
#pragma once
#include "rve_kernels.h"

namespace rve {

template <typename T>
using P1Fn = void (*)(const T*, const double*, int, const float*, Material<T>, cx<T>*, const cx<T>*, GridDims, int,
                      const MinresState*, double*);
template <typename T>
using P2Fn = void (*)(cx<T>*, cx<T>*, const cx<T>*, GridDims, int, long long, const MinresState*, MinresState*,
                      const double*, int, int);
template <typename T>
using P3Fn = void (*)(cx<T>*, const cx<T>*, FreqTables<T>, GridDims, int, T, const MinresState*);
template <typename T>
using P5Fn = void (*)(const cx<T>*, T*, const T*, const T*, double*, const cx<T>*, GridDims, int,
                      const MinresState*);

template <typename T>
using SCFn = void (*)(cx<T>*, long long, int, int, int, const cx<T>*, int);

template <typename T>
using RPFn = void (*)(cx<T>*, long long, const float*, long long, int, int, int, T, const cx<T>*, int);

template <typename T>
struct LenKernels {
  P1Fn<T> p1, p1t;  // p1t: with the per-voxel elastic-plastic tangent (Material::tan)
  P2Fn<T> p2f, p2i;
  P3Fn<T> p3, p3_ident;
  P3Fn<T> p3s, p3s_ident;  // components split over two halves of the block
  P3Fn<T> p3t, p3t_ident;  // components split over three groups of the block
  P5Fn<T> p5;
  SCFn<T> scf, sci;  // forward / inverse transforms along a strided axis (k_strided)
  RPFn<T> rowp;      // per-pair row pass along axis 2 (k_row_pair)
};

struct LenEntry {
  int n, na, nb;
  LenKernels<float> f;
  LenKernels<double> d;
  template <typename T>
  const LenKernels<T>& k() const;
};
template <>
inline const LenKernels<float>& LenEntry::k<float>() const { return f; }
template <>
inline const LenKernels<double>& LenEntry::k<double>() const { return d; }

void register_len(const LenEntry& e);
const LenEntry* find_len(int n, int variant = 0);
// the default factorisation of a length (the table is filled on first use), or nullptr
const LenEntry* lookup_len(int n);

}  // namespace rve

#define RVE_LEN_KERNELS(T_, NA_, NB_)                                                                  \
  {&rve::k_fwd_axis2<T_, NA_, NB_>, &rve::k_fwd_axis2<T_, NA_, NB_, true>, &rve::k_axis1<T_, NA_, NB_, -1>, &rve::k_axis1<T_, NA_, NB_, 1>, \
   &rve::k_axis0_project<T_, NA_, NB_, false>, &rve::k_axis0_project<T_, NA_, NB_, true>,              \
   &rve::k_axis0_project_split<T_, NA_, NB_, false>, &rve::k_axis0_project_split<T_, NA_, NB_, true>,  \
   &rve::k_axis0_project_split3<T_, NA_, NB_, false>, &rve::k_axis0_project_split3<T_, NA_, NB_, true>, \
   &rve::k_inv_axis2<T_, NA_, NB_>, &rve::k_strided<T_, NA_, NB_, -1>, &rve::k_strided<T_, NA_, NB_, 1>, \
   &rve::k_row_pair<T_, NA_, NB_>}
#define RVE_LEN_ENTRY(N_, NA_, NB_) \
  rve::LenEntry { N_, NA_, NB_, RVE_LEN_KERNELS(float, NA_, NB_), RVE_LEN_KERNELS(double, NA_, NB_) }
