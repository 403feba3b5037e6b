// Host-side launchers of the device kernels.  Each launcher is a template
// over the level L; its instances for one (level, kind) are compiled in their
// own translation unit (instances.hip built with PE_LEVEL and PE_KIND), so the
// library builds in parallel.  polyeval.hip only sees the declarations.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "eval_kernels.hpp"
#include "lstsq_kernels.hpp"
#include "newton_kernels.hpp"

namespace pe {

// The compiled launch shapes (level, segment length, chunks per workgroup).
// A workgroup of G chunks has G * 256 threads; G > 1 is compiled for up to
// 512 columns only.  Double double with segments of 16 and quad double with
// segments of 8 exist for monomials too wide for the shorter segments (up to
// 1024 and 512 variables in one wavefront); they hold many registers per lane.
#define PE_SHAPES(X) \
  X(1, 8, 1)         \
  X(1, 8, 4)         \
  X(1, 16, 1)        \
  X(1, 16, 2)        \
  X(2, 4, 1)         \
  X(2, 4, 4)         \
  X(2, 6, 1)         \
  X(2, 6, 2)         \
  X(2, 8, 1)         \
  X(2, 8, 2)         \
  X(2, 16, 1)        \
  X(4, 4, 1)         \
  X(4, 2, 1)         \
  X(4, 8, 1)

inline bool shape_compiled(int L, int seg, int G) {
#define PE_X(L_, S_, G_) \
  if (L == L_ && seg == S_ && G == G_) return true;
  PE_SHAPES(PE_X)
#undef PE_X
  return false;
}

// what a launch over one system needs to know about its plan
struct EvalShape {
  SysView view;
  int seg = 4, G = 1, cpl = 1;
  size_t lds = 0;   // dynamic LDS of a workgroup of G chunks
  size_t lds1 = 0;  // dynamic LDS of a one-chunk workgroup
  int64_t n_chunks = 0;  // chunks of the system (per-monomial output)
};

// one persistent launch over the items of a batch class
struct BatchShape {
  int seg = 4, G = 1, cpl = 1;
  int vw = 0;  // copy width of batch_small_kernel, 0: batch_rows_kernel
  size_t lds = 0;
  int64_t nitems = 0;
  const uint64_t* items = nullptr;
  const SysView* views = nullptr;
  const int64_t* x_off = nullptr;
  int* counter = nullptr;
};

template <int L>
hipError_t launch_rows(const EvalShape& sh, int P, const double* x, const OutView& O, int mode, hipStream_t st);

// per-monomial output (terms_waves_kernel)
template <int L>
hipError_t launch_terms(const EvalShape& sh, int P, const double* x, const OutView& O, hipStream_t st);
template <int L>
hipError_t launch_adjoint(const EvalShape& sh, int P, const double* x, const double* v, int NG, int gsize,
                          double* part, double* g, hipStream_t st);
template <int L>
hipError_t launch_batch(const BatchShape& b, int P, const double* x, const BatchOut& out, int mode,
                        hipStream_t st);
template <int L>
hipError_t launch_mgs(int P, int N, int n, double* W, int64_t w_pt, double* R, int64_t r_pt, double* Y,
                      int64_t y_pt, double* x, double* resid, hipStream_t st);
template <int L>
hipError_t launch_mgs_batch(int S, int P, int maxN, const BatchNewtonDesc* desc, const int* order, double* W,
                            double* R, double* Y, double* x, double* resid, hipStream_t st);

template <int L>
hipError_t launch_rhs_shift(double* W, int64_t w_pt, int64_t plane, int64_t ld, int N, int n, int P, const double* c,
                            double wF, double wc, hipStream_t st);

// Column-parallel least-squares solve of the augmented matrices [A b] given
// row-major at A (row stride ld, component plane stride a_plane, point stride
// a_pt; see lstsq_kernels.hpp), writing x (x_pt per point; add = 1 adds the
// solution to x, the Newton update), resid[P][2] and optionally R and Q.
// PE panel of pivots per launch: kLsPanel.
constexpr int kLsPanel = 32;
constexpr int kLsMaxRows = 4096;  // N limit of the column-parallel solve

template <int L>
hipError_t launch_lstsq(const LsLayout& lo, void* ws, const double* A, int64_t ld, int64_t a_plane, int64_t a_pt,
                        double* x, int64_t x_pt, int add, double* resid, double* Rout, double* Qout,
                        hipStream_t st);

#ifdef PE_LAUNCH_DEFINITIONS

template <typename K>
hipError_t allow_lds(K kern, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

template <int L, int SEG, int CPL, int G, int MODE>
hipError_t launch_rows_t(const EvalShape& sh, int P, const double* x, const OutView& O, hipStream_t st) {
  auto kern = eval_rows_kernel<L, SEG, CPL, G, MODE>;
  hipError_t e = allow_lds(kern, sh.lds);
  if (e != hipSuccess) return e;
  // F alone needs no column tiles (no owners): one workgroup per row-point
  SysView view = sh.view;
  if (MODE == MODE_FONLY) view.col_tiles = 1;
  const int64_t blocks = int64_t(P) * view.N * view.col_tiles;
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(G * kSub), sh.lds, st, view, O, x,
                     int64_t(width_of(L)) * sh.view.n);
  return hipGetLastError();
}

template <int L, int SEG, int G>
hipError_t rows_lsg(const EvalShape& sh, int P, const double* x, const OutView& O, int mode, hipStream_t st) {
  const int cpl = sh.cpl;
  if (mode == MODE_EVAL) {
    if (cpl == 1) return launch_rows_t<L, SEG, 1, G, MODE_EVAL>(sh, P, x, O, st);
    if (cpl == 2) return launch_rows_t<L, SEG, 2, G, MODE_EVAL>(sh, P, x, O, st);
    if (G == 1 && cpl == 4) return launch_rows_t<L, SEG, 4, 1, MODE_EVAL>(sh, P, x, O, st);
    if (G == 1 && cpl == 8) return launch_rows_t<L, SEG, 8, 1, MODE_EVAL>(sh, P, x, O, st);
  } else {
    if (cpl == 1) return launch_rows_t<L, SEG, 1, G, MODE_FONLY>(sh, P, x, O, st);
    if (cpl == 2) return launch_rows_t<L, SEG, 2, G, MODE_FONLY>(sh, P, x, O, st);
    if (G == 1 && cpl == 4) return launch_rows_t<L, SEG, 4, 1, MODE_FONLY>(sh, P, x, O, st);
    if (G == 1 && cpl == 8) return launch_rows_t<L, SEG, 8, 1, MODE_FONLY>(sh, P, x, O, st);
  }
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_rows(const EvalShape& sh, int P, const double* x, const OutView& O, int mode, hipStream_t st) {
#define PE_X(L_, S_, G_) \
  if constexpr (limbs_of(L) == L_) \
    if (sh.seg == S_ && sh.G == G_) return rows_lsg<L, S_, G_>(sh, P, x, O, mode, st);
  PE_SHAPES(PE_X)
#undef PE_X
  return hipErrorInvalidValue;
}

template <int L, int SEG>
hipError_t launch_terms_t(const EvalShape& sh, int P, const double* x, const OutView& O, hipStream_t st) {
  auto kern = terms_waves_kernel<L, SEG>;
  const SysView& V = sh.view;
  const size_t lds = size_t(V.tab_last >= V.tab_first ? V.tab_last - V.tab_first + 1 : 0) * (V.n + 1) *
                     width_of(L) * sizeof(double);
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  // about eight chunks per wavefront (the table is built once per
  // workgroup), and at least 2048 workgroups in all when there are chunks
  // enough
  const int64_t quads = (sh.n_chunks + 3) / 4;
  int64_t wpp = std::max<int64_t>((quads + 7) / 8, (2048 + P - 1) / P);
  // (and at most 2^31 - 1 in all: a workgroup then takes more chunks)
  wpp = std::max<int64_t>(1, std::min<int64_t>({wpp, quads, 0x7fffffffLL / std::max(P, 1)}));
  hipLaunchKernelGGL(kern, dim3(unsigned(int64_t(P) * wpp)), dim3(kSub), lds, st, V, O, x,
                     int64_t(width_of(L)) * V.n, int(wpp), uint32_t(sh.n_chunks));
  return hipGetLastError();
}

template <int L>
hipError_t launch_terms(const EvalShape& sh, int P, const double* x, const OutView& O, hipStream_t st) {
#define PE_X(L_, S_, G_) \
  if constexpr (limbs_of(L) == L_ && G_ == 1) \
    if (sh.seg == S_) return launch_terms_t<L, S_>(sh, P, x, O, st);
  PE_SHAPES(PE_X)
#undef PE_X
  return hipErrorInvalidValue;
}

template <int L, int SEG, int CPL, int G>
hipError_t launch_adj_t(const EvalShape& sh, int P, const double* x, const double* v, int NG, int gsize,
                        double* part, double* g, hipStream_t st) {
  auto kern = adjoint_rows_kernel<L, SEG, CPL, G>;
  const size_t lds = G > 1 ? sh.lds : sh.lds1;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int n = sh.view.n;
  hipLaunchKernelGGL(kern, dim3(unsigned(int64_t(P) * NG)), dim3(G * kSub), lds, st, sh.view, x,
                     int64_t(width_of(L)) * n, v, int64_t(width_of(L)) * sh.view.N, NG, gsize, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = int64_t(P) * n;
  hipLaunchKernelGGL(adjoint_reduce_kernel<L>, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, n, NG, P,
                     (const double*)part, g);
  return hipGetLastError();
}

// the adjoint runs with the evaluation plan's chunks per workgroup when that
// is 2 (at most 512 columns), else with one chunk at a time
template <int L, int SEG, int G>
hipError_t adj_lsg(const EvalShape& sh, int P, const double* x, const double* v, int NG, int gsize,
                   double* part, double* g, hipStream_t st) {
  if constexpr (G == 2) {
    switch (sh.cpl) {
      case 1: return launch_adj_t<L, SEG, 1, 2>(sh, P, x, v, NG, gsize, part, g, st);
      case 2: return launch_adj_t<L, SEG, 2, 2>(sh, P, x, v, NG, gsize, part, g, st);
    }
    return hipErrorInvalidValue;
  } else {
    switch (sh.cpl) {
      case 1: return launch_adj_t<L, SEG, 1, 1>(sh, P, x, v, NG, gsize, part, g, st);
      case 2: return launch_adj_t<L, SEG, 2, 1>(sh, P, x, v, NG, gsize, part, g, st);
      case 4: return launch_adj_t<L, SEG, 4, 1>(sh, P, x, v, NG, gsize, part, g, st);
      case 8: return launch_adj_t<L, SEG, 8, 1>(sh, P, x, v, NG, gsize, part, g, st);
    }
    return hipErrorInvalidValue;
  }
}

template <int L>
hipError_t launch_adjoint(const EvalShape& sh, int P, const double* x, const double* v, int NG, int gsize,
                          double* part, double* g, hipStream_t st) {
  const int G = sh.G == 2 ? 2 : 1;
#define PE_X(L_, S_, G_) \
  if constexpr (L == L_ && G_ <= 2) \
    if (sh.seg == S_ && G == G_) return adj_lsg<L, S_, G_>(sh, P, x, v, NG, gsize, part, g, st);
  PE_SHAPES(PE_X)
#undef PE_X
  return hipErrorInvalidValue;
}

// persistent grid: as many workgroups as fit on the device at once, at most
// one per item
template <typename Kern>
hipError_t persistent_grid(Kern kern, int threads, size_t lds, int64_t nitems, int64_t& grid) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, threads, lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  grid = std::max<int64_t>(1, std::min<int64_t>(int64_t(std::max(per_cu, 1)) * cus, nitems));
  return hipSuccess;
}

template <int L, int SEG, int CPL, int G, int MODE>
hipError_t launch_batch_t(const BatchShape& K, int P, const double* x, const BatchOut& out, hipStream_t st) {
  auto kern = batch_rows_kernel<L, SEG, CPL, G, MODE>;
  hipError_t e = allow_lds(kern, K.lds);
  if (e != hipSuccess) return e;
  int64_t grid = 0;
  if ((e = persistent_grid(kern, G * kSub, K.lds, K.nitems, grid)) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(G * kSub), K.lds, st, K.views, K.items, K.nitems, K.counter,
                     P, x, K.x_off, out);
  return hipGetLastError();
}

template <int L, int SEG, int VW, int MODE>
hipError_t launch_batch_small_t(const BatchShape& K, int P, const double* x, const BatchOut& out, hipStream_t st) {
  auto kern = batch_small_kernel<L, SEG, VW, MODE>;
  hipError_t e = allow_lds(kern, K.lds);
  if (e != hipSuccess) return e;
  int64_t grid = 0;
  if ((e = persistent_grid(kern, kSub, K.lds, K.nitems, grid)) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kSub), K.lds, st, K.views, K.items, K.nitems, K.counter, P, x,
                     K.x_off, out);
  return hipGetLastError();
}

template <int L, int SEG>
hipError_t batch_small_ls(const BatchShape& K, int P, const double* x, const BatchOut& out, int mode,
                          hipStream_t st) {
  switch (K.vw * 4 + mode) {
#define PE_CASE(VW, MODE) \
  case VW * 4 + MODE:     \
    return launch_batch_small_t<L, SEG, VW, MODE>(K, P, x, out, st);
    PE_CASE(32, MODE_EVAL)
    PE_CASE(32, MODE_FONLY)
    PE_CASE(64, MODE_EVAL)
    PE_CASE(64, MODE_FONLY)
    PE_CASE(128, MODE_EVAL)
    PE_CASE(128, MODE_FONLY)
    PE_CASE(256, MODE_EVAL)
    PE_CASE(256, MODE_FONLY)
#undef PE_CASE
  }
  return hipErrorInvalidValue;
}

template <int L, int SEG, int G>
hipError_t batch_lsg(const BatchShape& K, int P, const double* x, const BatchOut& out, int mode, hipStream_t st) {
  if constexpr (G == 1)
    if (K.vw > 0) return batch_small_ls<L, SEG>(K, P, x, out, mode, st);
  switch (K.cpl * 4 + mode) {
#define PE_CASE(CPL, MODE) \
  case CPL * 4 + MODE:     \
    return launch_batch_t<L, SEG, CPL, G, MODE>(K, P, x, out, st);
    PE_CASE(1, MODE_EVAL)
    PE_CASE(1, MODE_FONLY)
    PE_CASE(2, MODE_EVAL)
    PE_CASE(2, MODE_FONLY)
    PE_CASE(4, MODE_EVAL)
    PE_CASE(4, MODE_FONLY)
    PE_CASE(8, MODE_EVAL)
    PE_CASE(8, MODE_FONLY)
#undef PE_CASE
  }
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_batch(const BatchShape& K, int P, const double* x, const BatchOut& out, int mode,
                        hipStream_t st) {
#define PE_X(L_, S_, G_) \
  if constexpr (L == L_ && G_ <= 2) \
    if (K.seg == S_ && K.G == G_) return batch_lsg<L, S_, G_>(K, P, x, out, mode, st);
  PE_SHAPES(PE_X)
#undef PE_X
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_mgs(int P, int N, int n, double* W, int64_t w_pt, double* R, int64_t r_pt, double* Y,
                      int64_t y_pt, double* x, double* resid, hipStream_t st) {
  auto kern = mgs_solve_kernel<L, kMgsThreads>;
  const size_t lds = mgs_lds_bytes<L>(N);
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(P)), dim3(kMgsThreads), lds, st, N, n, W, w_pt, R, r_pt, Y, y_pt, x,
                     int64_t(width_of(L)) * n, resid);
  return hipGetLastError();
}

template <int L>
hipError_t launch_mgs_batch(int S, int P, int maxN, const BatchNewtonDesc* desc, const int* order, double* W,
                            double* R, double* Y, double* x, double* resid, hipStream_t st) {
  auto kern = mgs_solve_batch_kernel<L, kMgsThreads>;
  const size_t lds = mgs_lds_bytes<L>(maxN);
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(int64_t(S) * P)), dim3(kMgsThreads), lds, st, desc, order, P, W, R, Y, x,
                     resid);
  return hipGetLastError();
}

template <int L>
hipError_t launch_rhs_shift(double* W, int64_t w_pt, int64_t plane, int64_t ld, int N, int n, int P, const double* c,
                            double wF, double wc, hipStream_t st) {
  const int64_t tot = int64_t(P) * N;
  hipLaunchKernelGGL(rhs_shift_kernel<L>, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, W, w_pt, plane, ld, N, n,
                     P, c, wF, wc);
  return hipGetLastError();
}

template <int L, int T, int EPT>
hipError_t ls_sweep(const LsView& V, int P, hipStream_t st) {
  const int n = V.n;
  auto apply = [&](int k0, int k1, int j0, int j1) -> hipError_t {
    if (j1 <= j0) return hipSuccess;
    hipLaunchKernelGGL((ls_apply_kernel<L, T, EPT>), dim3(unsigned(int64_t(P) * (j1 - j0))), dim3(T), 0, st, V, k0,
                       k1, j0, j1);
    return hipGetLastError();
  };
  hipError_t e = apply(0, 0, 0, 1);  // the norm of column 0
  for (int k0 = 0; k0 < n && e == hipSuccess; k0 += kLsPanel) {
    const int k1 = std::min(k0 + kLsPanel, n);
    for (int c = k0; c + 1 < k1 && e == hipSuccess; ++c) e = apply(c, c + 1, c + 1, k1);
    if (e == hipSuccess) e = apply(k0, k1, k1, n + 1);
  }
  return e;
}

// threads and rows per thread of the sweep: T * EPT >= N, registers for the
// column and one pivot within about 128 VGPRs
template <int L>
hipError_t ls_sweep_for(const LsView& V, int P, hipStream_t st) {
  const int N = V.N;
  if constexpr (width_of(L) <= 4) {
    if (N <= 256) return ls_sweep<L, 256, 1>(V, P, st);
    if (N <= 512) return ls_sweep<L, 256, 2>(V, P, st);
    if (N <= 1024) return ls_sweep<L, 256, 4>(V, P, st);
    if (N <= 2048) return ls_sweep<L, 256, 8>(V, P, st);
    if (N <= 3072) return ls_sweep<L, 384, 8>(V, P, st);
    if (N <= 4096) return ls_sweep<L, 512, 8>(V, P, st);
  } else {
    if (N <= 256) return ls_sweep<L, 256, 1>(V, P, st);
    if (N <= 512) return ls_sweep<L, 256, 2>(V, P, st);
    if (N <= 1024) return ls_sweep<L, 256, 4>(V, P, st);
    if (N <= 2048) return ls_sweep<L, 256, 8>(V, P, st);
    if (N <= 4096) return ls_sweep<L, 256, 16>(V, P, st);
  }
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_lstsq(const LsLayout& lo, void* ws, const double* A, int64_t ld, int64_t a_plane, int64_t a_pt,
                        double* x, int64_t x_pt, int add, double* resid, double* Rout, double* Qout,
                        hipStream_t st) {
  const LsView V = ls_view(lo, ws);
  const int P = lo.P, N = lo.N, n = lo.n;
  const int tiles = ((n + 1 + 63) / 64) * ((N + 63) / 64);
  hipLaunchKernelGGL(ls_copy_in_kernel<L>, dim3(unsigned(tiles), unsigned(width_of(L)), unsigned(P)), dim3(256), 0, st, V,
                     A, ld, a_plane, a_pt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (resid) {
    hipLaunchKernelGGL(ls_bnorm_kernel<L>, dim3(unsigned(P)), dim3(256), 0, st, V, resid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = ls_sweep_for<L>(V, P, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(ls_init_y_kernel<L>, dim3(unsigned((n + 255) / 256), unsigned(P)), dim3(256), 0, st, V);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int end = n; end > 0; end -= kBs) {
    const int s = std::max(0, end - kBs);
    hipLaunchKernelGGL(ls_backsub_diag_kernel<L>, dim3(unsigned(P)), dim3(kBs), 0, st, V, s, end);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (s > 0) {
      hipLaunchKernelGGL(ls_backsub_update_kernel<L>, dim3(unsigned((s + kBs - 1) / kBs), unsigned(P)), dim3(kBs), 0,
                         st, V, s, end);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(ls_finish_kernel<L>, dim3(unsigned(P)), dim3(256), 0, st, V, x, x_pt, add, resid);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (Rout || Qout) {
    const int64_t cnt = std::max(int64_t(N) * n, int64_t(n) * (n + 1));
    hipLaunchKernelGGL(ls_export_kernel<L>, dim3(unsigned((cnt + 255) / 256), unsigned(P)), dim3(256), 0, st, V, Rout,
                       Qout);
    e = hipGetLastError();
  }
  return e;
}

#endif  // PE_LAUNCH_DEFINITIONS

}  // namespace pe
