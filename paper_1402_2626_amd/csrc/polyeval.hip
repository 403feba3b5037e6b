// C ABI of the polyeval library (include/polyeval.h): system loading,
// evaluation, adjoint, batches, Gauss-Newton steps and launch-shape tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/polyeval.h"
#include "eval_kernels.hpp"
#include "newton_kernels.hpp"
#include "packer.hpp"

using namespace pe;

// ------------------------------------------------------------------ errors

namespace {

thread_local std::string g_last_error;

pe_status fail(pe_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define PE_HIP(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(e_ == hipErrorOutOfMemory ? PE_ENOMEM : PE_EDEVICE,                              \
                  std::string(#call) + ": " + hipGetErrorString(e_));                              \
  } while (0)

// chunk slot budget per level: about 36 KB of LDS for D and DD (so that a
// workgroup can hold four chunks at once), 68 KB for QD
int default_seg(int L) { return L == 1 ? 8 : 4; }

int default_slots(int L) { return L == 1 ? 2304 : (L == 2 ? 1152 : 1088); }

int cpl_bucket(int ncols, int T) {
  int c = (ncols + T - 1) / T;
  if (c <= 1) return 1;
  if (c <= 2) return 2;
  if (c <= 4) return 4;
  if (c <= 8) return 8;
  return 0;
}

size_t device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return size_t(v);
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct Plan {
  int G = 1;  // chunks processed at once (workgroup of G * 256 threads)
  int seg = 4;
  int cpl = 1;
  int max_slots = 2048;
  int tab_last = 0;
  size_t lds = 0;   // this plan's workgroup LDS
  size_t lds1 = 0;  // LDS of a one-chunk workgroup (adjoint and batches)
};

struct pe_system {
  int device = 0;
  int level = 0;
  Packed host;  // kept for batches and tuning (structure only)
  Plan plan;
  SysView view{};
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  // adjoint workspace
  mutable std::mutex ws_mu;
  mutable void* adj_ws = nullptr;
  mutable size_t adj_ws_bytes = 0;
};

// ------------------------------------------------------------------ kernel dispatch

namespace {

template <int L, int SEG, int CPL, int G, int MODE>
hipError_t launch_rows_t(const pe_system* sys, int P, const double* x, const OutView& O, hipStream_t st) {
  auto kern = eval_rows_kernel<L, SEG, CPL, G, MODE>;
  const size_t lds = sys->plan.lds;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = int64_t(P) * sys->view.N;
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(G * kSub), lds, st, sys->view, O, x,
                     int64_t(2) * L * sys->view.n);
  return hipGetLastError();
}

template <int L, int SEG, int CPL>
hipError_t launch_adj_t(const pe_system* sys, int P, const double* x, const double* v, int NG, int gsize,
                        double* part, double* g, hipStream_t st) {
  auto kern = adjoint_rows_kernel<L, SEG, CPL>;
  const size_t lds = sys->plan.lds1;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  const int n = sys->view.n;
  hipLaunchKernelGGL(kern, dim3(unsigned(int64_t(P) * NG)), dim3(kSub), lds, st, sys->view, x,
                     int64_t(2) * L * n, v, int64_t(2) * L * sys->view.N, NG, gsize, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = int64_t(P) * n;
  hipLaunchKernelGGL(adjoint_reduce_kernel<L>, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, n, NG, P,
                     (const double*)part, g);
  return hipGetLastError();
}

// dispatch over (G, CPL, MODE) for a level
template <int L, int SEG>
hipError_t dispatch_rows_seg(const pe_system* sys, int P, const double* x, const OutView& O, int mode,
                             hipStream_t st) {
  const int G = sys->plan.G;
  switch ((G * 16 + sys->plan.cpl) * 4 + mode) {
#define PE_CASE(G_, CPL, MODE) \
  case (G_ * 16 + CPL) * 4 + MODE:  \
    return launch_rows_t<L, SEG, CPL, G_, MODE>(sys, P, x, O, st);
    PE_CASE(1, 1, MODE_EVAL)
    PE_CASE(1, 1, MODE_FONLY)
    PE_CASE(1, 2, MODE_EVAL)
    PE_CASE(1, 2, MODE_FONLY)
    PE_CASE(1, 4, MODE_EVAL)
    PE_CASE(1, 4, MODE_FONLY)
    PE_CASE(1, 8, MODE_EVAL)
    PE_CASE(1, 8, MODE_FONLY)
#undef PE_CASE
  }
  return hipErrorInvalidValue;
}

// the four-chunk workgroups exist for D and DD with up to 512 columns
template <int L, int SEG>
hipError_t dispatch_rows_seg_g4(const pe_system* sys, int P, const double* x, const OutView& O, int mode,
                                hipStream_t st) {
  switch (sys->plan.cpl * 4 + mode) {
    case 1 * 4 + MODE_EVAL: return launch_rows_t<L, SEG, 1, 4, MODE_EVAL>(sys, P, x, O, st);
    case 1 * 4 + MODE_FONLY: return launch_rows_t<L, SEG, 1, 4, MODE_FONLY>(sys, P, x, O, st);
    case 2 * 4 + MODE_EVAL: return launch_rows_t<L, SEG, 2, 4, MODE_EVAL>(sys, P, x, O, st);
    case 2 * 4 + MODE_FONLY: return launch_rows_t<L, SEG, 2, 4, MODE_FONLY>(sys, P, x, O, st);
  }
  return hipErrorInvalidValue;
}

template <int L, int SEG>
hipError_t dispatch_adj_seg(const pe_system* sys, int P, const double* x, const double* v, int NG, int gsize,
                            double* part, double* g, hipStream_t st) {
  switch (sys->plan.cpl) {
    case 1: return launch_adj_t<L, SEG, 1>(sys, P, x, v, NG, gsize, part, g, st);
    case 2: return launch_adj_t<L, SEG, 2>(sys, P, x, v, NG, gsize, part, g, st);
    case 4: return launch_adj_t<L, SEG, 4>(sys, P, x, v, NG, gsize, part, g, st);
    case 8: return launch_adj_t<L, SEG, 8>(sys, P, x, v, NG, gsize, part, g, st);
  }
  return hipErrorInvalidValue;
}

hipError_t dispatch_rows(const pe_system* sys, int P, const double* x, const OutView& O, int mode,
                         hipStream_t st) {
  const int L = sys->level, seg = sys->plan.seg, G = sys->plan.G;
  if (G == 4) {
    if (L == 1 && seg == 8) return dispatch_rows_seg_g4<1, 8>(sys, P, x, O, mode, st);
    if (L == 2 && seg == 4) return dispatch_rows_seg_g4<2, 4>(sys, P, x, O, mode, st);
    return hipErrorInvalidValue;
  }
  if (L == 1 && seg == 8) return dispatch_rows_seg<1, 8>(sys, P, x, O, mode, st);
  if (L == 2 && seg == 4) return dispatch_rows_seg<2, 4>(sys, P, x, O, mode, st);
  if (L == 4 && seg == 4) return dispatch_rows_seg<4, 4>(sys, P, x, O, mode, st);
  return hipErrorInvalidValue;
}

hipError_t dispatch_adj(const pe_system* sys, int P, const double* x, const double* v, int NG, int gsize,
                        double* part, double* g, hipStream_t st) {
  const int L = sys->level, seg = sys->plan.seg;
  if (L == 1 && seg == 8) return dispatch_adj_seg<1, 8>(sys, P, x, v, NG, gsize, part, g, st);
  if (L == 2 && seg == 4) return dispatch_adj_seg<2, 4>(sys, P, x, v, NG, gsize, part, g, st);
  if (L == 4 && seg == 4) return dispatch_adj_seg<4, 4>(sys, P, x, v, NG, gsize, part, g, st);
  return hipErrorInvalidValue;
}

template <typename T>
pe_status upload(pe_system* sys, const std::vector<T>& v, const T*& dst, hipStream_t st) {
  if (v.empty()) {
    dst = nullptr;
    return PE_OK;
  }
  void* p = nullptr;
  const size_t bytes = v.size() * sizeof(T);
  PE_HIP(hipMalloc(&p, bytes));
  sys->allocs.push_back(p);
  sys->device_bytes += bytes;
  PE_HIP(hipMemcpyAsync(p, v.data(), bytes, hipMemcpyHostToDevice, st));
  dst = static_cast<const T*>(p);
  return PE_OK;
}

// Launch shape: G chunks at once (G = 4 needs at least two chunks in some
// row, room in LDS for four slot regions and n + R <= 512 columns).
pe_status choose_plan(pe_system* sys, int seg, int force_G) {
  Packed& H = sys->host;
  Plan pl;
  pl.seg = seg;
  pl.max_slots = std::max(H.max_slots_used, 1);
  pl.cpl = cpl_bucket(H.ncols, kSub);
  if (pl.cpl == 0) return fail(PE_EUNSUPPORTED, "more than 2048 columns (n + R) is not supported");
  const size_t limit = device_lds_limit();
  const int L = H.level;
  auto lds_for = [&](int tab_last, int G) { return lds_bytes<1>(H.n, tab_last, pl.max_slots, H.R, G) * L; };
  pl.tab_last = 0;
  if (H.emax - 1 >= 2 && lds_for(H.emax - 1, 1) <= limit) pl.tab_last = H.emax - 1;
  int max_chunks = 0;
  for (int p = 0; p < H.N; ++p) max_chunks = std::max<int>(max_chunks, H.chunk_ptr[p + 1] - H.chunk_ptr[p]);
  pl.G = 1;
  const bool g4_ok = L <= 2 && pl.cpl <= 2 && H.ncols * 3 <= pl.max_slots * 4 && lds_for(pl.tab_last, 4) <= limit;
  if (force_G == 4 && !g4_ok) return fail(PE_EUNSUPPORTED, "four-chunk workgroups do not fit this system");
  if (force_G == 4 || (force_G == 0 && g4_ok && max_chunks >= 2)) pl.G = 4;  // force_G == 1 keeps 1
  pl.lds = lds_for(pl.tab_last, pl.G);
  pl.lds1 = lds_for(pl.tab_last, 1);
  if (pl.lds > limit) return fail(PE_EUNSUPPORTED, "workgroup LDS need exceeds the device limit");
  sys->plan = pl;
  return PE_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int32_t pe_abi_version(void) { return 1; }

const char* pe_last_error(void) { return g_last_error.c_str(); }

pe_status pe_system_create(pe_system** out, int32_t level, int32_t n_vars, int32_t n_polys,
                           const int64_t* poly_ptr, const int64_t* mon_ptr, const int32_t* var_idx,
                           const int32_t* exps, const double* coef, void* stream) {
  g_last_error.clear();
  if (!out) return fail(PE_EINVAL, "out is NULL");
  *out = nullptr;
  SysInput in;
  in.level = level;
  in.n_vars = n_vars;
  in.n_polys = n_polys;
  in.poly_ptr = poly_ptr;
  in.mon_ptr = mon_ptr;
  in.var_idx = var_idx;
  in.exps = exps;
  in.coef = coef;
  PackParams pp;
  pp.threads = kSub;
  pp.seg = (level == 1 || level == 2 || level == 4) ? default_seg(level) : 4;
  pp.max_slots = (level == 1 || level == 2 || level == 4) ? default_slots(level) : 2048;
  std::string msg;
  auto* sys = new (std::nothrow) pe_system();
  if (!sys) return fail(PE_ENOMEM, "host allocation failed");
  int st = pack_system(in, pp, sys->host, msg);
  if (st != kOk) {
    delete sys;
    return fail(st, msg);
  }
  sys->level = level;
  pe_status ps = choose_plan(sys, pp.seg, 0);
  if (ps != PE_OK) {
    delete sys;
    return ps;
  }
  hipError_t he = hipGetDevice(&sys->device);
  if (he != hipSuccess) {
    delete sys;
    return fail(PE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const Packed& H = sys->host;
  SysView& V = sys->view;
  V.n = H.n;
  V.N = H.N;
  V.R = H.R;
  V.ncols = H.ncols;
  V.emax = H.emax;
  V.tab_last = sys->plan.tab_last;
  V.max_slots = sys->plan.max_slots;
  pe_status e = PE_OK;
  if ((e = upload(sys, H.chunks, V.chunks, hs)) != PE_OK || (e = upload(sys, H.chunk_ptr, V.chunk_ptr, hs)) != PE_OK ||
      (e = upload(sys, H.occ, V.occ, hs)) != PE_OK || (e = upload(sys, H.mcoef, V.mcoef, hs)) != PE_OK ||
      (e = upload(sys, H.mmeta, V.mmeta, hs)) != PE_OK || (e = upload(sys, H.colptr, V.colptr, hs)) != PE_OK) {
    pe_system_destroy(sys);
    return e;
  }
  he = hipStreamSynchronize(hs);
  if (he != hipSuccess) {
    pe_system_destroy(sys);
    return fail(PE_EDEVICE, std::string("upload: ") + hipGetErrorString(he));
  }
  // the device copies are authoritative; keep only what batches and tuning need
  sys->host.occ.clear();
  sys->host.occ.shrink_to_fit();
  sys->host.mcoef.clear();
  sys->host.mcoef.shrink_to_fit();
  sys->host.colptr.clear();
  sys->host.colptr.shrink_to_fit();
  *out = sys;
  return PE_OK;
}

pe_status pe_system_destroy(pe_system* sys) {
  if (!sys) return PE_OK;
  for (void* p : sys->allocs) (void)hipFree(p);
  if (sys->adj_ws) (void)hipFree(sys->adj_ws);
  delete sys;
  return PE_OK;
}

pe_status pe_system_info(const pe_system* sys, int64_t info[10]) {
  if (!sys || !info) return fail(PE_EINVAL, "NULL argument");
  const Packed& H = sys->host;
  info[0] = sys->level;
  info[1] = H.n;
  info[2] = H.N;
  info[3] = H.M;
  info[4] = H.nnz;
  info[5] = H.emax;
  info[6] = H.kmax;
  info[7] = int64_t(sys->device_bytes);
  info[8] = sys->plan.G;
  info[9] = int64_t(sys->plan.lds);
  return PE_OK;
}

pe_status pe_system_set_shape(pe_system* sys, int32_t chunks_per_workgroup) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (chunks_per_workgroup != 0 && chunks_per_workgroup != 1 && chunks_per_workgroup != 4)
    return fail(PE_EINVAL, "chunks_per_workgroup must be 0, 1 or 4");
  Plan saved = sys->plan;
  pe_status st = choose_plan(sys, sys->plan.seg, chunks_per_workgroup);
  if (st != PE_OK) {
    sys->plan = saved;
    return st;
  }
  sys->view.tab_last = sys->plan.tab_last;
  sys->view.max_slots = sys->plan.max_slots;
  return PE_OK;
}

pe_status pe_eval(const pe_system* sys, int32_t P, const double* x, double* F, double* J, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0 || sys->view.N == 0) return PE_OK;
  if (!x || !F) return fail(PE_EINVAL, "x or F is NULL");
  if (int64_t(P) * sys->view.N > 0x7fffffffLL) return fail(PE_EUNSUPPORTED, "P * N too large");
  const int L = sys->level, n = sys->view.n, N = sys->view.N;
  OutView O;
  O.J = J;
  O.j_plane = int64_t(N) * n;
  O.j_pt = 2 * L * O.j_plane;
  O.j_row = n;
  O.F = F;
  O.f_plane = N;
  O.f_pt = 2 * L * int64_t(N);
  O.f_row = 1;
  O.f_sign = 1.0;
  hipError_t e = dispatch_rows(sys, P, x, O, J ? MODE_EVAL : MODE_FONLY, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("eval launch: ") + hipGetErrorString(e));
  return PE_OK;
}

pe_status pe_eval_adjoint(const pe_system* sys, int32_t P, const double* x, const double* v, double* g,
                          void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0) return PE_OK;
  if (!x || !v || !g) return fail(PE_EINVAL, "x, v or g is NULL");
  const int L = sys->level, n = sys->view.n, N = sys->view.N;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (N == 0) {
    PE_HIP(hipMemsetAsync(g, 0, size_t(P) * 2 * L * n * sizeof(double), hs));
    return PE_OK;
  }
  // groups of polynomials: enough workgroups to fill the device
  const int target = 4096;
  int gsize = int(std::max<int64_t>(1, (int64_t(N) * P + target - 1) / target));
  gsize = std::min(gsize, N);
  const int NG = (N + gsize - 1) / gsize;
  const size_t need = size_t(P) * NG * 2 * L * n * sizeof(double);
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lk(sys->ws_mu);
    if (sys->adj_ws_bytes < need) {
      if (sys->adj_ws) {
        PE_HIP(hipStreamSynchronize(hs));
        (void)hipFree(sys->adj_ws);
        sys->adj_ws = nullptr;
        sys->adj_ws_bytes = 0;
      }
      PE_HIP(hipMalloc(&sys->adj_ws, need));
      sys->adj_ws_bytes = need;
    }
    part = static_cast<double*>(sys->adj_ws);
  }
  hipError_t e = dispatch_adj(sys, P, x, v, NG, gsize, part, g, hs);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("adjoint launch: ") + hipGetErrorString(e));
  return PE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ Newton

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct NewtonLayout {
  size_t w_off, r_off, y_off, total;
  int64_t w_pt, r_pt, y_pt;  // in doubles
};

NewtonLayout newton_layout(int L, int N, int n, int P) {
  NewtonLayout lo;
  lo.w_pt = int64_t(2) * L * N * (n + 1);
  lo.r_pt = int64_t(n) * (n + 1) * 2 * L;
  lo.y_pt = int64_t(n) * 2 * L;
  lo.w_off = 0;
  lo.r_off = align256(lo.w_off + size_t(P) * lo.w_pt * sizeof(double));
  lo.y_off = align256(lo.r_off + size_t(P) * lo.r_pt * sizeof(double));
  lo.total = align256(lo.y_off + size_t(P) * lo.y_pt * sizeof(double));
  return lo;
}

template <int L>
hipError_t launch_mgs(int P, int N, int n, double* W, const NewtonLayout& lo, char* base, double* x,
                      double* resid, hipStream_t st) {
  auto kern = mgs_solve_kernel<L, kMgsThreads>;
  const size_t lds = mgs_lds_bytes<L>(N);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(unsigned(P)), dim3(kMgsThreads), lds, st, N, n, W, lo.w_pt,
                     reinterpret_cast<double*>(base + lo.r_off), lo.r_pt, reinterpret_cast<double*>(base + lo.y_off),
                     lo.y_pt, x, int64_t(2) * L * n, resid);
  return hipGetLastError();
}

pe_status newton_check(const pe_system* sys, int P) {
  const int n = sys->view.n, N = sys->view.N;
  if (N < n) return fail(PE_EUNSUPPORTED, "Gauss-Newton needs at least as many polynomials as variables");
  if (n + 1 > 1024) return fail(PE_EUNSUPPORTED, "Gauss-Newton supports n + 1 <= 1024");
  const int L = sys->level;
  const size_t lds = L == 1 ? mgs_lds_bytes<1>(N) : (L == 2 ? mgs_lds_bytes<2>(N) : mgs_lds_bytes<4>(N));
  if (lds > device_lds_limit()) return fail(PE_EUNSUPPORTED, "too many polynomials for the LDS pivot column");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  return PE_OK;
}

}  // namespace

extern "C" {

size_t pe_newton_workspace_bytes(const pe_system* sys, int32_t P) {
  if (!sys || P < 0) return 0;
  return newton_layout(sys->level, sys->view.N, sys->view.n, P).total;
}

pe_status pe_newton_step(const pe_system* sys, int32_t P, double* x_inout, void* workspace, double* resid_out,
                         void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  pe_status ps = newton_check(sys, P);
  if (ps != PE_OK) return ps;
  if (P == 0) return PE_OK;
  if (!x_inout || !workspace) return fail(PE_EINVAL, "x or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(PE_EINVAL, "workspace must be 256-byte aligned");
  const int L = sys->level, n = sys->view.n, N = sys->view.N;
  const NewtonLayout lo = newton_layout(L, N, n, P);
  char* base = static_cast<char*>(workspace);
  double* W = reinterpret_cast<double*>(base + lo.w_off);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  OutView O;
  O.J = W;
  O.j_row = n + 1;
  O.j_plane = int64_t(N) * (n + 1);
  O.j_pt = lo.w_pt;
  O.F = W + n;
  O.f_row = n + 1;
  O.f_plane = O.j_plane;
  O.f_pt = lo.w_pt;
  O.f_sign = -1.0;
  hipError_t e = dispatch_rows(sys, P, x_inout, O, MODE_EVAL, hs);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("newton eval launch: ") + hipGetErrorString(e));
  if (L == 1) e = launch_mgs<1>(P, N, n, W, lo, base, x_inout, resid_out, hs);
  if (L == 2) e = launch_mgs<2>(P, N, n, W, lo, base, x_inout, resid_out, hs);
  if (L == 4) e = launch_mgs<4>(P, N, n, W, lo, base, x_inout, resid_out, hs);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("newton solve launch: ") + hipGetErrorString(e));
  return PE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct pe_batch {
  int device = 0;
  int level = 0;
  int S = 0;
  int seg = 4;
  int cpl = 1;
  size_t lds = 0;
  int maxN = 0;
  std::vector<const pe_system*> systems;
  std::vector<int64_t> x_off, F_off, J_off;  // per point, doubles, [S+1]
  std::vector<BatchNewtonDesc> ndesc;        // per point offsets of the Newton workspace
  int64_t w_total = 0, r_total = 0, y_total = 0;  // per point, doubles
  int64_t nitems = 0;
  SysView* d_views = nullptr;
  uint64_t* d_items = nullptr;
  int64_t* d_offs = nullptr;  // x_off | F_off | J_off | W offsets, each [S+1]
  BatchNewtonDesc* d_ndesc = nullptr;
  int* d_order = nullptr;
  int* d_counter = nullptr;
  int grid = 0;
};

namespace {

template <int L, int SEG, int CPL, int MODE>
hipError_t launch_batch_t(const pe_batch* b, int P, const double* x, const BatchOut& out, hipStream_t st) {
  auto kern = batch_rows_kernel<L, SEG, CPL, MODE>;
  if (b->lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(b->lds));
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, kSub, b->lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(int64_t(std::max(per_cu, 1)) * cus, b->nitems));
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, b->d_counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kSub), b->lds, st, (const SysView*)b->d_views,
                     (const uint64_t*)b->d_items, b->nitems, b->d_counter, P, x, (const int64_t*)b->d_offs, out);
  return hipGetLastError();
}

template <int L, int SEG>
hipError_t dispatch_batch_seg(const pe_batch* b, int P, const double* x, const BatchOut& out, int mode,
                              hipStream_t st) {
  switch (b->cpl * 4 + mode) {
#define PE_CASE(CPL, MODE) \
  case CPL * 4 + MODE:     \
    return launch_batch_t<L, SEG, CPL, MODE>(b, P, x, out, st);
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

hipError_t dispatch_batch(const pe_batch* b, int P, const double* x, const BatchOut& out, int mode, hipStream_t st) {
  if (b->level == 1 && b->seg == 8) return dispatch_batch_seg<1, 8>(b, P, x, out, mode, st);
  if (b->level == 2 && b->seg == 4) return dispatch_batch_seg<2, 4>(b, P, x, out, mode, st);
  if (b->level == 4 && b->seg == 4) return dispatch_batch_seg<4, 4>(b, P, x, out, mode, st);
  return hipErrorInvalidValue;
}

void batch_free(pe_batch* b) {
  for (void* p : {(void*)b->d_views, (void*)b->d_items, (void*)b->d_offs, (void*)b->d_ndesc, (void*)b->d_order,
                  (void*)b->d_counter})
    if (p) (void)hipFree(p);
}

template <typename T>
pe_status upload_raw(const std::vector<T>& v, T** dst, hipStream_t st) {
  *dst = nullptr;
  if (v.empty()) return PE_OK;
  PE_HIP(hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T)));
  PE_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return PE_OK;
}

}  // namespace

extern "C" {

pe_status pe_batch_create(pe_batch** out, int32_t S, const pe_system* const* systems, void* stream) {
  if (!out) return fail(PE_EINVAL, "out is NULL");
  *out = nullptr;
  if (S < 1 || !systems) return fail(PE_EINVAL, "need at least one system");
  auto* b = new (std::nothrow) pe_batch();
  if (!b) return fail(PE_ENOMEM, "host allocation failed");
  b->S = S;
  b->systems.assign(systems, systems + S);
  for (int s = 0; s < S; ++s)
    if (!systems[s]) {
      delete b;
      return fail(PE_EINVAL, "system " + std::to_string(s) + " is NULL");
    }
  b->level = systems[0]->level;
  b->seg = systems[0]->plan.seg;
  b->device = systems[0]->device;
  int maxcols = 1;
  for (int s = 0; s < S; ++s) {
    const pe_system* y = systems[s];
    if (y->level != b->level || y->plan.seg != b->seg || y->device != b->device) {
      delete b;
      return fail(PE_EINVAL, "batched systems must share level, launch shape and device");
    }
    maxcols = std::max(maxcols, y->view.ncols);
    b->lds = std::max(b->lds, y->plan.lds1);
    b->maxN = std::max(b->maxN, y->view.N);
  }
  b->cpl = cpl_bucket(maxcols, kSub);
  const int L = b->level;
  // packed layout per point
  b->x_off.assign(S + 1, 0);
  b->F_off.assign(S + 1, 0);
  b->J_off.assign(S + 1, 0);
  std::vector<int64_t> w_off(S + 1, 0);
  b->ndesc.resize(S);
  int64_t ro = 0, yo = 0;
  for (int s = 0; s < S; ++s) {
    const int n = systems[s]->view.n, N = systems[s]->view.N;
    b->x_off[s + 1] = b->x_off[s] + int64_t(2) * L * n;
    b->F_off[s + 1] = b->F_off[s] + int64_t(2) * L * N;
    b->J_off[s + 1] = b->J_off[s] + int64_t(2) * L * N * n;
    w_off[s + 1] = w_off[s] + int64_t(2) * L * N * (n + 1);
    BatchNewtonDesc& d = b->ndesc[s];
    d.N = N;
    d.n = n;
    d.w_off = w_off[s];
    d.r_off = ro;
    d.y_off = yo;
    d.x_off = b->x_off[s];
    ro += int64_t(n) * (n + 1) * 2 * L;
    yo += int64_t(n) * 2 * L;
  }
  b->w_total = w_off[S];
  b->r_total = ro;
  b->y_total = yo;
  // work items in decreasing cost (longest processing time first)
  std::vector<std::pair<int64_t, uint64_t>> items;
  for (int s = 0; s < S; ++s) {
    const Packed& H = systems[s]->host;
    for (int p = 0; p < H.N; ++p) items.push_back({H.poly_cost[p], (uint64_t(s) << 32) | uint64_t(p)});
  }
  std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
  std::vector<uint64_t> it(items.size());
  for (size_t i = 0; i < items.size(); ++i) it[i] = items[i].second;
  b->nitems = int64_t(it.size());
  std::vector<SysView> views(S);
  for (int s = 0; s < S; ++s) views[s] = systems[s]->view;
  std::vector<int64_t> offs;
  offs.insert(offs.end(), b->x_off.begin(), b->x_off.end());
  offs.insert(offs.end(), b->F_off.begin(), b->F_off.end());
  offs.insert(offs.end(), b->J_off.begin(), b->J_off.end());
  offs.insert(offs.end(), w_off.begin(), w_off.end());
  std::vector<int> order(S);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return int64_t(systems[a]->view.n) * systems[a]->view.N > int64_t(systems[c]->view.n) * systems[c]->view.N;
  });
  hipStream_t hs = static_cast<hipStream_t>(stream);
  pe_status e = PE_OK;
  if ((e = upload_raw(views, &b->d_views, hs)) != PE_OK || (e = upload_raw(it, &b->d_items, hs)) != PE_OK ||
      (e = upload_raw(offs, &b->d_offs, hs)) != PE_OK || (e = upload_raw(b->ndesc, &b->d_ndesc, hs)) != PE_OK ||
      (e = upload_raw(order, &b->d_order, hs)) != PE_OK) {
    batch_free(b);
    delete b;
    return e;
  }
  hipError_t he = hipMalloc(reinterpret_cast<void**>(&b->d_counter), sizeof(int));
  if (he == hipSuccess) he = hipStreamSynchronize(hs);
  if (he != hipSuccess) {
    batch_free(b);
    delete b;
    return fail(PE_EDEVICE, std::string("batch upload: ") + hipGetErrorString(he));
  }
  *out = b;
  return PE_OK;
}

pe_status pe_batch_destroy(pe_batch* b) {
  if (!b) return PE_OK;
  batch_free(b);
  delete b;
  return PE_OK;
}

pe_status pe_batch_layout(const pe_batch* b, int64_t* x_off, int64_t* F_off, int64_t* J_off) {
  if (!b) return fail(PE_EINVAL, "batch is NULL");
  for (int s = 0; s <= b->S; ++s) {
    if (x_off) x_off[s] = b->x_off[s];
    if (F_off) F_off[s] = b->F_off[s];
    if (J_off) J_off[s] = b->J_off[s];
  }
  return PE_OK;
}

pe_status pe_batch_eval(const pe_batch* b, int32_t P, const double* x, double* F, double* J, void* stream) {
  if (!b) return fail(PE_EINVAL, "batch is NULL");
  if (P < 0) return fail(PE_EINVAL, "points_per_system must be nonnegative");
  if (P == 0 || b->nitems == 0) return PE_OK;
  if (!x || !F) return fail(PE_EINVAL, "x or F is NULL");
  BatchOut out;
  out.J = J;
  out.J_off = b->d_offs + 2 * (b->S + 1);
  out.F = F;
  out.F_off = b->d_offs + (b->S + 1);
  out.newton = 0;
  hipError_t e = dispatch_batch(b, P, x, out, J ? MODE_EVAL : MODE_FONLY, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
  return PE_OK;
}

size_t pe_batch_newton_workspace_bytes(const pe_batch* b, int32_t P) {
  if (!b || P < 0) return 0;
  // [W blocks][R blocks][y blocks]
  return align256(size_t(P) * b->w_total * 8) + align256(size_t(P) * b->r_total * 8) +
         align256(size_t(P) * b->y_total * 8);
}

pe_status pe_batch_newton_step(const pe_batch* b, int32_t P, double* x_inout, void* workspace, double* resid_out,
                               void* stream) {
  if (!b) return fail(PE_EINVAL, "batch is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0) return PE_OK;
  if (!x_inout || !workspace) return fail(PE_EINVAL, "x or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(PE_EINVAL, "workspace must be 256-byte aligned");
  for (const pe_system* y : b->systems) {
    pe_status ps = newton_check(y, P);
    if (ps != PE_OK) return ps;
  }
  const int L = b->level;
  char* base = static_cast<char*>(workspace);
  double* W = reinterpret_cast<double*>(base);
  double* Rw = reinterpret_cast<double*>(base + align256(size_t(P) * b->w_total * 8));
  double* Yw = reinterpret_cast<double*>(base + align256(size_t(P) * b->w_total * 8) + align256(size_t(P) * b->r_total * 8));
  hipStream_t hs = static_cast<hipStream_t>(stream);
  BatchOut out;
  out.J = W;
  out.J_off = b->d_offs + 3 * (b->S + 1);
  out.F = nullptr;
  out.F_off = nullptr;
  out.newton = 1;
  hipError_t e = dispatch_batch(b, P, x_inout, out, MODE_EVAL, hs);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("batch newton eval: ") + hipGetErrorString(e));
  size_t lds = L == 1 ? mgs_lds_bytes<1>(b->maxN) : (L == 2 ? mgs_lds_bytes<2>(b->maxN) : mgs_lds_bytes<4>(b->maxN));
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 65536) {
      hipError_t e2 = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e2 != hipSuccess) return e2;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(int64_t(b->S) * P)), dim3(kMgsThreads), lds, hs,
                       (const BatchNewtonDesc*)b->d_ndesc, (const int*)b->d_order, P, W, Rw, Yw, x_inout, resid_out);
    return hipGetLastError();
  };
  if (L == 1) e = go(mgs_solve_batch_kernel<1, kMgsThreads>);
  if (L == 2) e = go(mgs_solve_batch_kernel<2, kMgsThreads>);
  if (L == 4) e = go(mgs_solve_batch_kernel<4, kMgsThreads>);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("batch newton solve: ") + hipGetErrorString(e));
  return PE_OK;
}

pe_status pe_autotune(pe_system*, int32_t, void*) { return PE_OK; }
pe_status pe_set_plan_cache(const char*) { return PE_OK; }

}  // extern "C"
