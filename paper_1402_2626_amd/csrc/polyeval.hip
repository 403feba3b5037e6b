// C ABI of the polyeval library (include/polyeval.h): system loading,
// evaluation, adjoint, batches, Gauss-Newton steps and launch-shape tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "polyeval.h"
#include "launch.hpp"
#include "packer.hpp"

using namespace pe;

static_assert(PE_REAL == kRealCode && PE_REAL == kRealLevel, "one real flag for the ABI, the kernels and the packer");

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
int default_seg(int L) { return L == 1 ? 8 : (L == 2 ? 8 : 4); }

// Default segment length for a system: among the level's compiled lengths
// (in order of preference), the first for which a monomial of the most
// common size k fills all its lanes' segments exactly (then the monomial
// sweeps run without branches); else the level's default.
int default_seg_for(int L, const std::vector<int64_t>& mon_ptr) {
  std::vector<int64_t> hist(kMaxMonomialVars + 1, 0);
  for (size_t t = 0; t + 1 < mon_ptr.size(); ++t) {
    const int64_t k = mon_ptr[t + 1] - mon_ptr[t];
    if (k >= 1 && k <= kMaxMonomialVars) hist[size_t(k)] += k;
  }
  int kmode = 0;
  for (int k = 1; k <= kMaxMonomialVars; ++k)
    if (hist[size_t(k)] > hist[size_t(kmode)]) kmode = k;
  if (kmode == 0) return default_seg(L);
  static const int pref1[] = {8, 16}, pref2[] = {8, 6, 4}, pref4[] = {4, 2};
  const int* pref = L == 1 ? pref1 : (L == 2 ? pref2 : pref4);
  const int np = L == 1 ? 2 : (L == 2 ? 3 : 2);
  int chosen = default_seg(L);
  for (int i = 0; i < np; ++i) {
    const int seg = pref[i];
    const int s = lanes_for(kmode, seg);
    if (s <= kMaxWave && (kmode + s - 1) / s == seg) {
      chosen = seg;
      break;
    }
  }
  // a monomial must fit in one wavefront: the shortest compiled segment that
  // holds the largest monomial, when the chosen one does not
  int kmax = 0;
  for (size_t t = 0; t + 1 < mon_ptr.size(); ++t) kmax = std::max<int>(kmax, int(mon_ptr[t + 1] - mon_ptr[t]));
  if (kmax > 0 && lanes_for(kmax, chosen) > kMaxWave)
    for (int seg : {2, 4, 6, 8, 16})
      if (shape_compiled(L, seg, 1) && lanes_for(kmax, seg) <= kMaxWave) return seg;
  return chosen;
}

int default_slots(int L) { return L == 1 ? 2304 : (L == 2 ? 1152 : 1088); }

// A workgroup of G > 1 chunks adds the partial rows of sub-groups 1..G-1
// into sub-group 0's through the G contribution regions (reused once the
// chunks are done): (G - 1) partial rows of n columns must fit in G regions of
// max_slots slots, and the row accumulators of a multi-chunk kernel cover at
// most 2 * 256 columns.
bool multi_chunk_fits(int n, int cpl, int max_slots, int G) {
  if (G == 1) return true;
  return cpl <= 2 && int64_t(n) * (G - 1) <= int64_t(max_slots) * G;
}

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
  int tab_first = 2;
  int tab_last = 0;
  size_t lds = 0;   // this plan's workgroup LDS
  size_t lds1 = 0;  // LDS of a one-chunk workgroup (adjoint and batches)
};

struct pe_system {
  int device = 0;
  int level = 0;  // limbs per real part (1, 2, 4)
  int code = 0;   // level code: level, plus PE_REAL for real arithmetic
  int n_vars = 0;
  // the input as given (host copy), for repacking with another launch shape
  std::vector<int64_t> in_poly_ptr, in_mon_ptr;
  std::vector<int32_t> in_var, in_exp;
  std::vector<double> in_coef;
  Packed host;  // kept for batches and tuning (structure only)
  Plan plan;
  SysView view{};
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  // batches that hold a copy of this system's device view; while any is
  // alive the system may not be repacked or destroyed
  mutable std::atomic<int> batch_refs{0};
  // adjoint workspace
  mutable std::mutex ws_mu;
  mutable void* adj_ws = nullptr;
  mutable size_t adj_ws_bytes = 0;
  // input-order maps of the packed records and monomials (uploaded by the
  // first pe_eval_terms; freed with the packed arrays)
  mutable uint32_t* d_occ_orig = nullptr;
  mutable uint32_t* d_mon_orig = nullptr;
};

// ------------------------------------------------------------------ kernel dispatch

namespace {

EvalShape eval_shape(const pe_system* sys) {
  EvalShape sh;
  sh.view = sys->view;
  sh.seg = sys->plan.seg;
  sh.G = sys->plan.G;
  sh.cpl = sys->plan.cpl;
  sh.lds = sys->plan.lds;
  sh.lds1 = sys->plan.lds1;
  return sh;
}

hipError_t dispatch_rows(const pe_system* sys, int P, const double* x, const OutView& O, int mode,
                         hipStream_t st) {
  const EvalShape sh = eval_shape(sys);
  switch (sys->code) {
    case 1: return launch_rows<1>(sh, P, x, O, mode, st);
    case 2: return launch_rows<2>(sh, P, x, O, mode, st);
    case 4: return launch_rows<4>(sh, P, x, O, mode, st);
    case PE_REAL | 1: return launch_rows<PE_REAL | 1>(sh, P, x, O, mode, st);
    case PE_REAL | 2: return launch_rows<PE_REAL | 2>(sh, P, x, O, mode, st);
    case PE_REAL | 4: return launch_rows<PE_REAL | 4>(sh, P, x, O, mode, st);
  }
  return hipErrorInvalidValue;
}

hipError_t dispatch_adj(const pe_system* sys, int P, const double* x, const double* v, int NG, int gsize,
                        double* part, double* g, hipStream_t st) {
  const EvalShape sh = eval_shape(sys);
  switch (sys->code) {
    case 1: return launch_adjoint<1>(sh, P, x, v, NG, gsize, part, g, st);
    case 2: return launch_adjoint<2>(sh, P, x, v, NG, gsize, part, g, st);
    case 4: return launch_adjoint<4>(sh, P, x, v, NG, gsize, part, g, st);
  }
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

// Launch shape for a packed system: G chunks at once (G > 1 needs at least
// two chunks in some row, room in LDS for G slot regions and at most 512
// columns).  force_G = 0 picks the largest fitting G of the compiled shapes.
pe_status choose_plan(pe_system* sys, int seg, int force_G) {
  Packed& H = sys->host;
  Plan pl;
  pl.seg = seg;
  pl.max_slots = std::max(H.max_slots_used, 1);
  // owner columns per lane for one tile of at most kTileCols columns
  pl.cpl = cpl_bucket(std::min(H.n, kTileCols), kSub);
  const size_t limit = device_lds_limit();
  const int L = H.level;
  // lds_bytes<1> counts 2 doubles per number; the level's width is W
  const int W = width_of(H.code);
  auto lds_for = [&](int tf, int tl, int G) { return lds_bytes<1>(H.n, tf, tl, pl.max_slots, G) / 2 * W; };
  // table of powers in LDS, in order of preference: for D and DD x itself
  // first (its gathers are frequent next to cheap arithmetic) and then as
  // many powers as fit; for QD only powers >= 2.  In double precision, when
  // every exponent is 1 and a row has on average at most one occurrence per
  // variable (products of many variables), building the table would cost as
  // many loads as the gathers it serves: x is gathered from global memory
  // instead and the LDS holds the slots only.
  std::vector<std::pair<int, int>> tables;
  if (L == 1 && H.emax == 1 && H.nnz <= int64_t(H.N) * H.n) tables.push_back({2, 0});
  const int emax1 = std::max(H.emax - 1, 1);
  if (L <= 2)
    for (int tl = emax1; tl >= 1; --tl) tables.push_back({1, tl});
  for (int tl = emax1; tl >= 2; --tl) tables.push_back({2, tl});
  tables.push_back({2, 0});  // no table
  auto pick_table = [&](int G) -> int {
    for (size_t i = 0; i < tables.size(); ++i)
      if (lds_for(tables[i].first, tables[i].second, G) <= limit) return int(i);
    return -1;
  };
  int max_chunks = 0;
  for (int p = 0; p < H.N; ++p) max_chunks = std::max<int>(max_chunks, H.chunk_ptr[p + 1] - H.chunk_ptr[p]);
  auto fits = [&](int G) {
    if (!shape_compiled(L, seg, G)) return false;
    if (pick_table(G) < 0) return false;
    return multi_chunk_fits(H.n, pl.cpl, pl.max_slots, G);
  };
  if (force_G > 0) {
    if (!fits(force_G)) return fail(PE_EUNSUPPORTED, "this launch shape does not fit the system");
    pl.G = force_G;
  } else {
    pl.G = 1;
    for (int G : {4, 2})
      if (max_chunks >= 2 && fits(G)) {
        pl.G = G;
        break;
      }
  }
  const int ti = pick_table(pl.G);
  if (ti < 0) return fail(PE_EUNSUPPORTED, "workgroup LDS need exceeds the device limit");
  pl.tab_first = tables[ti].first;
  pl.tab_last = tables[ti].second;
  pl.lds = lds_for(pl.tab_first, pl.tab_last, pl.G);
  pl.lds1 = lds_for(pl.tab_first, pl.tab_last, 1);
  if (pl.lds > limit) return fail(PE_EUNSUPPORTED, "workgroup LDS need exceeds the device limit");
  sys->plan = pl;
  return PE_OK;
}

// slot budget of a chunk: about 36 KB (D, DD; 70 KB with segments of 6 or
// more) or 68 KB (QD) of LDS
int slots_for(int L, int seg) {
  if (L == 4) return 1088;
  const int bytes = (seg >= 6 && !(L == 1 && seg == 8)) ? 70 * 1024 : 36 * 1024;
  return std::max(kMaxMonomialVars + 1, bytes / (16 * L));
}

void free_device(pe_system* sys) {
  for (void* p : sys->allocs) (void)hipFree(p);
  sys->allocs.clear();
  sys->device_bytes = 0;
  for (uint32_t* p : {sys->d_occ_orig, sys->d_mon_orig})
    if (p) (void)hipFree(p);
  sys->d_occ_orig = sys->d_mon_orig = nullptr;
}

// the stored input as the packer takes it
SysInput stored_input(const pe_system* sys) {
  SysInput in;
  in.level = sys->code;
  in.n_vars = sys->n_vars;
  in.n_polys = int(sys->in_poly_ptr.size()) - 1;
  in.poly_ptr = sys->in_poly_ptr.data();
  in.mon_ptr = sys->in_mon_ptr.data();
  in.var_idx = sys->in_var.data();
  in.exps = sys->in_exp.data();
  in.coef = sys->in_coef.data();
  return in;
}

// (Re)pack the stored input for segment length `seg`, choose G and upload.
pe_status pack_and_upload(pe_system* sys, int seg, int force_G, hipStream_t hs) {
  const SysInput in = stored_input(sys);
  PackParams pp;
  pp.threads = kSub;
  pp.seg = seg;
  pp.max_slots = slots_for(sys->level, seg);
  Packed H;
  std::string msg;
  int st = pack_system(in, pp, H, msg);
  if (st != kOk) return fail(st, msg);
  Packed saved_host = std::move(sys->host);
  Plan saved_plan = sys->plan;
  sys->host = std::move(H);
  pe_status ps = choose_plan(sys, seg, force_G);
  if (ps != PE_OK) {
    sys->host = std::move(saved_host);
    sys->plan = saved_plan;
    return ps;
  }
  free_device(sys);
  const Packed& P = sys->host;
  SysView& V = sys->view;
  V = SysView{};
  V.n = P.n;
  V.N = P.N;
  V.emax = P.emax;
  V.tab_first = sys->plan.tab_first;
  V.tab_last = sys->plan.tab_last;
  V.max_slots = sys->plan.max_slots;
  V.col_tiles = (P.n + kTileCols - 1) / kTileCols;
  V.col0 = 0;
  pe_status e = PE_OK;
  if ((e = upload(sys, P.chunks, V.chunks, hs)) != PE_OK || (e = upload(sys, P.chunk_ptr, V.chunk_ptr, hs)) != PE_OK ||
      (e = upload(sys, P.rowdesc, V.rowdesc, hs)) != PE_OK ||
      (e = upload(sys, P.occ, V.occ, hs)) != PE_OK || (e = upload(sys, P.mcoef, V.mcoef, hs)) != PE_OK ||
      (e = upload(sys, P.colptr, V.colptr, hs)) != PE_OK)
    return e;
  // rows of very uneven cost (cyclic n-roots: row i holds monomials of i
  // variables) are started in decreasing cost, so that the longest rows do
  // not wait for a CU behind the short ones; even rows keep the identity
  // (no extra load before the first descriptors)
  {
    int64_t mx = 0, sum = 0;
    for (int64_t c : P.poly_cost) {
      mx = std::max(mx, c);
      sum += c;
    }
    if (P.N >= 2 && 2 * mx * P.N >= 3 * sum) {
      std::vector<uint32_t> order(size_t(P.N));
      for (int p = 0; p < P.N; ++p) order[size_t(p)] = uint32_t(p);
      std::stable_sort(order.begin(), order.end(),
                       [&](uint32_t a, uint32_t c) { return P.poly_cost[a] > P.poly_cost[c]; });
      if ((e = upload(sys, order, V.row_order, hs)) != PE_OK) return e;
    }
  }
  PE_HIP(hipStreamSynchronize(hs));
  // the device copies are authoritative; keep only what batches and tuning need
  sys->host.occ.clear();
  sys->host.occ.shrink_to_fit();
  sys->host.mcoef.clear();
  sys->host.mcoef.shrink_to_fit();
  sys->host.colptr.clear();
  sys->host.colptr.shrink_to_fit();
  sys->host.occ_orig.clear();
  sys->host.occ_orig.shrink_to_fit();
  sys->host.mon_orig.clear();
  sys->host.mon_orig.shrink_to_fit();
  return PE_OK;
}

// ------------------------------------------------------------------ plan cache

std::mutex g_cache_mu;
std::string g_cache_path;

std::string plan_key(const pe_system* sys) {
  const Packed& H = sys->host;
  std::ostringstream k;
  k << "L" << sys->code << " n" << H.n << " N" << H.N << " M" << H.M << " nnz" << H.nnz << " kmax" << H.kmax
    << " emax" << H.emax;
  return k.str();
}

// returns true and the shape if the cache has an entry for this system
bool cache_lookup(const std::string& key, int& seg, int& G) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cache_path.empty()) return false;
  std::ifstream f(g_cache_path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const size_t bar = line.find(" | ");
    if (bar == std::string::npos || line.compare(0, bar, key) != 0) continue;
    std::istringstream r(line.substr(bar + 3));
    int a = 0, b = 0;
    if (r >> a >> b) {
      seg = a;
      G = b;
      found = true;  // the last entry wins
    }
  }
  return found;
}

void cache_store(const std::string& key, int seg, int G, double us) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cache_path.empty()) return;
  std::ofstream f(g_cache_path, std::ios::app);
  f << key << " | " << seg << " " << G << " " << us << "\n";
}

// Groups of polynomials of the adjoint: gsize consecutive polynomials per
// workgroup, NG groups per point, enough workgroups (about 4096) to fill the
// device.
void adjoint_groups(int N, int P, int& NG, int& gsize) {
  const int target = 4096;
  gsize = int(std::max<int64_t>(1, (int64_t(N) * P + target - 1) / target));
  gsize = std::min(gsize, N);
  NG = (N + gsize - 1) / gsize;
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
  std::string msg;
  int st = validate(in, msg);
  if (st != kOk) return fail(st, msg);
  auto* sys = new (std::nothrow) pe_system();
  if (!sys) return fail(PE_ENOMEM, "host allocation failed");
  sys->level = level & ~PE_REAL;
  sys->code = level;
  sys->n_vars = n_vars;
  const int64_t M = poly_ptr[n_polys];
  const int64_t nnz = M > 0 ? mon_ptr[M] : 0;
  try {
    sys->in_poly_ptr.assign(poly_ptr, poly_ptr + n_polys + 1);
    if (M > 0) sys->in_mon_ptr.assign(mon_ptr, mon_ptr + M + 1);
    else sys->in_mon_ptr.assign(1, 0);
    sys->in_var.assign(var_idx, var_idx + nnz);
    sys->in_exp.assign(exps, exps + nnz);
    sys->in_coef.assign(coef, coef + size_t(M) * width_of(level));
  } catch (...) {
    delete sys;
    return fail(PE_ENOMEM, "host allocation failed");
  }
  hipError_t he = hipGetDevice(&sys->device);
  if (he != hipSuccess) {
    delete sys;
    return fail(PE_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
  }
  // launch shape: from the plan cache if it knows this system, else the default
  int seg = default_seg_for(sys->level, sys->in_mon_ptr), G = 0;
  pe_status ps = pack_and_upload(sys, seg, G, static_cast<hipStream_t>(stream));
  if (ps == PE_OK) {
    int cseg = 0, cG = 0;
    if (cache_lookup(plan_key(sys), cseg, cG) && (cseg != seg || cG != sys->plan.G))
      if (pack_and_upload(sys, cseg, cG, static_cast<hipStream_t>(stream)) != PE_OK)
        ps = pack_and_upload(sys, seg, G, static_cast<hipStream_t>(stream));
  }
  if (ps != PE_OK) {
    std::string keep = g_last_error;
    pe_system_destroy(sys);
    g_last_error = keep;
    return ps;
  }
  *out = sys;
  return PE_OK;
}

pe_status pe_system_destroy(pe_system* sys) {
  if (!sys) return PE_OK;
  if (sys->batch_refs.load() > 0) return fail(PE_EINVAL, "the system belongs to a live batch; destroy the batch first");
  free_device(sys);
  if (sys->adj_ws) (void)hipFree(sys->adj_ws);
  delete sys;
  return PE_OK;
}

pe_status pe_system_info(const pe_system* sys, int64_t info[11]) {
  if (!sys || !info) return fail(PE_EINVAL, "NULL argument");
  const Packed& H = sys->host;
  info[0] = sys->code;
  info[1] = H.n;
  info[2] = H.N;
  info[3] = H.M;
  info[4] = H.nnz;
  info[5] = H.emax;
  info[6] = H.kmax;
  info[7] = int64_t(sys->device_bytes);
  info[8] = sys->plan.G;
  info[9] = int64_t(sys->plan.lds);
  info[10] = sys->plan.seg;
  return PE_OK;
}

pe_status pe_system_set_shape(pe_system* sys, int32_t segment, int32_t chunks_per_workgroup, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (sys->batch_refs.load() > 0) return fail(PE_EINVAL, "the system belongs to a live batch; destroy the batch first");
  if (chunks_per_workgroup < 0 || chunks_per_workgroup > 4 || chunks_per_workgroup == 3 || segment < 0)
    return fail(PE_EINVAL, "invalid launch shape");
  const int seg = segment ? segment : default_seg_for(sys->level, sys->in_mon_ptr);
  if (!shape_compiled(sys->level, seg, chunks_per_workgroup ? chunks_per_workgroup : 1))
    return fail(PE_EUNSUPPORTED, "launch shape not compiled for this level");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (seg == sys->plan.seg) {
    Plan saved = sys->plan;
    pe_status st = choose_plan(sys, seg, chunks_per_workgroup);
    if (st != PE_OK) {
      sys->plan = saved;
      return st;
    }
    sys->view.tab_first = sys->plan.tab_first;
    sys->view.tab_last = sys->plan.tab_last;
    sys->view.max_slots = sys->plan.max_slots;
    return PE_OK;
  }
  PE_HIP(hipStreamSynchronize(hs));
  const int old_seg = sys->plan.seg, old_G = sys->plan.G;
  pe_status st = pack_and_upload(sys, seg, chunks_per_workgroup, hs);
  if (st != PE_OK) {
    std::string keep = g_last_error;
    if (pack_and_upload(sys, old_seg, old_G, hs) != PE_OK) keep += "; restoring the previous shape failed too";
    g_last_error = keep;
  }
  return st;
}

pe_status pe_eval(const pe_system* sys, int32_t P, const double* x, double* F, double* J, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0 || sys->view.N == 0) return PE_OK;
  if (!x || !F) return fail(PE_EINVAL, "x or F is NULL");
  // one workgroup per (point, row, column tile); F alone needs no tiles
  if (int64_t(P) * sys->view.N * (J ? sys->view.col_tiles : 1) > 0x7fffffffLL)
    return fail(PE_EUNSUPPORTED, "P * N (times the column tiles of J) too large");
  const int W = width_of(sys->code), n = sys->view.n, N = sys->view.N;
  OutView O;
  O.J = J;
  O.j_plane = int64_t(N) * n;
  O.j_pt = W * O.j_plane;
  O.j_row = n;
  O.F = F;
  O.f_plane = N;
  O.f_pt = W * int64_t(N);
  O.f_row = 1;
  O.f_sign = 1.0;
  hipError_t e = dispatch_rows(sys, P, x, O, J ? MODE_EVAL : MODE_FONLY, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("eval launch: ") + hipGetErrorString(e));
  return PE_OK;
}

pe_status pe_eval_terms(const pe_system* sys, int32_t P, const double* x, double* V, double* G, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  const Packed& H = sys->host;
  if (P == 0 || H.M == 0) return PE_OK;
  if (!x || !V || (!G && H.nnz > 0)) return fail(PE_EINVAL, "x, V or G is NULL");
  if (int64_t(P) * sys->view.N > 0x7fffffffLL) return fail(PE_EUNSUPPORTED, "P * N too large");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  {
    // the input-order maps: the packing is deterministic, so packing the
    // stored input again with the system's parameters gives the records'
    // order on the device
    std::lock_guard<std::mutex> lk(sys->ws_mu);
    if (!sys->d_mon_orig) {
      Packed R;
      std::string msg;
      const int st = pack_system(stored_input(sys), H.params, R, msg);
      if (st != kOk) return fail(st, msg);
      if (R.occ.size() != R.occ_orig.size() || R.chunks.size() != H.chunks.size())
        return fail(PE_EDEVICE, "repacking for the input order did not reproduce the packing");
      uint32_t *occ = nullptr, *mon = nullptr;
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&mon), R.mon_orig.size() * sizeof(uint32_t));
      if (e == hipSuccess && !R.occ_orig.empty())
        e = hipMalloc(reinterpret_cast<void**>(&occ), R.occ_orig.size() * sizeof(uint32_t));
      if (e == hipSuccess)
        e = hipMemcpyAsync(mon, R.mon_orig.data(), R.mon_orig.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs);
      if (e == hipSuccess && occ)
        e = hipMemcpyAsync(occ, R.occ_orig.data(), R.occ_orig.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs);
      if (e == hipSuccess) e = hipStreamSynchronize(hs);
      if (e != hipSuccess) {
        if (mon) (void)hipFree(mon);
        if (occ) (void)hipFree(occ);
        return fail(e == hipErrorOutOfMemory ? PE_ENOMEM : PE_EDEVICE,
                    std::string("input-order maps: ") + hipGetErrorString(e));
      }
      sys->d_occ_orig = occ;
      sys->d_mon_orig = mon;
    }
  }
  const int W = width_of(sys->code);
  EvalShape sh = eval_shape(sys);
  sh.view.occ_orig = sys->d_occ_orig;
  sh.view.mon_orig = sys->d_mon_orig;
  sh.n_chunks = int64_t(H.chunks.size());
  OutView O;
  O.F = V;
  O.f_plane = H.M;
  O.f_pt = W * H.M;
  O.f_row = 0;
  O.f_sign = 1.0;
  O.J = G;
  O.j_plane = H.nnz;
  O.j_pt = W * H.nnz;
  O.j_row = 0;
  hipError_t e = hipErrorInvalidValue;
  if (sh.n_chunks == 0) return PE_OK;
  switch (sys->code) {
    case 1: e = launch_terms<1>(sh, P, x, O, hs); break;
    case 2: e = launch_terms<2>(sh, P, x, O, hs); break;
    case 4: e = launch_terms<4>(sh, P, x, O, hs); break;
    case PE_REAL | 1: e = launch_terms<PE_REAL | 1>(sh, P, x, O, hs); break;
    case PE_REAL | 2: e = launch_terms<PE_REAL | 2>(sh, P, x, O, hs); break;
    case PE_REAL | 4: e = launch_terms<PE_REAL | 4>(sh, P, x, O, hs); break;
  }
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("terms launch: ") + hipGetErrorString(e));
  return PE_OK;
}

pe_status pe_eval_adjoint(const pe_system* sys, int32_t P, const double* x, const double* v, double* g,
                          void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0) return PE_OK;
  if (!x || !v || !g) return fail(PE_EINVAL, "x, v or g is NULL");
  if (is_real(sys->code)) return fail(PE_EUNSUPPORTED, "the adjoint is implemented for complex systems");
  if (sys->view.col_tiles > 1) return fail(PE_EUNSUPPORTED, "the adjoint supports at most 2048 variables");
  const int L = sys->level, n = sys->view.n, N = sys->view.N;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (N == 0) {
    PE_HIP(hipMemsetAsync(g, 0, size_t(P) * 2 * L * n * sizeof(double), hs));
    return PE_OK;
  }
  int NG = 0, gsize = 0;
  adjoint_groups(N, P, NG, gsize);
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

// ------------------------------------------------------------------ adjoint without allocation

namespace {

// The partial rows of pe_eval_adjoint_static live in this array: one copy
// per GPU, held until the process ends, shared by every call on that GPU.
// In host code its name is not a device address; host code uses only the
// per-device address that hipGetSymbolAddress returns (static_scratch).
constexpr size_t kStaticScratchBytes = PE_STATIC_SCRATCH_BYTES;
__device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the address of `scratch` on the calling thread's current device, looked up
// once per device
pe_status static_scratch(double** out) {
  int dev = 0;
  PE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PE_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PE_EDEVICE, std::string("address of the static scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PE_OK;
}

// g = 0 for a system without polynomials (a kernel, not a memset node, so
// that the call can be captured in a graph)
__global__ void zero_fill_kernel(double* __restrict__ a, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) a[i] = 0.0;
}

}  // namespace

extern "C" {

pe_status pe_eval_adjoint_static(const pe_system* sys, int32_t P, const double* x, const double* v, double* g,
                                 void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (P == 0) return PE_OK;
  if (!x || !v || !g) return fail(PE_EINVAL, "x, v or g is NULL");
  if (is_real(sys->code)) return fail(PE_EUNSUPPORTED, "the adjoint is implemented for complex systems");
  if (sys->view.col_tiles > 1) return fail(PE_EUNSUPPORTED, "the adjoint supports at most 2048 variables");
  const int L = sys->level, n = sys->view.n, N = sys->view.N;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t row_bytes = size_t(P) * 2 * L * n * sizeof(double);  // one partial row per point
  if (row_bytes > kStaticScratchBytes)
    return fail(PE_EUNSUPPORTED, "P * 16 L * n bytes exceed the static scratch of pe_eval_adjoint_static (" +
                                     std::to_string(kStaticScratchBytes >> 20) + " MiB)");
  if (N == 0) {
    const int64_t cnt = int64_t(P) * 2 * L * n;
    hipLaunchKernelGGL(zero_fill_kernel, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, hs, g, cnt);
    PE_HIP(hipGetLastError());
    return PE_OK;
  }
  double* part = nullptr;
  pe_status ps = static_scratch(&part);
  if (ps != PE_OK) return ps;
  // the groups of pe_eval_adjoint when their partial rows fit, else fewer
  // and larger groups
  int NG = 0, gsize = 0;
  adjoint_groups(N, P, NG, gsize);
  const int ng_fit = int(std::min<size_t>(kStaticScratchBytes / row_bytes, size_t(N)));
  if (NG > ng_fit) {
    gsize = (N + ng_fit - 1) / ng_fit;
    NG = (N + gsize - 1) / gsize;
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

// W: doubles per number of the level
NewtonLayout newton_layout(int W, int N, int n, int P) {
  NewtonLayout lo;
  lo.w_pt = int64_t(W) * N * (n + 1);
  lo.r_pt = int64_t(n) * (n + 1) * W;
  lo.y_pt = int64_t(n) * W;
  lo.w_off = 0;
  lo.r_off = align256(lo.w_off + size_t(P) * lo.w_pt * sizeof(double));
  lo.y_off = align256(lo.r_off + size_t(P) * lo.r_pt * sizeof(double));
  lo.total = align256(lo.y_off + size_t(P) * lo.y_pt * sizeof(double));
  return lo;
}

hipError_t dispatch_mgs(int code, int P, int N, int n, double* W, const NewtonLayout& lo, char* base, double* x,
                        double* resid, hipStream_t st) {
  double* R = reinterpret_cast<double*>(base + lo.r_off);
  double* Y = reinterpret_cast<double*>(base + lo.y_off);
  switch (code) {
#define PE_C(C_) \
  case C_: return launch_mgs<C_>(P, N, n, W, lo.w_pt, R, lo.r_pt, Y, lo.y_pt, x, resid, st);
    PE_C(1) PE_C(2) PE_C(4) PE_C(PE_REAL | 1) PE_C(PE_REAL | 2) PE_C(PE_REAL | 4)
#undef PE_C
  }
  return hipErrorInvalidValue;
}

size_t mgs_lds_for(int code, int N) {
  switch (code) {
    case 1: return mgs_lds_bytes<1>(N);
    case 2: return mgs_lds_bytes<2>(N);
    case 4: return mgs_lds_bytes<4>(N);
    case PE_REAL | 1: return mgs_lds_bytes<PE_REAL | 1>(N);
    case PE_REAL | 2: return mgs_lds_bytes<PE_REAL | 2>(N);
    case PE_REAL | 4: return mgs_lds_bytes<PE_REAL | 4>(N);
  }
  return 0;
}

// The one-workgroup solve (mgs_solve_kernel) for small systems; the
// column-parallel one (launch_lstsq) once a system has 128 variables or more,
// or when the one-workgroup kernel's limits (n + 1 <= 1024, the pivot column
// in LDS) do not hold.
bool newton_column_parallel(const pe_system* sys) {
  const int n = sys->view.n, N = sys->view.N;
  return n >= 128 || n + 1 > 1024 || mgs_lds_for(sys->code, N) > device_lds_limit();
}

pe_status newton_check(const pe_system* sys, int P) {
  const int n = sys->view.n, N = sys->view.N;
  if (P < 0) return fail(PE_EINVAL, "P must be nonnegative");
  if (N < n) return fail(PE_EUNSUPPORTED, "Gauss-Newton needs at least as many polynomials as variables");
  if (newton_column_parallel(sys) && N > kLsMaxRows)
    return fail(PE_EUNSUPPORTED, "the least-squares solve supports at most 4096 polynomials");
  if (P > 65535) return fail(PE_EUNSUPPORTED, "at most 65535 points per call");
  if (int64_t(P) * N * sys->view.col_tiles > 0x7fffffffLL)
    return fail(PE_EUNSUPPORTED, "P * N (times the column tiles of J) too large");
  return PE_OK;
}

hipError_t dispatch_lstsq(int code, const LsLayout& lo, void* ws, const double* A, int64_t ld, int64_t a_plane,
                          int64_t a_pt, double* x, int64_t x_pt, int add, double* resid, double* Rout, double* Qout,
                          hipStream_t st) {
  switch (code) {
#define PE_C(C_) \
  case C_: return launch_lstsq<C_>(lo, ws, A, ld, a_plane, a_pt, x, x_pt, add, resid, Rout, Qout, st);
    PE_C(1) PE_C(2) PE_C(4) PE_C(PE_REAL | 1) PE_C(PE_REAL | 2) PE_C(PE_REAL | 4)
#undef PE_C
  }
  return hipErrorInvalidValue;
}

}  // namespace

extern "C" {

size_t pe_newton_workspace_bytes(const pe_system* sys, int32_t P) {
  if (!sys || P < 0) return 0;
  const int W = width_of(sys->code), N = sys->view.N, n = sys->view.n;
  if (!newton_column_parallel(sys)) return newton_layout(W, N, n, P).total;
  // [J | -F] row-major as the evaluation writes it, then the solver's space
  return align256(size_t(P) * W * N * (n + 1) * sizeof(double)) + ls_layout(sys->code, N, n, P).total;
}

}  // extern "C"

namespace {

hipError_t dispatch_rhs_shift(int code, double* W, int64_t w_pt, int64_t plane, int64_t ld, int N, int n, int P,
                              const double* c, double wF, double wc, hipStream_t st) {
  switch (code) {
#define PE_C(C_) \
  case C_: return launch_rhs_shift<C_>(W, w_pt, plane, ld, N, n, P, c, wF, wc, st);
    PE_C(1) PE_C(2) PE_C(4) PE_C(PE_REAL | 1) PE_C(PE_REAL | 2) PE_C(PE_REAL | 4)
#undef PE_C
  }
  return hipErrorInvalidValue;
}

// One step x += dx with J(x) dx = b in the least-squares sense, where
// b = -f(x) (c null), or b = wF (-f(x)) + wc c (the homotopy f(x) - t c).
pe_status newton_step_impl(const pe_system* sys, int32_t P, double* x_inout, const double* c, double wF, double wc,
                           void* workspace, double* resid_out, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  pe_status ps = newton_check(sys, P);
  if (ps != PE_OK) return ps;
  if (P == 0) return PE_OK;
  if (!x_inout || !workspace) return fail(PE_EINVAL, "x or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(PE_EINVAL, "workspace must be 256-byte aligned");
  const int code = sys->code, Wd = width_of(code), n = sys->view.n, N = sys->view.N;
  const bool big = newton_column_parallel(sys);
  const NewtonLayout lo = newton_layout(Wd, N, n, P);
  char* base = static_cast<char*>(workspace);
  double* W = reinterpret_cast<double*>(base);  // [J | -F], row stride n + 1
  const int64_t w_pt = int64_t(Wd) * N * (n + 1);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  OutView O;
  O.J = W;
  O.j_row = n + 1;
  O.j_plane = int64_t(N) * (n + 1);
  O.j_pt = w_pt;
  O.F = W + n;
  O.f_row = n + 1;
  O.f_plane = O.j_plane;
  O.f_pt = w_pt;
  O.f_sign = -1.0;
  hipError_t e = dispatch_rows(sys, P, x_inout, O, MODE_EVAL, hs);
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("newton eval launch: ") + hipGetErrorString(e));
  if (c) {
    e = dispatch_rhs_shift(code, W, w_pt, O.j_plane, n + 1, N, n, P, c, wF, wc, hs);
    if (e != hipSuccess) return fail(PE_EDEVICE, std::string("homotopy right-hand side: ") + hipGetErrorString(e));
  }
  if (big) {
    void* ls = base + align256(size_t(P) * w_pt * sizeof(double));
    e = dispatch_lstsq(code, ls_layout(code, N, n, P), ls, W, n + 1, O.j_plane, w_pt, x_inout, int64_t(Wd) * n, 1,
                       resid_out, nullptr, nullptr, hs);
  } else {
    e = dispatch_mgs(code, P, N, n, W, lo, base, x_inout, resid_out, hs);
  }
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("newton solve launch: ") + hipGetErrorString(e));
  return PE_OK;
}

}  // namespace

extern "C" {

pe_status pe_newton_step(const pe_system* sys, int32_t P, double* x_inout, void* workspace, double* resid_out,
                         void* stream) {
  return newton_step_impl(sys, P, x_inout, nullptr, 1.0, 0.0, workspace, resid_out, stream);
}

pe_status pe_homotopy_newton_step(const pe_system* sys, int32_t P, double* x_inout, const double* c, double t,
                                  void* workspace, double* resid_out, void* stream) {
  if (!c) return fail(PE_EINVAL, "c is NULL");
  if (!std::isfinite(t)) return fail(PE_EINVAL, "t must be finite");
  return newton_step_impl(sys, P, x_inout, c, 1.0, t, workspace, resid_out, stream);
}

pe_status pe_homotopy_predict(const pe_system* sys, int32_t P, double* x_inout, const double* c, double dt,
                              void* workspace, double* resid_out, void* stream) {
  if (!c) return fail(PE_EINVAL, "c is NULL");
  if (!std::isfinite(dt)) return fail(PE_EINVAL, "dt must be finite");
  return newton_step_impl(sys, P, x_inout, c, 0.0, dt, workspace, resid_out, stream);
}

pe_status pe_homotopy_track(const pe_system* sys, int32_t P, double* x_inout, const double* c, int32_t steps,
                            int32_t corrector_iters, void* workspace, double* resid_out, void* stream) {
  if (steps < 1 || corrector_iters < 0) return fail(PE_EINVAL, "need steps >= 1 and corrector_iters >= 0");
  if (!c) return fail(PE_EINVAL, "c is NULL");
  for (int k = 1; k <= steps; ++k) {
    // t from 1 down to 0 in equal steps; t_k computed, not accumulated
    const double t0 = 1.0 - double(k - 1) / double(steps), t1 = k == steps ? 0.0 : 1.0 - double(k) / double(steps);
    pe_status st = newton_step_impl(sys, P, x_inout, c, 0.0, t1 - t0, workspace, resid_out, stream);
    for (int it = 0; it < corrector_iters && st == PE_OK; ++it)
      st = newton_step_impl(sys, P, x_inout, c, 1.0, t1, workspace, resid_out, stream);
    if (st != PE_OK) return st;
  }
  return PE_OK;
}

// level codes 1, 2, 4 (complex) and PE_REAL | 1, 2, 4 (real)
static bool valid_level(int level) {
  const int L = level & ~PE_REAL;
  return (level & ~(PE_REAL | 7)) == 0 && (L == 1 || L == 2 || L == 4);
}

size_t pe_lstsq_workspace_bytes(int32_t level, int32_t P, int32_t N, int32_t n) {
  if (!valid_level(level) || P < 0 || N < 1 || n < 1) return 0;
  return ls_layout(level, N, n, P).total;
}

pe_status pe_lstsq(int32_t level, int32_t P, int32_t N, int32_t n, const double* Ab, double* x, double* resid_out,
                   double* R_out, double* Q_out, void* workspace, void* stream) {
  if (!valid_level(level)) return fail(PE_EINVAL, "level must be 1, 2 or 4, optionally with PE_REAL");
  if (P < 0 || N < 1 || n < 1) return fail(PE_EINVAL, "need P >= 0, N >= 1, n >= 1");
  if (N < n) return fail(PE_EUNSUPPORTED, "least squares needs N >= n");
  if (N > kLsMaxRows) return fail(PE_EUNSUPPORTED, "the least-squares solve supports at most 4096 rows");
  if (P > 65535) return fail(PE_EUNSUPPORTED, "at most 65535 points per call");
  if (P == 0) return PE_OK;
  if (!Ab || !x || !workspace) return fail(PE_EINVAL, "Ab, x or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(PE_EINVAL, "workspace must be 256-byte aligned");
  const int64_t plane = int64_t(N) * (n + 1);
  hipError_t e = dispatch_lstsq(level, ls_layout(level, N, n, P), workspace, Ab, n + 1, plane, width_of(level) * plane,
                                x, int64_t(width_of(level)) * n, 0, resid_out, R_out, Q_out,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("least-squares launch: ") + hipGetErrorString(e));
  return PE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

// One persistent launch of a batch: the (system, polynomial) items of one
// class of systems, in decreasing cost.
struct BatchClass {
  int G = 1;  // chunks per workgroup
  int cpl = 1;
  int vw = 0;  // copy width of batch_small_kernel (0: batch_rows_kernel)
  size_t lds = 0;
  int64_t nitems = 0;
  uint64_t* d_items = nullptr;
};

struct pe_batch {
  int device = 0;
  int level = 0;
  int S = 0;
  int seg = 4;
  // class 0: systems with a row of two or more chunks (two chunks per
  // workgroup when compiled and fitting); class 1: the other systems with
  // more than 256 variables, one chunk per workgroup; classes 2..5: systems
  // whose rows are at most one chunk of at most VW lanes and that have at
  // most VW variables, VW = 32, 64, 128, 256 (batch_small_kernel, 256 / VW
  // points per pass)
  static constexpr int kClasses = 6;
  BatchClass cls[kClasses];
  int maxN = 0;
  std::vector<const pe_system*> systems;
  std::vector<int64_t> x_off, F_off, J_off;  // per point, doubles, [S+1]
  std::vector<BatchNewtonDesc> ndesc;        // per point offsets of the Newton workspace
  int64_t w_total = 0, r_total = 0, y_total = 0;  // per point, doubles
  int64_t nitems = 0;
  SysView* d_views = nullptr;
  int64_t* d_offs = nullptr;  // x_off | F_off | J_off | W offsets, each [S+1]
  BatchNewtonDesc* d_ndesc = nullptr;
  int* d_order = nullptr;
  int* d_counter = nullptr;  // [kClasses], one per class
};

namespace {

__global__ void reset_counter_kernel(int* counter, int count) {
  if (blockIdx.x == 0 && int(threadIdx.x) < count) counter[threadIdx.x] = 0;
}

hipError_t dispatch_batch_class(const pe_batch* b, int c, int P, const double* x, const BatchOut& out, int mode,
                                hipStream_t st) {
  const BatchClass& C = b->cls[c];
  BatchShape K;
  K.seg = b->seg;
  K.G = C.G;
  K.cpl = C.cpl;
  K.vw = C.vw;
  K.lds = C.lds;
  K.nitems = C.nitems;
  K.items = C.d_items;
  K.views = b->d_views;
  K.x_off = b->d_offs;
  K.counter = b->d_counter + c;
  switch (b->level) {
    case 1: return launch_batch<1>(K, P, x, out, mode, st);
    case 2: return launch_batch<2>(K, P, x, out, mode, st);
    case 4: return launch_batch<4>(K, P, x, out, mode, st);
  }
  return hipErrorInvalidValue;
}

// reset both queue counters (a kernel, so the launch can be captured), then
// one persistent launch per non-empty class
hipError_t dispatch_batch(const pe_batch* b, int P, const double* x, const BatchOut& out, int mode, hipStream_t st) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, b->d_counter, pe_batch::kClasses);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int c = 0; c < pe_batch::kClasses; ++c)
    if (b->cls[c].nitems > 0 && (e = dispatch_batch_class(b, c, P, x, out, mode, st)) != hipSuccess) return e;
  return hipSuccess;
}

void batch_free(pe_batch* b) {
  for (void* p : {(void*)b->d_views, (void*)b->d_offs, (void*)b->d_ndesc, (void*)b->d_order, (void*)b->d_counter})
    if (p) (void)hipFree(p);
  for (BatchClass& c : b->cls)
    if (c.d_items) (void)hipFree(c.d_items);
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
  for (int s = 0; s < S; ++s) {
    if (is_real(systems[s]->code)) {
      delete b;
      return fail(PE_EUNSUPPORTED, "batches are implemented for complex systems");
    }
    if (systems[s]->view.col_tiles > 1) {
      delete b;
      return fail(PE_EUNSUPPORTED, "batched systems have at most 2048 variables");
    }
  }
  b->device = systems[0]->device;
  for (int s = 0; s < S; ++s) {
    const pe_system* y = systems[s];
    if (y->level != b->level || y->plan.seg != b->seg || y->device != b->device) {
      delete b;
      return fail(PE_EINVAL, "batched systems must share level, segment length and device "
                             "(pe_system_set_shape sets a common segment length)");
    }
    b->maxN = std::max(b->maxN, y->view.N);
  }
  const int L = b->level;
  // classes: systems with a row of two or more chunks (class 0); systems of
  // one-chunk rows by the copy width VW they need (n and the widest chunk),
  // classes 2..5 for VW = 32 .. 256, class 1 beyond; per class the columns,
  // the LDS and, for class 0, two chunks per workgroup when compiled and when
  // every system's table and two slot regions fit in LDS
  constexpr int kVw[4] = {32, 64, 128, 256};
  std::vector<int> cls_of(S, 1);
  int maxcols[pe_batch::kClasses] = {1, 1, 1, 1, 1, 1};
  size_t lds2 = 0;
  bool two_fit = shape_compiled(L, b->seg, 2);
  for (int s = 0; s < S; ++s) {
    const pe_system* y = systems[s];
    int mc = 0, wmax = 0;
    for (int p = 0; p < y->view.N; ++p) mc = std::max<int>(mc, y->host.chunk_ptr[p + 1] - y->host.chunk_ptr[p]);
    for (const ChunkDesc& cd : y->host.chunks) wmax = std::max<int>(wmax, cd.width);
    int c = mc >= 2 ? 0 : 1;
    if (c == 1)
      for (int v = 0; v < 4; ++v)
        if (std::max(y->view.n, wmax) <= kVw[v]) {
          c = 2 + v;
          break;
        }
    cls_of[s] = c;
    maxcols[c] = std::max(maxcols[c], y->view.n);
    if (c >= 2) {
      // Q copies of [table][slots][F partials]
      const int vw = kVw[c - 2];
      const size_t per_copy = size_t(y->plan.tab_last >= y->plan.tab_first ? y->plan.tab_last - y->plan.tab_first + 1
                                                                            : 0) * (y->view.n + 1) +
                              size_t(y->view.max_slots) + size_t(std::max(1, vw / 64));
      b->cls[c].lds = std::max(b->cls[c].lds, per_copy * 2 * L * sizeof(double) * size_t(kSub / vw));
    } else {
      b->cls[c].lds = std::max(b->cls[c].lds, y->plan.lds1);
    }
    if (c == 0) {
      lds2 = std::max(lds2, lds_bytes<1>(y->view.n, y->view.tab_first, y->view.tab_last, y->view.max_slots, 2) * L);
      two_fit = two_fit && multi_chunk_fits(y->view.n, cpl_bucket(y->view.n, kSub), y->view.max_slots, 2);
    }
  }
  for (int c = 0; c < pe_batch::kClasses; ++c) {
    b->cls[c].cpl = c >= 2 ? 1 : cpl_bucket(maxcols[c], kSub);
    b->cls[c].vw = c >= 2 ? kVw[c - 2] : 0;
  }
  // two chunks per workgroup only when every system of the class fits that
  // shape as pe_eval would run it (same rule), so rows match pe_eval bit for bit
  if (two_fit && lds2 > 0 && lds2 <= device_lds_limit()) {
    b->cls[0].G = 2;
    b->cls[0].lds = lds2;
  }
  // a small class whose copies do not fit in LDS goes to class 1
  for (int c = 2; c < pe_batch::kClasses; ++c)
    if (b->cls[c].lds > device_lds_limit()) {
      for (int s = 0; s < S; ++s)
        if (cls_of[s] == c) {
          cls_of[s] = 1;
          b->cls[1].lds = std::max(b->cls[1].lds, systems[s]->plan.lds1);
          b->cls[1].cpl = std::max(b->cls[1].cpl, cpl_bucket(systems[s]->view.n, kSub));
        }
      b->cls[c].lds = 0;
    }
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
  // work items of each class in decreasing cost (longest processing time
  // first)
  std::vector<uint64_t> it[pe_batch::kClasses];
  for (int c = 0; c < pe_batch::kClasses; ++c) {
    std::vector<std::pair<int64_t, uint64_t>> items;
    for (int s = 0; s < S; ++s) {
      if (cls_of[s] != c) continue;
      const Packed& H = systems[s]->host;
      for (int p = 0; p < H.N; ++p) items.push_back({H.poly_cost[p], (uint64_t(s) << 32) | uint64_t(p)});
    }
    std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& q) { return a.first > q.first; });
    for (const auto& pr : items) it[c].push_back(pr.second);
    b->cls[c].nitems = int64_t(it[c].size());
  }
  b->nitems = 0;
  for (const BatchClass& c : b->cls) b->nitems += c.nitems;
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
  for (int c = 0; c < pe_batch::kClasses && e == PE_OK; ++c) e = upload_raw(it[c], &b->cls[c].d_items, hs);
  if (e != PE_OK || (e = upload_raw(views, &b->d_views, hs)) != PE_OK ||
      (e = upload_raw(offs, &b->d_offs, hs)) != PE_OK || (e = upload_raw(b->ndesc, &b->d_ndesc, hs)) != PE_OK ||
      (e = upload_raw(order, &b->d_order, hs)) != PE_OK) {
    batch_free(b);
    delete b;
    return e;
  }
  hipError_t he = hipMalloc(reinterpret_cast<void**>(&b->d_counter), pe_batch::kClasses * sizeof(int));
  if (he == hipSuccess) he = hipStreamSynchronize(hs);
  if (he != hipSuccess) {
    batch_free(b);
    delete b;
    return fail(PE_EDEVICE, std::string("batch upload: ") + hipGetErrorString(he));
  }
  for (const pe_system* y : b->systems) y->batch_refs.fetch_add(1);
  *out = b;
  return PE_OK;
}

pe_status pe_batch_destroy(pe_batch* b) {
  if (!b) return PE_OK;
  for (const pe_system* y : b->systems) y->batch_refs.fetch_sub(1);
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

pe_status pe_batch_info(const pe_batch* b, int64_t info[4]) {
  if (!b || !info) return fail(PE_EINVAL, "NULL argument");
  info[0] = b->S;
  info[1] = b->level;
  info[2] = b->seg;
  info[3] = b->cls[0].nitems > 0 ? b->cls[0].G : b->cls[1].G;
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
  // the batched step runs the one-workgroup solve for every system
  for (const pe_system* y : b->systems) {
    pe_status ps = newton_check(y, P);
    if (ps != PE_OK) return ps;
    if (y->view.n + 1 > 1024) return fail(PE_EUNSUPPORTED, "the batched Gauss-Newton step supports n + 1 <= 1024");
  }
  {
    const size_t lds = b->level == 1 ? mgs_lds_bytes<1>(b->maxN)
                                     : (b->level == 2 ? mgs_lds_bytes<2>(b->maxN) : mgs_lds_bytes<4>(b->maxN));
    if (lds > device_lds_limit()) return fail(PE_EUNSUPPORTED, "too many polynomials for the LDS pivot column");
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
  const BatchNewtonDesc* nd = b->d_ndesc;
  switch (L) {
    case 1: e = launch_mgs_batch<1>(b->S, P, b->maxN, nd, b->d_order, W, Rw, Yw, x_inout, resid_out, hs); break;
    case 2: e = launch_mgs_batch<2>(b->S, P, b->maxN, nd, b->d_order, W, Rw, Yw, x_inout, resid_out, hs); break;
    case 4: e = launch_mgs_batch<4>(b->S, P, b->maxN, nd, b->d_order, W, Rw, Yw, x_inout, resid_out, hs); break;
  }
  if (e != hipSuccess) return fail(PE_EDEVICE, std::string("batch newton solve: ") + hipGetErrorString(e));
  return PE_OK;
}

pe_status pe_autotune(pe_system* sys, int32_t P, void* stream) {
  if (!sys) return fail(PE_EINVAL, "system is NULL");
  if (sys->batch_refs.load() > 0) return fail(PE_EINVAL, "the system belongs to a live batch; destroy the batch first");
  if (P < 1) return fail(PE_EINVAL, "P must be positive");
  if (sys->view.N == 0) return PE_OK;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int L = sys->level, Wd = width_of(sys->code), n = sys->view.n, N = sys->view.N;
  // inputs: unit-modulus points (real systems: the cosines); outputs F and J
  const size_t xs = size_t(P) * Wd * n, fs = size_t(P) * Wd * N, js = fs * n;
  std::vector<double> hx(xs, 0.0);
  for (int pt = 0; pt < P; ++pt)
    for (int j = 0; j < n; ++j) {
      const double t = 0.7 + 0.013 * j + 0.1 * pt;
      hx[(size_t(pt) * Wd + 0) * n + j] = std::cos(t);
      if (!is_real(sys->code)) hx[(size_t(pt) * Wd + L) * n + j] = std::sin(t);
    }
  double *dx = nullptr, *dF = nullptr, *dJ = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (dx) (void)hipFree(dx);
    if (dF) (void)hipFree(dF);
    if (dJ) (void)hipFree(dJ);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t he = hipMalloc(&dx, xs * 8);
  if (he == hipSuccess) he = hipMalloc(&dF, fs * 8);
  if (he == hipSuccess) he = hipMalloc(&dJ, js * 8);
  if (he == hipSuccess) he = hipMemcpyAsync(dx, hx.data(), xs * 8, hipMemcpyHostToDevice, hs);
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    cleanup();
    return fail(PE_EDEVICE, std::string("autotune setup: ") + hipGetErrorString(he));
  }
  const int best_seg0 = sys->plan.seg, best_G0 = sys->plan.G;
  int best_seg = best_seg0, best_G = best_G0;
  double best_us = 1e300;
  for (int seg : {1, 2, 4, 6, 8, 16})
    for (int G : {1, 2, 4}) {
      if (!shape_compiled(L, seg, G)) continue;
      if (pe_system_set_shape(sys, seg, G, stream) != PE_OK) continue;
      double us = 1e300;
      for (int rep = 0; rep < 3; ++rep) {
        (void)pe_eval(sys, P, dx, dF, dJ, stream);
        (void)hipEventRecord(e0, hs);
        const int iters = 5;
        for (int it = 0; it < iters; ++it) (void)pe_eval(sys, P, dx, dF, dJ, stream);
        (void)hipEventRecord(e1, hs);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        us = std::min(us, 1e3 * ms / iters);
      }
      if (us < best_us) {
        best_us = us;
        best_seg = seg;
        best_G = G;
      }
    }
  cleanup();
  pe_status st = pe_system_set_shape(sys, best_seg, best_G, stream);
  if (st != PE_OK) return st;
  cache_store(plan_key(sys), best_seg, best_G, best_us);
  return PE_OK;
}

pe_status pe_set_plan_cache(const char* path) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache_path = path ? path : "";
  return PE_OK;
}

}  // extern "C"
