// Host-side loading of a sparse polynomial system (see packer.hpp).
//
// Input form: sparse distributed form, only nonzero monomials (Problem
// Statement, Sec. 1); each monomial a coefficient and (variable, exponent)
// pairs with positive exponents (Sec. 2.1, eq. (1)).
#include "packer.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

namespace pe {

int lanes_for(int k, int seg) {
  int need = (k + seg - 1) / seg;
  int s = 1;
  while (s < need) s <<= 1;
  return s;
}

int validate(const SysInput& in, std::string& msg) {
  // level codes: 1, 2, 4 complex; 8 | 1, 8 | 2, 8 | 4 real (layout.hpp)
  if ((in.level & ~kRealLevel) != 1 && (in.level & ~kRealLevel) != 2 && (in.level & ~kRealLevel) != 4) {
    msg = "level must be 1, 2 or 4, optionally with the real flag 8";
    return kEinval;
  }
  if (in.n_vars < 1) {
    msg = "n_vars must be at least 1";
    return kEinval;
  }
  if (in.n_vars > kMaxVars) {
    msg = "n_vars above 65535 is not supported";
    return kEunsupported;
  }
  if (in.n_polys < 0) {
    msg = "n_polys must be nonnegative";
    return kEinval;
  }
  if (!in.poly_ptr) {
    msg = "poly_ptr is NULL";
    return kEinval;
  }
  if (in.poly_ptr[0] != 0) {
    msg = "poly_ptr[0] must be 0";
    return kEinval;
  }
  for (int p = 0; p < in.n_polys; ++p)
    if (in.poly_ptr[p + 1] < in.poly_ptr[p]) {
      msg = "poly_ptr is not nondecreasing at polynomial " + std::to_string(p);
      return kEinval;
    }
  const int64_t M = in.poly_ptr[in.n_polys];
  if (M > 0 && (!in.mon_ptr || !in.coef)) {
    msg = "mon_ptr or coef is NULL";
    return kEinval;
  }
  if (M > (int64_t(1) << 31)) {
    msg = "more than 2^31 monomials is not supported";
    return kEunsupported;
  }
  if (M > 0 && in.mon_ptr[0] != 0) {
    msg = "mon_ptr[0] must be 0";
    return kEinval;
  }
  for (int64_t t = 0; t < M; ++t)
    if (in.mon_ptr[t + 1] < in.mon_ptr[t]) {
      msg = "mon_ptr is not nondecreasing at monomial " + std::to_string(t);
      return kEinval;
    }
  const int64_t nnz = M > 0 ? in.mon_ptr[M] : 0;
  if (nnz > 0 && (!in.var_idx || !in.exps)) {
    msg = "var_idx or exps is NULL";
    return kEinval;
  }
  if (nnz > (int64_t(1) << 32)) {
    msg = "more than 2^32 occurrences is not supported";
    return kEunsupported;
  }
  std::vector<int32_t> seen(in.n_vars, -1);
  for (int64_t t = 0; t < M; ++t) {
    const int64_t a = in.mon_ptr[t], b = in.mon_ptr[t + 1];
    if (b - a > kMaxMonomialVars) {
      msg = "monomial " + std::to_string(t) + " has more than 1024 variables";
      return kEunsupported;
    }
    for (int64_t o = a; o < b; ++o) {
      const int32_t v = in.var_idx[o], d = in.exps[o];
      if (v < 0 || v >= in.n_vars) {
        msg = "variable index out of range in monomial " + std::to_string(t);
        return kEinval;
      }
      if (d < 1 || d > 65535) {
        msg = "exponent outside 1..65535 in monomial " + std::to_string(t);
        return kEinval;
      }
      if (seen[v] == int32_t(t & 0x7fffffff)) {
        msg = "duplicate variable in monomial " + std::to_string(t);
        return kEinval;
      }
      seen[v] = int32_t(t & 0x7fffffff);
    }
  }
  return kOk;
}

namespace {

struct Occ {
  int var, exp;
  int64_t orig;  // index of the occurrence in the input
};

}  // namespace

int pack_system(const SysInput& in, const PackParams& pp, Packed& out, std::string& msg) {
  int st = validate(in, msg);
  if (st != kOk) return st;
  const int L = in.level & ~kRealLevel, n = in.n_vars, N = in.n_polys;
  const int ncomp = (in.level & kRealLevel) ? 1 : 2;  // real or complex
  const int W = ncomp * L;                             // doubles per number
  const int64_t M = in.poly_ptr[N];
  const int64_t nnz = M > 0 ? in.mon_ptr[M] : 0;
  const int T = pp.threads, seg = pp.seg;
  if (T < 64 || T > 1024 || (T & 63) || seg < 1 || seg > kMaxSeg) {
    msg = "invalid launch shape";
    return kEinval;
  }

  out = Packed();
  out.level = L;
  out.code = in.level;
  out.n = n;
  out.N = N;
  out.M = M;
  out.nnz = nnz;
  out.params = pp;

  // largest exponent and monomial size, mean size
  int emax = 1, kmax = 0;
  for (int64_t o = 0; o < nnz; ++o) emax = std::max(emax, int(in.exps[o]));
  for (int64_t t = 0; t < M; ++t) kmax = std::max<int>(kmax, int(in.mon_ptr[t + 1] - in.mon_ptr[t]));
  out.emax = emax;
  out.kmax = kmax;
  if (lanes_for(std::max(kmax, 1), seg) > kMaxWave) {
    msg = "monomial too large for the segment length";
    return kEunsupported;
  }
  const int max_slots = pp.max_slots;
  if (max_slots < kMaxMonomialVars + 1 || max_slots > 65535) {
    msg = "slot budget must be in 1025..65535";
    return kEinval;
  }

  out.mcoef.resize(size_t(M) * W);
  out.mmeta.resize(size_t(M));
  out.mon_orig.resize(size_t(M));
  out.chunk_ptr.assign(size_t(N) + 1, 0);
  out.poly_cost.assign(size_t(N), 0);

  std::vector<int64_t> order;
  std::vector<Occ> occ_sorted;
  struct Contrib {
    int col, g, r;
  };
  std::vector<Contrib> contribs;
  std::vector<int> counts;
  std::vector<std::vector<int>> slot_of;

  int64_t packed_t = 0;
  for (int p = 0; p < N; ++p) {
    const int64_t t0 = in.poly_ptr[p], t1 = in.poly_ptr[p + 1];
    order.resize(size_t(t1 - t0));
    std::iota(order.begin(), order.end(), t0);
    // larger monomials first so that chunks are homogeneous in k
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return (in.mon_ptr[a + 1] - in.mon_ptr[a]) > (in.mon_ptr[b + 1] - in.mon_ptr[b]);
    });
    out.chunk_ptr[p] = uint32_t(out.chunks.size());
    size_t i = 0;
    while (i < order.size()) {
      const int kfirst = int(in.mon_ptr[order[i] + 1] - in.mon_ptr[order[i]]);
      const int s = lanes_for(std::max(kfirst, 1), seg);
      const int cap = T / s;
      // one slot per partial derivative; slot index `slots` (one past the
      // last) is the chunk's dummy slot, so at most max_slots - 1 are used
      int count = 0, slots = 0;
      size_t j = i;
      while (j < order.size() && count < cap) {
        const int k = int(in.mon_ptr[order[j] + 1] - in.mon_ptr[order[j]]);
        if (slots + k + 1 > max_slots) break;
        slots += k;
        ++count;
        ++j;
      }
      // build the chunk from order[i..j)
      ChunkDesc cd{};
      cd.poly = uint32_t(p);
      cd.count = uint16_t(count);
      cd.s = uint8_t(s);
      cd.width = uint16_t(count * s);
      cd.mon_base = uint32_t(packed_t);
      cd.nslots = uint16_t(slots);
      const int segc = kfirst > 0 ? (kfirst + s - 1) / s : 1;
      cd.seg = uint8_t(segc);
      out.max_seg_used = std::max(out.max_seg_used, segc);
      out.max_slots_used = std::max(out.max_slots_used, slots + 1);
      cd.occ_base = uint32_t(out.occ.size());
      if (out.occ.size() + size_t(segc) * cd.width > (size_t(1) << 32)) {
        msg = "packed occurrence array too large";
        return kEunsupported;
      }
      cd.colptr_base = uint32_t(out.colptr.size());

      // contributions: (column, monomial in chunk, position) -> slot
      contribs.clear();
      slot_of.resize(size_t(count));
      for (int g = 0; g < count; ++g) {
        const int64_t t = order[i + g];
        const int64_t a = in.mon_ptr[t], b = in.mon_ptr[t + 1];
        occ_sorted.clear();
        for (int64_t o = a; o < b; ++o) occ_sorted.push_back({in.var_idx[o], in.exps[o], o});
        std::sort(occ_sorted.begin(), occ_sorted.end(), [](const Occ& x, const Occ& y) { return x.var < y.var; });
        for (int r = 0; r < int(occ_sorted.size()); ++r) contribs.push_back({occ_sorted[r].var, g, r});
        slot_of[size_t(g)].assign(occ_sorted.size(), 0);
      }
      std::stable_sort(contribs.begin(), contribs.end(), [](const Contrib& x, const Contrib& y) {
        if (x.col != y.col) return x.col < y.col;
        if (x.g != y.g) return x.g < y.g;
        return x.r < y.r;
      });
      // slot of (g, r): position in the sorted list
      counts.assign(size_t(n) + 1, 0);
      for (int sidx = 0; sidx < int(contribs.size()); ++sidx) {
        const Contrib& c = contribs[size_t(sidx)];
        slot_of[size_t(c.g)][size_t(c.r)] = sidx;
        counts[size_t(c.col) + 1]++;
      }
      for (int c = 0; c < n; ++c) counts[size_t(c) + 1] += counts[size_t(c)];
      for (int c = 0; c <= n; ++c) out.colptr.push_back(uint16_t(counts[size_t(c)]));

      // occurrence records, lane-major; positions past a lane's segment hold
      // the neutral record (variable n, whose value is 1, exponent 1, the
      // dummy slot)
      const size_t rec0 = out.occ.size();
      const OccRec pad{uint16_t(n), 1, uint16_t(slots), 0};
      out.occ.resize(rec0 + size_t(segc) * cd.width, pad);
      out.occ_orig.resize(rec0 + size_t(segc) * cd.width, kNoOcc);
      int64_t cost = 0;
      for (int g = 0; g < count; ++g) {
        const int64_t t = order[i + g];
        const int64_t a = in.mon_ptr[t], b = in.mon_ptr[t + 1];
        const int k = int(b - a);
        occ_sorted.clear();
        for (int64_t o = a; o < b; ++o) occ_sorted.push_back({in.var_idx[o], in.exps[o], o});
        std::sort(occ_sorted.begin(), occ_sorted.end(), [](const Occ& x, const Occ& y) { return x.var < y.var; });
        // lane q of the group takes occurrences q, q + s, q + 2s, ... (in
        // variable order): a wavefront's gathers and slot stores at one step
        // then touch neighbouring variables when a monomial's variables are
        // runs of consecutive indices, instead of addresses a segment apart
        const int base = k / s, extra = k % s;
        for (int q = 0; q < s; ++q) {
          const int len = base + (q < extra ? 1 : 0);
          const int lane = g * s + q;
          for (int ii = 0; ii < len; ++ii) {
            const int r = q + ii * s;
            const Occ& oc = occ_sorted[size_t(r)];
            OccRec& rec = out.occ[rec0 + size_t(ii) * cd.width + size_t(lane)];
            rec.var = uint16_t(oc.var);
            rec.exp = uint16_t(oc.exp);
            rec.slot = uint16_t(slot_of[size_t(g)][size_t(r)]);
            out.occ_orig[rec0 + size_t(ii) * cd.width + size_t(lane)] = uint32_t(oc.orig);
          }
        }
        // packed monomial: coefficient and metadata
        for (int c = 0; c < ncomp; ++c)
          for (int l = 0; l < L; ++l)
            out.mcoef[size_t(packed_t + g) * W + size_t(c) * L + l] = in.coef[(size_t(c) * L + l) * size_t(M) + size_t(t)];
        out.mmeta[size_t(packed_t + g)] = mon_meta(uint32_t(k));
        out.mon_orig[size_t(packed_t + g)] = uint32_t(t);
        cost += k;
      }
      out.poly_cost[p] += int64_t(segc) * s * count + cost;
      out.chunks.push_back(cd);
      packed_t += count;
      i = j;
    }
  }
  out.chunk_ptr[N] = uint32_t(out.chunks.size());
  out.rowdesc.assign(size_t(N) * kRowDesc, ChunkDesc{});
  for (int p = 0; p < N; ++p)
    for (uint32_t j = 0; j < uint32_t(kRowDesc) && out.chunk_ptr[p] + j < out.chunk_ptr[p + 1]; ++j)
      out.rowdesc[size_t(p) * kRowDesc + j] = out.chunks[out.chunk_ptr[p] + j];
  return kOk;
}

}  // namespace pe
