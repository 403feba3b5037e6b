// Host fuzz driver of the library's validator and packer, built with the
// address and undefined-behaviour sanitizers by the test suite: random
// well-formed systems (empty polynomials, constants, monomials up to the size
// limit, large exponents) are packed at every segment length, malformed ones
// must be rejected, and the packed layout is checked for in-range records and
// slot permutations.  Exit status 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../paper_1402_2626_amd/csrc/packer.hpp"

using namespace pe;

namespace {

struct Sys {
  int level = 2, n = 1;
  std::vector<int64_t> poly_ptr{0}, mon_ptr{0};
  std::vector<int32_t> var, exp;
  std::vector<double> coef;
};

Sys random_sys(std::mt19937_64& g, int level) {
  Sys s;
  s.level = level;
  s.n = 1 + int(g() % 700);
  const int N = int(g() % 12);
  for (int p = 0; p < N; ++p) {
    const int m = (g() % 5 == 0) ? 0 : 1 + int(g() % 300);
    for (int t = 0; t < m; ++t) {
      int kmax = std::min(s.n, (g() % 7 == 0) ? 1024 : 40);
      int k = int(g() % (kmax + 1));
      std::vector<int> perm(s.n);
      for (int i = 0; i < s.n; ++i) perm[i] = i;
      for (int i = 0; i < k; ++i) std::swap(perm[i], perm[i + g() % (s.n - i)]);
      for (int i = 0; i < k; ++i) {
        s.var.push_back(perm[i]);
        s.exp.push_back(g() % 9 == 0 ? 1 + int(g() % 65535) : 1 + int(g() % 4));
      }
      s.mon_ptr.push_back(int64_t(s.var.size()));
    }
    s.poly_ptr.push_back(int64_t(s.mon_ptr.size() - 1));
  }
  s.coef.assign((s.mon_ptr.size() - 1) * 2 * level, 0.5);
  return s;
}

SysInput input_of(const Sys& s) {
  SysInput in;
  in.level = s.level;
  in.n_vars = s.n;
  in.n_polys = int(s.poly_ptr.size()) - 1;
  in.poly_ptr = s.poly_ptr.data();
  in.mon_ptr = s.mon_ptr.data();
  in.var_idx = s.var.data();
  in.exps = s.exp.data();
  in.coef = s.coef.data();
  return in;
}

int fails = 0;

void check(bool ok, const char* what, int trial) {
  if (!ok) {
    std::printf("FAIL %s (trial %d)\n", what, trial);
    ++fails;
  }
}

}  // namespace

int main() {
  std::mt19937_64 g(20141402);
  for (int trial = 0; trial < 300; ++trial) {
    const int level = (trial % 3 == 0) ? 1 : (trial % 3 == 1 ? 2 : 4);
    Sys s = random_sys(g, level);
    SysInput in = input_of(s);
    std::string msg;
    check(validate(in, msg) == kOk, "valid system accepted", trial);
    for (int seg : {1, 2, 4, 6, 8, 16}) {
      PackParams pp;
      pp.seg = seg;
      pp.max_slots = 1025 + int(g() % 3000);
      Packed P;
      int st = pack_system(in, pp, P, msg);
      int kmax = 0;
      for (size_t t = 0; t + 1 < s.mon_ptr.size(); ++t) kmax = std::max<int>(kmax, int(s.mon_ptr[t + 1] - s.mon_ptr[t]));
      if (lanes_for(std::max(kmax, 1), seg) > kMaxWave) {
        check(st == kEunsupported, "monomial too wide for the segment rejected", trial);
        continue;
      }
      check(st == kOk, "pack succeeded", trial);
      if (st != kOk) continue;
      for (const ChunkDesc& c : P.chunks) {
        check(c.nslots + 1 <= pp.max_slots, "slot budget", trial);
        check(size_t(c.occ_base) + size_t(c.seg) * c.width <= P.occ.size(), "records in range", trial);
        check(size_t(c.colptr_base) + s.n + 1 <= P.colptr.size(), "column pointers in range", trial);
        std::vector<int> hit(c.nslots + 1, 0);
        for (int i = 0; i < c.seg; ++i)
          for (int l = 0; l < c.width; ++l) {
            const OccRec& r = P.occ[c.occ_base + size_t(i) * c.width + l];
            check(r.var <= s.n && r.slot <= c.nslots && r.exp >= 1, "record fields in range", trial);
            if (r.slot < c.nslots) hit[r.slot]++;
          }
        for (int k = 0; k < c.nslots; ++k) check(hit[k] == 1, "every slot written once", trial);
      }
    }
    // malformed variants must be rejected
    if (!s.var.empty()) {
      Sys b = s;
      b.var[g() % b.var.size()] = b.n;
      SysInput bi = input_of(b);
      check(validate(bi, msg) == kEinval, "out-of-range variable rejected", trial);
      Sys e = s;
      e.exp[g() % e.exp.size()] = 0;
      SysInput ei = input_of(e);
      check(validate(ei, msg) == kEinval, "zero exponent rejected", trial);
    }
    if (s.mon_ptr.size() > 2) {
      Sys m = s;
      m.mon_ptr[1] = m.mon_ptr[2] + 1;
      SysInput mi = input_of(m);
      check(validate(mi, msg) != kOk, "non-monotone offsets rejected", trial);
    }
  }
  std::printf("%s\n", fails ? "FAILED" : "OK");
  return fails ? 1 : 0;
}
