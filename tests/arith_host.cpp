// Host build of the library's arithmetic header, for exact checks from the
// test suite (g++ -ffp-contract=off).  Each entry point applies one
// operation to `count` operand pairs given as [count][2][L] limbs.
#include <cstdint>
#include "../paper_1402_2626_amd/csrc/mdarith.hpp"

using namespace pe;

template <int L>
static C<L> load(const double* p) {
  C<L> c;
  for (int i = 0; i < L; ++i) { c.re.x[i] = p[i]; c.im.x[i] = p[L + i]; }
  return c;
}
template <int L>
static void store(double* p, const C<L>& c) {
  for (int i = 0; i < L; ++i) { p[i] = c.re.x[i]; p[L + i] = c.im.x[i]; }
}
template <int L>
static R<L> loadr(const double* p) {
  R<L> r;
  for (int i = 0; i < L; ++i) r.x[i] = p[i];
  return r;
}
template <int L>
static void storer(double* p, const R<L>& r) {
  for (int i = 0; i < L; ++i) p[i] = r.x[i];
}

template <int L>
static void run(int op, int64_t count, const double* a, const double* b, double* out) {
  for (int64_t t = 0; t < count; ++t) {
    const double* pa = a + t * 2 * L;
    const double* pb = b + t * 2 * L;
    double* po = out + t * 2 * L;
    switch (op) {
      case 0: store<L>(po, c_mul(load<L>(pa), load<L>(pb))); break;
      case 1: store<L>(po, c_add(load<L>(pa), load<L>(pb))); break;
      case 2: store<L>(po, c_mul_d(load<L>(pa), pb[0])); break;
      case 3: {  // real ops on the re parts: mul, add
        storer<L>(po, r_mul(loadr<L>(pa), loadr<L>(pb)));
        storer<L>(po + L, r_add(loadr<L>(pa), loadr<L>(pb)));
        break;
      }
      case 4: {  // reciprocal and square root of the re part of a
        storer<L>(po, r_recip(loadr<L>(pa)));
        storer<L>(po + L, r_sqrt(loadr<L>(pa)));
        break;
      }
    }
  }
}

extern "C" int pe_test_arith(int level, int op, int64_t count, const double* a, const double* b, double* out) {
  switch (level) {
    case 1: run<1>(op, count, a, b, out); return 0;
    case 2: run<2>(op, count, a, b, out); return 0;
    case 4: run<4>(op, count, a, b, out); return 0;
  }
  return -1;
}
