// Complex double (L=1), double double (L=2) and quad double (L=4) arithmetic
// built from FP64 error-free transformations.
//
// The paper motivates double double and quad double arithmetic to offset
// roundoff in large systems (Section 1) and names the error-free
// transformations behind it without giving algorithms.  The algorithms here
// are restated from the published literature:
//   * TwoSum (Knuth, TAOCP vol. 2): s = fl(a+b) and the exact error e, any a, b.
//   * FastTwoSum (Dekker 1971): the same in 3 operations when the exponent
//     of a is at least that of b.
//   * TwoProd with FMA: p = fl(a*b), e = fma(a, b, -p), exact.
//   * double-word addition and multiplication in the style of Joldes, Muller
//     and Popescu (ACM TOMS 2017): "sloppy" addition (one TwoSum on the high
//     parts) and the FMA product that drops the low*low term;
//   * quad-double addition and multiplication in the style of Hida, Li and
//     Bailey (2001): limb-wise TwoSums or TwoProds grouped by order of
//     magnitude, errors carried to the next order, then a renormalisation.
//
// Accuracy contract (what the evaluation needs): every operation is accurate
// NORMWISE, i.e. |computed - exact| <= c * u_L * (|a| + |b|) for additions
// and <= c * u_L * |a| * |b| for products, with u_1 = 2^-53, u_2 = 2^-106,
// u_4 = 2^-212 up to small factors, and outputs are nonoverlapping
// expansions.  Relative accuracy under catastrophic cancellation is not
// needed because errors are measured against the sum of absolute values of
// the terms.  The host test suite checks these bounds against exact
// arithmetic on random and cancellation-heavy operands.
//
// Complex numbers use the four-real-product form (ac - bd, ad + bc).  For
// L = 2 each component is one fused "two-product sum" with a single final
// normalisation.
//
// Build rules: no fast-math, no flush of denormals, and floating-point
// contraction off (products that must be fused are written with fma()).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define PE_HD __host__ __device__ __forceinline__
#define PE_FMA(a, b, c) __builtin_fma((a), (b), (c))
#define PE_SQRT(a) __builtin_sqrt(a)
#else
#include <cmath>
#define PE_HD inline
#define PE_FMA(a, b, c) std::fma((a), (b), (c))
#define PE_SQRT(a) std::sqrt(a)
#endif

namespace pe {

// ------------------------------------------------------------------ EFTs

PE_HD void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

PE_HD void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}

PE_HD void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = PE_FMA(a, b, -p);
}

// ------------------------------------------------------------------ real level-L

template <int L>
struct R {
  double x[L];
};

template <int L>
PE_HD R<L> r_zero() {
  R<L> r;
#pragma unroll
  for (int i = 0; i < L; ++i) r.x[i] = 0.0;
  return r;
}

template <int L>
PE_HD R<L> r_from_double(double a) {
  R<L> r = r_zero<L>();
  r.x[0] = a;
  return r;
}

template <int L>
PE_HD R<L> r_neg(const R<L>& a) {
  R<L> r;
#pragma unroll
  for (int i = 0; i < L; ++i) r.x[i] = -a.x[i];
  return r;
}

// --- L = 1

PE_HD R<1> r_add(const R<1>& a, const R<1>& b) { return R<1>{{a.x[0] + b.x[0]}}; }
PE_HD R<1> r_mul(const R<1>& a, const R<1>& b) { return R<1>{{a.x[0] * b.x[0]}}; }
PE_HD R<1> r_mul_d(const R<1>& a, double d) { return R<1>{{a.x[0] * d}}; }

// --- L = 2 (double word: hi, lo)

// sloppy double-word addition: one TwoSum on the high parts, the low parts
// added in plain arithmetic, then FastTwoSum.  Normwise error O(u^2)(|a|+|b|).
PE_HD R<2> r_add(const R<2>& a, const R<2>& b) {
  double s, e;
  two_sum(a.x[0], b.x[0], s, e);
  e += a.x[1] + b.x[1];
  R<2> r;
  fast_two_sum(s, e, r.x[0], r.x[1]);
  return r;
}

// double-word product with FMA; the lo*lo term (order u^2) is dropped.
PE_HD R<2> r_mul(const R<2>& a, const R<2>& b) {
  double p, e;
  two_prod(a.x[0], b.x[0], p, e);
  e = PE_FMA(a.x[0], b.x[1], e);
  e = PE_FMA(a.x[1], b.x[0], e);
  R<2> r;
  fast_two_sum(p, e, r.x[0], r.x[1]);
  return r;
}

// product by a double (exact small integers and reciprocals alike)
PE_HD R<2> r_mul_d(const R<2>& a, double d) {
  double p, e;
  two_prod(a.x[0], d, p, e);
  e = PE_FMA(a.x[1], d, e);
  R<2> r;
  fast_two_sum(p, e, r.x[0], r.x[1]);
  return r;
}

// --- L = 4 (quad double)

// Renormalise five components c0 (largest) .. c4 into four limbs: a
// bottom-up pass of TwoSums (error free for any ordering) and a top-down pass
// that compresses the errors.
PE_HD R<4> renorm5(double c0, double c1, double c2, double c3, double c4) {
  double x, e1, e2, e3, e4;
  two_sum(c3, c4, x, e4);
  two_sum(c2, x, x, e3);
  two_sum(c1, x, x, e2);
  double x0;
  two_sum(c0, x, x0, e1);
  R<4> r;
  double y;
  fast_two_sum(x0, e1, r.x[0], y);
  two_sum(y, e2, r.x[1], y);
  two_sum(y, e3, r.x[2], y);
  r.x[3] = y + e4;
  return r;
}

// Renormalisation for products, whose components decrease by order: two
// passes of FastTwoSum.
PE_HD R<4> renorm4_ordered(double c0, double c1, double c2, double c3) {
  double x, e1, e2, e3, x0;
  fast_two_sum(c2, c3, x, e3);
  fast_two_sum(c1, x, x, e2);
  fast_two_sum(c0, x, x0, e1);
  R<4> r;
  double y;
  r.x[0] = x0;
  fast_two_sum(e1, e2, r.x[1], y);
  fast_two_sum(y, e3, r.x[2], r.x[3]);
  return r;
}

// Quad-double addition: limb-wise TwoSums, errors carried order by order
// (exact down to order 2, plain sum at order 3), then renormalisation.
PE_HD R<4> r_add(const R<4>& a, const R<4>& b) {
  double s0, s1, s2, s3, t0, t1, t2, t3;
  two_sum(a.x[0], b.x[0], s0, t0);
  two_sum(a.x[1], b.x[1], s1, t1);
  two_sum(a.x[2], b.x[2], s2, t2);
  two_sum(a.x[3], b.x[3], s3, t3);
  // order 1: s1 + t0
  double u1, f2;
  two_sum(s1, t0, u1, f2);
  // order 2: s2 + t1 + f2
  double u2, g3, h3;
  two_sum(s2, t1, u2, g3);
  two_sum(u2, f2, u2, h3);
  // order 3 (plain)
  double u3 = s3 + t2 + (g3 + h3);
  return renorm5(s0, u1, u2, u3, t3);
}

// Quad-double product: TwoProds for the order 0..2 partial products, plain
// FMAs for order 3, order-4 terms dropped.
PE_HD R<4> r_mul(const R<4>& a, const R<4>& b) {
  double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
  two_prod(a.x[0], b.x[0], p0, q0);
  two_prod(a.x[0], b.x[1], p1, q1);
  two_prod(a.x[1], b.x[0], p2, q2);
  two_prod(a.x[0], b.x[2], p3, q3);
  two_prod(a.x[1], b.x[1], p4, q4);
  two_prod(a.x[2], b.x[0], p5, q5);
  double o3 = PE_FMA(a.x[0], b.x[3], PE_FMA(a.x[1], b.x[2], PE_FMA(a.x[2], b.x[1], a.x[3] * b.x[0])));
  // order 1: p1 + p2 + q0
  double s1, e_a, e_b;
  two_sum(p1, p2, s1, e_a);
  two_sum(s1, q0, s1, e_b);
  // order 2: p3 + p4 + p5 + q1 + q2 + e_a + e_b
  double s2, f0, f1, f2, f3, f4, f5;
  two_sum(p3, p4, s2, f0);
  two_sum(s2, p5, s2, f1);
  two_sum(s2, q1, s2, f2);
  two_sum(s2, q2, s2, f3);
  two_sum(s2, e_a, s2, f4);
  two_sum(s2, e_b, s2, f5);
  // order 3 (plain)
  double s3 = o3 + (q3 + q4 + q5) + ((f0 + f1) + (f2 + f3) + (f4 + f5));
  return renorm4_ordered(p0, s1, s2, s3);
}

// product by a double
PE_HD R<4> r_mul_d(const R<4>& a, double d) {
  double p0, q0, p1, q1, p2, q2;
  two_prod(a.x[0], d, p0, q0);
  two_prod(a.x[1], d, p1, q1);
  two_prod(a.x[2], d, p2, q2);
  double p3 = a.x[3] * d;
  double s1, e1;
  two_sum(p1, q0, s1, e1);
  double s2, e2, e3;
  two_sum(p2, q1, s2, e2);
  two_sum(s2, e1, s2, e3);
  double s3 = p3 + q2 + (e2 + e3);
  return renorm4_ordered(p0, s1, s2, s3);
}

template <int L>
PE_HD R<L> r_sub(const R<L>& a, const R<L>& b) {
  return r_add(a, r_neg(b));
}

// reciprocal by Newton's iteration y <- y + y (1 - a y), starting from the
// double reciprocal; each step doubles the number of correct bits.
template <int L>
PE_HD R<L> r_recip(const R<L>& a) {
  R<L> y = r_from_double<L>(1.0 / a.x[0]);
  const int steps = (L == 1) ? 0 : (L == 2 ? 1 : 2);
  for (int i = 0; i < steps; ++i) {
    R<L> one = r_from_double<L>(1.0);
    R<L> t = r_sub(one, r_mul(a, y));
    y = r_add(y, r_mul(y, t));
  }
  return y;
}

// square root via the inverse square root iteration
// z <- z + z (1 - a z^2) / 2, then sqrt(a) = a z with one correction.
template <int L>
PE_HD R<L> r_sqrt(const R<L>& a) {
  if (!(a.x[0] > 0.0)) return r_zero<L>();
  if (L == 1) return r_from_double<L>(PE_SQRT(a.x[0]));
  R<L> z = r_from_double<L>(1.0 / PE_SQRT(a.x[0]));
  const int steps = (L == 2 ? 1 : 2);
  for (int i = 0; i < steps; ++i) {
    R<L> one = r_from_double<L>(1.0);
    R<L> t = r_sub(one, r_mul(a, r_mul(z, z)));
    z = r_add(z, r_mul_d(r_mul(z, t), 0.5));
  }
  // s = a z, then one correction s <- s + z (a - s^2) / 2
  R<L> s = r_mul(a, z);
  R<L> d = r_sub(a, r_mul(s, s));
  return r_add(s, r_mul_d(r_mul(z, d), 0.5));
}

// ------------------------------------------------------------------ level codes
//
// A level code names the number type of a kernel instance: 1, 2, 4 are
// complex numbers of L = 1, 2, 4 limbs per real part; 8 | L (9, 10, 12) are
// real numbers of L limbs.  Real numbers use the same interface as complex
// ones (C<code> with only a real part), so every kernel is written once.

constexpr int kRealCode = 8;
constexpr int limbs_of(int code) { return code & 7; }
constexpr bool is_real(int code) { return (code & kRealCode) != 0; }
// doubles per number
constexpr int width_of(int code) { return is_real(code) ? limbs_of(code) : 2 * limbs_of(code); }

// ------------------------------------------------------------------ complex (or real) level-L

template <int L, bool REAL = is_real(L)>
struct C;

template <int L>
struct C<L, false> {
  R<L> re, im;
};

template <int L>
struct C<L, true> {
  R<limbs_of(L)> re;
};

template <int L>
PE_HD C<L> c_zero() {
  if constexpr (is_real(L))
    return C<L>{r_zero<limbs_of(L)>()};
  else
    return C<L>{r_zero<L>(), r_zero<L>()};
}

template <int L>
PE_HD C<L> c_one() {
  if constexpr (is_real(L))
    return C<L>{r_from_double<limbs_of(L)>(1.0)};
  else
    return C<L>{r_from_double<L>(1.0), r_zero<L>()};
}

template <int L>
PE_HD C<L> c_conj(const C<L>& a) {
  if constexpr (is_real(L))
    return a;
  else
    return C<L>{a.re, r_neg(a.im)};
}

template <int L>
PE_HD C<L> c_neg(const C<L>& a) {
  if constexpr (is_real(L))
    return C<L>{r_neg(a.re)};
  else
    return C<L>{r_neg(a.re), r_neg(a.im)};
}

template <int L>
PE_HD C<L> c_add(const C<L>& a, const C<L>& b) {
  if constexpr (is_real(L))
    return C<L>{r_add(a.re, b.re)};
  else
    return C<L>{r_add(a.re, b.re), r_add(a.im, b.im)};
}

template <int L>
PE_HD C<L> c_sub(const C<L>& a, const C<L>& b) {
  if constexpr (is_real(L))
    return C<L>{r_sub(a.re, b.re)};
  else
    return C<L>{r_sub(a.re, b.re), r_sub(a.im, b.im)};
}

// product by a real double (small integer exponents, real scalings)
template <int L>
PE_HD C<L> c_mul_d(const C<L>& a, double d) {
  if constexpr (is_real(L))
    return C<L>{r_mul_d(a.re, d)};
  else
    return C<L>{r_mul_d(a.re, d), r_mul_d(a.im, d)};
}

template <int L>
PE_HD C<L> c_mul_r(const C<L>& a, const R<limbs_of(L)>& d) {
  if constexpr (is_real(L))
    return C<L>{r_mul(a.re, d)};
  else
    return C<L>{r_mul(a.re, d), r_mul(a.im, d)};
}

// |a|^2 as a real level-L number
template <int L>
PE_HD R<limbs_of(L)> c_norm2(const C<L>& a) {
  if constexpr (is_real(L))
    return r_mul(a.re, a.re);
  else
    return r_add(r_mul(a.re, a.re), r_mul(a.im, a.im));
}

// generic product: for complex numbers four real products and two real
// additions; for real numbers the real product
template <int L>
PE_HD C<L> c_mul(const C<L>& a, const C<L>& b) {
  if constexpr (is_real(L)) {
    return C<L>{r_mul(a.re, b.re)};
  } else {
    R<L> ac = r_mul(a.re, b.re), bd = r_mul(a.im, b.im);
    R<L> ad = r_mul(a.re, b.im), bc = r_mul(a.im, b.re);
    return C<L>{r_sub(ac, bd), r_add(ad, bc)};
  }
}

// L = 1: contraction written explicitly
template <>
PE_HD C<1> c_mul<1>(const C<1>& a, const C<1>& b) {
  C<1> r;
  r.re.x[0] = PE_FMA(a.re.x[0], b.re.x[0], -(a.im.x[0] * b.im.x[0]));
  r.im.x[0] = PE_FMA(a.re.x[0], b.im.x[0], a.im.x[0] * b.re.x[0]);
  return r;
}

// L = 2: each component is x1*y1 + sgn*x2*y2 of double words, computed with
// exact high products, one TwoSum, the cross terms accumulated with FMAs and
// a single FastTwoSum at the end.  Normwise error O(u^2)(|x1 y1| + |x2 y2|).
PE_HD R<2> dd_dot2(const R<2>& x1, const R<2>& y1, const R<2>& x2, const R<2>& y2, double sgn) {
  double p1, e1, p2, e2;
  two_prod(x1.x[0], y1.x[0], p1, e1);
  two_prod(x2.x[0], y2.x[0], p2, e2);
  double s, t;
  two_sum(p1, sgn * p2, s, t);
  double l1 = PE_FMA(x1.x[0], y1.x[1], PE_FMA(x1.x[1], y1.x[0], e1));
  double l2 = PE_FMA(x2.x[0], y2.x[1], PE_FMA(x2.x[1], y2.x[0], e2));
  double lo = PE_FMA(sgn, l2, l1) + t;
  R<2> r;
  fast_two_sum(s, lo, r.x[0], r.x[1]);
  return r;
}

template <>
PE_HD C<2> c_mul<2>(const C<2>& a, const C<2>& b) {
  return C<2>{dd_dot2(a.re, b.re, a.im, b.im, -1.0), dd_dot2(a.re, b.im, a.im, b.re, 1.0)};
}

// Renormalise four components of any relative size (a fused sum may cancel
// at order 0): a bottom-up pass of TwoSums, then a top-down compression.
PE_HD R<4> renorm4(double c0, double c1, double c2, double c3) {
  double x, e1, e2, e3, x0;
  two_sum(c2, c3, x, e3);
  two_sum(c1, x, x, e2);
  two_sum(c0, x, x0, e1);
  R<4> r;
  double y;
  fast_two_sum(x0, e1, r.x[0], y);
  two_sum(y, e2, r.x[1], y);
  two_sum(y, e3, r.x[2], r.x[3]);
  return r;
}

// L = 4: each component is a*b + c*d of quad doubles, computed as one sum
// of partial products grouped by order (the order of a_i b_j is i + j):
// orders 0..2 by TwoProd with their sums taken exactly by TwoSum chains (the
// errors of a chain belong to the next order), order 3 in plain arithmetic,
// order 4 and beyond dropped, and one renormalisation at the end, instead
// of two rounded products and a rounded sum.  Normwise error O(u^4)(|ab| +
// |cd|), u = 2^-53.
PE_HD R<4> qd_dot2(const R<4>& a, const R<4>& b, const R<4>& c, const R<4>& d) {
  // order 0
  double p0a, q0a, p0c, q0c, s0, e0;
  two_prod(a.x[0], b.x[0], p0a, q0a);
  two_prod(c.x[0], d.x[0], p0c, q0c);
  two_sum(p0a, p0c, s0, e0);
  // order 1: four products, their order-0 neighbours' errors and e0
  double p1[4], q1[4];
  two_prod(a.x[0], b.x[1], p1[0], q1[0]);
  two_prod(a.x[1], b.x[0], p1[1], q1[1]);
  two_prod(c.x[0], d.x[1], p1[2], q1[2]);
  two_prod(c.x[1], d.x[0], p1[3], q1[3]);
  double f[6], s1;
  two_sum(p1[0], p1[1], s1, f[0]);
  two_sum(s1, p1[2], s1, f[1]);
  two_sum(s1, p1[3], s1, f[2]);
  two_sum(s1, q0a, s1, f[3]);
  two_sum(s1, q0c, s1, f[4]);
  two_sum(s1, e0, s1, f[5]);
  // order 2: six products, the order-1 products' errors and the chain's
  // errors; the TwoSum errors of this chain are order-3 terms
  double p2[6], q2[6];
  two_prod(a.x[0], b.x[2], p2[0], q2[0]);
  two_prod(a.x[1], b.x[1], p2[1], q2[1]);
  two_prod(a.x[2], b.x[0], p2[2], q2[2]);
  two_prod(c.x[0], d.x[2], p2[3], q2[3]);
  two_prod(c.x[1], d.x[1], p2[4], q2[4]);
  two_prod(c.x[2], d.x[0], p2[5], q2[5]);
  double s2 = p2[0], g = 0.0, e;
#pragma unroll
  for (int i = 1; i < 6; ++i) {
    two_sum(s2, p2[i], s2, e);
    g += e;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    two_sum(s2, q1[i], s2, e);
    g += e;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    two_sum(s2, f[i], s2, e);
    g += e;
  }
  // order 3 (plain)
  double o3 = PE_FMA(a.x[0], b.x[3], PE_FMA(a.x[1], b.x[2], PE_FMA(a.x[2], b.x[1], a.x[3] * b.x[0])));
  o3 = PE_FMA(c.x[0], d.x[3], PE_FMA(c.x[1], d.x[2], PE_FMA(c.x[2], d.x[1], PE_FMA(c.x[3], d.x[0], o3))));
  const double s3 = o3 + ((q2[0] + q2[1]) + (q2[2] + q2[3]) + (q2[4] + q2[5])) + g;
  return renorm4(s0, s1, s2, s3);
}

template <>
PE_HD C<4> c_mul<4>(const C<4>& a, const C<4>& b) {
  return C<4>{qd_dot2(a.re, b.re, r_neg(a.im), b.im), qd_dot2(a.re, b.im, a.im, b.re)};
}

// ------------------------------------------------------------------ operation counts
// FP64 operations per call of each primitive as written above (an FMA counts
// once here; flop counts with FMA = 2 are derived from the FMA share).
// {instructions, fma count}
template <int L>
struct OpCount;
template <>
struct OpCount<1> {
  static constexpr int cmul = 4, cmul_fma = 2, cadd = 2, cscal = 2, cscal_fma = 0;
};
template <>
struct OpCount<2> {
  // dd_dot2: 2 two_prod (2 mul + 2 fma) + sgn*p2 (1 mul) + two_sum (6) +
  // 4 fma + fma + add + fast_two_sum (3) = 20, 7 of them FMAs
  static constexpr int cmul = 40, cmul_fma = 14;
  // r_add: two_sum (6) + 2 adds + fast_two_sum (3) = 11
  static constexpr int cadd = 22;
  // r_mul_d: two_prod (2) + fma + fast_two_sum (3) = 6, 2 FMAs
  static constexpr int cscal = 12, cscal_fma = 4;
};
template <>
struct OpCount<4> {
  // qd_dot2: 12 two_prod (24) + 22 two_sum (132) + 15 error adds + o3 (1
  // mul + 7 fma) + 8 adds + renorm4 (5 two_sum + 1 fast_two_sum = 33) =
  // 220, 19 FMAs; c_mul = 2 qd_dot2 + 4 negations
  // r_add: 4 two_sum (24) + 3 two_sum (18) + 3 adds + renorm5 (6 two_sum +
  // 1 fast_two_sum + 1 add = 40) = 85
  static constexpr int cmul = 2 * 220 + 4, cmul_fma = 38;
  static constexpr int cadd = 170;
  // r_mul_d: 3 two_prod (6) + 1 mul + 3 two_sum (18) + 3 adds + 15 = 43, 3 FMAs
  static constexpr int cscal = 86, cscal_fma = 6;
};

}  // namespace pe
