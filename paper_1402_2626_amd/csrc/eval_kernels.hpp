// Evaluation and differentiation kernels (gfx950).
//
// One workgroup owns one polynomial (row of F and J) at one point, or, for
// the adjoint, a group of polynomials at one point.  It walks the row's
// chunks (layout.hpp); per chunk:
//   1. every monomial gets s consecutive lanes; lane q loads its segment of
//      variables, gathers x and the powers for the common factor (Sec. 2.1,
//      eq. (1): the factor prod x_j^(d_j - 1) divides every partial
//      derivative), and forms the forward products of its segment;
//   2. the s segment products (times their common factors, the coefficient
//      folded into lane 0's) are combined across the lane group by a
//      butterfly, which gives every lane the product of all other segments:
//      the product tree of Sec. 2.2 / Fig. 1-2, with its levels mapped onto
//      cross-lane exchanges instead of shared memory;
//   3. each lane runs the reverse sweep of Speelpenning's product over its
//      segment (Sec. 2.2, the 3n-5 scheme) seeded with coefficient x common
//      factor x other segments, so each partial derivative comes out already
//      multiplied by the common factor and the coefficient; it is then
//      multiplied by its exponent (Sec. 2.3) and written to its LDS slot; the
//      monomial's value is what the sweep leaves at the end, and lane 0 of
//      the group adds it to its running sum of F terms (a register);
//   4. after a barrier the owner lanes add the slots of their columns in a
//      fixed order (the sum reduction of Sec. 2.3), keeping row accumulators
//      in registers across chunks.
// At the end the row of J is written with coalesced stores, and F is the sum
// of the lanes' running sums, pairwise within each wavefront and then over
// the wavefronts in order.
//
// The table of pure powers x_j^e (Sec. 2.1) is built in LDS by every
// workgroup when it fits; otherwise powers are formed by binary powering from
// x.  It has one extra column, variable n, holding the constant 1: the
// neutral records that pad short segments point there.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "mdarith.hpp"

namespace pe {

enum : int { MODE_EVAL = 0, MODE_FONLY = 1, MODE_ADJ = 2 };

struct SysView {
  int n, N;
  int emax;
  int tab_first;  // powers tab_first..tab_last of every variable are in the
  int tab_last;   // LDS table (tab_first = 1: x itself too; none if last < first)
  int max_slots;  // slots of a contribution region (largest nslots + 1)
  const ChunkDesc* chunks;
  const uint32_t* chunk_ptr;
  const ChunkDesc* rowdesc;  // [N][kRowDesc], see layout.hpp
  const OccRec* occ;
  const double* mcoef;  // [M][2L]
  const uint16_t* colptr;
  const uint32_t* row_order;  // [N] rows in decreasing cost (workgroup b of a
                              // point takes row row_order[b]), or null: row b
};

// output addressing: element (pt, c, l, row, col) of J is at
// J[pt * j_pt + (c * L + l) * j_plane + row * j_row + col]
struct OutView {
  double* J;
  int64_t j_pt, j_plane, j_row;
  double* F;
  int64_t f_pt, f_plane, f_row;
  double f_sign;  // -1 writes b = -F for Newton
};

// ------------------------------------------------------------------ helpers

template <int L>
__device__ __forceinline__ C<L> load_planar(const double* __restrict__ base, int64_t plane, int64_t idx) {
  C<L> r;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    r.re.x[l] = base[l * plane + idx];
    r.im.x[l] = base[(L + l) * plane + idx];
  }
  return r;
}

template <int L>
__device__ __forceinline__ void store_planar(double* __restrict__ base, int64_t plane, int64_t idx, const C<L>& v) {
#pragma unroll
  for (int l = 0; l < L; ++l) {
    base[l * plane + idx] = v.re.x[l];
    base[(L + l) * plane + idx] = v.im.x[l];
  }
}

template <int L>
__device__ __forceinline__ C<L> load_aos(const double* p) {
  C<L> r;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    r.re.x[l] = p[l];
    r.im.x[l] = p[L + l];
  }
  return r;
}

template <int L>
__device__ __forceinline__ void store_aos(double* p, const C<L>& v) {
#pragma unroll
  for (int l = 0; l < L; ++l) {
    p[l] = v.re.x[l];
    p[L + l] = v.im.x[l];
  }
}

// LDS arrays of complex multi-doubles.  D and DD are planar (component k of
// element i at base[k * stride + i], components re limbs then im limbs): a
// wavefront's gather then reads 8-byte words spread over all banks, where
// 16- or 32-byte records map every lane's access onto a fraction of them.
// QD keeps one 64-byte record per element (base[i * 8 + k]), which moves the
// same bytes in half as many LDS instructions and measured faster.
template <int L>
__device__ __forceinline__ C<L> lds_ld(const double* base, int stride, int i) {
  if constexpr (L == 4)
    return load_aos<L>(base + size_t(i) * (2 * L));
  else
    return load_planar<L>(base, stride, i);
}

template <int L>
__device__ __forceinline__ void lds_st(double* base, int stride, int i, const C<L>& v) {
  if constexpr (L == 4)
    store_aos(base + size_t(i) * (2 * L), v);
  else
    store_planar(base, stride, i, v);
}

template <int L>
__device__ __forceinline__ C<L> shfl_xor_c(const C<L>& v, int mask) {
  C<L> r;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    r.re.x[l] = __shfl_xor(v.re.x[l], mask);
    r.im.x[l] = __shfl_xor(v.im.x[l], mask);
  }
  return r;
}

// x^e for e >= 1 by binary powering
template <int L>
__device__ C<L> c_pow(const C<L>& x, int e) {
  C<L> r = x, b = x;
  e -= 1;
  while (e > 0) {
    if (e & 1) r = c_mul(r, b);
    e >>= 1;
    if (e) b = c_mul(b, b);
  }
  return r;
}

__device__ __forceinline__ int tab_entries(const SysView& S) {
  return S.tab_last >= S.tab_first ? S.tab_last - S.tab_first + 1 : 0;
}

// the power table has n + 1 columns: the variables and the constant 1
__device__ __forceinline__ int tab_cols(const SysView& S) { return S.n + 1; }

// powers x_v^e, e = tab_first..tab_last: table block e - tab_first holds
// 2L planes of n + 1 doubles
template <int L>
__device__ __forceinline__ const double* tab_block(const SysView& S, const double* tab, int e) {
  return tab + size_t(e - S.tab_first) * (2 * L) * tab_cols(S);
}

// the table holds x itself and every power a common factor needs
__device__ __forceinline__ bool tab_full(const SysView& S) {
  return S.tab_first == 1 && S.tab_last >= S.emax - 1;
}

// x^e (e >= 2) from the LDS table, from the table's highest power times x,
// or by binary powering
template <int L>
__device__ __forceinline__ C<L> power_of(const SysView& S, const double* tab, int v, int e, const C<L>& xv) {
  if (e >= S.tab_first && e <= S.tab_last) return lds_ld<L>(tab_block<L>(S, tab, e), tab_cols(S), v);
  if (e == S.tab_last + 1 && S.tab_last >= S.tab_first && S.tab_last >= 2)
    return c_mul(lds_ld<L>(tab_block<L>(S, tab, S.tab_last), tab_cols(S), v), xv);
  return c_pow(xv, e);
}

// x_v for a gathered variable (v = n: the constant 1): from the LDS table
// when it holds x
template <int L>
__device__ __forceinline__ C<L> load_x(const SysView& S, const double* __restrict__ xpt, const double* tab, int v) {
  if (S.tab_first == 1 && S.tab_last >= 1) return lds_ld<L>(tab, tab_cols(S), v);
  return v < S.n ? load_planar<L>(xpt, S.n, v) : c_one<L>();
}

// value of column v = threadIdx.x of the power table's first block (x_v, or 1
// for v = n), loaded ahead of the table build
template <int L>
__device__ __forceinline__ C<L> table_first_x(const SysView& S, const double* __restrict__ xpt) {
  if (tab_entries(S) == 0 || int(threadIdx.x) >= S.n) return c_one<L>();
  return load_planar<L>(xpt, S.n, int(threadIdx.x));
}

// Build the power table x_v^e, e = tab_first..tab_last, v = 0..n (x_n = 1),
// for the point in LDS; x0 = table_first_x(S, xpt).
template <int L, int T>
__device__ void build_power_table(const SysView& S, const double* __restrict__ xpt, double* tab, const C<L>& x0) {
  if (tab_entries(S) == 0) return;
  for (int v = threadIdx.x; v <= S.n; v += T) {
    const C<L> x1 = v == int(threadIdx.x) ? x0 : (v < S.n ? load_planar<L>(xpt, S.n, v) : c_one<L>());
    C<L> p = x1;
    for (int e = 1; e <= S.tab_last; ++e) {
      if (e > 1) p = c_mul(p, x1);
      if (e >= S.tab_first) lds_st(const_cast<double*>(tab_block<L>(S, tab, e)), tab_cols(S), v, p);
    }
  }
}

// ------------------------------------------------------------------ one chunk
//
// A chunk is processed by a SUB-GROUP of kSub = 256 threads (lt = local
// thread index).  A workgroup of G sub-groups works on G consecutive chunks of
// its row at once, each sub-group with its own LDS slot region and its own
// register accumulators; the G partial rows are added in sub-group order at
// the end, so the result does not depend on timing.

constexpr int kSub = 256;

// sub-group of the calling thread, as a wavefront-uniform value (kSub is a
// multiple of the wavefront size)
__device__ __forceinline__ int sub_group() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kSub); }

// Everything a lane reads from global memory for one chunk.  The loads are
// issued well before their first use (before the power table is built, or
// while the previous chunk's owners add), so their latencies overlap.
template <int L, int SEG, int CPL>
struct ChunkLoads {
  ChunkDesc cd;      // wavefront-uniform
  OccRec rec[SEG];   // the lane's records (neutral past its segment)
  C<L> coef;         // coefficient on lane 0 of a monomial's group, else 1
  C<L> vp;           // adjoint weight v_p of the chunk's polynomial
  int cb[CPL], ce[CPL];  // slot ranges of the lane's owned columns
};

// the lane's loads for the chunk with descriptor `cd` (act false: no chunk)
template <int L, int SEG, int CPL, int MODE>
__device__ __forceinline__ void load_chunk_of(const SysView& S, const ChunkDesc& cd_in, bool act, int lt,
                                              const double* __restrict__ vpt, ChunkLoads<L, SEG, CPL>& cl) {
  if (act) {
    cl.cd = cd_in;
  } else {
    cl.cd = ChunkDesc{};
    cl.cd.s = 1;
  }
  const ChunkDesc& cd = cl.cd;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int c = lt + cc * kSub;
    const bool use = MODE != MODE_FONLY && act && c < S.n;
    cl.cb[cc] = use ? int(S.colptr[cd.colptr_base + c]) : 0;
    cl.ce[cc] = use ? int(S.colptr[cd.colptr_base + c + 1]) : 0;
  }
  const int s = cd.s;
  const int g = lt / s;
  const int q = lt & (s - 1);
  const bool active = g < int(cd.count);
  cl.coef = (active && q == 0) ? load_aos<L>(S.mcoef + size_t(cd.mon_base + g) * (2 * L)) : c_one<L>();
  if (MODE == MODE_ADJ) cl.vp = act ? load_planar<L>(vpt, S.N, cd.poly) : c_zero<L>();
  // lanes past the chunk's last group get neutral records; records are
  // moved as 64-bit words (var | exp << 16 | slot << 32)
  const uint64_t pad = uint64_t(S.n) | (uint64_t(1) << 16) | (uint64_t(cd.nslots) << 32);
  const int segc = cd.seg;
  const bool in_chunk = lt < int(cd.width);
  const uint64_t* occ = reinterpret_cast<const uint64_t*>(S.occ);
#pragma unroll
  for (int i = 0; i < SEG; ++i) {
    uint64_t r = pad;
    if (in_chunk) r = occ[cd.occ_base + size_t(min(i, max(segc - 1, 0))) * cd.width + lt];
    cl.rec[i].var = uint16_t(r);
    cl.rec[i].exp = uint16_t(r >> 16);
    cl.rec[i].slot = uint16_t(r >> 32);
    cl.rec[i].pad = 0;
  }
}

// the lane's loads for chunk `ch` (wavefront-uniform)
template <int L, int SEG, int CPL, int MODE>
__device__ __forceinline__ void load_chunk(const SysView& S, uint32_t ch, bool act, int lt,
                                           const double* __restrict__ vpt, ChunkLoads<L, SEG, CPL>& cl) {
  const uint32_t chu = uint32_t(__builtin_amdgcn_readfirstlane(int(ch)));
  ChunkDesc cd{};
  if (act) cd = S.chunks[chu];
  load_chunk_of<L, SEG, CPL, MODE>(S, cd, act, lt, vpt, cl);
}

// A partial derivative times its exponent d (a small positive integer).
// Double-double leaves the product unnormalized, (p, e) with p = fl(hi d) and
// e = the exact error of that product plus lo d: |e| stays within about one
// unit in the last place of p, which every consumer of a slot (the owners'
// compensated sums, the double-double additions) accepts.
template <int L>
__device__ __forceinline__ C<L> scale_by_exponent(const C<L>& a, double d) {
  if constexpr (L == 2) {
    C<2> r;
    r.re.x[0] = a.re.x[0] * d;
    r.re.x[1] = PE_FMA(a.re.x[1], d, PE_FMA(a.re.x[0], d, -r.re.x[0]));
    r.im.x[0] = a.im.x[0] * d;
    r.im.x[1] = PE_FMA(a.im.x[1], d, PE_FMA(a.im.x[0], d, -r.im.x[0]));
    return r;
  } else {
    return c_mul_d(a, d);
  }
}

// x_v^(d-1) for the common factor when the table holds x and every power
// needed: x^0 = 1 is column n of the x block
template <int L>
__device__ __forceinline__ C<L> cf_factor_full(const SysView& S, const double* tab, int v, int d) {
  const int e = d > 1 ? d - 1 : 1;
  return lds_ld<L>(tab_block<L>(S, tab, e), tab_cols(S), d > 1 ? v : S.n);
}

// Monomial phase of one chunk: writes every partial derivative of the chunk
// into its LDS slot (planar, plane stride max_slots) and adds the values of
// the lane's monomials to facc.  All lanes of the sub-group call it (the
// butterfly needs the whole wavefront).  Every lane walks the chunk's `seg`
// records (a wavefront-uniform count; short segments are padded with neutral
// records).  In MODE_ADJ the coefficient of a monomial of polynomial p is
// multiplied by conj(v_p).
//
// FAST: the chunk's segments have exactly SEG records and the power table
// holds every power the common factors need, so the sweeps have no branches
// at all and the compiler can interleave the independent product chains.
// POW false (FAST only): every exponent of the system is 1, so there is no
// common factor and no exponent to multiply by.
// GX (double precision, with POW false only): there is no LDS table and x is
// gathered from global memory (neighbouring lanes take neighbouring occurrences, so the
// gathers of a monomial whose variables are consecutive coalesce).
template <int L, int SEG, int CPL, int MODE, bool FAST, bool POW = true, bool GX = false>
__device__ __forceinline__ void chunk_monomials_body(const SysView& S, const ChunkLoads<L, SEG, CPL>& cl, int lt,
                                                     const double* __restrict__ xpt, const double* tab,
                                                     double* contrib, C<L>& facc) {
  const ChunkDesc& cd = cl.cd;
  const int s = cd.s;
  const int g = lt / s;
  const int q = lt & (s - 1);
  const bool active = g < int(cd.count);
  const int segc = FAST ? SEG : __builtin_amdgcn_readfirstlane(int(cd.seg));
  C<L> cf = cl.coef;
  if (MODE == MODE_ADJ && active && q == 0) cf = c_mul(cf, c_conj(cl.vp));
  const int ms = S.max_slots;
  const bool full = FAST || tab_full(S);

  // every gather of the segment before any arithmetic, so that the LDS
  // latencies overlap
  C<L> xv[SEG];
  if (GX) {
    // padding records name column n, the constant 1
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
      const int v = cl.rec[i].var;
      const C<L> t = load_planar<L>(xpt, S.n, v < S.n ? v : 0);
      xv[i] = v < S.n ? t : c_one<L>();
    }
  } else {
#pragma unroll
    for (int i = 0; i < SEG; ++i)
      xv[i] = (FAST || i < segc)
                  ? (FAST ? lds_ld<L>(tab, tab_cols(S), cl.rec[i].var) : load_x<L>(S, xpt, tab, cl.rec[i].var))
                  : c_one<L>();
  }

  C<L> pre[SEG > 1 ? SEG - 1 : 1];
  C<L> A = c_one<L>();
#pragma unroll
  for (int i = 0; i < SEG; ++i) {
    if (FAST || i < segc) {
      const int v = cl.rec[i].var, d = cl.rec[i].exp;
      if (!POW) {
      } else if (full) {
        cf = c_mul(cf, cf_factor_full<L>(S, tab, v, d));
      } else if (d >= 2) {
        cf = c_mul(cf, d == 2 ? xv[i] : power_of<L>(S, tab, v, d - 1, xv[i]));
      }
      if (i == 0)
        A = xv[0];
      else
        A = c_mul(A, xv[i]);
      if (i < SEG - 1) pre[i] = A;
    }
  }
  // segment product times its common factor; the butterfly gives every lane
  // the product over the other segments of the monomial
  C<L> B = c_mul(A, cf);
  C<L> E = c_one<L>();
  for (int m = 1; m < s; m <<= 1) {
    C<L> Bp = shfl_xor_c(B, m);
    if (m == 1)
      E = Bp;
    else
      E = c_mul(E, Bp);
    B = c_mul(B, Bp);
  }
  if (MODE == MODE_FONLY) {
    // B is now the monomial's value on every lane of the group
    if (active && q == 0) facc = c_add(facc, B);
    return;
  }
  // reverse sweep of Speelpenning's product over the segment
  C<L> Sx = (s > 1) ? c_mul(cf, E) : cf;
#pragma unroll
  for (int i = SEG - 1; i >= 1; --i) {
    if (FAST || i < segc) {
      C<L> gi = c_mul(pre[i - 1], Sx);
      Sx = c_mul(Sx, xv[i]);
      lds_st(contrib, ms, cl.rec[i].slot, POW ? scale_by_exponent(gi, double(cl.rec[i].exp)) : gi);
    }
  }
  if (FAST || segc >= 1) {
    C<L> g0 = Sx;
    Sx = c_mul(Sx, xv[0]);
    lds_st(contrib, ms, cl.rec[0].slot, POW ? scale_by_exponent(g0, double(cl.rec[0].exp)) : g0);
  }
  if (MODE == MODE_EVAL && active && q == 0) facc = c_add(facc, Sx);
}

template <int L, int SEG, int CPL, int MODE>
__device__ __forceinline__ void chunk_monomials(const SysView& S, const ChunkLoads<L, SEG, CPL>& cl, int lt,
                                                const double* __restrict__ xpt, const double* tab,
                                                double* contrib, C<L>& facc) {
  // a wavefront whose lanes all lie past the chunk's last monomial has
  // nothing to contribute (its records are all neutral)
  if (__builtin_amdgcn_readfirstlane(lt & ~63) >= int(cl.cd.width)) return;
  if (int(cl.cd.seg) == SEG && tab_full(S)) {
    if (S.emax >= 2)
      chunk_monomials_body<L, SEG, CPL, MODE, true, true>(S, cl, lt, xpt, tab, contrib, facc);
    else
      chunk_monomials_body<L, SEG, CPL, MODE, true, false>(S, cl, lt, xpt, tab, contrib, facc);
    return;
  }
  if constexpr (L == 1) {
    if (int(cl.cd.seg) == SEG && S.emax == 1 && tab_entries(S) == 0) {
      chunk_monomials_body<L, SEG, CPL, MODE, true, false, true>(S, cl, lt, xpt, tab, contrib, facc);
      return;
    }
  }
  chunk_monomials_body<L, SEG, CPL, MODE, false>(S, cl, lt, xpt, tab, contrib, facc);
}

// Double-double column sum: compensated summation (Ogita, Rump and Oishi's
// Sum2 carried to double-double inputs): the high parts go through TwoSum,
// whose errors and the low parts are added in a plain running sum, and the
// pair is renormalized once at the end.  For m terms the error is about
// m^2 u^2 times the sum of their absolute values (u = 2^-53), far inside the
// double-double bound for the column lengths of a chunk, and the only serial
// dependence is one addition per slot.
__device__ __forceinline__ void dd_sum_slots(double& hi, double& lo, const double* __restrict__ phi,
                                             const double* __restrict__ plo, int b, int e) {
  int sl = b;
  for (; sl + 3 < e; sl += 4) {
    double h[4], l[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h[j] = phi[sl + j];
      l[j] = plo[sl + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double s, err;
      two_sum(hi, h[j], s, err);
      hi = s;
      lo += err + l[j];
    }
  }
  for (; sl < e; ++sl) {
    double s, err;
    two_sum(hi, phi[sl], s, err);
    hi = s;
    lo += err + plo[sl];
  }
}

// Owner phase: add the chunk's slots into the register accumulators in slot
// order.  Double-double uses the compensated sum above; the other levels add
// four slots per step as acc + ((a + b) + (c + d)) (the tail one by one), so
// that the loads of a step are in flight together and the additions form
// short chains.  The order depends only on the slot layout.
template <int L, int CPL>
__device__ __forceinline__ void chunk_owners(const int (&cb)[CPL], const int (&ce)[CPL], const double* contrib,
                                             int ms, C<L> (&acc)[CPL]) {
  if constexpr (L == 2) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      if (cb[cc] >= ce[cc]) continue;
      double rh = acc[cc].re.x[0], rl = acc[cc].re.x[1], ih = acc[cc].im.x[0], il = acc[cc].im.x[1];
      dd_sum_slots(rh, rl, contrib, contrib + ms, cb[cc], ce[cc]);
      dd_sum_slots(ih, il, contrib + 2 * ms, contrib + 3 * ms, cb[cc], ce[cc]);
      two_sum(rh, rl, acc[cc].re.x[0], acc[cc].re.x[1]);
      two_sum(ih, il, acc[cc].im.x[0], acc[cc].im.x[1]);
    }
    return;
  }
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    int sl = cb[cc];
    for (; sl + 3 < ce[cc]; sl += 4) {
      const C<L> a = lds_ld<L>(contrib, ms, sl);
      const C<L> b = lds_ld<L>(contrib, ms, sl + 1);
      const C<L> c = lds_ld<L>(contrib, ms, sl + 2);
      const C<L> d = lds_ld<L>(contrib, ms, sl + 3);
      acc[cc] = c_add(acc[cc], c_add(c_add(a, b), c_add(c, d)));
    }
    for (; sl < ce[cc]; ++sl) acc[cc] = c_add(acc[cc], lds_ld<L>(contrib, ms, sl));
  }
}

// F: each wavefront adds its lanes' running sums pairwise and stores the
// result as its F partial (fpart[w], planar with plane stride kMaxWaves)
constexpr int kMaxWaves = 16;

template <int L>
__device__ __forceinline__ void store_wave_f(const C<L>& facc, double* fpart) {
  C<L> f = facc;
  if constexpr (L == 2) {
    // double-double: TwoSum on the high parts, low parts and errors in a
    // plain sum, renormalized once (the compensated summation of the owners)
    double rh = f.re.x[0], rl = f.re.x[1], ih = f.im.x[0], il = f.im.x[1];
    for (int m = 1; m < 64; m <<= 1) {
      const double orh = __shfl_xor(rh, m), orl = __shfl_xor(rl, m);
      const double oih = __shfl_xor(ih, m), oil = __shfl_xor(il, m);
      double s, e;
      two_sum(rh, orh, s, e);
      rh = s;
      rl = (rl + orl) + e;
      two_sum(ih, oih, s, e);
      ih = s;
      il = (il + oil) + e;
    }
    two_sum(rh, rl, f.re.x[0], f.re.x[1]);
    two_sum(ih, il, f.im.x[0], f.im.x[1]);
  } else {
    for (int m = 1; m < 64; m <<= 1) f = c_add(f, shfl_xor_c(f, m));
  }
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64);
  if ((threadIdx.x & 63) == 0) lds_st(fpart, kMaxWaves, w, f);
}

// Process chunks [ch0, ch1) into the accumulators; sub-group sg takes chunks
// ch0 + sg, ch0 + sg + G, ...  `cl` holds the loads of the sub-group's first
// chunk, issued by the caller; the loads of each next chunk are issued after
// the wavefront's monomial phase (DD), before the owner phase (D) or after it
// (QD).  After the monomial phase of the last
// chunk (before the barrier the fast wavefronts wait at anyway) every
// wavefront stores its F partial, unless fpart is null.  F-only evaluation
// writes no slots and needs no barriers here.
template <int L, int SEG, int CPL, int G, int MODE>
__device__ __forceinline__ void process_chunks(const SysView& S, uint32_t ch0, uint32_t ch1,
                                               const double* __restrict__ xpt, const double* __restrict__ vpt,
                                               const double* tab, double* contrib_base, C<L> (&acc)[CPL],
                                               double* fpart, ChunkLoads<L, SEG, CPL>& cl) {
  const int sg = sub_group();
  const int lt = int(threadIdx.x) - sg * kSub;
  double* contrib = contrib_base + size_t(sg) * S.max_slots * 2 * L;
  C<L> facc = c_zero<L>();
  if (MODE != MODE_ADJ && fpart && ch0 >= ch1) store_wave_f(facc, fpart);
  for (uint32_t base = ch0; base < ch1; base += G) {
    chunk_monomials<L, SEG, CPL, MODE>(S, cl, lt, xpt, tab, contrib, facc);
    if (MODE != MODE_ADJ && fpart && base + G >= ch1) store_wave_f(facc, fpart);
    if (MODE == MODE_FONLY) {
      if (base + G < ch1) load_chunk<L, SEG, CPL, MODE>(S, base + G + sg, base + G + sg < ch1, lt, vpt, cl);
      continue;
    }
    int cb[CPL], ce[CPL];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      cb[cc] = cl.cb[cc];
      ce[cc] = cl.ce[cc];
    }
    // the next chunk's loads: DD issues them as soon as the wavefront's
    // monomial phase is done (a wavefront that waits at the barrier has them
    // in flight meanwhile), D after the barrier (its four-chunk kernels have
    // no registers to spare across it), QD, whose registers are already
    // spilled to the accumulation registers, after the owners add
    constexpr int kWhen = L == 2 ? 0 : (L == 1 ? 1 : 2);
    if (kWhen == 0 && base + G < ch1) load_chunk<L, SEG, CPL, MODE>(S, base + G + sg, base + G + sg < ch1, lt, vpt, cl);
    __syncthreads();
    if (kWhen == 1 && base + G < ch1) load_chunk<L, SEG, CPL, MODE>(S, base + G + sg, base + G + sg < ch1, lt, vpt, cl);
    chunk_owners<L, CPL>(cb, ce, contrib, S.max_slots, acc);
    if (kWhen == 2 && base + G < ch1) load_chunk<L, SEG, CPL, MODE>(S, base + G + sg, base + G + sg < ch1, lt, vpt, cl);
    __syncthreads();
  }
}

// LDS layout of a workgroup: [power table][G contribution regions][F partials
// of the 4G wavefronts]
template <int L>
__host__ __device__ inline size_t lds_bytes(int n, int tab_first, int tab_last, int max_slots, int G) {
  const size_t tab = tab_last >= tab_first ? size_t(tab_last - tab_first + 1) * (n + 1) : 0;
  return (tab + size_t(G) * max_slots + kMaxWaves) * 2 * L * sizeof(double);
}

__device__ __forceinline__ size_t tab_doubles(const SysView& S, int L) {
  return size_t(tab_entries(S)) * tab_cols(S) * 2 * L;
}

// Write row p of J and F (EVAL / FONLY).  F: the first thread of the last
// wavefront adds the wavefronts' F partials (fpart, stored by
// process_chunks) in order.  J: with G > 1 sub-groups 1..G-1 first hand
// their partial rows to sub-group 0 through LDS (the contribution regions
// are free by then), which adds them in order.
template <int L, int CPL, int G, int MODE>
__device__ __forceinline__ void write_row(const SysView& S, const OutView& O, int pt, int p, C<L> (&acc)[CPL],
                                          double* scratch, const double* fpart) {
  const int sg = sub_group();
  const int lt = int(threadIdx.x) - sg * kSub;
  if (MODE == MODE_EVAL && G > 1 && sg > 0) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = lt + cc * kSub;
      if (c < S.n) lds_st(scratch + size_t(sg - 1) * (2 * L) * S.n, S.n, c, acc[cc]);
    }
  }
  __syncthreads();
  if (MODE == MODE_EVAL && sg == 0) {
    if (G > 1) {
      for (int o = 1; o < G; ++o) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          const int c = lt + cc * kSub;
          if (c < S.n) acc[cc] = c_add(acc[cc], lds_ld<L>(scratch + size_t(o - 1) * (2 * L) * S.n, S.n, c));
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = lt + cc * kSub;
      if (c < S.n) store_planar(O.J + pt * O.j_pt + int64_t(p) * O.j_row, O.j_plane, c, acc[cc]);
    }
  }
  if (int(threadIdx.x) == (4 * G - 1) * 64) {
    C<L> F = lds_ld<L>(fpart, kMaxWaves, 0);
    for (int o = 1; o < 4 * G; ++o) F = c_add(F, lds_ld<L>(fpart, kMaxWaves, o));
    if (O.f_sign < 0) F = c_neg(F);
    store_planar(O.F + pt * O.f_pt + int64_t(p) * O.f_row, O.f_plane, 0, F);
  }
}

// ------------------------------------------------------------------ kernels

// grid: P * N workgroups of G * 256 threads; block (pt, b) = (blockIdx.x / N,
// blockIdx.x % N) evaluates row p = row_order[b] (p = b without an order) at
// point pt
template <int L, int SEG, int CPL, int G, int MODE>
__global__ __launch_bounds__(G * kSub) void eval_rows_kernel(SysView S, OutView O, const double* __restrict__ x,
                                                             int64_t x_pt) {
  static_assert(G <= kRowDesc, "the first chunk of every sub-group comes from the row-ordered descriptors");
  static_assert(4 * G <= kMaxWaves, "F partials region");
  extern __shared__ double lds[];
  const int pt = blockIdx.x / S.N;
  const int b = blockIdx.x - pt * S.N;
  const int p = S.row_order ? int(S.row_order[b]) : b;
  const double* xpt = x + pt * x_pt;
  double* tab = lds;
  double* contrib = lds + tab_doubles(S, L);
  double* fpart = contrib + size_t(G) * S.max_slots * 2 * L;
  // loads first, in the order they are needed: x for the table, the row's
  // first chunk descriptors (row-ordered copy, no dependence on chunk_ptr),
  // then the lane's records; the table is built while they are in flight
  const C<L> x0 = table_first_x<L>(S, xpt);
  const int sg = sub_group();
  const ChunkDesc cd0 = S.rowdesc[size_t(p) * kRowDesc + sg];
  ChunkLoads<L, SEG, CPL> cl;
  load_chunk_of<L, SEG, CPL, MODE>(S, cd0, cd0.count > 0, int(threadIdx.x) - sg * kSub, nullptr, cl);
  const uint32_t ch0 = S.chunk_ptr[p], ch1 = S.chunk_ptr[p + 1];
  build_power_table<L, G * kSub>(S, xpt, tab, x0);
  __syncthreads();
  C<L> acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
  process_chunks<L, SEG, CPL, G, MODE>(S, ch0, ch1, xpt, nullptr, tab, contrib, acc, fpart, cl);
  write_row<L, CPL, G, MODE>(S, O, pt, p, acc, contrib, fpart);
}

// Adjoint: grid P * NG workgroups of G * 256 threads; group gi covers
// polynomials [gi * gsize, min(N, (gi+1) * gsize)), its chunks taken G at a
// time.  The G sub-groups' column sums are added in sub-group order, and the
// result is written as the partial row part[(pt * NG + gi)][2][L][n]
// (planar, plane stride n).
template <int L, int SEG, int CPL, int G>
__global__ __launch_bounds__(G * kSub) void adjoint_rows_kernel(SysView S, const double* __restrict__ x, int64_t x_pt,
                                                                const double* __restrict__ v, int64_t v_pt, int NG,
                                                                int gsize, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int pt = blockIdx.x / NG;
  const int gi = blockIdx.x - pt * NG;
  const double* xpt = x + pt * x_pt;
  const double* vpt = v + pt * v_pt;
  double* tab = lds;
  double* contrib = lds + tab_doubles(S, L);
  const int p0 = gi * gsize;
  const int p1 = min(S.N, p0 + gsize);
  const uint32_t ch0 = S.chunk_ptr[p0], ch1 = S.chunk_ptr[p1];
  const int sg = sub_group();
  const int lt = int(threadIdx.x) - sg * kSub;
  ChunkLoads<L, SEG, CPL> cl;
  const C<L> x0 = table_first_x<L>(S, xpt);
  load_chunk<L, SEG, CPL, MODE_ADJ>(S, ch0 + sg, ch0 + sg < ch1, lt, vpt, cl);
  build_power_table<L, G * kSub>(S, xpt, tab, x0);
  __syncthreads();
  C<L> acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
  process_chunks<L, SEG, CPL, G, MODE_ADJ>(S, ch0, ch1, xpt, vpt, tab, contrib, acc, nullptr, cl);
  if (G > 1) {
    // the slot regions are free (process_chunks ends with a barrier)
    if (sg > 0) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int c = lt + cc * kSub;
        if (c < S.n) lds_st(contrib + size_t(sg - 1) * (2 * L) * S.n, S.n, c, acc[cc]);
      }
    }
    __syncthreads();
    if (sg > 0) return;
    for (int o = 1; o < G; ++o) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int c = lt + cc * kSub;
        if (c < S.n) acc[cc] = c_add(acc[cc], lds_ld<L>(contrib + size_t(o - 1) * (2 * L) * S.n, S.n, c));
      }
    }
  }
  double* out = part + size_t(pt * NG + gi) * 2 * L * S.n;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int c = lt + cc * kSub;
    if (c < S.n) store_planar(out, S.n, c, acc[cc]);
  }
}

// g[pt][.][.][j] = conj(sum over groups of part[pt][gi][.][.][j]) in group order
template <int L>
__global__ void adjoint_reduce_kernel(int n, int NG, int P, const double* __restrict__ part, double* __restrict__ g) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(P) * n) return;
  const int pt = int(idx / n);
  const int j = int(idx - int64_t(pt) * n);
  C<L> s = c_zero<L>();
  for (int gi = 0; gi < NG; ++gi) s = c_add(s, load_planar<L>(part + size_t(pt * NG + gi) * 2 * L * n, n, j));
  store_planar(g + size_t(pt) * 2 * L * n, n, j, c_conj(s));
}

// ------------------------------------------------------------------ batches

// Outputs of a batch: system s's F/J blocks start at P * F_off[s] and
// P * J_off[s] (doubles).  In Newton mode J points at the workspace of
// augmented matrices [J | -F] (row stride n + 1) and F is unused.
struct BatchOut {
  double* J;
  const int64_t* J_off;
  double* F;
  const int64_t* F_off;
  int newton;
};

// Persistent kernel: workgroups of G sub-groups take (system, polynomial)
// items from a device counter in the order of `items` (decreasing cost) until
// none is left; each item is evaluated at all P points.  When the row has at
// most G chunks, every sub-group loads its chunk's records once and keeps
// them in registers for all P points.  Every workgroup reaches the exit test
// after every item, so the grid drains.
template <int L, int SEG, int CPL, int G, int MODE>
__global__ __launch_bounds__(G * kSub) void batch_rows_kernel(const SysView* __restrict__ views,
                                                              const uint64_t* __restrict__ items, int64_t nitems,
                                                              int* counter, int P, const double* __restrict__ x,
                                                              const int64_t* __restrict__ x_off, BatchOut out) {
  static_assert(4 * G <= kMaxWaves, "F partials region");
  extern __shared__ double lds[];
  __shared__ int64_t item_sh;
  const int sg = sub_group();
  const int lt = int(threadIdx.x) - sg * kSub;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int64_t it = item_sh;
    __syncthreads();
    if (it >= nitems) break;
    const uint64_t w = items[it];
    const int s = int(w >> 32);
    const int p = int(w & 0xffffffffu);
    const SysView S = views[s];
    const int n = S.n, N = S.N;
    OutView O;
    if (out.newton) {
      const int64_t ld = n + 1;
      O.J = out.J + out.J_off[s] * P;
      O.j_row = ld;
      O.j_plane = int64_t(N) * ld;
      O.j_pt = 2 * L * O.j_plane;
      O.F = O.J + n;
      O.f_row = ld;
      O.f_plane = O.j_plane;
      O.f_pt = O.j_pt;
      O.f_sign = -1.0;
    } else {
      O.J = out.J ? out.J + out.J_off[s] * P : nullptr;
      O.j_row = n;
      O.j_plane = int64_t(N) * n;
      O.j_pt = 2 * L * O.j_plane;
      O.F = out.F + out.F_off[s] * P;
      O.f_row = 1;
      O.f_plane = N;
      O.f_pt = 2 * L * int64_t(N);
      O.f_sign = 1.0;
    }
    double* tab = lds;
    double* contrib = lds + tab_doubles(S, L);
    double* fpart = contrib + size_t(G) * S.max_slots * 2 * L;
    const uint32_t ch0 = S.chunk_ptr[p], ch1 = S.chunk_ptr[p + 1];
    const bool resident = ch1 - ch0 <= uint32_t(G);
    ChunkLoads<L, SEG, CPL> cl;
    if (resident) load_chunk<L, SEG, CPL, MODE>(S, ch0 + sg, ch0 + sg < ch1, lt, nullptr, cl);
    const double* xs = x + x_off[s] * P;
    C<L> x0 = table_first_x<L>(S, xs);
    for (int pt = 0; pt < P; ++pt) {
      const double* xpt = xs + int64_t(pt) * 2 * L * n;
      if (!resident) load_chunk<L, SEG, CPL, MODE>(S, ch0 + sg, ch0 + sg < ch1, lt, nullptr, cl);
      // the previous point's write_row is done with the LDS before any
      // thread passes this barrier
      build_power_table<L, G * kSub>(S, xpt, tab, x0);
      __syncthreads();
      // the next point's first table column is loaded while this one runs
      if (pt + 1 < P) x0 = table_first_x<L>(S, xpt + 2 * L * n);
      C<L> acc[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
      process_chunks<L, SEG, CPL, G, MODE>(S, ch0, ch1, xpt, nullptr, tab, contrib, acc, fpart, cl);
      write_row<L, CPL, G, MODE>(S, O, pt, p, acc, contrib, fpart);
    }
  }
}

}  // namespace pe
