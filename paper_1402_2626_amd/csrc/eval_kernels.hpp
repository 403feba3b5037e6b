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

// EVAL: F and J; FONLY: F; ADJ: J^H v; TERMS: every monomial's value and
// partial derivatives, unsummed, in the input order
enum : int { MODE_EVAL = 0, MODE_FONLY = 1, MODE_ADJ = 2, MODE_TERMS = 3 };

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
  const uint32_t* occ_orig;   // like occ: input index of each record's occurrence
  const uint32_t* mon_orig;   // [M] input index of each packed monomial
  int col_tiles;  // tiles of kTileCols columns of a row of J (1 when n <= kTileCols)
  int col0;       // first column of the tile a workgroup owns (0 on the host)
};

// A row of J wider than kTileCols columns is evaluated by one workgroup per
// tile of kTileCols columns: every tile's workgroup runs the row's monomial
// phase (F and the partials), and its owner lanes add the slots of their
// tile's columns only (256 lanes x at most 8 columns each).
constexpr int kTileCols = 2048;

// destinations of the TERMS mode at one point: the value of input monomial t
// at V[t] (planes v_plane apart), the partial derivative of input occurrence
// o at G[o] (planes g_plane apart)
struct TermsOut {
  double* V = nullptr;
  int64_t v_plane = 0;
  double* G = nullptr;
  int64_t g_plane = 0;
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

// A level-L number (level code L: complex or real, see mdarith.hpp) in a
// planar array: limb l of the real part at base[l * plane + idx], of the
// imaginary part at base[(limbs + l) * plane + idx].
template <int L>
__device__ __forceinline__ C<L> load_planar(const double* __restrict__ base, int64_t plane, int64_t idx) {
  constexpr int NL = limbs_of(L);
  C<L> r;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    r.re.x[l] = base[l * plane + idx];
    if constexpr (!is_real(L)) r.im.x[l] = base[(NL + l) * plane + idx];
  }
  return r;
}

template <int L>
__device__ __forceinline__ void store_planar(double* __restrict__ base, int64_t plane, int64_t idx, const C<L>& v) {
  constexpr int NL = limbs_of(L);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    base[l * plane + idx] = v.re.x[l];
    if constexpr (!is_real(L)) base[(NL + l) * plane + idx] = v.im.x[l];
  }
}

// one number as consecutive doubles: real limbs, then imaginary limbs
template <int L>
__device__ __forceinline__ C<L> load_aos(const double* p) {
  constexpr int NL = limbs_of(L);
  C<L> r;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    r.re.x[l] = p[l];
    if constexpr (!is_real(L)) r.im.x[l] = p[NL + l];
  }
  return r;
}

template <int L>
__device__ __forceinline__ void store_aos(double* p, const C<L>& v) {
  constexpr int NL = limbs_of(L);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    p[l] = v.re.x[l];
    if constexpr (!is_real(L)) p[NL + l] = v.im.x[l];
  }
}

// LDS arrays of multi-doubles.  D and DD are planar (component k of element
// i at base[k * stride + i], components re limbs then im limbs): a
// wavefront's gather then reads 8-byte words spread over all banks, where
// 16- or 32-byte records map every lane's access onto a fraction of them.
// Complex QD keeps one 64-byte record per element (base[i * 8 + k]), which
// moves the same bytes in half as many LDS instructions and measured faster.
template <int L>
__device__ __forceinline__ C<L> lds_ld(const double* base, int stride, int i) {
  if constexpr (L == 4)
    return load_aos<L>(base + size_t(i) * width_of(L));
  else
    return load_planar<L>(base, stride, i);
}

template <int L>
__device__ __forceinline__ void lds_st(double* base, int stride, int i, const C<L>& v) {
  if constexpr (L == 4)
    store_aos(base + size_t(i) * width_of(L), v);
  else
    store_planar(base, stride, i, v);
}

template <int L>
__device__ __forceinline__ C<L> shfl_xor_c(const C<L>& v, int mask) {
  C<L> r;
#pragma unroll
  for (int l = 0; l < limbs_of(L); ++l) {
    r.re.x[l] = __shfl_xor(v.re.x[l], mask);
    if constexpr (!is_real(L)) r.im.x[l] = __shfl_xor(v.im.x[l], mask);
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
  return tab + size_t(e - S.tab_first) * width_of(L) * tab_cols(S);
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
  uint32_t orig[SEG];    // input occurrence of each record (TERMS mode only)
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
    const int c = S.col0 + lt + cc * kSub;
    const bool use = MODE != MODE_FONLY && MODE != MODE_TERMS && act && c < S.n;
    cl.cb[cc] = use ? int(S.colptr[cd.colptr_base + c]) : 0;
    cl.ce[cc] = use ? int(S.colptr[cd.colptr_base + c + 1]) : 0;
  }
  const int s = cd.s;
  const int g = lt / s;
  const int q = lt & (s - 1);
  const bool active = g < int(cd.count);
  cl.coef = (active && q == 0) ? load_aos<L>(S.mcoef + size_t(cd.mon_base + g) * width_of(L)) : c_one<L>();
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
    if (MODE == MODE_TERMS)
      cl.orig[i] = in_chunk ? S.occ_orig[cd.occ_base + size_t(min(i, max(segc - 1, 0))) * cd.width + lt] : kNoOcc;
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
  if constexpr (limbs_of(L) == 2) {
    auto scale = [d](const R<2>& v) {
      R<2> r;
      r.x[0] = v.x[0] * d;
      r.x[1] = PE_FMA(v.x[1], d, PE_FMA(v.x[0], d, -r.x[0]));
      return r;
    };
    C<L> r;
    r.re = scale(a.re);
    if constexpr (!is_real(L)) r.im = scale(a.im);
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
                                                     double* contrib, C<L>& facc, const TermsOut& to) {
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
  // reverse sweep of Speelpenning's product over the segment; a partial
  // goes to its LDS slot, or in TERMS mode to its input position
  auto put = [&](int i, const C<L>& gval) {
    if constexpr (MODE == MODE_TERMS) {
      if (cl.orig[i] != kNoOcc) store_planar(to.G, to.g_plane, cl.orig[i], gval);
    } else {
      lds_st(contrib, ms, cl.rec[i].slot, gval);
    }
  };
  C<L> Sx = (s > 1) ? c_mul(cf, E) : cf;
#pragma unroll
  for (int i = SEG - 1; i >= 1; --i) {
    if (FAST || i < segc) {
      C<L> gi = c_mul(pre[i - 1], Sx);
      Sx = c_mul(Sx, xv[i]);
      put(i, POW ? scale_by_exponent(gi, double(cl.rec[i].exp)) : gi);
    }
  }
  if (FAST || segc >= 1) {
    C<L> g0 = Sx;
    Sx = c_mul(Sx, xv[0]);
    put(0, POW ? scale_by_exponent(g0, double(cl.rec[0].exp)) : g0);
  }
  if (MODE == MODE_EVAL && active && q == 0) facc = c_add(facc, Sx);
  if (MODE == MODE_TERMS && active && q == 0) store_planar(to.V, to.v_plane, S.mon_orig[cd.mon_base + g], Sx);
}

template <int L, int SEG, int CPL, int MODE>
__device__ __forceinline__ void chunk_monomials(const SysView& S, const ChunkLoads<L, SEG, CPL>& cl, int lt,
                                                const double* __restrict__ xpt, const double* tab,
                                                double* contrib, C<L>& facc, const TermsOut& to = TermsOut{}) {
  // a wavefront whose lanes all lie past the chunk's last monomial has
  // nothing to contribute (its records are all neutral)
  if (__builtin_amdgcn_readfirstlane(lt & ~63) >= int(cl.cd.width)) return;
  if (int(cl.cd.seg) == SEG && tab_full(S)) {
    if (S.emax >= 2)
      chunk_monomials_body<L, SEG, CPL, MODE, true, true>(S, cl, lt, xpt, tab, contrib, facc, to);
    else
      chunk_monomials_body<L, SEG, CPL, MODE, true, false>(S, cl, lt, xpt, tab, contrib, facc, to);
    return;
  }
  if constexpr (limbs_of(L) == 1) {
    if (int(cl.cd.seg) == SEG && S.emax == 1 && tab_entries(S) == 0) {
      chunk_monomials_body<L, SEG, CPL, MODE, true, false, true>(S, cl, lt, xpt, tab, contrib, facc, to);
      return;
    }
  }
  chunk_monomials_body<L, SEG, CPL, MODE, false>(S, cl, lt, xpt, tab, contrib, facc, to);
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
  if constexpr (limbs_of(L) == 2) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      if (cb[cc] >= ce[cc]) continue;
      double rh = acc[cc].re.x[0], rl = acc[cc].re.x[1];
      dd_sum_slots(rh, rl, contrib, contrib + ms, cb[cc], ce[cc]);
      two_sum(rh, rl, acc[cc].re.x[0], acc[cc].re.x[1]);
      if constexpr (!is_real(L)) {
        double ih = acc[cc].im.x[0], il = acc[cc].im.x[1];
        dd_sum_slots(ih, il, contrib + 2 * ms, contrib + 3 * ms, cb[cc], ce[cc]);
        two_sum(ih, il, acc[cc].im.x[0], acc[cc].im.x[1]);
      }
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

// Sum of a value over groups of SPAN neighbouring lanes (SPAN a power of two
// up to 64) by an XOR butterfly; every lane of a group gets the same sum.
// Double-double: TwoSum on the high parts, low parts and errors in a plain
// sum, renormalized once (the compensated summation of the owners).
template <int L, int SPAN>
__device__ __forceinline__ C<L> lane_group_sum(const C<L>& v) {
  C<L> f = v;
  if constexpr (limbs_of(L) == 2) {
    auto sum = [](R<2>& x) {
      double h = x.x[0], l = x.x[1];
      for (int m = 1; m < SPAN; m <<= 1) {
        const double oh = __shfl_xor(h, m), ol = __shfl_xor(l, m);
        double s, e;
        two_sum(h, oh, s, e);
        h = s;
        l = (l + ol) + e;
      }
      two_sum(h, l, x.x[0], x.x[1]);
    };
    sum(f.re);
    if constexpr (!is_real(L)) sum(f.im);
  } else {
    for (int m = 1; m < SPAN; m <<= 1) f = c_add(f, shfl_xor_c(f, m));
  }
  return f;
}

template <int L>
__device__ __forceinline__ void store_wave_f(const C<L>& facc, double* fpart) {
  const C<L> f = lane_group_sum<L, 64>(facc);
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
  double* contrib = contrib_base + size_t(sg) * S.max_slots * width_of(L);
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
    constexpr int kWhen = limbs_of(L) == 2 ? 0 : (limbs_of(L) == 1 ? 1 : 2);
    const bool more = base + G < ch1;
    const bool act = base + G + sg < ch1;
    if (kWhen == 0 && more) load_chunk<L, SEG, CPL, MODE>(S, base + G + sg, act, lt, vpt, cl);
    // D and QD: the next chunk's descriptor (scalar registers) is fetched
    // before the barrier, so that only the records' load waits after it
    ChunkDesc nd{};
    if (kWhen != 0 && more && act) nd = S.chunks[uint32_t(__builtin_amdgcn_readfirstlane(int(base + G + sg)))];
    __syncthreads();
    if (kWhen == 1 && more) load_chunk_of<L, SEG, CPL, MODE>(S, nd, act, lt, vpt, cl);
    chunk_owners<L, CPL>(cb, ce, contrib, S.max_slots, acc);
    if (kWhen == 2 && more) load_chunk_of<L, SEG, CPL, MODE>(S, nd, act, lt, vpt, cl);
    __syncthreads();
  }
}

// LDS layout of a workgroup: [power table][G contribution regions][F partials
// of the 4G wavefronts]
template <int L>
__host__ __device__ inline size_t lds_bytes(int n, int tab_first, int tab_last, int max_slots, int G) {
  const size_t tab = tab_last >= tab_first ? size_t(tab_last - tab_first + 1) * (n + 1) : 0;
  return (tab + size_t(G) * max_slots + kMaxWaves) * width_of(L) * sizeof(double);
}

__device__ __forceinline__ size_t tab_doubles(const SysView& S, int L) {
  return size_t(tab_entries(S)) * tab_cols(S) * width_of(L);
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
  // columns of this workgroup's tile: S.col0 .. S.col0 + nt - 1
  const int nt = min(S.n - S.col0, kTileCols);
  if (MODE == MODE_EVAL && G > 1 && sg > 0) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = lt + cc * kSub;
      if (c < nt) lds_st(scratch + size_t(sg - 1) * width_of(L) * nt, nt, c, acc[cc]);
    }
  }
  __syncthreads();
  if (MODE == MODE_EVAL && sg == 0) {
    if (G > 1) {
      for (int o = 1; o < G; ++o) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          const int c = lt + cc * kSub;
          if (c < nt) acc[cc] = c_add(acc[cc], lds_ld<L>(scratch + size_t(o - 1) * width_of(L) * nt, nt, c));
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = lt + cc * kSub;
      if (c < nt) store_planar(O.J + pt * O.j_pt + int64_t(p) * O.j_row, O.j_plane, S.col0 + c, acc[cc]);
    }
  }
  if (int(threadIdx.x) == (4 * G - 1) * 64 && S.col0 == 0) {
    C<L> F = lds_ld<L>(fpart, kMaxWaves, 0);
    for (int o = 1; o < 4 * G; ++o) F = c_add(F, lds_ld<L>(fpart, kMaxWaves, o));
    if (O.f_sign < 0) F = c_neg(F);
    store_planar(O.F + pt * O.f_pt + int64_t(p) * O.f_row, O.f_plane, 0, F);
  }
}

// ------------------------------------------------------------------ kernels

// grid: P * N * col_tiles workgroups of G * 256 threads; block (pt, b, tile)
// (blockIdx.x = (pt * N + b) * col_tiles + tile) evaluates row
// p = row_order[b] (p = b without an order) at point pt, columns of J from
// tile * kTileCols; F is written by tile 0
template <int L, int SEG, int CPL, int G, int MODE>
__global__ __launch_bounds__(G * kSub) void eval_rows_kernel(SysView S, OutView O, const double* __restrict__ x,
                                                             int64_t x_pt) {
  static_assert(G <= kRowDesc, "the first chunk of every sub-group comes from the row-ordered descriptors");
  static_assert(4 * G <= kMaxWaves, "F partials region");
  extern __shared__ double lds[];
  const int rb = blockIdx.x / S.col_tiles;
  S.col0 = (blockIdx.x - rb * S.col_tiles) * kTileCols;
  const int pt = rb / S.N;
  const int b = rb - pt * S.N;
  const int p = S.row_order ? int(S.row_order[b]) : b;
  const double* xpt = x + pt * x_pt;
  double* tab = lds;
  double* contrib = lds + tab_doubles(S, L);
  double* fpart = contrib + size_t(G) * S.max_slots * width_of(L);
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

// Per-monomial output (values and partials written to their input
// positions; no slots, no owners, no row sums): the four wavefronts of a
// workgroup take chunks of any row one after another, each chunk in slices
// of 64 lanes (the monomials of a chunk are aligned groups of s lanes, s a
// power of two <= 64, so a slice holds whole monomials), and slice j of a
// chunk runs exactly as lanes 64 j .. 64 j + 63 of a chunk-processing
// sub-group would.  There is no barrier after the power table, which each
// workgroup builds once per point.  grid: P * wpp workgroups of 256
// threads; workgroup b of point pt takes chunks 4 b + w, 4 b + w + 4 wpp, ...
// (w its wavefront) of the nch chunks.
template <int L, int SEG>
__global__ __launch_bounds__(kSub) void terms_waves_kernel(SysView S, OutView O, const double* __restrict__ x,
                                                           int64_t x_pt, int wpp, uint32_t nch) {
  extern __shared__ double lds[];
  const int pt = blockIdx.x / wpp;
  const int b = blockIdx.x - pt * wpp;
  const double* xpt = x + pt * x_pt;
  double* tab = lds;
  const C<L> x0 = table_first_x<L>(S, xpt);
  build_power_table<L, kSub>(S, xpt, tab, x0);
  __syncthreads();
  TermsOut to;
  to.V = O.F + pt * O.f_pt;
  to.v_plane = O.f_plane;
  to.G = O.J + pt * O.j_pt;
  to.g_plane = O.j_plane;
  const uint32_t w = uint32_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6));
  const int lane = int(threadIdx.x) & 63;
  for (uint32_t ch = uint32_t(b) * 4 + w; ch < nch; ch += uint32_t(wpp) * 4) {
    const ChunkDesc cd = S.chunks[ch];
    for (int j = 0; 64 * j < int(cd.width); ++j) {
      ChunkLoads<L, SEG, 1> cl;
      load_chunk_of<L, SEG, 1, MODE_TERMS>(S, cd, true, 64 * j + lane, nullptr, cl);
      C<L> facc = c_zero<L>();
      chunk_monomials<L, SEG, 1, MODE_TERMS>(S, cl, 64 * j + lane, xpt, tab, nullptr, facc, to);
    }
  }
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
        if (c < S.n) lds_st(contrib + size_t(sg - 1) * width_of(L) * S.n, S.n, c, acc[cc]);
      }
    }
    __syncthreads();
    if (sg > 0) return;
    for (int o = 1; o < G; ++o) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int c = lt + cc * kSub;
        if (c < S.n) acc[cc] = c_add(acc[cc], lds_ld<L>(contrib + size_t(o - 1) * width_of(L) * S.n, S.n, c));
      }
    }
  }
  double* out = part + size_t(pt * NG + gi) * width_of(L) * S.n;
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
  for (int gi = 0; gi < NG; ++gi) s = c_add(s, load_planar<L>(part + size_t(pt * NG + gi) * width_of(L) * n, n, j));
  store_planar(g + size_t(pt) * width_of(L) * n, n, j, c_conj(s));
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
      O.j_pt = width_of(L) * O.j_plane;
      O.F = O.J + n;
      O.f_row = ld;
      O.f_plane = O.j_plane;
      O.f_pt = O.j_pt;
      O.f_sign = -1.0;
    } else {
      O.J = out.J ? out.J + out.J_off[s] * P : nullptr;
      O.j_row = n;
      O.j_plane = int64_t(N) * n;
      O.j_pt = width_of(L) * O.j_plane;
      O.F = out.F + out.F_off[s] * P;
      O.f_row = 1;
      O.f_plane = N;
      O.f_pt = width_of(L) * int64_t(N);
      O.f_sign = 1.0;
    }
    double* tab = lds;
    double* contrib = lds + tab_doubles(S, L);
    double* fpart = contrib + size_t(G) * S.max_slots * width_of(L);
    const uint32_t ch0 = S.chunk_ptr[p], ch1 = S.chunk_ptr[p + 1];
    const bool resident = ch1 - ch0 <= uint32_t(G);
    ChunkLoads<L, SEG, CPL> cl;
    if (resident) load_chunk<L, SEG, CPL, MODE>(S, ch0 + sg, ch0 + sg < ch1, lt, nullptr, cl);
    const double* xs = x + x_off[s] * P;
    C<L> x0 = table_first_x<L>(S, xs);
    for (int pt = 0; pt < P; ++pt) {
      const double* xpt = xs + int64_t(pt) * width_of(L) * n;
      if (!resident) load_chunk<L, SEG, CPL, MODE>(S, ch0 + sg, ch0 + sg < ch1, lt, nullptr, cl);
      // the previous point's write_row is done with the LDS before any
      // thread passes this barrier
      build_power_table<L, G * kSub>(S, xpt, tab, x0);
      __syncthreads();
      // the next point's first table column is loaded while this one runs
      if (pt + 1 < P) x0 = table_first_x<L>(S, xpt + width_of(L) * n);
      C<L> acc[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
      process_chunks<L, SEG, CPL, G, MODE>(S, ch0, ch1, xpt, nullptr, tab, contrib, acc, fpart, cl);
      write_row<L, CPL, G, MODE>(S, O, pt, p, acc, contrib, fpart);
    }
  }
}


// Output view of batch system s (the evaluation layout, or the augmented
// Newton matrices [J | -F] with row stride n + 1)
template <int L>
__device__ __forceinline__ OutView batch_out_view(const BatchOut& out, int s, int n, int N, int P) {
  OutView O;
  if (out.newton) {
    const int64_t ld = n + 1;
    O.J = out.J + out.J_off[s] * P;
    O.j_row = ld;
    O.j_plane = int64_t(N) * ld;
    O.j_pt = width_of(L) * O.j_plane;
    O.F = O.J + n;
    O.f_row = ld;
    O.f_plane = O.j_plane;
    O.f_pt = O.j_pt;
    O.f_sign = -1.0;
  } else {
    O.J = out.J ? out.J + out.J_off[s] * P : nullptr;
    O.j_row = n;
    O.j_plane = int64_t(N) * n;
    O.j_pt = width_of(L) * O.j_plane;
    O.F = out.F + out.F_off[s] * P;
    O.f_row = 1;
    O.f_plane = N;
    O.f_pt = width_of(L) * int64_t(N);
    O.f_sign = 1.0;
  }
  return O;
}

// Persistent kernel for small rows: systems whose rows are at most one chunk
// of at most VW lanes and that have at most VW variables.  The 256 threads of
// a workgroup hold Q = 256 / VW copies of the row, copy q (threads
// q VW .. q VW + VW - 1) at point pt0 + q, so that Q points are evaluated in
// one pass instead of one point per 256 lanes.  Each copy has its own power
// table, slot region and F partials in LDS; lane v of a copy does what lane
// v of a one-chunk workgroup of eval_rows_kernel does (the same records, the
// same monomial phase, the same owner column v), so every row equals
// pe_eval's bit for bit.  The records are loaded again for every pass (an
// L2 hit): kept in registers across the passes they pushed the kernel past
// the 256 registers of two wavefronts per SIMD and into scratch.  Every
// workgroup reaches the exit test after every item, so the grid drains.
template <int L, int SEG, int VW, int MODE>
__global__ __launch_bounds__(kSub, 2) void batch_small_kernel(const SysView* __restrict__ views,
                                                              const uint64_t* __restrict__ items, int64_t nitems,
                                                              int* counter, int P, const double* __restrict__ x,
                                                              const int64_t* __restrict__ x_off, BatchOut out) {
  static_assert(VW == 32 || VW == 64 || VW == 128 || VW == 256, "copy width");
  constexpr int Q = kSub / VW;
  constexpr int WPC = VW >= 64 ? VW / 64 : 1;  // F partials per copy (wavefront parts)
  extern __shared__ double lds[];
  __shared__ int64_t item_sh;
  const int qi = int(threadIdx.x) / VW;
  const int lv = int(threadIdx.x) - qi * VW;
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
    const OutView O = batch_out_view<L>(out, s, n, N, P);
    // copy qi's LDS: [table][slots][F partials]
    const size_t per_copy = tab_doubles(S, L) + size_t(S.max_slots) * width_of(L) + size_t(WPC) * width_of(L);
    double* tab = lds + per_copy * qi;
    double* contrib = tab + tab_doubles(S, L);
    double* fpart = contrib + size_t(S.max_slots) * width_of(L);
    const uint32_t ch0 = S.chunk_ptr[p], ch1 = S.chunk_ptr[p + 1];
    const double* xs = x + x_off[s] * P;
    for (int pt0 = 0; pt0 < P; pt0 += Q) {
      ChunkLoads<L, SEG, 1> cl;
      load_chunk<L, SEG, 1, MODE>(S, ch0, ch0 < ch1, lv, nullptr, cl);
      const int pt = pt0 + qi;
      const bool live = pt < P;
      const double* xpt = xs + int64_t(live ? pt : 0) * width_of(L) * n;
      // the power table of copy qi (the previous pass's owners and writes
      // are done with the LDS before any thread passes the barrier below)
      if (tab_entries(S) > 0) {
        for (int v = lv; v <= n; v += VW) {
          const C<L> x1 = v < n ? load_planar<L>(xpt, n, v) : c_one<L>();
          C<L> pw = x1;
          for (int e = 1; e <= S.tab_last; ++e) {
            if (e > 1) pw = c_mul(pw, x1);
            if (e >= S.tab_first) lds_st(const_cast<double*>(tab_block<L>(S, tab, e)), tab_cols(S), v, pw);
          }
        }
      }
      __syncthreads();
      C<L> facc = c_zero<L>();
      if (ch0 < ch1) chunk_monomials<L, SEG, 1, MODE>(S, cl, lv, xpt, tab, contrib, facc);
      // F partial of each wavefront part of the copy (lanes of one copy
      // only; the order is that of store_wave_f, lanes of other copies
      // excluded)
      {
        constexpr int span = VW < 64 ? VW : 64;
        const C<L> f = lane_group_sum<L, span>(facc);
        if ((lv & (span - 1)) == 0) lds_st(fpart, WPC, lv / span, f);
      }
      __syncthreads();
      if (MODE == MODE_EVAL) {
        C<L> acc[1] = {c_zero<L>()};
        int cb[1] = {cl.cb[0]}, ce[1] = {cl.ce[0]};
        chunk_owners<L, 1>(cb, ce, contrib, S.max_slots, acc);
        if (live && lv < n) store_planar(O.J + pt * O.j_pt + int64_t(p) * O.j_row, O.j_plane, lv, acc[0]);
      }
      if (live && lv == 0) {
        C<L> F = lds_ld<L>(fpart, WPC, 0);
        for (int o = 1; o < WPC; ++o) F = c_add(F, lds_ld<L>(fpart, WPC, o));
        if (O.f_sign < 0) F = c_neg(F);
        store_planar(O.F + pt * O.f_pt + int64_t(p) * O.f_row, O.f_plane, 0, F);
      }
    }
  }
}

}  // namespace pe
