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
//      monomial's value is what the sweep leaves at the end;
//   4. after a barrier the owner lanes add the slots of their columns in a
//      fixed order (the sum reduction of Sec. 2.3), keeping row accumulators
//      in registers across chunks.
// At the end the row of J is written with coalesced stores and F is the
// ordered sum of the R partial columns.
//
// The table of pure powers x_j^e (Sec. 2.1) for e = 2 .. emax-1 is built in
// LDS by every workgroup when it fits; otherwise powers are formed by binary
// powering from x.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "mdarith.hpp"

namespace pe {

enum : int { MODE_EVAL = 0, MODE_FONLY = 1, MODE_ADJ = 2 };

struct SysView {
  int n, N, R, ncols;
  int emax;
  int tab_first;  // powers tab_first..tab_last of every variable are in the
  int tab_last;   // LDS table (tab_first = 1: x itself too; none if last < first)
  int max_slots;
  const ChunkDesc* chunks;
  const uint32_t* chunk_ptr;
  const OccRec* occ;
  const double* mcoef;  // [M][2L]
  const uint32_t* mmeta;
  const uint16_t* colptr;
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

// x^e (e >= 2) from the LDS table, from the table's highest power times x,
// or by binary powering
template <int L>
__device__ __forceinline__ C<L> power_of(const SysView& S, const double* tab, int v, int e, const C<L>& xv) {
  if (e >= S.tab_first && e <= S.tab_last) return load_aos<L>(tab + (size_t(e - S.tab_first) * S.n + v) * (2 * L));
  if (e == S.tab_last + 1 && S.tab_last >= S.tab_first && S.tab_last >= 2)
    return c_mul(load_aos<L>(tab + (size_t(S.tab_last - S.tab_first) * S.n + v) * (2 * L)), xv);
  return c_pow(xv, e);
}

// x_v for a gathered variable: from the LDS table when it holds x
template <int L>
__device__ __forceinline__ C<L> load_x(const SysView& S, const double* __restrict__ xpt, const double* tab, int v) {
  if (S.tab_first == 1 && S.tab_last >= 1) return load_aos<L>(tab + size_t(v) * (2 * L));
  return load_planar<L>(xpt, S.n, v);
}

// Build the power table x_v^e, e = tab_first..tab_last, for the point in LDS.
template <int L, int T>
__device__ void build_power_table(const SysView& S, const double* __restrict__ xpt, double* tab) {
  if (tab_entries(S) == 0) return;
  for (int v = threadIdx.x; v < S.n; v += T) {
    const C<L> x1 = load_planar<L>(xpt, S.n, v);
    C<L> p = x1;
    for (int e = 1; e <= S.tab_last; ++e) {
      if (e > 1) p = c_mul(p, x1);
      if (e >= S.tab_first) store_aos(tab + (size_t(e - S.tab_first) * S.n + v) * (2 * L), p);
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

// Monomial phase of one chunk: writes every contribution of the chunk into
// its LDS slot.  All lanes of the sub-group call it (the butterfly needs the
// whole wavefront).  In MODE_ADJ the coefficient of a monomial of polynomial
// p is multiplied by conj(v_p).
template <int L, int SEG, int MODE>
__device__ __forceinline__ void chunk_monomials(const SysView& S, const ChunkDesc& cd, int lt,
                                                const double* __restrict__ xpt,
                                                const double* __restrict__ vpt, const double* tab,
                                                double* contrib) {
  const int s = cd.s;
  const int g = lt / s;
  const int q = lt & (s - 1);
  const bool active = g < int(cd.count);

  int k = 0, fslot = 0;
  C<L> cf = c_one<L>();
  if (active) {
    const uint32_t meta = S.mmeta[cd.mon_base + g];
    k = int(meta & 0xffffu);
    fslot = int(meta >> 16);
    if (q == 0) {
      cf = load_aos<L>(S.mcoef + size_t(cd.mon_base + g) * (2 * L));
      if (MODE == MODE_ADJ) cf = c_mul(cf, c_conj(load_planar<L>(vpt, S.N, cd.poly)));
    }
  }
  const int base = k / s, extra = k - base * s;
  const int len = base + (q < extra ? 1 : 0);

  // Issue every load of the lane before any arithmetic: the occurrence
  // records (indices clamped inside the chunk, so lanes past their segment or
  // past the chunk read valid padding records) and then the variables.
  // Keeping the loads out of the per-variable branches lets their latencies
  // overlap instead of adding up.
  OccRec rec[SEG];
  if (cd.width > 0) {
    const int lane_c = min(lt, int(cd.width) - 1);
    const int segc = cd.seg;
#pragma unroll
    for (int i = 0; i < SEG; ++i) rec[i] = S.occ[cd.occ_base + size_t(min(i, segc - 1)) * cd.width + lane_c];
  } else {
#pragma unroll
    for (int i = 0; i < SEG; ++i) rec[i] = OccRec{0, 0, 0, 0};
  }
  C<L> xv[SEG];
#pragma unroll
  for (int i = 0; i < SEG; ++i) xv[i] = load_x<L>(S, xpt, tab, rec[i].var);

  C<L> pre[SEG > 1 ? SEG - 1 : 1];
  C<L> A = c_one<L>();
#pragma unroll
  for (int i = 0; i < SEG; ++i) {
    if (i < len) {
      const int v = rec[i].var, d = rec[i].exp;
      if (d >= 2) cf = c_mul(cf, d == 2 ? xv[i] : power_of<L>(S, tab, v, d - 1, xv[i]));
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
    if (active && q == 0) store_aos(contrib + size_t(fslot) * (2 * L), B);
    return;
  }
  // reverse sweep of Speelpenning's product over the segment
  C<L> Sx = (s > 1) ? c_mul(cf, E) : cf;
#pragma unroll
  for (int i = SEG - 1; i >= 1; --i) {
    if (i < len) {
      C<L> gi = c_mul(pre[i - 1], Sx);
      Sx = c_mul(Sx, xv[i]);
      store_aos(contrib + size_t(rec[i].slot) * (2 * L), c_mul_d(gi, double(rec[i].exp)));
    }
  }
  if (len >= 1) {
    C<L> g0 = Sx;
    Sx = c_mul(Sx, xv[0]);
    store_aos(contrib + size_t(rec[0].slot) * (2 * L), c_mul_d(g0, double(rec[0].exp)));
  }
  if (MODE == MODE_EVAL && active && q == 0) store_aos(contrib + size_t(fslot) * (2 * L), Sx);
}

// Owner phase: add the chunk's slots into the register accumulators.
template <int L, int CPL>
__device__ __forceinline__ void chunk_owners(const int (&cb)[CPL], const int (&ce)[CPL], const double* contrib,
                                             C<L> (&acc)[CPL]) {
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    // two slots per step: both loads are issued before the additions
    int sl = cb[cc];
    for (; sl + 1 < ce[cc]; sl += 2) {
      const C<L> a = load_aos<L>(contrib + size_t(sl) * (2 * L));
      const C<L> b = load_aos<L>(contrib + size_t(sl + 1) * (2 * L));
      acc[cc] = c_add(c_add(acc[cc], a), b);
    }
    if (sl < ce[cc]) acc[cc] = c_add(acc[cc], load_aos<L>(contrib + size_t(sl) * (2 * L)));
  }
}

// Columns of the accumulator slot cc of local thread lt: lt + cc * kSub.
template <int CPL, int MODE>
__device__ __forceinline__ void chunk_colptr(const SysView& S, const ChunkDesc& cd, bool act, int lt,
                                             int (&cb)[CPL], int (&ce)[CPL]) {
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int c = lt + cc * kSub;
    bool use = act && c < S.ncols;
    if (MODE == MODE_FONLY) use = use && c >= S.n;
    if (MODE == MODE_ADJ) use = use && c < S.n;
    if (use) {
      cb[cc] = S.colptr[cd.colptr_base + c];
      ce[cc] = S.colptr[cd.colptr_base + c + 1];
    } else {
      cb[cc] = 0;
      ce[cc] = 0;
    }
  }
}

// Process chunks [ch0, ch1) into the accumulators; sub-group sg takes chunks
// ch0 + sg, ch0 + sg + G, ...
template <int L, int SEG, int CPL, int G, int MODE>
__device__ __forceinline__ void process_chunks(const SysView& S, uint32_t ch0, uint32_t ch1, const double* __restrict__ xpt,
                               const double* __restrict__ vpt, const double* tab, double* contrib_base,
                               C<L> (&acc)[CPL]) {
  const int sg = threadIdx.x / kSub;
  const int lt = threadIdx.x - sg * kSub;
  double* contrib = contrib_base + size_t(sg) * S.max_slots * 2 * L;
  for (uint32_t base = ch0; base < ch1; base += G) {
    const uint32_t ch = base + sg;
    const bool act = ch < ch1;
    ChunkDesc cd;
    if (act) {
      cd = S.chunks[ch];
    } else {
      cd = ChunkDesc{};
      cd.s = 1;
    }
    int cb[CPL], ce[CPL];
    chunk_colptr<CPL, MODE>(S, cd, act, lt, cb, ce);
    chunk_monomials<L, SEG, MODE>(S, cd, lt, xpt, vpt, tab, contrib);
    __syncthreads();
    chunk_owners<L, CPL>(cb, ce, contrib, acc);
    __syncthreads();
  }
}

// Write row p of J and F from the accumulators (EVAL / FONLY).  With G > 1
// sub-groups 1..G-1 first hand their partial rows to sub-group 0 through
// LDS (the contribution region is free by then), which adds them in order.
template <int L, int CPL, int G, int MODE>
__device__ __forceinline__ void write_row(const SysView& S, const OutView& O, int pt, int p, C<L> (&acc)[CPL], double* scratch,
                          double* fpart) {
  const int sg = threadIdx.x / kSub;
  const int lt = threadIdx.x - sg * kSub;
  if (G > 1) {
    if (sg > 0) {
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int c = lt + cc * kSub;
        if (c < S.ncols) store_aos(scratch + (size_t(sg - 1) * S.ncols + c) * (2 * L), acc[cc]);
      }
    }
    __syncthreads();
    if (sg == 0) {
      for (int o = 1; o < G; ++o) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          const int c = lt + cc * kSub;
          if (c < S.ncols) acc[cc] = c_add(acc[cc], load_aos<L>(scratch + (size_t(o - 1) * S.ncols + c) * (2 * L)));
        }
      }
    }
  }
  if (sg == 0) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int c = lt + cc * kSub;
      if (c < S.n) {
        if (MODE == MODE_EVAL) store_planar(O.J + pt * O.j_pt + int64_t(p) * O.j_row, O.j_plane, c, acc[cc]);
      } else if (c < S.ncols) {
        store_aos(fpart + size_t(c - S.n) * (2 * L), acc[cc]);
      }
    }
  }
  __syncthreads();
  // F = sum of the R partial columns, added pairwise across the lanes of the
  // first wavefront (R <= 32)
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    C<L> f = r < S.R ? load_aos<L>(fpart + size_t(r) * (2 * L)) : c_zero<L>();
    for (int m = 1; m < 32; m <<= 1) f = c_add(f, shfl_xor_c(f, m));
    if (r == 0) {
      if (O.f_sign < 0) f = c_neg(f);
      store_planar(O.F + pt * O.f_pt + int64_t(p) * O.f_row, O.f_plane, 0, f);
    }
  }
  __syncthreads();
}

// LDS layout of a workgroup: [power table][G contribution regions][F partials]
template <int L>
__host__ __device__ inline size_t lds_bytes(int n, int tab_first, int tab_last, int max_slots, int R, int G) {
  const size_t tab = tab_last >= tab_first ? size_t(tab_last - tab_first + 1) * n : 0;
  return (tab + size_t(G) * max_slots + size_t(R)) * 2 * L * sizeof(double);
}

__device__ __forceinline__ size_t tab_doubles(const SysView& S, int L) {
  return size_t(tab_entries(S)) * S.n * 2 * L;
}

// ------------------------------------------------------------------ kernels

// grid: P * N workgroups of G * 256 threads, block (pt, p) = (blockIdx.x / N,
// blockIdx.x % N)
template <int L, int SEG, int CPL, int G, int MODE>
__global__ __launch_bounds__(G * kSub) void eval_rows_kernel(SysView S, OutView O, const double* __restrict__ x,
                                                             int64_t x_pt) {
  extern __shared__ double lds[];
  const int pt = blockIdx.x / S.N;
  const int p = blockIdx.x - pt * S.N;
  const double* xpt = x + pt * x_pt;
  double* tab = lds;
  double* contrib = lds + tab_doubles(S, L);
  double* fpart = contrib + size_t(G) * S.max_slots * 2 * L;
  build_power_table<L, G * kSub>(S, xpt, tab);
  __syncthreads();
  C<L> acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
  process_chunks<L, SEG, CPL, G, MODE>(S, S.chunk_ptr[p], S.chunk_ptr[p + 1], xpt, nullptr, tab, contrib, acc);
  write_row<L, CPL, G, MODE>(S, O, pt, p, acc, contrib, fpart);
}

// Adjoint: grid P * NG workgroups of 256 threads; group gi covers
// polynomials [gi * gsize, min(N, (gi+1) * gsize)).  Writes partial rows
// part[(pt * NG + gi)][2][L][n] (planar, plane stride n).
template <int L, int SEG, int CPL>
__global__ __launch_bounds__(kSub) void adjoint_rows_kernel(SysView S, const double* __restrict__ x, int64_t x_pt,
                                                            const double* __restrict__ v, int64_t v_pt, int NG,
                                                            int gsize, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int pt = blockIdx.x / NG;
  const int gi = blockIdx.x - pt * NG;
  const double* xpt = x + pt * x_pt;
  const double* vpt = v + pt * v_pt;
  double* tab = lds;
  double* contrib = lds + tab_doubles(S, L);
  build_power_table<L, kSub>(S, xpt, tab);
  __syncthreads();
  C<L> acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
  const int p0 = gi * gsize;
  const int p1 = min(S.N, p0 + gsize);
  process_chunks<L, SEG, CPL, 1, MODE_ADJ>(S, S.chunk_ptr[p0], S.chunk_ptr[p1], xpt, vpt, tab, contrib, acc);
  double* out = part + size_t(pt * NG + gi) * 2 * L * S.n;
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    const int c = threadIdx.x + cc * kSub;
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

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Persistent kernel: workgroups take (system, polynomial) items from a
// device counter in the order of `items` (decreasing cost) until none is
// left; each item is evaluated at all P points.  Every workgroup reaches the
// exit test after every item, so the grid drains.
template <int L, int SEG, int CPL, int MODE>
__global__ __launch_bounds__(kSub) void batch_rows_kernel(const SysView* __restrict__ views,
                                                          const uint64_t* __restrict__ items, int64_t nitems,
                                                          int* counter, int P, const double* __restrict__ x,
                                                          const int64_t* __restrict__ x_off, BatchOut out) {
  extern __shared__ double lds[];
  __shared__ int64_t item_sh;
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
    double* fpart = contrib + size_t(S.max_slots) * 2 * L;
    for (int pt = 0; pt < P; ++pt) {
      const double* xpt = x + x_off[s] * P + int64_t(pt) * 2 * L * n;
      build_power_table<L, kSub>(S, xpt, tab);
      __syncthreads();
      C<L> acc[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) acc[cc] = c_zero<L>();
      process_chunks<L, SEG, CPL, 1, MODE>(S, S.chunk_ptr[p], S.chunk_ptr[p + 1], xpt, nullptr, tab, contrib, acc);
      write_row<L, CPL, 1, MODE>(S, O, pt, p, acc, contrib, fpart);
    }
  }
}

}  // namespace pe
