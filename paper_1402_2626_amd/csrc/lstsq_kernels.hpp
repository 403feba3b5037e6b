// Least-squares solve of A x = b by modified Gram-Schmidt on the augmented
// matrix [A b] (Sec. 3, Fig. 4, eq. (2)), column-parallel, for systems too
// large for one workgroup, followed by a multi-stage back substitution
// (eq. (4)).
//
// The augmented matrix is first copied to a column-major working copy W.  The
// algorithm is right-looking, one workgroup per column: the workgroup that
// owns column j holds it in registers (thread t keeps rows t, t + T, ...),
// and for each pivot column c < j in turn computes the inner product
// a_c^H a_j over all N rows (each thread its rows, then a reduction across the
// workgroup: the rounds of tiled partial sums of eq. (3)), and updates
// a_j -= (a_c^H a_j / |a_c|^2) a_c.  As in the paper's delayed
// normalisation, pivot columns are never normalised in memory:
// r_cj = a_c^H a_j / |a_c| and the projection divides by |a_c|^2, so no
// workgroup ever waits for a normalised pivot.  The squared norm of a column
// is computed by its owner right after its last update, and read by every
// workgroup that uses it as a pivot.
//
// Pivots are applied in panels: a launch applies the pivots [k0, k1) to the
// columns [j0, j1), each workgroup loading its column once and applying the
// panel's pivots in increasing order; columns inside the panel first receive
// the panel's earlier pivots one launch per pivot.  Every column therefore
// receives exactly the updates of Fig. 4 in the same order as the one-column-
// at-a-time algorithm (the arithmetic is that of Fig. 4, only the loops are
// blocked), with the column read and written once per panel instead of once
// per pivot.
//
// Back substitution R x = y (y = column n of R): blocks of kBs rows from the
// bottom; a one-workgroup kernel solves the diagonal block, then a kernel of
// one workgroup per kBs rows above it subtracts the block's contribution
// (R[0:s, s:e] x[s:e]) from y -- the paper's stages of L, L - 1, ... blocks.
#pragma once
#include <hip/hip_runtime.h>

#include "eval_kernels.hpp"
#include "mdarith.hpp"
#include "newton_kernels.hpp"

namespace pe {

// ------------------------------------------------------------------ layout

// Workspace of one least-squares solve of an N x (n + 1) augmented matrix at
// P points, in doubles from the base (each region 256-byte aligned):
//   W     [P][2L][n + 1][N]   column-major working copy (column c plane-major)
//   R     [P][2L][n + 1][n]   R column-major: entry (i, j) at [j][i]; column n
//                             is y = Q^H b
//   nrm   [P][n + 1][4][L]    per pivot column: its squared norm s, sqrt(s),
//                             1 / sqrt(s) and 1 / s (computed once by the
//                             column's owner, read by every later column)
//   rmax  [P][n + 1]          largest |r_cc| up to and including column c
//   yw    [P][2L][n]          right-hand side of the back substitution
//   flag  [P]                 int: 1 when a pivot was numerically zero
struct LsLayout {
  int L = 1, N = 0, n = 0, P = 0;
  int64_t w_pt = 0, r_pt = 0, nrm_pt = 0, rmax_pt = 0, y_pt = 0;  // per point, doubles
  size_t w_off = 0, r_off = 0, nrm_off = 0, rmax_off = 0, y_off = 0, flag_off = 0, total = 0;  // bytes
};

__host__ __device__ inline size_t ls_align256(size_t b) { return (b + 255) & ~size_t(255); }

inline LsLayout ls_layout(int L, int N, int n, int P) {
  LsLayout lo;
  lo.L = L;
  lo.N = N;
  lo.n = n;
  lo.P = P;
  lo.w_pt = int64_t(width_of(L)) * (n + 1) * N;
  lo.r_pt = int64_t(width_of(L)) * (n + 1) * n;
  lo.nrm_pt = int64_t(n + 1) * 4 * limbs_of(L);
  lo.rmax_pt = n + 1;
  lo.y_pt = int64_t(width_of(L)) * n;
  size_t off = 0;
  lo.w_off = off;
  off = ls_align256(off + size_t(P) * lo.w_pt * 8);
  lo.r_off = off;
  off = ls_align256(off + size_t(P) * lo.r_pt * 8);
  lo.nrm_off = off;
  off = ls_align256(off + size_t(P) * lo.nrm_pt * 8);
  lo.rmax_off = off;
  off = ls_align256(off + size_t(P) * lo.rmax_pt * 8);
  lo.y_off = off;
  off = ls_align256(off + size_t(P) * lo.y_pt * 8);
  lo.flag_off = off;
  off = ls_align256(off + size_t(P) * sizeof(int));
  lo.total = off;
  return lo;
}

// device pointers into a workspace
struct LsView {
  int N, n;
  double* W;
  int64_t w_pt;
  double* R;
  int64_t r_pt;
  double* nrm;
  int64_t nrm_pt;
  double* rmax;
  int64_t rmax_pt;
  double* y;
  int64_t y_pt;
  int* flag;
};

inline LsView ls_view(const LsLayout& lo, void* base) {
  char* b = static_cast<char*>(base);
  LsView v;
  v.N = lo.N;
  v.n = lo.n;
  v.W = reinterpret_cast<double*>(b + lo.w_off);
  v.w_pt = lo.w_pt;
  v.R = reinterpret_cast<double*>(b + lo.r_off);
  v.r_pt = lo.r_pt;
  v.nrm = reinterpret_cast<double*>(b + lo.nrm_off);
  v.nrm_pt = lo.nrm_pt;
  v.rmax = reinterpret_cast<double*>(b + lo.rmax_off);
  v.rmax_pt = lo.rmax_pt;
  v.y = reinterpret_cast<double*>(b + lo.y_off);
  v.y_pt = lo.y_pt;
  v.flag = reinterpret_cast<int*>(b + lo.flag_off);
  return v;
}

template <int L>
__host__ __device__ constexpr double ls_unit() {
  return limbs_of(L) == 1 ? 0x1p-53 : (limbs_of(L) == 2 ? 0x1p-104 : 0x1p-206);
}

// ------------------------------------------------------------------ copy in

// Augmented matrix [A b] in the row-major planar layout of the evaluation
// ([P][2L][N][ld], row stride ld, point stride a_pt) -> column-major W.  Tiles
// of 64 rows x 64 columns through LDS so that both sides are coalesced; grid
// (ceil((n+1)/64) * ceil(N/64), 2L, P), 256 threads.  Also clears the
// singular flag of the point.
template <int L>
__global__ __launch_bounds__(256) void ls_copy_in_kernel(LsView V, const double* __restrict__ A, int64_t ld,
                                                          int64_t a_plane, int64_t a_pt) {
  __shared__ double tile[64][65];
  const int ncol = V.n + 1;
  const int tc = (ncol + 63) / 64;
  const int bt = blockIdx.x;
  const int c0 = (bt % tc) * 64, r0 = (bt / tc) * 64;
  const int comp = blockIdx.y, p = blockIdx.z;
  const double* src = A + p * a_pt + comp * a_plane;
  double* dst = V.W + p * V.w_pt + int64_t(comp) * ncol * V.N;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int row = r0 + r, col = c0 + tx;
    tile[r][tx] = (row < V.N && col < ncol) ? src[int64_t(row) * ld + col] : 0.0;
  }
  __syncthreads();
  for (int c = ty; c < 64; c += 4) {
    const int col = c0 + c, row = r0 + tx;
    if (row < V.N && col < ncol) dst[int64_t(col) * V.N + row] = tile[tx][c];
  }
  if (bt == 0 && comp == 0 && threadIdx.x == 0) V.flag[p] = 0;
}

// ------------------------------------------------------------------ reductions

// Sum of a value held by every thread of a workgroup of T threads, the same
// result in every thread: XOR butterfly in each wavefront (the additions are
// commutative, so both lanes of a pair compute the same sum), then the
// wavefront sums added in order by every thread.  `red` holds T / 64 values
// of type V.  With REUSE the buffer is free again on return (two barriers);
// without, one barrier, and the caller alternates between two buffers: a
// thread writes buffer b again only after the barrier of the sum in between,
// which every thread reaches after its reads of b.
template <int T, bool REUSE = true, typename V, typename Add, typename Shfl>
__device__ __forceinline__ V wg_sum(V v, V* red, Add add, Shfl shfl) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = add(v, shfl(v, m));
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  V s = red[0];
#pragma unroll
  for (int i = 1; i < T / 64; ++i) s = add(s, red[i]);
  if (REUSE) __syncthreads();
  return s;
}

template <int NL>
__device__ __forceinline__ R<NL> shfl_xor_r(const R<NL>& v, int mask) {
  R<NL> r;
#pragma unroll
  for (int l = 0; l < NL; ++l) r.x[l] = __shfl_xor(v.x[l], mask);
  return r;
}

// ------------------------------------------------------------------ the sweep

// Apply pivots [k0, k1) to the columns [j0, j1) (only the pivots c < j), for
// every point; grid P * (j1 - j0), T threads, EPT rows per thread (N <= T *
// EPT).  The workgroup of column j == k1 (when k1 <= n) also computes that
// column's squared norm: it is the next pivot.  `uL_n` = n u_L, the relative
// threshold below which a pivot counts as zero.
template <int L, int T, int EPT>
__global__ __launch_bounds__(T) void ls_apply_kernel(LsView V, int k0, int k1, int j0, int j1) {
  using RL = R<limbs_of(L)>;
  constexpr int NL = limbs_of(L);
  __shared__ C<L> red_c[2][T / 64];
  __shared__ RL red_r[T / 64];
  const int ncol = V.n + 1;
  const int cols = j1 - j0;
  const int p = blockIdx.x / cols;
  const int j = j0 + int(blockIdx.x - p * cols);
  if (V.flag[p]) return;  // a zero pivot was met earlier: the point is done
  const int N = V.N;
  const int64_t plane = int64_t(ncol) * N;  // doubles per component plane
  double* Wp = V.W + p * V.w_pt;
  const int tid = threadIdx.x;
  C<L> a[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = e * T + tid;
    a[e] = i < N ? load_planar<L>(Wp + int64_t(j) * N, plane, i) : c_zero<L>();
  }
  const int cend = min(k1, j);
  auto cadd = [](const C<L>& x, const C<L>& y) { return c_add(x, y); };
  auto cshf = [](const C<L>& x, int m) { return shfl_xor_c(x, m); };
  auto radd = [](const RL& x, const RL& y) { return r_add(x, y); };
  auto rshf = [](const RL& x, int m) { return shfl_xor_r(x, m); };
  const double thresh = double(V.n) * ls_unit<L>();
  // the pivot's rows: kept in registers for the update in double and
  // double double; quad double loads them again (an L2 hit) so that the
  // column alone fills the registers.  Up to 2 rows per thread the next
  // pivot's rows are loaded while the current one is applied.
  constexpr bool kKeep = width_of(L) <= 4;
  constexpr bool kPre = kKeep && EPT <= 2;
  const double* pvb = V.nrm + p * V.nrm_pt;
  auto load_q = [&](int c, C<L>* q) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = e * T + tid;
      q[e] = i < N ? load_planar<L>(Wp + int64_t(c) * N, plane, i) : c_zero<L>();
    }
  };
  C<L> qn[kPre ? EPT : 1];
  if (kPre && k0 < cend) load_q(k0, qn);
  for (int c = k0; c < cend; ++c) {
    const double* pv = pvb + int64_t(c) * 4 * NL;
    RL rcc, inv_r, inv_n;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      rcc.x[l] = pv[NL + l];
      inv_r.x[l] = pv[2 * NL + l];
      inv_n.x[l] = pv[3 * NL + l];
    }
    const double rmax = V.rmax[p * V.rmax_pt + c];
    if (!(rcc.x[0] > thresh * rmax)) {
      if (j == c + 1 && tid == 0) V.flag[p] = 1;
      return;  // uniform: every thread read the same values
    }
    C<L> q[kKeep ? EPT : 1];
    if constexpr (kPre) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) q[e] = qn[e];
      if (c + 1 < cend) load_q(c + 1, qn);
    }
    // the thread's rows in NA independent partial sums (a dependent chain
    // of EPT additions would leave the SIMD waiting on each), added
    // pairwise at the end
    constexpr int NA = EPT < 4 ? EPT : 4;
    C<L> part[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) part[k] = c_zero<L>();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      C<L> qe;
      if constexpr (kPre) {
        qe = q[e];
      } else {
        const int i = e * T + tid;
        qe = i < N ? load_planar<L>(Wp + int64_t(c) * N, plane, i) : c_zero<L>();
        if constexpr (kKeep) q[e] = qe;
      }
      part[e % NA] = c_add(part[e % NA], c_mul(c_conj(qe), a[e]));
    }
#pragma unroll
    for (int h = 1; h < NA; h <<= 1) {
#pragma unroll
      for (int k = 0; k + h < NA; k += 2 * h) part[k] = c_add(part[k], part[k + h]);
    }
    const C<L> dot = wg_sum<T, false>(part[0], red_c[c & 1], cadd, cshf);
    double* Rp = V.R + p * V.r_pt;
    const int64_t rplane = int64_t(ncol) * V.n;
    if (tid == 0) {
      store_planar(Rp + int64_t(j) * V.n, rplane, c, c_mul_r(dot, inv_r));
      if (j == c + 1) store_planar(Rp + int64_t(c) * V.n, rplane, c, c_from_r<L>(rcc));
    }
    const C<L> f = c_neg(c_mul_r(dot, inv_n));
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      if constexpr (kKeep) {
        a[e] = c_add(a[e], c_mul(f, q[e]));
      } else {
        const int i = e * T + tid;
        const C<L> qe = i < N ? load_planar<L>(Wp + int64_t(c) * N, plane, i) : c_zero<L>();
        a[e] = c_add(a[e], c_mul(f, qe));
      }
    }
  }
  if (cend > k0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = e * T + tid;
      if (i < N) store_planar(Wp + int64_t(j) * N, plane, i, a[e]);
    }
  }
  if (j == k1) {
    RL s = r_zero<NL>();
#pragma unroll
    for (int e = 0; e < EPT; ++e) s = r_add(s, c_norm2(a[e]));
    s = wg_sum<T>(s, red_r, radd, rshf);
    if (tid == 0) {
      const RL r = r_sqrt(s);
      const RL ir = r_recip(r);
      const RL is = r_recip(s);
      double* pv = V.nrm + p * V.nrm_pt + int64_t(j) * 4 * NL;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        pv[l] = s.x[l];
        pv[NL + l] = r.x[l];
        pv[2 * NL + l] = ir.x[l];
        pv[3 * NL + l] = is.x[l];
      }
      const double prev = j > 0 ? V.rmax[p * V.rmax_pt + j - 1] : 0.0;
      V.rmax[p * V.rmax_pt + j] = fmax(prev, r.x[0]);
    }
  }
}

// ------------------------------------------------------------------ back substitution

constexpr int kBs = 256;  // rows per back-substitution block

// y <- column n of R (y = Q^H b); grid ceil(n/256) x P
template <int L>
__global__ void ls_init_y_kernel(LsView V) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const int64_t rplane = int64_t(V.n + 1) * V.n;
  const C<L> y = load_planar<L>(V.R + p * V.r_pt + int64_t(V.n) * V.n, rplane, i);
  store_planar(V.y + p * V.y_pt, V.n, i, y);
}

// Solve the diagonal block [s, e) of R x = y: x_i = y_i / r_ii from the
// bottom, each solved value subtracted from the block's rows above it.  The
// solution overwrites y[s, e).  The diagonal r_jj is the norm of pivot column
// j, whose reciprocal the sweep stored; the block's reciprocals are staged in
// LDS and each thread loads its entry of the next column of R while the
// current one is applied, so the serial loop waits on no global load.  Grid
// P, kBs threads.
template <int L>
__global__ __launch_bounds__(kBs) void ls_backsub_diag_kernel(LsView V, int s, int e) {
  using RL = R<limbs_of(L)>;
  constexpr int NL = limbs_of(L);
  __shared__ C<L> ysh[kBs];
  __shared__ RL dinv[kBs];
  __shared__ C<L> xj;
  const int p = blockIdx.x;
  if (V.flag[p]) return;
  const int tid = threadIdx.x;
  const int64_t rplane = int64_t(V.n + 1) * V.n;
  const double* Rp = V.R + p * V.r_pt;
  double* yp = V.y + p * V.y_pt;
  const int i = s + tid;
  if (i < e) {
    ysh[tid] = load_planar<L>(yp, V.n, i);
    const double* pv = V.nrm + p * V.nrm_pt + int64_t(i) * 4 * NL + 2 * NL;
    RL d;
#pragma unroll
    for (int l = 0; l < NL; ++l) d.x[l] = pv[l];
    dinv[tid] = d;
  }
  C<L> rcol = i < e - 1 ? load_planar<L>(Rp + int64_t(e - 1) * V.n, rplane, i) : c_zero<L>();
  __syncthreads();
  for (int j = e - 1; j >= s; --j) {
    if (tid == 0) {
      xj = c_mul_r(ysh[j - s], dinv[j - s]);
      ysh[j - s] = xj;
    }
    __syncthreads();
    const C<L> rnext = (j > s && i < j - 1) ? load_planar<L>(Rp + int64_t(j - 1) * V.n, rplane, i) : c_zero<L>();
    if (i < j) ysh[tid] = c_sub(ysh[tid], c_mul(rcol, xj));
    rcol = rnext;
    __syncthreads();
  }
  if (i < e) store_planar(yp, V.n, i, ysh[tid]);
}

// y[0, s) -= R[0:s, s:e] x[s:e] (x[s:e] already in y[s:e]), one row per
// thread, the block's columns in increasing order.  Grid ceil(s/kBs) x P.
template <int L>
__global__ __launch_bounds__(kBs) void ls_backsub_update_kernel(LsView V, int s, int e) {
  __shared__ C<L> xs[kBs];
  const int p = blockIdx.y;
  if (V.flag[p]) return;
  const int tid = threadIdx.x;
  const int64_t rplane = int64_t(V.n + 1) * V.n;
  const double* Rp = V.R + p * V.r_pt;
  double* yp = V.y + p * V.y_pt;
  if (s + tid < e) xs[tid] = load_planar<L>(yp, V.n, s + tid);
  __syncthreads();
  const int i = blockIdx.x * kBs + tid;
  if (i >= s) return;
  C<L> acc = c_zero<L>();
  for (int j = s; j < e; ++j) acc = c_add(acc, c_mul(load_planar<L>(Rp + int64_t(j) * V.n, rplane, i), xs[j - s]));
  store_planar(yp, V.n, i, c_sub(load_planar<L>(yp, V.n, i), acc));
}

// Finish: x_out (+)= dx for every point (add = 1: Newton update x += dx;
// add = 0: x = dx), dx = 0 when a pivot was zero.  resid[p] = {|b|_2 from the
// leading limbs of the original right-hand side (column n of A, read before
// the sweep by ls_bnorm_kernel), |dx|_inf or -1 if singular}.  Grid P, 256
// threads.
template <int L>
__global__ __launch_bounds__(256) void ls_finish_kernel(LsView V, double* __restrict__ x, int64_t x_pt, int add,
                                                        double* __restrict__ resid) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const bool singular = V.flag[p] != 0;
  double dmax = 0.0;
  for (int j = tid; j < V.n; j += 256) {
    const C<L> d = singular ? c_zero<L>() : load_planar<L>(V.y + p * V.y_pt, V.n, j);
    double* xp = x + p * x_pt;
    store_planar(xp, V.n, j, add ? c_add(load_planar<L>(xp, V.n, j), d) : d);
    dmax = fmax(dmax, fmax(fabs(d.re.x[0]), fabs(im_lead(d))));
  }
  red[tid] = dmax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  if (tid == 0 && resid) resid[2 * p + 1] = singular ? -1.0 : red[0];
}

// |b|_2 of the right-hand side (column n of W, before the sweep) from the
// leading limbs into resid[p][0]; grid P, 256 threads
template <int L>
__global__ __launch_bounds__(256) void ls_bnorm_kernel(LsView V, double* __restrict__ resid) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t plane = int64_t(V.n + 1) * V.N;
  const double* b = V.W + p * V.w_pt + int64_t(V.n) * V.N;
  double s = 0.0;
  for (int i = tid; i < V.N; i += 256) {
    const double re = b[i], im = is_real(L) ? 0.0 : b[int64_t(limbs_of(L)) * plane + i];
    s += re * re + im * im;
  }
  red[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0 && resid) resid[2 * p] = sqrt(red[0]);
}

// Copy out R (row-major [P][2L][n][n+1], upper triangle and y, zeros below)
// and, if Q is not null, Q = the final pivot columns divided by their norms
// (row-major [P][2L][N][n]): the delayed normalisation of the last columns.
// Grid (ceil(max(N, n) * (n + 1) / 256), P).
template <int L>
__global__ void ls_export_kernel(LsView V, double* __restrict__ Rout, double* __restrict__ Qout) {
  const int p = blockIdx.y;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int ncol = V.n + 1;
  const int64_t rplane = int64_t(ncol) * V.n;
  if (Rout && idx < int64_t(V.n) * ncol) {
    const int i = int(idx / ncol), j = int(idx - int64_t(i) * ncol);
    const C<L> r = (i <= j) ? load_planar<L>(V.R + p * V.r_pt + int64_t(j) * V.n, rplane, i) : c_zero<L>();
    store_planar(Rout + p * (int64_t(width_of(L)) * rplane), rplane, idx, r);
  }
  if (Qout && idx < int64_t(V.N) * V.n) {
    const int i = int(idx / V.n), c = int(idx - int64_t(i) * V.n);
    constexpr int NL = limbs_of(L);
    R<NL> ir;
#pragma unroll
    for (int l = 0; l < NL; ++l) ir.x[l] = V.nrm[p * V.nrm_pt + int64_t(c) * 4 * NL + 2 * NL + l];
    const int64_t plane = int64_t(ncol) * V.N;
    const C<L> q = c_mul_r(load_planar<L>(V.W + p * V.w_pt + int64_t(c) * V.N, plane, i), ir);
    store_planar(Qout + p * (int64_t(width_of(L)) * V.N * V.n), int64_t(V.N) * V.n, idx, q);
  }
}

}  // namespace pe
