// Gauss-Newton step on the device: modified Gram-Schmidt on the augmented
// matrix [A b] with A = J(x), b = -F(x) (Sec. 3, Fig. 4 and eq. (2)), back
// substitution R dx = y, and the update x += dx (Sec. 4).
//
// One workgroup per (system, point); thread t owns columns t, t + T, ... of
// [A b].  As in the paper's delayed
// normalisation, the pivot column is never normalised in memory: the
// projection coefficient of column j is (a_k^H a_j) / |a_k|^2 and
// r_kj = (a_k^H a_j) / |a_k|, which is all the least-squares solve needs
// (Q itself is not returned).  Step k first updates column k + 1 with pivot
// k, all threads together, and stages it in LDS beside pivot k; then every
// later column is updated with pivot k and, in the same pass over its rows,
// its inner product with column k + 1 (the next pivot) is accumulated.  So a
// column is read and written once per pivot instead of read twice, with the
// arithmetic (and its order) of the plain loop for the inner products
// (summed over the rows in order); the squared norm of the next pivot is a
// workgroup sum (each thread's rows, then an XOR butterfly per wavefront,
// then the wavefronts in order).
#pragma once
#include <hip/hip_runtime.h>

#include "eval_kernels.hpp"
#include "mdarith.hpp"

namespace pe {

constexpr int kMgsThreads = 256;

template <int L>
__device__ __forceinline__ R<L> r_load_aos(const double* p) {
  R<L> r;
#pragma unroll
  for (int l = 0; l < L; ++l) r.x[l] = p[l];
  return r;
}

template <int L>
__device__ __forceinline__ void r_store_aos(double* p, const R<L>& v) {
#pragma unroll
  for (int l = 0; l < L; ++l) p[l] = v.x[l];
}

template <int L>
__device__ __forceinline__ C<L> c_mul_conj_a(const C<L>& a, const C<L>& b) {
  return c_mul(c_conj(a), b);
}

// leading limb of the imaginary part (0 for a real number)
template <int L>
__device__ __forceinline__ double im_lead(const C<L>& a) {
  if constexpr (is_real(L))
    return 0.0;
  else
    return a.im.x[0];
}

// a real level-L number as a complex (or real) one
template <int L>
__device__ __forceinline__ C<L> c_from_r(const R<limbs_of(L)>& r) {
  C<L> d = c_zero<L>();
  d.re = r;
  return d;
}

// unit roundoff of the level: 2^-53, 2^-104, 2^-206 for 1, 2, 4 limbs
template <int L>
__host__ __device__ constexpr double level_unit() {
  return limbs_of(L) == 1 ? 0x1p-53 : (limbs_of(L) == 2 ? 0x1p-104 : 0x1p-206);
}

// Per point: A (planar [2][L][N][ld], ld = n + 1, column n = b) is
// overwritten; Rw gets R as [n][n+1] complex AoS (diagonal real); yw is
// [n] complex AoS scratch for the back substitution; x is updated.
template <int L, int T>
__device__ void mgs_solve_point(int N, int n, double* __restrict__ A, double* __restrict__ Rm,
                                double* __restrict__ Y, double* __restrict__ xp, double* __restrict__ res2,
                                double* lds) {
  using RL = R<limbs_of(L)>;
  constexpr int W = width_of(L);
  const int tid = threadIdx.x;
  const int ld = n + 1;
  const int64_t plane = int64_t(N) * ld;
  double* colk = lds;                             // N numbers, AoS: pivot k
  double* coln = colk + size_t(N) * W;            // N numbers: column k + 1
  double* sh = coln + size_t(N) * W;              // |a_k|^2 of the pivot
  double* dpub = sh + W;                          // a_k^H a_{k+1}
  double* red = dpub + W;                         // T doubles for reductions
  double* wsum = red + T;                         // T / 64 wavefront sums of limbs_of(L) doubles
  int* flag = reinterpret_cast<int*>(wsum + (T / 64) * 4);  // singular flag

  // |F|_2 from the leading limbs of b = -F
  double fs = 0.0;
  for (int i = tid; i < N; i += T) {
    const double re = A[0 * plane + int64_t(i) * ld + n];
    const double im = is_real(L) ? 0.0 : A[int64_t(limbs_of(L)) * plane + int64_t(i) * ld + n];
    fs += re * re + im * im;
  }
  red[tid] = fs;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int s = T / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double fnorm = sqrt(red[0]);
  __syncthreads();

  // squared norm of column 0, and column 0 staged as the first pivot
  if (tid == 0) {
    RL s2 = r_zero<limbs_of(L)>();
    for (int i = 0; i < N; ++i) s2 = r_add(s2, c_norm2(load_planar<L>(A, plane, int64_t(i) * ld)));
    r_store_aos(sh, s2);
  }
  for (int i = tid; i < N; i += T) store_aos(colk + size_t(i) * W, load_planar<L>(A, plane, int64_t(i) * ld));
  __syncthreads();
  // inner products of the pivot with the thread's columns j >= 1, kept
  // (unscaled) in R's row 0 until step 0 scales them; the one with column 1
  // also goes to LDS (dpub) for the cooperative update
  for (int j = tid; j <= n; j += T) {
    if (j < 1) continue;
    C<L> d = c_zero<L>();
    for (int i = 0; i < N; ++i)
      d = c_add(d, c_mul_conj_a(load_aos<L>(colk + size_t(i) * W), load_planar<L>(A, plane, int64_t(i) * ld + j)));
    store_aos(Rm + size_t(j) * W, d);
    if (j == 1) store_aos(dpub, d);
  }
  __syncthreads();
  double rmax = 0.0;
  const double uL = level_unit<L>();

  for (int k = 0; k < n; ++k) {
    const RL nk = r_load_aos<limbs_of(L)>(sh);
    const RL rkk = r_sqrt(nk);
    rmax = fmax(rmax, rkk.x[0]);
    if (!(rkk.x[0] > double(n) * uL * rmax)) {
      if (tid == 0) *flag = 1;
      break;  // uniform: every thread reads the same values
    }
    const RL inv_n = r_recip(nk);
    const RL inv_r = r_recip(rkk);
    // column k + 1 (the next pivot; the right-hand side when k + 1 = n)
    // updated with pivot k by all threads and staged in LDS
    const C<L> d1 = load_aos<L>(dpub);
    const C<L> cr1 = c_neg(c_mul_r(d1, inv_n));
    RL s2 = r_zero<limbs_of(L)>();  // the thread's rows of |a_{k+1}|^2
    for (int i = tid; i < N; i += T) {
      C<L> a = load_planar<L>(A, plane, int64_t(i) * ld + k + 1);
      a = c_add(a, c_mul(cr1, load_aos<L>(colk + size_t(i) * W)));
      store_planar(A, plane, int64_t(i) * ld + k + 1, a);
      store_aos(coln + size_t(i) * W, a);
      s2 = r_add(s2, c_norm2(a));
    }
    // wavefront sums by an XOR butterfly, then the wavefronts' in order
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      RL o;
#pragma unroll
      for (int l = 0; l < limbs_of(L); ++l) o.x[l] = __shfl_xor(s2.x[l], m);
      s2 = r_add(s2, o);
    }
    if ((tid & 63) == 0) r_store_aos(wsum + (tid / 64) * 4, s2);
    if (tid == 0) {
      store_aos(Rm + (size_t(k) * ld + k) * W, c_from_r<L>(rkk));
      store_aos(Rm + (size_t(k) * ld + k + 1) * W, c_mul_r(d1, inv_r));
    }
    __syncthreads();  // column k + 1 staged; sh and dpub read by everyone
    if (tid == 0) {
      RL t2 = r_load_aos<limbs_of(L)>(wsum);
      for (int w = 1; w < T / 64; ++w) t2 = r_add(t2, r_load_aos<limbs_of(L)>(wsum + w * 4));
      r_store_aos(sh, t2);
    }
    // columns k + 2 .. n: update with pivot k (whose inner product with the
    // column the previous step left unscaled in R's row k) and, in the same
    // pass, the inner product with column k + 1, left unscaled in row k + 1
    for (int j = tid; j <= n; j += T) {
      if (j < k + 2) continue;
      double* rkj = Rm + (size_t(k) * ld + j) * W;
      const C<L> d = load_aos<L>(rkj);
      store_aos(rkj, c_mul_r(d, inv_r));
      const C<L> cr = c_neg(c_mul_r(d, inv_n));
      C<L> dn = c_zero<L>();
      for (int i = 0; i < N; ++i) {
        C<L> a = load_planar<L>(A, plane, int64_t(i) * ld + j);
        a = c_add(a, c_mul(cr, load_aos<L>(colk + size_t(i) * W)));
        store_planar(A, plane, int64_t(i) * ld + j, a);
        dn = c_add(dn, c_mul_conj_a(load_aos<L>(coln + size_t(i) * W), a));
      }
      store_aos(Rm + (size_t(k + 1) * ld + j) * W, dn);
      if (j == k + 2) store_aos(dpub, dn);
    }
    __syncthreads();
    double* t = colk;
    colk = coln;
    coln = t;
  }
  __syncthreads();
  const bool singular = *flag != 0;

  // back substitution R dx = y, y = column n of R; dx overwrites Y
  if (!singular) {
    for (int i = tid; i < n; i += T) store_aos(Y + size_t(i) * W, load_aos<L>(Rm + (size_t(i) * ld + n) * W));
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
      if (tid == 0) {
        const RL rkk = load_aos<L>(Rm + (size_t(k) * ld + k) * W).re;
        store_aos(Y + size_t(k) * W, c_mul_r(load_aos<L>(Y + size_t(k) * W), r_recip(rkk)));
      }
      __syncthreads();
      const C<L> dk = load_aos<L>(Y + size_t(k) * W);
      for (int i = tid; i < k; i += T) {
        const C<L> t = c_mul(load_aos<L>(Rm + (size_t(i) * ld + k) * W), dk);
        store_aos(Y + size_t(i) * W, c_sub(load_aos<L>(Y + size_t(i) * W), t));
      }
      __syncthreads();
    }
  }
  // update x and the step size
  double dmax = 0.0;
  for (int j = tid; j < n; j += T) {
    if (!singular) {
      const C<L> d = load_aos<L>(Y + size_t(j) * W);
      store_planar(xp, n, j, c_add(load_planar<L>(xp, n, j), d));
      dmax = fmax(dmax, fmax(fabs(d.re.x[0]), fabs(im_lead(d))));
    }
  }
  red[tid] = dmax;
  __syncthreads();
  for (int s = T / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  if (tid == 0 && res2) {
    res2[0] = fnorm;
    res2[1] = singular ? -1.0 : red[0];
  }
}

// one system, P points: block pt solves point pt
template <int L, int T>
__global__ __launch_bounds__(T) void mgs_solve_kernel(int N, int n, double* __restrict__ W, int64_t w_pt,
                                                      double* __restrict__ Rw, int64_t r_pt,
                                                      double* __restrict__ yw, int64_t y_pt,
                                                      double* __restrict__ X, int64_t x_pt,
                                                      double* __restrict__ resid) {
  extern __shared__ double lds[];
  const int pt = blockIdx.x;
  mgs_solve_point<L, T>(N, n, W + pt * w_pt, Rw + pt * r_pt, yw + pt * y_pt, X + pt * x_pt,
                        resid ? resid + 2 * pt : nullptr, lds);
}

// Per-system description of a batched Newton step (offsets in doubles for
// one point; a system's block for P points starts at P times its offset).
struct BatchNewtonDesc {
  int N, n;
  int64_t w_off, r_off, y_off, x_off;
};

// batch: block b solves point (b % P) of system order[b / P]
template <int L, int T>
__global__ __launch_bounds__(T) void mgs_solve_batch_kernel(const BatchNewtonDesc* __restrict__ desc,
                                                            const int* __restrict__ order, int P,
                                                            double* __restrict__ W, double* __restrict__ Rw,
                                                            double* __restrict__ yw, double* __restrict__ X,
                                                            double* __restrict__ resid) {
  extern __shared__ double lds[];
  const int s = order[blockIdx.x / P];
  const int pt = blockIdx.x - (blockIdx.x / P) * P;
  const BatchNewtonDesc d = desc[s];
  const int64_t w_pt = int64_t(width_of(L)) * d.N * (d.n + 1);
  const int64_t r_pt = int64_t(d.n) * (d.n + 1) * width_of(L);
  const int64_t y_pt = int64_t(d.n) * width_of(L);
  const int64_t x_pt = int64_t(width_of(L)) * d.n;
  mgs_solve_point<L, T>(d.N, d.n, W + d.w_off * P + pt * w_pt, Rw + d.r_off * P + pt * r_pt,
                        yw + d.y_off * P + pt * y_pt, X + d.x_off * P + pt * x_pt,
                        resid ? resid + (int64_t(s) * P + pt) * 2 : nullptr, lds);
}

// Right-hand side of a Newton step on the homotopy h(x, t) = f(x) - t c
// (Sec. 5.3: c = f(z), so z solves h at t = 1).  The evaluation has written
// b = -f(x) into column n of the augmented matrices (row-major planar, point
// stride w_pt, plane stride plane, row stride ld); this replaces it by
// wF b + wc c_p with wF in {0, 1}: (1, t) is the corrector at t, (0, dt) the
// Euler predictor J dx = c dt.  c is [P][components][N]; grid over P * N.
template <int L>
__global__ void rhs_shift_kernel(double* __restrict__ W, int64_t w_pt, int64_t plane, int64_t ld, int N, int n, int P,
                                 const double* __restrict__ c, double wF, double wc) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(P) * N) return;
  const int p = int(idx / N), i = int(idx - int64_t(p) * N);
  double* b = W + p * w_pt + int64_t(i) * ld + n;
  const C<L> sc = c_mul_d(load_planar<L>(c + int64_t(p) * width_of(L) * N, N, i), wc);
  store_planar(b, plane, 0, wF == 0.0 ? sc : c_add(load_planar<L>(b, plane, 0), sc));
}

template <int L>
__host__ __device__ inline size_t mgs_lds_bytes(int N) {
  return 2 * size_t(N) * width_of(L) * sizeof(double) + 2 * width_of(L) * sizeof(double) +
         kMgsThreads * sizeof(double) + (kMgsThreads / 64) * 4 * sizeof(double) + 16;
}

}  // namespace pe
