// One-workgroup FP64 small linear algebra between two fibre passes of the
// ALS mode solve (Algorithm 3.3), so that a sweep costs one fused pass, one
// reduction and one launch of this kernel:
//   SOLVE  L_{k+1} = L_acc (R_k^T R_k)^{-1} with G_V = R_k^T R_k (Cholesky,
//          explicit inverse of the r x r factor),
//          the residual from the trace identity ||B||^2 - tr(Gq^{-1} G_V)
//          (or the explicit sum);
//   QR     reduced QR of a tall matrix by CholeskyQR2 (diag(R_hat) > 0),
//          used for the initial guess (Section 5) and the returned factor;
//   PREP   for the next sweep: L~ = L (L^T L)^{-1} quantised to the compute
//          type, the Cholesky factor of the Gram of the quantised L~ and,
//          for the explicit residual, L in the compute type.
// Every Cholesky applies the pivot test of Remark 3 (squared pivot at most
// PIVOT_TOL times the largest diagonal entry: rank deficient).  Matrices are
// m x r row-major FP64 in global memory (m up to a few thousand, r <= 64);
// the r x r factors, their inverses and inverse Grams live in LDS, and every
// m x r result is a plain product with one of them (independent output
// elements, no per-thread solve state).  All sums have a fixed order.
#include <math.h>

#include "tk_kernels.h"

namespace tk {
namespace {

constexpr int NT = 1024;
constexpr int LD = 65;     // LDS row stride of the r x r matrices
constexpr int TR = 64;     // rows per staged tile
constexpr int PPT = 3;     // Gram pairs per thread (r (r + 1) / 2 <= 2080 <= 3 NT)

// sum_{l < n} x[l * sx] * y[l * sy] with four independent partial sums
// (combined in a fixed order).
__device__ __forceinline__ double dot4(const double* x, int sx, const double* y, int sy, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int l = 0;
  for (; l + 3 < n; l += 4) {
    s0 += x[l * sx] * y[l * sy];
    s1 += x[(l + 1) * sx] * y[(l + 1) * sy];
    s2 += x[(l + 2) * sx] * y[(l + 2) * sy];
    s3 += x[(l + 3) * sx] * y[(l + 3) * sy];
  }
  for (; l < n; ++l) s0 += x[l * sx] * y[l * sy];
  return (s0 + s1) + (s2 + s3);
}

// G = X^T X (r x r, LDS, stride LD) of the m x r matrix X (type T, global):
// thread t owns the upper-triangle pairs t, t + NT, ... (at most PPT).
template <typename T>
__device__ void bgram(const T* __restrict__ X, int64_t m, int r, double* G, double* tile) {
  const int npair = r * (r + 1) / 2;
  double acc[PPT];
  int pa[PPT], pb[PPT];
  int cnt = 0;
#pragma unroll
  for (int c = 0; c < PPT; ++c) {
    const int t = (int)threadIdx.x + NT * c;
    int a = 0, rem = t < npair ? t : 0;
    while (rem >= r - a) { rem -= r - a; ++a; }
    pa[c] = a;
    pb[c] = a + rem;
    acc[c] = 0.0;
    if (t < npair) cnt = c + 1;
  }
  for (int64_t i0 = 0; i0 < m; i0 += TR) {
    const int rows = (int)((m - i0) < TR ? (m - i0) : TR);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * r; e += NT)
      tile[e] = (double)Elem<T>::load(X + i0 * r + e);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PPT; ++c)
      if (c < cnt) acc[c] += dot4(tile + pa[c], r, tile + pb[c], r, rows);
  }
#pragma unroll
  for (int c = 0; c < PPT; ++c) {
    if (c < cnt) {
      G[pa[c] * LD + pb[c]] = acc[c];
      G[pb[c] * LD + pa[c]] = acc[c];
    }
  }
  __syncthreads();
}

// In-place lower Cholesky of the LDS matrix a (stride LD).  Returns true
// (uniformly over the block) when the pivot test fails; the flag is only
// written by thread 0 in a phase where no other thread reads it.
__device__ bool bchol(double* a, int r, int* flag, double* dmax) {
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int k = 0; k < r; ++k) mx = fmax(mx, a[k * LD + k]);
    *dmax = mx;
    *flag = !(mx > 0.0) || !isfinite(mx);
  }
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    if (threadIdx.x == 0 && !*flag) {
      const double d = a[k * LD + k];
      if (!(d > PIVOT_TOL * *dmax) || !isfinite(d)) *flag = 1;
      else a[k * LD + k] = sqrt(d);
    }
    __syncthreads();
    if (*flag) break;
    const double dk = a[k * LD + k];
    for (int i = k + 1 + threadIdx.x; i < r; i += NT) a[i * LD + k] /= dk;
    __syncthreads();
    const int n = r - k - 1;
    for (int e = threadIdx.x; e < n * n; e += NT) {
      const int i = k + 1 + e / n, j = k + 1 + e % n;
      if (j <= i) a[i * LD + j] -= a[i * LD + k] * a[j * LD + k];
    }
    __syncthreads();
  }
  const bool bad = *flag != 0;
  if (!bad)
    for (int e = threadIdx.x; e < r * r; e += NT)
      if (e % r > e / r) a[(e / r) * LD + e % r] = 0.0;
  __syncthreads();
  return bad;
}

// W = C^{-1} (lower, zeros above the diagonal) of the LDS lower factor C;
// thread j solves column j by forward substitution.
__device__ void binv(const double* C, int r, double* W) {
  const int j = threadIdx.x;
  if (j < r) {
    for (int k = 0; k < j; ++k) W[k * LD + j] = 0.0;
    for (int k = j; k < r; ++k) {
      const double v = ((k == j) ? 1.0 : 0.0) - dot4(C + k * LD + j, 1, W + j * LD + j, LD, k - j);
      W[k * LD + j] = v / C[k * LD + k];
    }
  }
  __syncthreads();
}

// M = W^T W (r x r, LDS): with W = C^{-1}, M = (C C^T)^{-1}.
__device__ void bwtw(const double* W, int r, double* M) {
  for (int e = threadIdx.x; e < r * r; e += NT) {
    const int a = e / r, b = e % r;
    const int k0 = a > b ? a : b;
    M[a * LD + b] = dot4(W + k0 * LD + a, LD, W + k0 * LD + b, LD, r - k0);
  }
  __syncthreads();
}

// X = B W (trans = 0) or X = B W^T (trans = 1) with W r x r in LDS; B is
// m x r FP64 (global, staged through LDS TR rows at a time), X has element
// type TO.  One output element per thread and step, r products each.
template <typename TO>
__device__ void bapply(const double* __restrict__ B, int64_t m, int r, const double* W,
                       int trans, TO* __restrict__ X, double* tile) {
  const int si = trans ? LD : 1, sl = trans ? 1 : LD;
  for (int64_t i0 = 0; i0 < m; i0 += TR) {
    const int rows = (int)((m - i0) < TR ? (m - i0) : TR);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * r; e += NT) tile[e] = B[i0 * r + e];
    __syncthreads();
    for (int e = threadIdx.x; e < rows * r; e += NT) {
      const int ii = e / r, k = e - ii * r;
      X[i0 * r + e] = Store<TO>::cvt(dot4(tile + ii * r, 1, W + k * si, sl, r));
    }
  }
  __syncthreads();
}

template <typename TQ>
__global__ void __launch_bounds__(NT) k_mode_step(StepArgs a) {
  __shared__ double A1[64 * LD];
  __shared__ double A2[64 * LD];
  __shared__ double W[64 * LD];
  __shared__ double tile[TR * 64];
  __shared__ double red[NT];
  __shared__ double dmax;
  __shared__ int flag;
  const int r = a.r;
  const int64_t m = a.m;
  const double* src = a.Qin;    // PREP source unless SOLVE or QR runs

  if (a.ops & STEP_SOLVE) {
    for (int e = threadIdx.x; e < r * r; e += NT) A1[(e / r) * LD + e % r] = a.GV[e];
    for (int e = threadIdx.x; e < r * r; e += NT) A2[(e / r) * LD + e % r] = a.Cq[e];
    __syncthreads();
    if (bchol(A1, r, &flag, &dmax)) {
      if (threadIdx.x == 0) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    binv(A1, r, W);
    // tr(Gq^{-1} G_V) = ||Cq^{-1} D||_F^2 with Gq = Cq Cq^T, G_V = D D^T:
    // thread `col` solves Cq z = D[:, col] in place in column col of A1
    // (D is lower, so z vanishes above the diagonal)
    double s = 0.0;
    const int col = threadIdx.x;
    if (col < r) {
      for (int k = col; k < r; ++k) {
        double v = A1[k * LD + col] - dot4(A2 + k * LD + col, 1, A1 + col * LD + col, LD, k - col);
        v /= A2[k * LD + k];
        A1[k * LD + col] = v;
        s += v * v;
      }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double e = 0.0;
      for (int t = 0; t < r; ++t) e += red[t];
      a.res2[0] = a.rsum ? a.rsum[0] : (a.norm2 - e);
      a.res2[1] = e;
    }
    // L_{k+1} = L_acc (D D^T)^{-1}
    bwtw(W, r, A1);
    bapply<double>(a.Lacc, m, r, A1, 0, a.Lnext, tile);
    src = a.Lnext;
  }

  if (a.ops & STEP_QR) {
    // CholeskyQR2: Q1 = L C1^{-T}, Q = Q1 C2^{-T}
    bgram<double>(a.Qin, m, r, A1, tile);
    if (bchol(A1, r, &flag, &dmax)) {
      if (threadIdx.x == 0) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    binv(A1, r, W);
    bapply<double>(a.Qin, m, r, W, 1, a.Q1, tile);
    bgram<double>(a.Q1, m, r, A1, tile);
    if (bchol(A1, r, &flag, &dmax)) {
      if (threadIdx.x == 0) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    binv(A1, r, W);
    bapply<double>(a.Q1, m, r, W, 1, a.Qout, tile);
    src = a.Qout;
  }

  if ((a.ops & STEP_PREP) && src) {
    int* pst = (a.ops & STEP_PREP_SPECULATIVE) ? a.prep_status : a.status;
    bgram<double>(src, m, r, A1, tile);
    if (bchol(A1, r, &flag, &dmax)) {
      if (threadIdx.x == 0) *pst = TK_ERR_RANK_DEFICIENT;
      return;
    }
    binv(A1, r, W);
    bwtw(W, r, A1);
    TQ* Lq = (TQ*)a.Lq;
    bapply<TQ>(src, m, r, A1, 0, Lq, tile);
    if (a.Lr) {
      TQ* Lr = (TQ*)a.Lr;
      for (int64_t e = threadIdx.x; e < m * r; e += NT) Lr[e] = Store<TQ>::cvt(src[e]);
    }
    bgram<TQ>(Lq, m, r, A2, tile);
    if (bchol(A2, r, &flag, &dmax)) {
      if (threadIdx.x == 0) *pst = TK_ERR_RANK_DEFICIENT;
      return;
    }
    for (int e = threadIdx.x; e < r * r; e += NT) a.Cq[e] = A2[(e / r) * LD + e % r];
  }
}

}  // namespace

void launch_mode_step(const StepArgs& a, int q_dtype, hipStream_t s) {
  if (q_dtype == TK_F64) hipLaunchKernelGGL(k_mode_step<double>, dim3(1), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL(k_mode_step<float>, dim3(1), dim3(NT), 0, s, a);
}

}  // namespace tk
