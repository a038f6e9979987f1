// FP64 small dense linear algebra of the ALS mode solve (Algorithm 3.3's
// (L^T L)^{-1} and (R^T R)^{-1}, the reduced QR of Algorithms 3.4/3.5).
// Matrices are tall (m <= a few thousand rows) by r <= 64 columns, row-major.
#include "tk_kernels.h"

namespace tk {

// ---------------------------------------------------------------------------
// Gram G = X^T X (r x r, FP64) of a tall m x r matrix with element type T.
// One workgroup; rows are staged through LDS 32 at a time.
template <typename T>
__global__ void __launch_bounds__(256) k_gram(const T* __restrict__ X, int64_t m,
                                              int r, double* __restrict__ G) {
  __shared__ double tile[32 * 64];
  const int npair = r * (r + 1) / 2;
  double acc[9];
  int pa[9], pb[9];
  int cnt = 0;
  for (int t = threadIdx.x; t < npair && cnt < 9; t += blockDim.x, ++cnt) {
    // pair index t -> (a, b) with a <= b
    int a = 0, rem = t;
    while (rem >= r - a) { rem -= r - a; ++a; }
    pa[cnt] = a;
    pb[cnt] = a + rem;
    acc[cnt] = 0.0;
  }
  for (int64_t i0 = 0; i0 < m; i0 += 32) {
    int rows = (int)((m - i0) < 32 ? (m - i0) : 32);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * r; e += blockDim.x)
      tile[e] = (double)Elem<T>::load(X + i0 * r + e);
    __syncthreads();
    for (int c = 0; c < cnt; ++c) {
      double s = 0.0;
      for (int i = 0; i < rows; ++i) s += tile[i * r + pa[c]] * tile[i * r + pb[c]];
      acc[c] += s;
    }
  }
  for (int c = 0; c < cnt; ++c) {
    G[pa[c] * r + pb[c]] = acc[c];
    G[pb[c] * r + pa[c]] = acc[c];
  }
}

// ---------------------------------------------------------------------------
// In-place Cholesky G = C C^T (lower C) of an r x r SPD matrix in FP64, one
// workgroup.  The Gram is declared singular (Remark 3) when a squared pivot
// C_kk^2 falls to PIVOT_TOL * max_k G_kk or below, or is not finite; then
// *status gets TK_ERR_RANK_DEFICIENT and C is replaced by the identity so
// later kernels stay finite.
__global__ void __launch_bounds__(256) k_chol(double* __restrict__ G, int r,
                                              int* __restrict__ status) {
  __shared__ double a[64 * 65];
  __shared__ double dmax;
  __shared__ int bad;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x)
    a[(e / r) * 65 + (e % r)] = G[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int k = 0; k < r; ++k) mx = fmax(mx, a[k * 65 + k]);
    dmax = mx;
    bad = !(mx > 0.0) || !isfinite(mx);
  }
  __syncthreads();
  for (int k = 0; k < r && !bad; ++k) {
    if (threadIdx.x == 0) {
      double d = a[k * 65 + k];
      if (!(d > PIVOT_TOL * dmax) || !isfinite(d)) bad = 1;
      else a[k * 65 + k] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    double dk = a[k * 65 + k];
    for (int i = k + 1 + threadIdx.x; i < r; i += blockDim.x) a[i * 65 + k] /= dk;
    __syncthreads();
    int n = r - k - 1;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      int i = k + 1 + e / n, j = k + 1 + e % n;
      if (j <= i) a[i * 65 + j] -= a[i * 65 + k] * a[j * 65 + k];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    for (int e = threadIdx.x; e < r * r; e += blockDim.x)
      G[e] = (e / r == e % r) ? 1.0 : 0.0;
    if (threadIdx.x == 0) *status = TK_ERR_RANK_DEFICIENT;
    return;
  }
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    int i = e / r, j = e % r;
    G[e] = (j <= i) ? a[i * 65 + j] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Row-wise solves with a Cholesky factor C (r x r lower, FP64).
//  mode GRAM  : X = B (C C^T)^{-1}  (each row solves C C^T x^T = b^T)
//  mode UPPER : X = B C^{-T}        (each row solves C x^T = b^T)
// B is m x r FP64; X gets element type TO (and optionally an FP64 copy Xd).
template <int RM, typename TO>
__global__ void __launch_bounds__(256) k_row_solve(const double* __restrict__ B,
                                                   int64_t m, int r,
                                                   const double* __restrict__ C,
                                                   int gram, TO* __restrict__ X,
                                                   double* __restrict__ Xd) {
  __shared__ double c[RM * RM];
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) c[(e / r) * RM + e % r] = C[e];
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double y[RM];
#pragma unroll
  for (int k = 0; k < RM; ++k) y[k] = (k < r) ? B[i * r + k] : 0.0;
  // forward: C y = b
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    if (k < r) {
      double s = y[k];
#pragma unroll
      for (int l = 0; l < k; ++l) s -= c[k * RM + l] * y[l];
      y[k] = s / c[k * RM + k];
    }
  }
  if (gram) {
    // backward: C^T x = y
#pragma unroll
    for (int k = RM - 1; k >= 0; --k) {
      if (k < r) {
        double s = y[k];
#pragma unroll
        for (int l = k + 1; l < RM; ++l)
          if (l < r) s -= c[l * RM + k] * y[l];
        y[k] = s / c[k * RM + k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    if (k < r) {
      X[i * r + k] = Store<TO>::cvt(y[k]);
      if (Xd) Xd[i * r + k] = y[k];
    }
  }
}

// ---------------------------------------------------------------------------
// Captured energy tr(Gq^{-1} G_V) = ||Cq^{-1} D||_F^2 with Gq = Cq Cq^T and
// G_V = D D^T (both lower Cholesky factors), then
// res2 = norm2 - energy (trace form), or res2 = explicit_sum when the sweep
// accumulated the residual directly.  One workgroup, r <= 64.
__global__ void __launch_bounds__(64) k_trace_resid(const double* __restrict__ Cq,
                                                    const double* __restrict__ D,
                                                    int r, double norm2,
                                                    const double* __restrict__ explicit_sum,
                                                    double* __restrict__ out) {
  __shared__ double part[64];
  int col = threadIdx.x;
  double s = 0.0;
  if (col < r) {
    double z[64];
    for (int k = 0; k < r; ++k) {
      double v = (k >= col) ? D[k * r + col] : 0.0;
      for (int l = 0; l < k; ++l) v -= Cq[k * r + l] * z[l];
      z[k] = v / Cq[k * r + k];
      s += z[k] * z[k];
    }
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int t = 0; t < 64; ++t) e += part[t];
    out[0] = explicit_sum ? explicit_sum[0] : (norm2 - e);
    out[1] = e;
  }
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of `parts` partial arrays of length n:
// out[e] = sum_{w=0}^{parts-1} in[w*stride + e].  Deterministic.
template <typename T>
__global__ void __launch_bounds__(256) k_reduce_parts(const T* __restrict__ in,
                                                      int parts, int64_t n,
                                                      int64_t stride,
                                                      double* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int w = 0; w < parts; ++w) s += (double)in[(int64_t)w * stride + e];
  out[e] = s;
}

// Identity factor (R_n == I_n) in element type T.
template <typename T>
__global__ void k_identity(T* __restrict__ U, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) U[e] = Store<T>::cvt((e / n == e % n) ? 1.0 : 0.0);
}

// Element-type conversion of an FP64 array.
template <typename T>
__global__ void k_convert(const double* __restrict__ in, int64_t n, T* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = Store<T>::cvt(in[e]);
}

// ---------------------------------------------------------------------------
// host launchers

template <typename T>
void launch_gram(const T* X, int64_t m, int r, double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_gram<T>, dim3(1), dim3(256), 0, s, X, m, r, G);
}
template void launch_gram<double>(const double*, int64_t, int, double*, hipStream_t);
template void launch_gram<float>(const float*, int64_t, int, double*, hipStream_t);
template void launch_gram<bf16_t>(const bf16_t*, int64_t, int, double*, hipStream_t);

void launch_chol(double* G, int r, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, s, G, r, status);
}

template <typename TO>
void launch_row_solve(const double* B, int64_t m, int r, const double* C, int gram,
                      TO* X, double* Xd, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(m, 256));
  if (r <= 16)
    hipLaunchKernelGGL((k_row_solve<16, TO>), grid, dim3(256), 0, s, B, m, r, C, gram, X, Xd);
  else if (r <= 32)
    hipLaunchKernelGGL((k_row_solve<32, TO>), grid, dim3(256), 0, s, B, m, r, C, gram, X, Xd);
  else
    hipLaunchKernelGGL((k_row_solve<64, TO>), grid, dim3(256), 0, s, B, m, r, C, gram, X, Xd);
}
template void launch_row_solve<double>(const double*, int64_t, int, const double*, int,
                                       double*, double*, hipStream_t);
template void launch_row_solve<float>(const double*, int64_t, int, const double*, int,
                                      float*, double*, hipStream_t);
template void launch_row_solve<bf16_t>(const double*, int64_t, int, const double*, int,
                                       bf16_t*, double*, hipStream_t);

void launch_trace_resid(const double* Cq, const double* D, int r, double norm2,
                        const double* explicit_sum, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_resid, dim3(1), dim3(64), 0, s, Cq, D, r, norm2,
                     explicit_sum, out);
}

template <typename T>
void launch_reduce_parts(const T* in, int parts, int64_t n, int64_t stride, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_parts<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     in, parts, n, stride, out);
}
template void launch_reduce_parts<float>(const float*, int, int64_t, int64_t, double*,
                                         hipStream_t);
template void launch_reduce_parts<double>(const double*, int, int64_t, int64_t, double*,
                                          hipStream_t);

template <typename T>
void launch_identity(T* U, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_identity<T>, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s,
                     U, n);
}
template void launch_identity<double>(double*, int64_t, hipStream_t);
template void launch_identity<float>(float*, int64_t, hipStream_t);

template <typename T>
void launch_convert(const double* in, int64_t n, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, in,
                     n, out);
}
template void launch_convert<double>(const double*, int64_t, double*, hipStream_t);
template void launch_convert<float>(const double*, int64_t, float*, hipStream_t);

}  // namespace tk
