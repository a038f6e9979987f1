// Singular vectors of a mode unfolding inside an orthonormal basis Q of its dominant
// subspace (Section 3, the optional replacement of the factor step of Algorithm 3.4).
// With C = Q^T A_(n), the left singular vectors of C are the eigenvectors W of the R x R
// FP64 Gram M = C C^T (one streaming pass with L~ = Q produces it), and U^(n) = Q W.
#include <algorithm>

#include "tk_kernels.h"

namespace tk {
namespace {

constexpr int EIG_THREADS = 1024;
constexpr int EIG_LD = 65;           // odd row stride of the LDS matrices
constexpr int EIG_MAX_SWEEPS = 40;

// Cyclic Jacobi on the symmetric r x r matrix M (r <= 64) in one workgroup.  Each round
// rotates rp/2 disjoint index pairs at once (round-robin tournament: slot 0 fixed, the
// other rp - 1 slots shifted by the round; rp = r rounded up to even, and a pair holding
// the padding index is idle), first on the rows, then on the columns of the matrix and
// of the accumulated rotations V.  A pair is rotated when |m_pq| > 2^-53 sqrt(|m_pp m_qq|)
// and |m_pq| > 2^-50 max_i |M_ii| (the rounding level of the whole matrix, below which the
// relative test could ask for more than double precision holds); the sweeps stop after
// one without a rotation.  W (r x r row-major) receives the columns of V in descending
// order of the eigenvalues, each signed so that its entry of largest magnitude (the first
// such) is positive; evals the eigenvalues in that order.
__global__ void __launch_bounds__(EIG_THREADS)
k_sym_eig(const double* __restrict__ M, int r, double* __restrict__ W,
          double* __restrict__ evals, int* __restrict__ status) {
  __shared__ double a[64 * EIG_LD];
  __shared__ double v[64 * EIG_LD];
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ double d[64];
  // rotation flags of three consecutive sweeps: the slot of sweep s + 1 is cleared
  // during sweep s, long after its previous reader (sweep s - 2) has finished
  __shared__ int rot[3];
  const int t = threadIdx.x;
  const int rp = r + (r & 1);
  const int np = rp / 2;
  for (int e = t; e < r * r; e += EIG_THREADS) {
    const int i = e / r, j = e - (e / r) * r;
    a[i * EIG_LD + j] = M[e];
    v[i * EIG_LD + j] = i == j ? 1.0 : 0.0;
  }
  if (t < 3) rot[t] = 0;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < r; ++i) dmax = fmax(dmax, fabs(a[i * EIG_LD + i]));
  const double floor_abs = 0x1p-50 * dmax;
  for (int sweep = 0; sweep < EIG_MAX_SWEEPS; ++sweep) {
    const int cur = sweep % 3;
    if (t == 0) rot[(sweep + 1) % 3] = 0;
    for (int round = 0; round < rp - 1; ++round) {
      if (t < np) {
        const int k0 = t, k1 = rp - 1 - t;
        int p = k0 == 0 ? 0 : 1 + (k0 - 1 + round) % (rp - 1);
        int q = 1 + (k1 - 1 + round) % (rp - 1);
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < r) {
          const double apq = a[p * EIG_LD + q];
          const double app = a[p * EIG_LD + p], aqq = a[q * EIG_LD + q];
          if (fabs(apq) > floor_abs && fabs(apq) > 0x1p-53 * sqrt(fabs(app * aqq))) {
            // the rotation [c s; -s c] that zeroes m_pq (symmetric 2 x 2 Schur step)
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            rot[cur] = 1;
          }
        }
        cs[t] = c; sn[t] = s; pp[t] = p; qq[t] = q;
      }
      __syncthreads();
      for (int e = t; e < np * r; e += EIG_THREADS) {
        const int i = e / r, k = e - (e / r) * r;
        const double s = sn[i];
        if (s != 0.0) {
          const double c = cs[i];
          const int p = pp[i], q = qq[i];
          const double x = a[p * EIG_LD + k], y = a[q * EIG_LD + k];
          a[p * EIG_LD + k] = c * x - s * y;
          a[q * EIG_LD + k] = s * x + c * y;
        }
      }
      __syncthreads();
      for (int e = t; e < np * r; e += EIG_THREADS) {
        const int i = e / r, k = e - (e / r) * r;
        const double s = sn[i];
        if (s != 0.0) {
          const double c = cs[i];
          const int p = pp[i], q = qq[i];
          const double x = a[k * EIG_LD + p], y = a[k * EIG_LD + q];
          a[k * EIG_LD + p] = c * x - s * y;
          a[k * EIG_LD + q] = s * x + c * y;
          const double vx = v[k * EIG_LD + p], vy = v[k * EIG_LD + q];
          v[k * EIG_LD + p] = c * vx - s * vy;
          v[k * EIG_LD + q] = s * vx + c * vy;
        }
      }
      __syncthreads();
    }
    if (!rot[cur]) break;  // every thread reads the same flag after the last barrier
  }
  if (t < r) d[t] = a[t * EIG_LD + t];
  __syncthreads();
  if (t < r) {
    const double di = d[t];
    int rank = 0;
    for (int j = 0; j < r; ++j) rank += (d[j] > di) || (d[j] == di && j < t);
    int kmax = 0;
    double vmax = -1.0;
    for (int k = 0; k < r; ++k) {
      const double x = fabs(v[k * EIG_LD + t]);
      if (x > vmax) { vmax = x; kmax = k; }
    }
    const double sg = v[kmax * EIG_LD + t] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < r; ++k) W[k * r + rank] = sg * v[k * EIG_LD + t];
    evals[rank] = di;
    if (!isfinite(di)) *status = TK_ERR_NONFINITE;
  }
}

// out = Q W: Q m x r and W r x r row-major FP64, out m x r FP64.
__global__ void __launch_bounds__(256)
k_rotate(const double* __restrict__ Q, int64_t m, int r, const double* __restrict__ W,
         double* __restrict__ out) {
  __shared__ double w[64 * 64];
  for (int e = threadIdx.x; e < r * r; e += 256) w[e] = W[e];
  __syncthreads();
  const int64_t n = m * r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / r;
    const int c = (int)(e - i * r);
    const double* q = Q + i * r;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc = fma(q[k], w[k * r + c], acc);
    out[e] = acc;
  }
}

}  // namespace

void launch_sym_eig(const double* M, int r, double* W, double* evals, int* status,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_sym_eig, dim3(1), dim3(EIG_THREADS), 0, s, M, r, W, evals, status);
}

void launch_rotate(const double* Q, int64_t m, int r, const double* W, double* out,
                   hipStream_t s) {
  const int64_t n = m * r;
  const int grid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_rotate, dim3(grid), dim3(256), 0, s, Q, m, r, W, out);
}

}  // namespace tk
