// FP64 small linear algebra between two fibre passes of the ALS mode solve
// (Algorithm 3.3), so that a sweep costs one fused pass, one reduction and one
// launch of this kernel:
//   SOLVE  L_{k+1} = L_acc (R_k^T R_k)^{-1} with G_V = R_k^T R_k, and the
//          residual from the trace identity ||B||^2 - tr(Gq^{-1} G_V)
//          (or the explicit sum);
//   QR     reduced QR of a tall matrix by CholeskyQR2 (diag(R_hat) > 0),
//          used for the initial guess (Section 5) and the returned factor;
//   PREP   for the next sweep: L~ = L (L^T L)^{-1} quantised to the compute
//          type (to BF16 precision for BF16 storage, whose sweeps multiply
//          the BF16 tensor by L~ as one BF16 term), the inverse Cholesky
//          factor of the Gram of the quantised L~
//          and, for the explicit residual, L in the compute type.
// Every r x r Gram G is factored by one Gaussian elimination of [G | I]
// without pivoting (G = Lu Dp Lu^T): the pivots Dp give the test of Remark 3
// (pivot at most PIVOT_TOL times the largest diagonal entry: rank
// deficient), the upper part gives the Cholesky factor C = Lu Dp^{1/2} and
// the right block gives W = C^{-1} = Dp^{-1/2} Lu^{-1}, so G^{-1} = W^T W.
// The m x r matrices (row-major FP64 in global memory, m up to a few
// thousand, r <= 64) are streamed through LDS in tiles of rows with several
// tiles in flight; each pass multiplies the tile by an r x r LDS matrix on
// the FP64 matrix cores and accumulates the Gram of the result, so that a
// sweep reads L_acc once and L_{k+1} once.  All sums have a fixed order.
// With a partial buffer and more than one row tile the kernel runs as a
// cooperative grid of G workgroups: workgroup b streams a fixed contiguous
// range of the row tiles (the same range in every pass, so it reads back only
// rows it wrote), writes its Gram partial to the buffer, and after a grid
// barrier every workgroup adds the G partials in workgroup order.  The r x r
// work is repeated in every workgroup on identical values, so all of them
// take the same decisions (the rank test included); workgroup 0 writes the
// scalar and r x r outputs.
#include <math.h>

#include <hip/hip_cooperative_groups.h>

#include "tk_kernels.h"

namespace tk {
namespace {

constexpr int NT = 1024;            // one workgroup of sixteen waves
constexpr int NW = NT / 64;
constexpr int EPT = 4;              // staged elements per thread and tile (TR r <= NT EPT)
constexpr int PF = 2;               // staged tiles in flight
constexpr int POOL = 20224;         // LDS doubles (158 KiB)

typedef double d4 __attribute__((ext_vector_type(4)));
// LDS pointers keep their address space through the (non-inlined) helpers,
// so that their accesses compile to LDS instructions.
typedef __attribute__((address_space(3))) double ldsd;
// Global output pointers (plain global stores, which do not count against
// the LDS wait counter as generic stores do).
template <typename T> using gptr = __attribute__((address_space(1))) T*;

// The helpers below are not inlined, and their arguments arrive in vector
// registers; these re-establish that they are uniform over the workgroup
// (scalar loop control, scalar buffer descriptors).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint64_t u = (uint64_t)x;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  return (T*)uni((int64_t)(uintptr_t)p);
}
__device__ __forceinline__ ldsd* uni(ldsd* p) {
  return (ldsd*)(uintptr_t)(uint32_t)uni((int)(uint32_t)(uintptr_t)p);
}
__device__ __forceinline__ const ldsd* uni(const ldsd* p) { return uni((ldsd*)p); }

// v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// result register v of lane l is D[l / 16 + 4 v][l % 16].
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS row stride of the r x r matrices and the tiles (odd: the strided
// column reads of the matrix-core operands spread over the banks).
__host__ __device__ inline int lds_ld(int r) { return (r & 1) ? r : r + 1; }

// Rows per staged tile: a multiple of 16, at most NT EPT / r and 256, and
// small enough for four r x r matrices and two tiles in POOL.
__host__ __device__ inline int tile_rows(int r) {
  const int ld = lds_ld(r);
  int tr = ((NT * EPT) / r) & ~15;
  if (tr > 256) tr = 256;
  const int fit = ((POOL - 4 * r * ld) / (2 * ld)) & ~15;
  return tr < fit ? tr : fit;     // >= 16 for r <= 64
}

struct Lay {
  int r, ld, tr;
  ldsd *A, *B, *C, *M, *Ti, *To;   // contiguous in this order
};

// tr: rows per staged tile (0: tile_rows(r); else a multiple of 16 below it)
__device__ __forceinline__ Lay make_lay(int r, int tr, ldsd* pool) {
  Lay L;
  L.r = r;
  L.ld = lds_ld(r);
  L.tr = tr ? tr : tile_rows(r);
  const int mat = r * L.ld;
  L.A = pool;
  L.B = L.A + mat;
  L.C = L.B + mat;
  L.M = L.C + mat;
  L.Ti = L.M + mat;
  L.To = L.Ti + L.tr * L.ld;
  return L;
}

// Gaussian elimination without pivoting of [A | B] with B = I, A the SPD
// r x r matrix in LDS (only its upper triangle is read or written).  Step k
// subtracts multiples of row k from the rows below it.  Thread (i, c) keeps
// the entries j = c QN ... c QN + QN - 1 of row i of A and B in registers
// and publishes the row to LDS at the step after which it no longer
// changes, so that a step costs one barrier and one round of LDS reads.  On
// return the upper triangle of A holds U = Dp Lu^T (pivots on the diagonal)
// and B holds Lu^{-1} (unit lower).  Returns true when a pivot fails the
// test of Remark 3 or A has a non-finite or non-positive diagonal; the
// decision is uniform since every thread reads the same values.
template <int QN>
__device__ bool belim_q(ldsd* A, ldsd* B, int r, int ld, double dmax) {
  A = uni(A); B = uni(B); r = uni(r); ld = uni(ld);
  const int tid = threadIdx.x, tpr = NT / r;
  const int i = tid / tpr, c = tid - (tid / tpr) * tpr;
  const bool own = i < r;
  const int ic = own ? i : r - 1;          // clamped row: every load is in range
  int jc[QN];                              // clamped columns
  double ar[QN], br[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int j = c * QN + q;
    jc[q] = j < r ? j : r - 1;
    ar[q] = A[ic * ld + jc[q]];
    br[q] = (j == i) ? 1.0 : 0.0;
    if (own && j < r && i == 0) B[j] = br[q];
  }
  __syncthreads();
  // Row k of A (upper part) and of B (zeros past column k) are published by
  // step k.  The updates below also touch entries left of the diagonal of A
  // (never read again) and entries of B right of column k (B[k][j] = 0
  // there), so no entry needs a mask.
  for (int k = 0; k < r; ++k) {
    const double d = A[k * ld + k];
    const double aki = A[k * ld + ic];
    double ak[QN], bk[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      ak[q] = A[k * ld + jc[q]];
      bk[q] = B[k * ld + jc[q]];
    }
    const double f = (own && i > k) ? aki / d : 0.0;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      ar[q] -= f * ak[q];
      br[q] -= f * bk[q];
    }
    if (own && i == k + 1) {
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int j = c * QN + q;
        if (j < r) {
          if (j >= i) A[i * ld + j] = ar[q];
          B[i * ld + j] = br[q];
        }
      }
    }
    if (!(d > PIVOT_TOL * dmax) || !isfinite(d)) return true;
    __syncthreads();
  }
  return false;
}

__device__ bool belim(ldsd* A, ldsd* B, int r, int ld) {
  A = uni(A); B = uni(B); r = uni(r); ld = uni(ld);
  double dmax = 0.0;
  bool bad = false;
#pragma unroll 8
  for (int k = 0; k < r; ++k) {
    const double d = A[k * ld + k];
    dmax = fmax(dmax, d);
    bad = bad || !isfinite(d);
  }
  if (bad || !(dmax > 0.0)) return true;
  const int tpr = NT / r, qn = (r + tpr - 1) / tpr;
  if (qn <= 1) return belim_q<1>(A, B, r, ld, dmax);
  if (qn <= 2) return belim_q<2>(A, B, r, ld, dmax);
  return belim_q<4>(A, B, r, ld, dmax);      // NT / r >= 16 for r <= 64
}

// B (= Lu^{-1} from belim) -> W = C^{-1} = Dp^{-1/2} Lu^{-1}, zeros above
// the diagonal; Dp is the diagonal of U.
__device__ void bscale(const ldsd* U, ldsd* B, int r, int ld) {
  U = uni(U); B = uni(B); r = uni(r); ld = uni(ld);
  const int tid = threadIdx.x, tpr = NT / r;
  const int i = tid / tpr, c = tid - (tid / tpr) * tpr;
  if (i < r) {
    const double s = 1.0 / sqrt(U[i * ld + i]);
    for (int j = c; j < r; j += tpr) B[i * ld + j] = (j <= i) ? B[i * ld + j] * s : 0.0;
  }
  __syncthreads();
}

// M = W^T W (exactly symmetric) for the lower triangular W: with W = C^{-1},
// M = (C C^T)^{-1}.
__device__ void bwtw(const ldsd* W, int r, int ld, ldsd* M) {
  W = uni(W); M = uni(M); r = uni(r); ld = uni(ld);
  const int tid = threadIdx.x, tpr = NT / r;
  const int a = tid / tpr, c = tid - (tid / tpr) * tpr;
  if (a < r) {
    for (int b = a + c; b < r; b += tpr) {
      double s0 = 0.0, s1 = 0.0;
      int k = b;
      for (; k + 1 < r; k += 2) {
        s0 += W[k * ld + a] * W[k * ld + b];
        s1 += W[(k + 1) * ld + a] * W[(k + 1) * ld + b];
      }
      if (k < r) s0 += W[k * ld + a] * W[k * ld + b];
      const double s = s0 + s1;
      M[a * ld + b] = s;
      M[b * ld + a] = s;
    }
  }
  __syncthreads();
}

// One pass over the m x r FP64 matrix S (global): per staged tile of rows,
//   Y = S_tile M (wsel = W_M) or S_tile B^T (wsel = W_BT) on the FP64
//       matrix cores, with M, B the LDS matrices of the layout; Y = S_tile
//       for wsel = W_NONE;
//   Out = Y in type TO (when given), Out2 = S_tile in type TO (when given);
//   A = Yq^T Yq with Yq = Y rounded to TO (when gram; the LDS matrix A,
//       written exactly symmetric at the end).
// PF tiles are loaded ahead into registers.  Wave w computes the output
// tiles w, w + NW, ... of each staged tile.  For the Gram, wave w owns the
// upper 16 x 16 block w % nb and the K steps w / nb, w / nb + S, ... of every
// tile (S = NW / nb splits); the S partial blocks are added in a fixed order
// at the end.
enum { W_NONE = 0, W_M = 1, W_BT = 2 };

// With rbf16 the product written to Outp (and kept for the Gram) is rounded to
// BF16 precision (round to nearest even) before it is stored in TO.
// gp: the Gram partials of a cooperative grid ([G][nb][256], null for one
// workgroup).
template <typename TO>
__device__ __forceinline__ void stream_pass(const Lay& L, const double* __restrict__ S, int64_t m,
                                            int wsel, TO* Outp, TO* Out2p, bool gram,
                                            double* gp, bool rbf16 = false) {
  const int r = L.r, ld = L.ld, tr = L.tr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nt = (r + 15) >> 4, nb = nt * (nt + 1) / 2;
  const int nk = (r + 3) >> 2;             // K steps of the product (<= 16)
  const int cap = tr * r;                  // elements of a full tile
  const int64_t ntile = (m + tr - 1) / tr;
  // this workgroup's row tiles [t_lo, t_hi)
  const int64_t nwg = gridDim.x, wg = blockIdx.x;
  const int64_t t_lo = ntile * wg / nwg, t_hi = ntile * (wg + 1) / nwg;
  const bool apply = wsel != W_NONE;
  const int trans = wsel == W_BT;
  const ldsd* Wm = (wsel == W_BT) ? L.B : L.M;
  ldsd* Ti = L.Ti;
  ldsd* To = L.To;
  gptr<TO> Out = (gptr<TO>)Outp;
  gptr<TO> Out2 = (gptr<TO>)Out2p;

  // LDS offsets of this thread's staged elements (the same for every tile)
  int off[EPT];
  {
    int row = tid / r, col = tid - (tid / r) * r;
    const int dr = NT / r, dc = NT - (NT / r) * r;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      off[j] = row * ld + col;
      row += dr;
      col += dc;
      if (col >= r) { col -= r; ++row; }
    }
  }
  // Gram block and K split of this wave; the partial blocks are gathered at
  // the end in C, M and the tiles (contiguous, and free by then)
  const int part_room = (2 * r * ld + 2 * tr * ld) / 256;
  int nsplit = NW / nb;
  if (nsplit * nb > part_room) nsplit = part_room / nb;
  const bool gact = gram && wv < nb * nsplit;
  const int blk = wv % nb, ks = wv / nb;
  int ta = 0, tb = 0;
  for (int p = 0, x = 0; x < nt; ++x)
    for (int y = x; y < nt; ++y, ++p)
      if (p == blk) { ta = x; tb = y; }
  const int ca = 16 * ta + lr, cb = 16 * tb + lr;
  const int cac = ca < r ? ca : r - 1, cbc = cb < r ? cb : r - 1;
  d4 gacc = {0.0, 0.0, 0.0, 0.0};

  // Tile t is loaded through a buffer resource spanning exactly its rows:
  // the loads past its end return zero (the whole offset is in the
  // range-checked vector offset).
  double buf[PF][EPT];
  auto load = [&](double* dst, int64_t t) {
    const int64_t rem = (m - t * tr) * (int64_t)r;
    const int cnt = (int)(rem < (int64_t)cap ? rem : (int64_t)cap);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(S + t * tr * (int64_t)r), (short)0, cnt * 8, 0x00020000);
#pragma unroll
    for (int j = 0; j < EPT; ++j)
      dst[j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (j * NT + tid) * 8, 0, 0));
  };
#pragma unroll
  for (int b = 0; b < PF; ++b)
    if (t_lo + b < t_hi) load(buf[b], t_lo + b);

  for (int64_t t0 = t_lo; t0 < t_hi; t0 += PF) {
#pragma unroll
    for (int b = 0; b < PF; ++b) {
      const int64_t t = t0 + b;
      if (t < t_hi) {
        const int64_t i0 = t * tr;
        const int rows = (int)((m - i0) < tr ? (m - i0) : tr);
        const int cnt = rows * r;
        __syncthreads();
        // rows past the end of the matrix are staged as zeros (the loads past
        // the end of the tile return zero)
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (j * NT + tid < cap) Ti[off[j]] = buf[b][j];
        if (t + PF < t_hi) load(buf[b], t + PF);
        __syncthreads();
        if (Out2p) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) {
            const int e = j * NT + tid;
            if (e < cnt) Out2[i0 * r + e] = Store<TO>::cvt(Ti[off[j]]);
          }
        }
        const ldsd* Y = Ti;
        if (apply) {
          const int nrt = (rows + 15) >> 4;
          for (int ot = wv; ot < nrt * nt; ot += NW) {
            const int rt = ot / nt, ct = ot - (ot / nt) * nt;
            const int arow = 16 * rt + lr, col = 16 * ct + lr;
            const int colc = col < r ? col : r - 1;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              double av[4], bv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int kk = 4 * h + u;
                if (kk < nk) {
                  const int k = 4 * kk + lk;
                  const int kc = k < r ? k : r - 1;
                  const double xa = Ti[arow * ld + kc];
                  const double xb = Wm[(trans ? colc : kc) * ld + (trans ? kc : colc)];
                  av[u] = (k < r) ? xa : 0.0;
                  bv[u] = (k < r && col < r) ? xb : 0.0;
                }
              }
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (4 * h + u < nk) acc = mfma64(av[u], bv[u], acc);
            }
            if (col < r) {
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int orow = 16 * rt + lk + 4 * v;
                TO q = Store<TO>::cvt(acc[v]);
                if (rbf16) q = (TO)bf16_to_f32(f32_to_bf16((float)q));
                To[orow * ld + col] = (double)q;
                if (Outp && orow < rows) Out[(i0 + orow) * r + col] = q;
              }
            }
          }
          Y = To;
          if (gram) __syncthreads();
        }
        if (gact) {
          // rows past `rows` (up to the next multiple of 16) are zero in Ti,
          // and so in To
          const int nkr = (rows + 3) >> 2;
          for (int k0 = ks; k0 < nkr; k0 += 4 * nsplit) {
            double xa[4], xb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int kk = k0 + u * nsplit;
              const int i = 4 * (kk < nkr ? kk : 0) + lk;
              const double ya = Y[i * ld + cac];
              const double yb = Y[i * ld + cbc];
              xa[u] = (kk < nkr && ca < r) ? ya : 0.0;
              xb[u] = (kk < nkr && cb < r) ? yb : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) gacc = mfma64(xa[u], xb[u], gacc);
          }
        }
      }
    }
  }
  if (gram) {
    __syncthreads();
    ldsd* part = L.C;                      // [nsplit][nb][16 x 16]
    if (gact) {
#pragma unroll
      for (int v = 0; v < 4; ++v) part[(ks * nb + blk) * 256 + (lk + 4 * v) * 16 + lr] = gacc[v];
    }
    __syncthreads();
    if (gp) {
      // this workgroup's partial to the buffer, then the grid's in order
      for (int e = tid; e < nb * 256; e += NT) {
        double sum = 0.0;
        for (int q = 0; q < nsplit; ++q) sum += part[q * nb * 256 + e];
        gp[wg * nb * 256 + e] = sum;
      }
      cooperative_groups::this_grid().sync();
    }
    ldsd* G = L.A;
    for (int e = tid; e < nb * 256; e += NT) {
      const int bq = e >> 8, rc = e & 255, row = rc >> 4, col = rc & 15;
      double sum = 0.0;
      if (gp) {
#pragma unroll 8
        for (int64_t q = 0; q < nwg; ++q) sum += gp[q * nb * 256 + e];
      } else {
        for (int q = 0; q < nsplit; ++q) sum += part[(q * nb + bq) * 256 + rc];
      }
      int xa = 0, xb = 0;
      for (int p = 0, x = 0; x < nt; ++x)
        for (int y = x; y < nt; ++y, ++p)
          if (p == bq) { xa = x; xb = y; }
      const int ga = 16 * xa + row, gb = 16 * xb + col;
      if (ga < r && gb < r && (xa < xb || row <= col)) {
        G[ga * ld + gb] = sum;
        G[gb * ld + ga] = sum;
      }
    }
  }
  __syncthreads();
}

template <typename TQ>
__global__ __launch_bounds__(NT, 1) void k_mode_step(StepArgs a) {
  __shared__ double pool[POOL];
  __shared__ double red[NW];
  const Lay L = make_lay(a.r, a.tr, (ldsd*)pool);
  const int r = a.r, ld = L.ld, tid = threadIdx.x;
  const int64_t m = a.m;
  const int tpr = NT / r;
  const int ri = tid / tpr, rc = tid - (tid / tpr) * tpr;
  const double* src = a.Qin;    // PREP source unless SOLVE or QR runs
  bool have_gram = false;       // L.A holds the Gram of src
  const bool prep = (a.ops & STEP_PREP) != 0;
  const bool lead = tid == 0 && blockIdx.x == 0;   // writes the scalar outputs
  double* gp = gridDim.x > 1 ? a.gpart : nullptr;

  if (a.ops & STEP_SOLVE) {
    if (ri < r)
      for (int j = rc; j < r; j += tpr) {
        L.A[ri * ld + j] = a.GV[ri * r + j];
        L.C[ri * ld + j] = a.Wq[ri * r + j];
      }
    __syncthreads();
    if (belim(L.A, L.B, r, ld)) {
      if (lead) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    // tr(Gq^{-1} G_V) = ||Wq D||_F^2 with Wq = Cq^{-1} (Gq = Cq Cq^T) and
    // D the Cholesky factor of G_V: D[l][j] = U[j][l] / sqrt(U[j][j]).  Both
    // are lower triangular, so (Wq D)[i][j] sums over j <= l <= i.
    double e2 = 0.0;
    if (ri < r)
      for (int j = rc; j <= ri; j += tpr) {
        double z = 0.0;
        for (int l = j; l <= ri; ++l) z += L.C[ri * ld + l] * L.A[j * ld + l];
        z /= sqrt(L.A[j * ld + j]);
        e2 += z * z;
      }
    // fixed-order sum: butterfly within each wave, then over the waves
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e2 += __shfl_xor(e2, o);
    if ((tid & 63) == 0) red[tid >> 6] = e2;
    __syncthreads();
    if (lead) {
      double e = 0.0;
      for (int w = 0; w < NW; ++w) e += red[w];
      a.res2[0] = a.rsum ? a.rsum[0] : ((a.norm2p ? a.norm2p[0] : a.norm2) - e);
      a.res2[1] = e;
    }
    // L_{k+1} = L_acc G_V^{-1}, with the Gram of L_{k+1} for PREP
    bscale(L.A, L.B, r, ld);
    bwtw(L.B, r, ld, L.M);
    stream_pass<double>(L, a.Lacc, m, W_M, a.Lnext, nullptr, prep, gp);
    have_gram = prep;
    src = a.Lnext;
  }

  if (a.ops & STEP_QR) {
    // CholeskyQR2: Q1 = L C1^{-T}, Q = Q1 C2^{-T}
    stream_pass<double>(L, a.Qin, m, W_NONE, nullptr, nullptr, true, gp);
    if (belim(L.A, L.B, r, ld)) {
      if (lead) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    bscale(L.A, L.B, r, ld);
    stream_pass<double>(L, a.Qin, m, W_BT, a.Q1, nullptr, true, gp);
    if (belim(L.A, L.B, r, ld)) {
      if (lead) *a.status = TK_ERR_RANK_DEFICIENT;
      return;
    }
    bscale(L.A, L.B, r, ld);
    stream_pass<double>(L, a.Q1, m, W_BT, a.Qout, nullptr, prep, gp);
    have_gram = prep;
    src = a.Qout;
  }

  if (prep && src) {
    int* pst = (a.ops & STEP_PREP_SPECULATIVE) ? a.prep_status : a.status;
    if (!have_gram) stream_pass<double>(L, src, m, W_NONE, nullptr, nullptr, true, gp);
    if (belim(L.A, L.B, r, ld)) {
      if (lead) *pst = TK_ERR_RANK_DEFICIENT;
      return;
    }
    bscale(L.A, L.B, r, ld);
    bwtw(L.B, r, ld, L.M);
    // L~ = L (L^T L)^{-1} in TQ (BF16 precision with lq_bf16), with the Gram
    // of the quantised L~
    stream_pass<TQ>(L, src, m, W_M, (TQ*)a.Lq, (TQ*)a.Lr, true, gp, a.lq_bf16 != 0);
    if (belim(L.A, L.B, r, ld)) {
      if (lead) *pst = TK_ERR_RANK_DEFICIENT;
      return;
    }
    bscale(L.A, L.B, r, ld);
    if (ri < r && blockIdx.x == 0)
      for (int j = rc; j < r; j += tpr) a.Wq[ri * r + j] = L.B[ri * ld + j];
  }
}

}  // namespace

constexpr int GRID_MAX = 32;      // workgroups of a cooperative mode step
constexpr int GRID_ROWS = 64;     // rows per workgroup it aims at
// A cooperative launch leaves about 11 us idle before and after the kernel on
// this runtime (measured in kernel traces; plain launches follow each other
// without a gap), so the grid is used only where the m x r passes take a few
// hundred microseconds on one workgroup: m r^2 at least GRID_MIN_WORK (the
// 1024 x 48 mode step passes take about 230 us there, 200 x 20 about 40 us).
constexpr int64_t GRID_MIN_WORK = 1000000;

void launch_mode_step(const StepArgs& a, int q_dtype, hipStream_t s) {
  // with a partial buffer: one row tile of about GRID_ROWS rows per
  // workgroup (at most GRID_MAX workgroups, partials within the buffer)
  StepArgs arg = a;
  arg.tr = 0;
  int g = 1;
  if (a.gpart && a.m > GRID_ROWS && a.m * a.r * a.r >= GRID_MIN_WORK) {
    const int nt = (a.r + 15) / 16, nb = nt * (nt + 1) / 2;
    const int trmax = tile_rows(a.r);
    int64_t gm = ceil_div(a.m, GRID_ROWS);
    if (gm > GRID_MAX) gm = GRID_MAX;
    if (gm * nb * 256 > a.gpart_cap) gm = a.gpart_cap / (nb * 256);
    if (gm > 1) {
      int tr = (int)(ceil_div(ceil_div(a.m, gm), 16) * 16);
      if (tr > trmax) tr = trmax;
      const int64_t ntile = ceil_div(a.m, tr);
      g = (int)(ntile < gm ? ntile : gm);
      if (g > 1) arg.tr = tr;
      else g = 1;
    }
  }
  const void* fn = q_dtype == TK_F64 ? (const void*)k_mode_step<double>
                                     : (const void*)k_mode_step<float>;
  void* args[] = {&arg};
  if (g > 1) {
    if (hipLaunchCooperativeKernel(fn, dim3(g), dim3(NT), args, 0, s) == hipSuccess) return;
    // no cooperative launch: the one-workgroup form computes the same step
    (void)hipGetLastError();
    arg.tr = 0;
  }
  (void)hipLaunchKernel(fn, dim3(1), dim3(NT), args, 0, s);
}

}  // namespace tk
