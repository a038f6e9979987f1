// Fused ALS sweep on the gfx950 matrix cores.
//
// One sweep of Algorithm 3.3 on the mode-n view [P, I, Q] reads every fibre
// a_j (a column of A_(n)) from HBM once and uses it twice (row-wise update
// rule of Section 3):
//    v_j   = Lq^T a_j                (row j of R_k; never written out)
//    G_V  += v_j v_j^T               (R_k^T R_k, flushed to FP64 per tile)
//    L_acc += a_j v_j^T              (A_(n) R_k, per-workgroup partial)
// and optionally accumulates the explicit residual sum_j ||a_j - L v_j||^2.
// The init variant replaces v_j by row j of the Section 5 sketch S.
//
// Work layout: a workgroup of 4 waves walks 64-fibre tiles (persistent grid).
// The tile X (I x 64, FP32 in LDS) is filled from registers that were
// prefetched during the previous tile.  Wave w owns mode rows
// [w*IW, (w+1)*IW), IW = ceil(I/4):
//   R-update  v_mfma_f32_4x4x1f32, 16 blocks, lane = fibre, 4 r per block:
//             K-split over the wave's rows, partials summed through LDS;
//   L-update  same instruction, lane = mode row, 4 r per block, one fibre
//             per instruction;
//   Gram      one instruction per fibre covers 16 upper-triangle 4x4 blocks.
// All reductions are in a fixed order (deterministic, no atomics).
#include "tk_kernels.h"

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 256;      // threads per workgroup
constexpr int TJ = 64;       // fibres per tile
constexpr int XLD = 65;      // LDS row stride of the X tile
constexpr int NWG = 256;     // persistent workgroups (one per CU)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ float to_f(T x);
template <> __device__ __forceinline__ float to_f<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f<bf16_t>(bf16_t x) { return bf16_to_f32(x); }

struct Lds {
  int xs, lq, lr, vp, vf, total;  // offsets in floats
};

__host__ __device__ inline Lds lds_layout(int I, int RG, int mode) {
  const int IW = (I + 3) / 4;
  const int RP = 4 * RG;
  Lds l;
  l.xs = 0;
  l.lq = l.xs + 4 * IW * XLD;
  l.lr = l.lq + (mode != 2 ? I * RP : 0);
  l.vp = l.lr + (mode == 1 ? 4 * IW * RP : 0);
  l.vf = l.vp + (mode != 2 ? 4 * TJ * (RP + 1) : 0);
  l.total = l.vf + TJ * (RP + 1);
  return l;
}

// Prefetch of one tile into registers: a fixed number of unconditional
// loads per lane whose row / fibre indices are clamped into the tensor, so
// the compiler issues them back to back (duplicates of the clamped row hit
// the caches; only the LDS stores are guarded).
//  LAYOUT 0 (Q > 1): wave w loads rows ii = 4k + w (k < 64) of fibre
//          j0 + lane (coalesced along q); lanes past the last fibre read
//          fibre j0 and are zeroed in the stash.
//  LAYOUT 1 (Q == 1): wave w loads fibres jj = w + 4k (k < 16), rows
//          lane + 64c (c < 4) of each contiguous fibre.
template <typename T, int LAYOUT>
__device__ __forceinline__ void prefetch(const T* __restrict__ X, const View& v, int64_t j0,
                                         int lane, int w, T* pf, bool& ok) {
  const int64_t J = v.J();
  const int I = (int)v.I;
  if (LAYOUT == 0) {
    const int64_t j = j0 + lane;
    ok = j < J;
    const int64_t base = v.fibre_base(ok ? j : j0);
    const T* b = X + base;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const int ii = min(4 * k + w, I - 1);
      pf[k] = b[(int64_t)ii * v.Q];
    }
  } else {
    ok = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int64_t j = min(j0 + w + 4 * k, J - 1);
      const T* b = X + j * I;
#pragma unroll
      for (int c = 0; c < 4; ++c) pf[4 * k + c] = b[min(lane + 64 * c, I - 1)];
    }
  }
}

template <typename T, int LAYOUT>
__device__ __forceinline__ void stash(const View& v, int64_t j0, int lane, int w, const T* pf,
                                      bool ok, float* Xs) {
  const int I = (int)v.I;
  if (LAYOUT == 0) {
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const int ii = 4 * k + w;
      if (ii < I) Xs[ii * XLD + lane] = ok ? to_f<T>(pf[k]) : 0.0f;
    }
  } else {
    const int64_t J = v.J();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const bool fok = j0 + w + 4 * k < J;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int ii = lane + 64 * c;
        if (ii < I) Xs[ii * XLD + w + 4 * k] = fok ? to_f<T>(pf[4 * k + c]) : 0.0f;
      }
    }
  }
}

// MODE 0: sweep; 1: sweep + explicit residual; 2: init (sketch, no Gram).
template <typename T, int RG, int MODE, int LAYOUT>
__global__ void __launch_bounds__(NT, 1) k_fused(FusedArgs a) {
  extern __shared__ float smem[];
  constexpr int RP = 4 * RG;
  constexpr int VS = RP + 1;                 // V row stride (odd: no conflicts)
  constexpr int NP = RG * (RG + 1) / 2;      // upper-triangle 4x4 blocks
  constexpr int NM = (NP + 15) / 16;         // Gram instructions per fibre
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63, l4 = lane & 3;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int IW = (I + 3) / 4;
  const int i0 = w * IW;
  const int iend = (i0 + IW < I) ? i0 + IW : I;
  const int IWw = iend > i0 ? iend - i0 : 0;
  const Lds L = lds_layout(I, RG, MODE);
  float* Xs = smem + L.xs;
  float* Lq = smem + L.lq;
  float* Lr = smem + L.lr;
  float* Vp = smem + L.vp;
  float* Vf = smem + L.vf;

  // ---- once per kernel: zero the X tile (pad rows stay zero), load Lq/Lr
  for (int e = threadIdx.x; e < 4 * IW * XLD; e += NT) Xs[e] = 0.0f;
  if (MODE != 2) {
    // Lq[i][c*RG + g] = L~(i, 4g + c): a lane reads its RG values contiguously
    for (int e = threadIdx.x; e < I * RP; e += NT) {
      const int i = e / RP, r = e % RP;
      Lq[i * RP + (r & 3) * RG + (r >> 2)] = (r < R) ? a.Lq[i * R + r] : 0.0f;
    }
  }
  if (MODE == 1) {
    for (int e = threadIdx.x; e < 4 * IW * RP; e += NT) {
      const int i = e / RP, r = e % RP;
      Lr[e] = (i < I && r < R) ? -a.Lr[i * R + r] : 0.0f;
    }
  }

  f4 lacc[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) lacc[g] = f4{0, 0, 0, 0};
  double gd[NM][4];
  f4 gacc[NM];
  int gbi[NM], gbj[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    gacc[m] = f4{0, 0, 0, 0};
    gd[m][0] = gd[m][1] = gd[m][2] = gd[m][3] = 0.0;
    int p = 16 * m + (lane >> 2), bi = 0;
    if (p >= NP) p = 0;
    while (p >= RG - bi) { p -= RG - bi; ++bi; }
    gbi[m] = bi;
    gbj[m] = bi + p;
  }
  double rsum = 0.0;

  const T* X = (const T*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  const int nwg = gridDim.x;
  T pf[64];
  bool pf_ok = false;
  int64_t tile = blockIdx.x;
  if (tile < ntiles) prefetch<T, LAYOUT>(X, v, tile * TJ, lane, w, pf, pf_ok);

  for (; tile < ntiles; tile += nwg) {
    const int64_t j0 = tile * TJ;
    __syncthreads();
    stash<T, LAYOUT>(v, j0, lane, w, pf, pf_ok, Xs);
    __syncthreads();
    if (tile + nwg < ntiles) prefetch<T, LAYOUT>(X, v, (tile + nwg) * TJ, lane, w, pf, pf_ok);

    if (MODE != 2) {
      // R-update partial over this wave's rows: V_w[j][r], lane = fibre j.
      // Four rows per step; the LDS operands of step s+1 are read before
      // the MFMAs of step s.  Rows past the wave's range get a zero B.
      f4 vacc[RG];
#pragma unroll
      for (int g = 0; g < RG; ++g) vacc[g] = f4{0, 0, 0, 0};
      float bc[4], lc[4][RG], bn[4], ln[4][RG];
      auto rows4 = [&](int k, float (&b)[4], float (&l)[4][RG]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k + u;
          const int i = i0 + (kk < IWw ? kk : 0);
          b[u] = (kk < IWw) ? Xs[i * XLD + lane] : 0.0f;
          const float* lq = Lq + i * RP + l4 * RG;
#pragma unroll
          for (int g = 0; g < RG; ++g) l[u][g] = lq[g];
        }
      };
      rows4(0, bc, lc);
      for (int k = 0; k < IWw; k += 4) {
        rows4(k + 4, bn, ln);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int g = 0; g < RG; ++g) vacc[g] = mfma4(lc[u][g], bc[u], vacc[g]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          bc[u] = bn[u];
#pragma unroll
          for (int g = 0; g < RG; ++g) lc[u][g] = ln[u][g];
        }
      }
      float* vp = Vp + (w * TJ + lane) * VS;
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) vp[4 * g + q] = vacc[g][q];
      __syncthreads();
      // fixed-order sum of the four partials for fibres 16w..16w+15
#pragma unroll
      for (int k = 0; k < RG; ++k) {
        const int e = lane + 64 * k;
        const int jl = 16 * w + e / RP, r = e % RP;
        float s = Vp[(0 * TJ + jl) * VS + r];
        s += Vp[(1 * TJ + jl) * VS + r];
        s += Vp[(2 * TJ + jl) * VS + r];
        s += Vp[(3 * TJ + jl) * VS + r];
        Vf[jl * VS + (r & 3) * RG + (r >> 2)] = s;
      }
    } else {
      // init: V = the Section 5 sketch rows of this tile
#pragma unroll
      for (int k = 0; k < RG; ++k) {
        const int e = lane + 64 * k;
        const int jl = 16 * w + e / RP, r = e % RP;
        const int64_t j = j0 + jl;
        float s = 0.0f;
        if (j < J && r < R)
          s = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        Vf[jl * VS + (r & 3) * RG + (r >> 2)] = s;
      }
    }
    __syncthreads();

    // L-update: L_acc[i0 + lane-row][r] += X[i][j] V[j][r], lane = mode row.
    // Operands of four fibres are read before their MFMAs.
#pragma unroll
    for (int jb = 0; jb < TJ; jb += 4) {
      float x[4], vv[4][RG];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = Xs[(i0 + lane) * XLD + jb + u];
        const float* vf = Vf + (jb + u) * VS + l4 * RG;
#pragma unroll
        for (int g = 0; g < RG; ++g) vv[u][g] = vf[g];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int g = 0; g < RG; ++g) lacc[g] = mfma4(x[u], vv[u][g], lacc[g]);
    }

    if (MODE != 2) {
      // Gram of this wave's 16 fibres, FP32 within the tile, FP64 across.
#pragma unroll
      for (int jb = 16 * w; jb < 16 * w + 16; jb += 8) {
        float ga[8][NM], gb[8][NM];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float* vf = Vf + (jb + u) * VS + l4 * RG;
#pragma unroll
          for (int m = 0; m < NM; ++m) { ga[u][m] = vf[gbi[m]]; gb[u][m] = vf[gbj[m]]; }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int m = 0; m < NM; ++m) gacc[m] = mfma4(ga[u][m], gb[u][m], gacc[m]);
      }
#pragma unroll
      for (int m = 0; m < NM; ++m) {
#pragma unroll
        for (int q = 0; q < 4; ++q) gd[m][q] += (double)gacc[m][q];
        gacc[m] = f4{0, 0, 0, 0};
      }
    }

    if (MODE == 1) {
      // explicit residual: a_j - L v_j for this wave's rows, lane = fibre.
      float vj[RP];
      const float* vr = Vf + lane * VS;
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int c = 0; c < 4; ++c) vj[4 * g + c] = vr[c * RG + g];
      for (int t = 0; t < IWw; t += 4) {
        const int ib = i0 + t;
        f4 c4;
#pragma unroll
        for (int q = 0; q < 4; ++q) c4[q] = (t + q < IWw) ? Xs[(ib + q) * XLD + lane] : 0.0f;
        const float* lr = Lr + (ib + l4) * RP;
#pragma unroll
        for (int r = 0; r < RP; ++r) c4 = mfma4(lr[r], vj[r], c4);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (t + q < IWw) rsum += (double)c4[q] * (double)c4[q];
      }
    }
  }

  // ---- per-workgroup outputs
  const int wg = blockIdx.x;
  float* lp = a.lacc_parts + (int64_t)wg * I * R;
#pragma unroll
  for (int g = 0; g < RG; ++g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 4 * (lane >> 2) + q;
      const int r = 4 * g + l4;
      if (i < iend && r < R) lp[i * R + r] = lacc[g][q];
    }
  }
  if (MODE != 2) {
    // the upper-triangle 4x4 blocks and their mirrors cover every entry
    double* gp = a.gv_parts + (int64_t)(wg * 4 + w) * R * R;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      if (16 * m + (lane >> 2) >= NP) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 4 * gbi[m] + q, col = 4 * gbj[m] + l4;
        if (row < R && col < R) {
          gp[row * R + col] = gd[m][q];
          gp[col * R + row] = gd[m][q];
        }
      }
    }
  }
  if (MODE == 1) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rsum += __shfl_xor(rsum, off, 64);
    if (lane == 0) a.resid_parts[wg * 4 + w] = rsum;
  }
}

template <typename T, int RG, int MODE>
void launch_mode(const FusedArgs& a, int nwg, size_t bytes, hipStream_t s) {
  if (a.v.Q != 1) {
    hipFuncSetAttribute((const void*)k_fused<T, RG, MODE, 0>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused<T, RG, MODE, 0>), dim3(nwg), dim3(NT), bytes, s, a);
  } else {
    hipFuncSetAttribute((const void*)k_fused<T, RG, MODE, 1>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused<T, RG, MODE, 1>), dim3(nwg), dim3(NT), bytes, s, a);
  }
}

template <typename T, int RG>
int launch_rg(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  const Lds L = lds_layout((int)a.v.I, RG, mode);
  const size_t bytes = (size_t)L.total * 4;
  if (mode == 0) launch_mode<T, RG, 0>(a, nwg, bytes, s);
  else if (mode == 1) launch_mode<T, RG, 1>(a, nwg, bytes, s);
  else launch_mode<T, RG, 2>(a, nwg, bytes, s);
  return nwg;
}

// R is padded up to 4*RG with RG from a fixed list (zero columns).
inline int rg_of(int R) {
  const int g = (R + 3) / 4;
  if (g <= 6) return g;
  if (g <= 8) return 8;
  if (g <= 10) return 10;
  return 12;
}

template <typename T>
int launch_t(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  switch (rg_of(a.R)) {
    case 1: return launch_rg<T, 1>(a, mode, nwg, s);
    case 2: return launch_rg<T, 2>(a, mode, nwg, s);
    case 3: return launch_rg<T, 3>(a, mode, nwg, s);
    case 4: return launch_rg<T, 4>(a, mode, nwg, s);
    case 5: return launch_rg<T, 5>(a, mode, nwg, s);
    case 6: return launch_rg<T, 6>(a, mode, nwg, s);
    case 8: return launch_rg<T, 8>(a, mode, nwg, s);
    case 10: return launch_rg<T, 10>(a, mode, nwg, s);
    case 12: return launch_rg<T, 12>(a, mode, nwg, s);
  }
  return 0;
}

}  // namespace

constexpr int LDS_MAX_BYTES = 160 * 1024;

bool fused_supported(int x_dtype, const View& v, int R, int resid_mode) {
  if (x_dtype != TK_F32 && x_dtype != TK_BF16) return false;
  if (v.I > 256 || v.I < 1 || R < 1 || R > 48) return false;
  const int RG = rg_of(R);
  const int mode = resid_mode == TK_RESID_EXPLICIT ? 1 : 0;
  return (size_t)lds_layout((int)v.I, RG, mode).total * 4 <= (size_t)LDS_MAX_BYTES;
}

int fused_workgroups(const View& v) {
  int64_t ntiles = ceil_div(v.J(), TJ);
  return (int)(ntiles < NWG ? ntiles : NWG);
}

int launch_fused(const FusedArgs& a, int nwg_max, hipStream_t s) {
  int nwg = fused_workgroups(a.v);
  if (nwg > nwg_max / 4) nwg = nwg_max / 4;
  const int mode = a.sketch ? 2 : (a.Lr ? 1 : 0);
  if (a.x_dtype == TK_F32) return launch_t<float>(a, mode, nwg, s);
  return launch_t<bf16_t>(a, mode, nwg, s);
}

}  // namespace tk
