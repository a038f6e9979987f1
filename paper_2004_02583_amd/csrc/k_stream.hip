// Tensor-streaming kernels on the strided mode-n view (no unfolding is ever
// materialised; the row-wise update rule of Section 3 lets every fibre be
// processed independently).  These are the generic VALU kernels: any dtype,
// any mode size.  The matrix-core fused sweep lives in k_fused.hip.
#include "tk_kernels.h"

namespace tk {

namespace {

constexpr int TJ = 64;   // fibres per tile
constexpr int TI = 64;   // mode-index rows per tile
constexpr int LDX = 65;  // padded LDS row stride of an X tile

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Fibre base offsets of tile [j0, j0+TJ) for view v (0 past the end).
__device__ __forceinline__ void tile_bases(const View& v, int64_t j0, int64_t* fb) {
  if (threadIdx.x < TJ) {
    int64_t j = j0 + threadIdx.x;
    fb[threadIdx.x] = (j < v.J()) ? v.fibre_base(j) : 0;
  }
}

// X[i0+ii, j0+jj] -> tile[ii*LDX + jj] for ii < TI, jj < TJ, zero outside.
// Coalesced along q when Q > 1 and along i when Q == 1.
template <typename T, typename C>
__device__ __forceinline__ void load_tile(const T* __restrict__ X, const View& v,
                                          int64_t i0, int64_t j0,
                                          const int64_t* __restrict__ fb, C* tile) {
  const int64_t J = v.J();
  if (v.Q == 1) {
    for (int e = threadIdx.x; e < TI * TJ; e += blockDim.x) {
      int ii = e % TI, jj = e / TI;
      int64_t i = i0 + ii, j = j0 + jj;
      C val = 0;
      if (i < v.I && j < J) val = (C)Elem<T>::load(X + fb[jj] + i);
      tile[ii * LDX + jj] = val;
    }
  } else {
    for (int e = threadIdx.x; e < TI * TJ; e += blockDim.x) {
      int jj = e % TJ, ii = e / TJ;
      int64_t i = i0 + ii, j = j0 + jj;
      C val = 0;
      if (i < v.I && j < J) val = (C)Elem<T>::load(X + fb[jj] + i * v.Q);
      tile[ii * LDX + jj] = val;
    }
  }
}

// The X and W elements of one row step (rows i0 .. i0 + TI - 1) that thread
// tid stages, loaded into registers (zero outside), and their LDS stores:
// while a step is computed from LDS the next step's loads are in flight.
template <typename T, typename C, int OM>
struct StepRegs {
  static constexpr int NX = TI * TJ / 256, NW = TI * OM / 256;
  C x[NX], w[NW];
};

// Element k of thread tid: X row i0 + tid / TJ + 4k of fibre j0 + tid % TJ
// (Q > 1), or row i0 + tid % TI of fibre j0 + tid / TI + 4k (Q == 1); W row
// i0 + tid / OM + (256 / OM) k, output o0 + tid % OM.  The per-thread bases
// pass through empty asm statements, so that each step forms its addresses
// from them plus wave-uniform offsets instead of keeping per-element
// addresses hoisted out of the row loop (they would take the registers).
template <typename T, typename C, int OM>
__device__ __forceinline__ void step_load(const T* __restrict__ X, const C* __restrict__ W,
                                          const VpassArgs& a, const View& v, int64_t i0,
                                          int64_t j0, int64_t o0,
                                          const int64_t* __restrict__ fb,
                                          StepRegs<T, C, OM>& sr) {
  const int64_t J = v.J();
  const int tid = (int)threadIdx.x;
  if (v.Q == 1) {
    const int ii = tid % TI;
    const int64_t i = i0 + ii;
#pragma unroll
    for (int k = 0; k < StepRegs<T, C, OM>::NX; ++k) {
      const int jj = tid / TI + 4 * k;
      C val = 0;
      if (i < v.I && j0 + jj < J) val = (C)Elem<T>::load(X + fb[jj] + i);
      sr.x[k] = val;
    }
  } else {
    const int jj = tid % TJ;
    const bool jok = j0 + jj < J;
    const int64_t ib = i0 + tid / TJ;
    const T* xb = X + fb[jj] + ib * v.Q;
    asm volatile("" : "+v"(xb));
#pragma unroll
    for (int k = 0; k < StepRegs<T, C, OM>::NX; ++k) {
      C val = 0;
      if (jok && ib + 4 * k < v.I) val = (C)Elem<T>::load(xb + (int64_t)(4 * k) * v.Q);
      sr.x[k] = val;
    }
  }
  const int64_t iw = i0 + tid / OM, o = o0 + tid % OM;
  const bool ook = o < a.O;
  const C* wb = W + iw * a.w_ldi + o * a.w_ldo;
  asm volatile("" : "+v"(wb));
#pragma unroll
  for (int k = 0; k < StepRegs<T, C, OM>::NW; ++k) {
    constexpr int DI = 256 / OM;
    sr.w[k] = (ook && iw + DI * k < v.I) ? wb[(int64_t)(DI * k) * a.w_ldi] : (C)0;
  }
}

template <typename T, typename C, int OM>
__device__ __forceinline__ void step_store(const View& v, const StepRegs<T, C, OM>& sr, C* xt,
                                           C* wt) {
#pragma unroll
  for (int k = 0; k < StepRegs<T, C, OM>::NX; ++k) {
    const int e = (int)threadIdx.x + 256 * k;
    int ii, jj;
    if (v.Q == 1) { ii = e % TI; jj = e / TI; }
    else { jj = e % TJ; ii = e / TJ; }
    xt[ii * LDX + jj] = sr.x[k];
  }
#pragma unroll
  for (int k = 0; k < StepRegs<T, C, OM>::NW; ++k) wt[(int)threadIdx.x + 256 * k] = sr.w[k];
}

// ---------------------------------------------------------------------------
// out(j, o) = sum_i W(i, o) X[j-th fibre][i]; thread (jh, oh) owns outputs
// o = o0 + oh + 8k of fibres j0 + jh and j0 + jh + 32 (two fibres per
// thread: each W value read from LDS serves two products).  Row steps of TI
// rows; the next step's X and W elements are loaded into registers while a
// step is computed.
template <typename T, typename C, int OM>
__global__ void __launch_bounds__(256) k_vpass(VpassArgs a) {
  __shared__ C xt[TI * LDX];
  __shared__ C wt[TI * OM];
  __shared__ int64_t fb[TJ];
  __shared__ double red[256];
  const T* X = (const T*)a.X;
  const C* W = (const C*)a.W;
  const View v = a.v;
  const int64_t J = v.J();
  const int jj = threadIdx.x % TJ, oq = threadIdx.x / TJ;    // residual
  constexpr int HJ = TJ / 2;
  const int jh = threadIdx.x % HJ, oh = threadIdx.x / HJ;    // products
  const int64_t ntiles = ceil_div(J, TJ);
  double rsum = 0.0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t j0 = tile * TJ;
    __syncthreads();
    tile_bases(v, j0, fb);
    __syncthreads();
    const int64_t j = j0 + jj;
    for (int64_t o0 = 0; o0 < a.O; o0 += OM) {
      C acc0[OM / 8], acc1[OM / 8];
#pragma unroll
      for (int k = 0; k < OM / 8; ++k) acc0[k] = acc1[k] = 0;
      StepRegs<T, C, OM> sr;
      step_load<T, C, OM>(X, W, a, v, 0, j0, o0, fb, sr);
      for (int64_t i0 = 0; i0 < v.I; i0 += TI) {
        __syncthreads();
        step_store<T, C, OM>(v, sr, xt, wt);
        __syncthreads();
        if (i0 + TI < v.I) step_load<T, C, OM>(X, W, a, v, i0 + TI, j0, o0, fb, sr);
        const int rows = (int)((v.I - i0) < TI ? (v.I - i0) : TI);
        // (a modest unroll: the registers go to the loads in flight)
#pragma unroll 4
        for (int ii = 0; ii < rows; ++ii) {
          const C x0 = xt[ii * LDX + jh], x1 = xt[ii * LDX + jh + HJ];
#pragma unroll
          for (int k = 0; k < OM / 8; ++k) {
            const C ww = wt[ii * OM + oh + 8 * k];
            acc0[k] += ww * x0;
            acc1[k] += ww * x1;
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t jo = j0 + jh + HJ * h;
        if (jo < J) {
          const int64_t p = jo / v.Q, q = jo - (jo / v.Q) * v.Q;
#pragma unroll
          for (int k = 0; k < OM / 8; ++k) {
            const int64_t o = o0 + oh + 8 * k;
            const C val = h ? acc1[k] : acc0[k];
            if (o < a.O) {
              if (a.out_kind == 0) ((C*)a.out)[jo * a.O + o] = val;
              else ((C*)a.out)[(p * a.O + o) * v.Q + q] = val;
            }
          }
        }
      }
    }
    if (a.Lr) {
      // explicit residual of this tile: sum_j ||x_j - Lr v_j||^2 (O <= OM).
      // v_j comes back from the output into LDS with an odd row stride (a
      // stride of OM would put every lane of a read on one bank) and then
      // into this thread's registers; Lr and X stream by row steps as above.
      const C* V = (const C*)a.out;
      __shared__ C vt[TJ * (OM + 1)];
      __syncthreads();
      for (int e = threadIdx.x; e < TJ * OM; e += blockDim.x) {
        int jl = e / OM, o = e % OM;
        vt[jl * (OM + 1) + o] = (j0 + jl < J && o < a.O) ? V[(j0 + jl) * a.O + o] : (C)0;
      }
      __syncthreads();
      C vr[OM];
#pragma unroll
      for (int o = 0; o < OM; ++o) vr[o] = vt[jj * (OM + 1) + o];
      VpassArgs ar = a;
      ar.W = a.Lr;
      ar.w_ldi = a.O;
      ar.w_ldo = 1;
      StepRegs<T, C, OM> sr;
      step_load<T, C, OM>(X, (const C*)a.Lr, ar, v, 0, j0, 0, fb, sr);
      for (int64_t i0 = 0; i0 < v.I; i0 += TI) {
        __syncthreads();
        step_store<T, C, OM>(v, sr, xt, wt);
        __syncthreads();
        if (i0 + TI < v.I) step_load<T, C, OM>(X, (const C*)a.Lr, ar, v, i0 + TI, j0, 0, fb, sr);
        const int rows = (int)((v.I - i0) < TI ? (v.I - i0) : TI);
        if (j < J) {
          for (int ii = oq; ii < rows; ii += 4) {
            C d = xt[ii * LDX + jj];
#pragma unroll
            for (int o = 0; o < OM; ++o) d -= wt[ii * OM + o] * vr[o];
            rsum += (double)d * (double)d;
          }
        }
      }
    }
  }
  if (a.resid_parts) {
    double t = block_sum(rsum, red);
    if (threadIdx.x == 0) a.resid_parts[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Partial L(i, r) = sum_{j in chunk} X[j-th fibre][i] V(j, r); grid =
// (i-blocks, fibre chunks); thread (ii, rq) owns r = rq + 8k of rows i0 + ii
// and i0 + ii + 32 (two rows per thread: each V value read from LDS serves
// two products).
template <typename T, typename C, int RM, int VK>
__global__ void __launch_bounds__(256) k_lpass(LpassArgs a, int64_t tiles_per_chunk) {
  __shared__ C xt[TI * LDX];
  __shared__ C vt[TJ * RM];
  __shared__ int64_t fb[TJ];
  __shared__ int64_t fby[TJ];
  __shared__ double red[256];
  const T* X = (const T*)a.X;
  const View v = a.v;
  const int64_t J = v.J(), R = a.R;
  constexpr int HR = TI / 2;                 // second row of a thread
  const int ii = threadIdx.x % HR, rq = threadIdx.x / HR;
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int64_t c = blockIdx.y;
  const int64_t ntiles = ceil_div(J, TJ);
  const int64_t t_beg = c * tiles_per_chunk;
  const int64_t t_end = (t_beg + tiles_per_chunk < ntiles) ? t_beg + tiles_per_chunk : ntiles;
  C acc0[RM / 8], acc1[RM / 8];
#pragma unroll
  for (int k = 0; k < RM / 8; ++k) acc0[k] = acc1[k] = 0;
  double nsum = 0.0;
  for (int64_t tile = t_beg; tile < t_end; ++tile) {
    const int64_t j0 = tile * TJ;
    __syncthreads();
    tile_bases(v, j0, fb);
    if (VK == 2 && threadIdx.x < TJ) {
      int64_t j = j0 + threadIdx.x;
      int64_t p = (j < J) ? j / v.Q : 0;
      int64_t q = (j < J) ? j - p * v.Q : 0;
      fby[threadIdx.x] = (p * R) * v.Q + q;
    }
    __syncthreads();
    load_tile<T, C>(X, v, i0, j0, fb, xt);
    for (int e = threadIdx.x; e < TJ * RM; e += blockDim.x) {
      int jl = e / RM, r = e % RM;
      int64_t j = j0 + jl;
      C val = 0;
      if (j < J && r < R) {
        if (VK == 0) val = ((const C*)a.V)[j * R + r];
        else if (VK == 1)
          val = (C)sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        else val = (C)Elem<T>::load((const T*)a.V + fby[jl] + r * v.Q);
      }
      vt[e] = val;
    }
    __syncthreads();
    if (a.norm2_parts) {
      for (int e = threadIdx.x; e < TI * TJ; e += blockDim.x) {
        double x = (double)xt[(e / TJ) * LDX + (e % TJ)];
        nsum += x * x;
      }
    }
    for (int jl = 0; jl < TJ; ++jl) {
      const C x0 = xt[ii * LDX + jl], x1 = xt[(ii + HR) * LDX + jl];
#pragma unroll
      for (int k = 0; k < RM / 8; ++k) {
        const C vv = vt[jl * RM + rq + 8 * k];
        acc0[k] += x0 * vv;
        acc1[k] += x1 * vv;
      }
    }
  }
  C* out = (C*)a.parts + c * v.I * R;
#pragma unroll
  for (int k = 0; k < RM / 8; ++k) {
    const int64_t r = rq + 8 * k;
    if (r < R) {
      if (i0 + ii < v.I) out[(i0 + ii) * R + r] = acc0[k];
      if (i0 + ii + HR < v.I) out[(i0 + ii + HR) * R + r] = acc1[k];
    }
  }
  if (a.norm2_parts) {
    double t = block_sum(nsum, red);
    if (threadIdx.x == 0) a.norm2_parts[c * gridDim.x + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// G = V^T V partials over row chunks (FP64 accumulation).
template <typename C>
__global__ void __launch_bounds__(256) k_gram_parts(const C* __restrict__ V, int64_t J,
                                                    int64_t R, int64_t rows_per_chunk,
                                                    double* __restrict__ parts) {
  __shared__ double vt[64 * 64];
  const int npair = (int)(R * (R + 1) / 2);
  double acc[9];
  int pa[9], pb[9];
  int cnt = 0;
  for (int t = threadIdx.x; t < npair && cnt < 9; t += blockDim.x, ++cnt) {
    int x = 0, rem = t;
    while (rem >= R - x) { rem -= (int)(R - x); ++x; }
    pa[cnt] = x;
    pb[cnt] = x + rem;
    acc[cnt] = 0.0;
  }
  const int64_t r0 = blockIdx.x * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < J) ? r0 + rows_per_chunk : J;
  for (int64_t b = r0; b < r1; b += 64) {
    int rows = (int)((r1 - b) < 64 ? (r1 - b) : 64);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * R; e += blockDim.x) vt[e] = (double)V[b * R + e];
    __syncthreads();
    for (int c = 0; c < cnt; ++c) {
      double s = 0.0;
      for (int i = 0; i < rows; ++i) s += vt[i * R + pa[c]] * vt[i * R + pb[c]];
      acc[c] += s;
    }
  }
  double* out = parts + blockIdx.x * R * R;
  for (int c = 0; c < cnt; ++c) {
    out[pa[c] * R + pb[c]] = acc[c];
    out[pb[c] * R + pa[c]] = acc[c];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_norm2_parts(const T* __restrict__ X, int64_t n,
                                                     double* __restrict__ parts) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double x = (double)Elem<T>::load(X + e);
    s += x * x;
  }
  double t = block_sum(s, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

template <typename T, typename C>
int vpass_dispatch(const VpassArgs& a, int nwg, hipStream_t s) {
  if (a.O <= 16)
    hipLaunchKernelGGL((k_vpass<T, C, 16>), dim3(nwg), dim3(256), 0, s, a);
  else if (a.O <= 32)
    hipLaunchKernelGGL((k_vpass<T, C, 32>), dim3(nwg), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_vpass<T, C, 64>), dim3(nwg), dim3(256), 0, s, a);
  return 0;
}

template <typename T, typename C, int VK>
void lpass_dispatch(const LpassArgs& a, int chunks, int64_t tpc, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(a.v.I, TI), (unsigned)chunks);
  if (a.R <= 16)
    hipLaunchKernelGGL((k_lpass<T, C, 16, VK>), grid, dim3(256), 0, s, a, tpc);
  else if (a.R <= 32)
    hipLaunchKernelGGL((k_lpass<T, C, 32, VK>), grid, dim3(256), 0, s, a, tpc);
  else
    hipLaunchKernelGGL((k_lpass<T, C, 64, VK>), grid, dim3(256), 0, s, a, tpc);
}

template <typename T, typename C>
void lpass_vk(const LpassArgs& a, int chunks, int64_t tpc, hipStream_t s) {
  if (a.v_kind == 0) lpass_dispatch<T, C, 0>(a, chunks, tpc, s);
  else if (a.v_kind == 1) lpass_dispatch<T, C, 1>(a, chunks, tpc, s);
  else lpass_dispatch<T, C, 2>(a, chunks, tpc, s);
}

}  // namespace

int launch_vpass(const VpassArgs& a, int nwg_max, int* nwg_used, hipStream_t s) {
  int64_t ntiles = ceil_div(a.v.J(), TJ);
  int nwg = (int)(ntiles < nwg_max ? ntiles : nwg_max);
  if (nwg < 1) nwg = 1;
  if (nwg_used) *nwg_used = nwg;
  if (a.Lr && a.O > 64) return TK_ERR_INVALID_ARG;
  switch (a.x_dtype) {
    case TK_F64: return vpass_dispatch<double, double>(a, nwg, s);
    case TK_F32: return vpass_dispatch<float, float>(a, nwg, s);
    case TK_BF16: return vpass_dispatch<bf16_t, float>(a, nwg, s);
  }
  return TK_ERR_UNSUPPORTED_DTYPE;
}

int lpass_chunks(const View& v, int64_t R, int nwg_max) {
  (void)R;
  int64_t ntiles = ceil_div(v.J(), TJ);
  int64_t iblocks = ceil_div(v.I, TI);
  int64_t want = nwg_max / (iblocks > 0 ? iblocks : 1);
  if (want < 1) want = 1;
  // at least 4 tiles per chunk so partial traffic stays small
  int64_t byt = ceil_div(ntiles, 4);
  if (want > byt) want = byt;
  if (want < 1) want = 1;
  return (int)want;
}

int lpass_blocks(const View& v, int chunks) {
  return (int)(chunks * ceil_div(v.I, TI));
}

void launch_lpass(const LpassArgs& a, int chunks, hipStream_t s) {
  int64_t ntiles = ceil_div(a.v.J(), TJ);
  int64_t tpc = ceil_div(ntiles, chunks);
  switch (a.x_dtype) {
    case TK_F64: lpass_vk<double, double>(a, chunks, tpc, s); break;
    case TK_F32: lpass_vk<float, float>(a, chunks, tpc, s); break;
    case TK_BF16: lpass_vk<bf16_t, float>(a, chunks, tpc, s); break;
  }
}

void launch_gram_parts(const void* V, int c_dtype, int64_t J, int64_t R, int chunks,
                       double* parts, hipStream_t s) {
  int64_t rpc = ceil_div(J, chunks);
  if (c_dtype == TK_F64)
    hipLaunchKernelGGL(k_gram_parts<double>, dim3(chunks), dim3(256), 0, s,
                       (const double*)V, J, R, rpc, parts);
  else
    hipLaunchKernelGGL(k_gram_parts<float>, dim3(chunks), dim3(256), 0, s,
                       (const float*)V, J, R, rpc, parts);
}

void launch_norm2_parts(const void* X, int x_dtype, int64_t n, int chunks, double* parts,
                        hipStream_t s) {
  switch (x_dtype) {
    case TK_F64:
      hipLaunchKernelGGL(k_norm2_parts<double>, dim3(chunks), dim3(256), 0, s,
                         (const double*)X, n, parts);
      break;
    case TK_F32:
      hipLaunchKernelGGL(k_norm2_parts<float>, dim3(chunks), dim3(256), 0, s,
                         (const float*)X, n, parts);
      break;
    case TK_BF16:
      hipLaunchKernelGGL(k_norm2_parts<bf16_t>, dim3(chunks), dim3(256), 0, s,
                         (const bf16_t*)X, n, parts);
      break;
  }
}

}  // namespace tk
