// Fused ALS sweep for large modes (256 < I_n <= 1024) on the gfx950 matrix
// cores.  The products are those of k_fused.hip (one HBM read of every fibre
// a_j per sweep, row-wise rule of Section 3: v_j = Lq^T a_j, G_V += v_j v_j^T,
// L_acc += a_j v_j^T; the init variant uses the Section 5 sketch rows and
// adds up ||A||^2; the TTM variant writes v_j out), but a tile of 64 fibres no
// longer fits LDS whole, so each tile is streamed in chunks of 128 rows:
//   pass 1  V = sum over chunks of X_c^T Lq_c  (R-update; X_c and the matching
//           rows of Lq staged in LDS, the next chunk of both prefetched in
//           registers while the current one is worked on);
//   Gram    G_V += V^T V from the finished V (FP32 per tile, FP64 across;
//           wave w < NR (NR + 1) / 2 owns one 16 x 16 block pair);
//   pass 2  L_acc[chunk rows] += X_c V  (L-update), the chunks read again,
//           last-loaded first, partly from the caches (a tile's 256 KiB per
//           workgroup overflows the XCD's L2).
// L_acc stays in registers for the whole launch: wave w owns, in every chunk,
// the output tiles (16 rows x 16 ranks) w, w + 8, ... of the 8 NR tiles of the
// chunk.  The R-update splits each chunk's 128 rows in two 64-row halves so the
// 4 NR (fibre block, rank tile) products spread over the 8 waves as 8 NR units.
// All products are v_mfma_f32_16x16x4f32 with FP32 accumulation; BF16
// storage is widened to FP32 when staged.  Every reduction has a fixed order.
#include "tk_kernels.h"

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 512;
constexpr int NW = NT / 64;
static_assert(NW == FUSED_WAVES, "partial buffers are sized for FUSED_WAVES waves");
constexpr int TJ = 64;            // fibres per tile
constexpr int CH = 128;           // rows per chunk
constexpr int NCHM = 8;           // chunks per mode, at most (I <= 1024)
constexpr int XLD = 65;           // LDS row stride of the chunk
constexpr int NWG = 256;
constexpr int SL = CH / NW;       // row slots per wave and chunk (16)

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ float to_f(T x);
template <> __device__ __forceinline__ float to_f<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f<bf16_t>(bf16_t x) { return bf16_to_f32(x); }

__host__ __device__ constexpr int rank_stride(int RP) { return (RP % 32 == 0) ? RP + 16 : RP; }

struct LdsG {
  int xs, lq, vf, vp, total;  // offsets in floats
};

__host__ __device__ inline LdsG lds_big(int NR, int mode) {
  const int RP = 16 * NR;
  const int RS = rank_stride(RP);
  LdsG l;
  l.xs = 0;
  l.lq = l.xs + CH * XLD;
  l.vf = l.lq + (mode != 2 ? 2 * CH * RS : 0);      // two chunk buffers
  l.vp = l.vf + (mode == 3 ? RP * (TJ + 1) : TJ * RS);
  l.total = l.vp + (mode != 2 ? 2 * TJ * RS : 0);   // the two R-update halves
  return l;
}

// Chunk c of tile j0 into registers: slot k is row 128 c + 8 k + w (clamped
// into the mode) of fibre j0 + lane (Q > 1, coalesced along q), or rows
// 128 c + lane + 64 h of the 8 fibres j0 + w + 8 f (Q == 1, slot k = 2 f + h).
// Lanes past the last fibre read fibre j0 and are zeroed in the stash.
template <typename T, int LAYOUT>
__device__ __forceinline__ void load_chunk(const T* __restrict__ X, const View& v, int64_t j0,
                                           int c, int lane, int w, T* pf, bool& ok) {
  const int64_t J = v.J();
  const int I = (int)v.I;
  if (LAYOUT == 0) {
    const int64_t j = j0 + lane;
    ok = j < J;
    const T* b = X + v.fibre_base(ok ? j : j0);
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int ii = min(CH * c + NW * k + w, I - 1);
      pf[k] = b[(int64_t)ii * v.Q];
    }
  } else {
    ok = true;
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int f = k / 2, h = k % 2;
      const int64_t j = min(j0 + w + NW * f, J - 1);
      pf[k] = X[j * I + min(CH * c + lane + 64 * h, I - 1)];
    }
  }
}

// Copy of rows CH c .. CH c + 127 of Lq into an LDS buffer of CH x RS floats
// by direct global -> LDS loads (no registers; the copy lands while the
// previous chunk is worked on).  Instruction m of wave w fills the PER x 64
// floats from PER * 64 (NW m + w) on, PER floats per lane; lane l's source is
// that element's (row, rank), clamped into the factor, so rows past I and
// ranks past R hold finite duplicates: the stash zeroes the matching X rows,
// and ranks past R only reach outputs that are never written.  VEC moves 16
// bytes per lane (Lq rows 16-byte aligned, ranks contiguous), else 4.
template <int RS, bool VEC>
__device__ __forceinline__ void issue_lq(const float* __restrict__ Lq, int I, int R, int64_t ldi,
                                         int64_t ldo, int c, float* dst, int lane, int w) {
  constexpr int PER = VEC ? 4 : 1;
  static_assert((CH * RS) % (NT * PER) == 0, "the chunk splits evenly over the threads");
  constexpr int NI = CH * RS / (NT * PER);
#pragma unroll
  for (int m = 0; m < NI; ++m) {
    const int base = PER * 64 * (NW * m + w);
    const int f = base + PER * lane;
    const int r = f / RS, col = f - (f / RS) * RS;
    const float* src = Lq + min(CH * c + r, I - 1) * ldi + min(col, R - PER) * ldo;
    auto* d = (__attribute__((address_space(3))) void*)(dst + base);
    if constexpr (VEC) __builtin_amdgcn_global_load_lds(src, d, 16, 0, 0);
    else __builtin_amdgcn_global_load_lds(src, d, 4, 0, 0);
  }
}

// s_waitcnt with vmcnt(0) (expcnt and lgkmcnt left at their maxima): this
// wave's outstanding global loads, the direct-to-LDS copies included, are done.
__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Rows past I are written as zeros (no branches): the staged Lq rows there
// are duplicates.  With NORM the squares of the chunk's elements are added to
// nsum.
template <typename T, int LAYOUT, bool NORM>
__device__ __forceinline__ void stash_chunk(const View& v, int64_t j0, int c, int lane, int w,
                                            const T* pf, bool ok, float* Xs, double& nsum) {
  const int I = (int)v.I;
  // (the squares go to four partial sums: one FP64 chain would wait out the
  // FMA latency at every element)
  double ns[4] = {0.0, 0.0, 0.0, 0.0};
  if (LAYOUT == 0) {
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int r = NW * k + w;
      const bool in = CH * c + r < I;
      const float x = ok && in ? to_f<T>(pf[k]) : 0.0f;
      Xs[r * XLD + lane] = x;
      if (NORM && in) ns[k & 3] += (double)x * (double)x;
    }
  } else {
    const int64_t J = v.J();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int f = k / 2, h = k % 2;
      const bool fok = j0 + w + NW * f < J;
      const int r = lane + 64 * h;
      const bool in = CH * c + r < I;
      const float x = fok && in ? to_f<T>(pf[k]) : 0.0f;
      Xs[r * XLD + w + NW * f] = x;
      if (NORM && in) ns[k & 3] += (double)x * (double)x;
    }
  }
  if (NORM) nsum += (ns[0] + ns[1]) + (ns[2] + ns[3]);
}

// MODE 0: sweep; 2: init (sketch, norm, no Gram); 3: TTM.
template <typename T, int NR, int MODE, int LAYOUT>
__global__ void __launch_bounds__(NT, 1) k_fused_big(FusedArgs a) {
  extern __shared__ float smem[];
  constexpr int RP = 16 * NR;
  constexpr int RS = rank_stride(RP);
  constexpr int NG = NR * (NR + 1) / 2;
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int NCH = (I + CH - 1) / CH;
  const LdsG L = lds_big(NR, MODE);
  float* Xs = smem + L.xs;
  float* Lq = smem + L.lq;
  float* Vf = smem + L.vf;
  float* Vp = smem + L.vp;
  const int64_t ldi = a.lq_ldi ? a.lq_ldi : R, ldo = a.lq_ldi ? a.lq_ldo : 1;

  for (int e = threadIdx.x; e < CH * XLD; e += NT) Xs[e] = 0.0f;

  f4 lacc[NCHM][NR];
#pragma unroll
  for (int c = 0; c < NCHM; ++c)
#pragma unroll
    for (int u = 0; u < NR; ++u) lacc[c][u] = f4{0, 0, 0, 0};
  // G_V: wave w < NG owns block pair w = (ga, gb), ga <= gb, over all fibres
  int ga = 0, gb = 0;
  for (int p = 0, na = 0; na < NR; ++na)
    for (int nb = na; nb < NR; ++nb, ++p)
      if (p == w) { ga = na; gb = nb; }
  double gd[4] = {0.0, 0.0, 0.0, 0.0};
  double nsum = 0.0;
  const bool want_norm = MODE == 2 && a.norm2_parts != nullptr;

  const T* X = (const T*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  T pf[SL];
  bool pf_ok = false;
  const bool lq_vec = ldo == 1 && ldi % 4 == 0 && R % 4 == 0 && ((uintptr_t)a.Lq & 15) == 0;
  auto lq_copy = [&](int c) __attribute__((always_inline)) {
    float* dst = Lq + (c & 1) * CH * RS;
    if (lq_vec) issue_lq<RS, true>(a.Lq, I, R, ldi, ldo, c, dst, lane, w);
    else issue_lq<RS, false>(a.Lq, I, R, ldi, ldo, c, dst, lane, w);
  };

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t j0 = tile * TJ;

    if (MODE != 2) {
      // ---- pass 1: V = sum_c X_c^T Lq_c; unit u = w + 8 k -> (fibre block
      // fb, rank tile n, half h) with 2 (NR fb + n) + h = u.
      f4 vacc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) vacc[k] = f4{0, 0, 0, 0};
      load_chunk<T, LAYOUT>(X, v, j0, 0, lane, w, pf, pf_ok);
      lq_copy(0);
      for (int c = 0; c < NCH; ++c) {
        // buffer (c + 1) & 1 was last read by chunk c - 1's products, which
        // every wave has finished at the first barrier
        __syncthreads();
        stash_chunk<T, LAYOUT, false>(v, j0, c, lane, w, pf, pf_ok, Xs, nsum);
        wait_vm0();
        __syncthreads();
        if (c + 1 < NCH) {
          load_chunk<T, LAYOUT>(X, v, j0, c + 1, lane, w, pf, pf_ok);
          lq_copy(c + 1);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          const int u = w + NW * k;
          const int h = u & 1, t = u >> 1;
          const int fb = t / NR, n = t % NR;
          const float* xa = Xs + (64 * h + lk) * XLD + 16 * fb + lr;
          const float* lb = Lq + (c & 1) * CH * RS + (64 * h + lk) * RS + 16 * n + lr;
          f4 acc = vacc[k];
#pragma unroll
          for (int ks = 0; ks < 16; ++ks) acc = mfma16(xa[4 * ks * XLD], lb[4 * ks * RS], acc);
          vacc[k] = acc;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // V = half 0 + half 1 (V[16 fb + 4 lk + q][16 n + lr])
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int u = w + NW * k;
        const int h = u & 1, t = u >> 1;
        const int fb = t / NR, n = t % NR;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Vp[h * TJ * RS + (16 * fb + 4 * lk + q) * RS + 16 * n + lr] = vacc[k][q];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < TJ * RP; e += NT) {
        const int jl = e / RP, r = e - (e / RP) * RP;
        const float s = Vp[jl * RS + r] + Vp[TJ * RS + jl * RS + r];
        if (MODE == 3) Vf[r * (TJ + 1) + jl] = s;
        else Vf[jl * RS + r] = s;
      }
      __syncthreads();
    } else {
      // init: V = the Section 5 sketch rows of this tile
      __syncthreads();
      for (int e = threadIdx.x; e < TJ * RP; e += NT) {
        const int jl = e / RP, r = e - (e / RP) * RP;
        const int64_t j = j0 + jl;
        float s = 0.0f;
        if (j < J && r < R)
          s = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        Vf[jl * RS + r] = s;
      }
    }

    if (MODE == 3) {
      // fibre j of Y = B x_n U^T: Y[p, r, q] = V[j, r], coalesced along q
      float* Y = a.y;
      if (LAYOUT == 0) {
        const int64_t j = j0 + lane;
        if (j < J) {
          const int64_t p = j / v.Q, q = j - p * v.Q;
          float* yb = Y + p * (int64_t)R * v.Q + q;
          for (int r = w; r < R; r += NW) yb[(int64_t)r * v.Q] = Vf[r * (TJ + 1) + lane];
        }
      } else {
        for (int e = threadIdx.x; e < TJ * R; e += NT) {
          const int jl = e / R, r = e - jl * R;
          if (j0 + jl < J) Y[(j0 + jl) * R + r] = Vf[r * (TJ + 1) + jl];
        }
      }
      continue;
    }

    if (MODE == 0 && w < NG) {
      // block (ga, gb) of G_V over the tile's 64 fibres (16 K steps)
      const float* va = Vf + lk * RS + 16 * ga + lr;
      const float* vb = Vf + lk * RS + 16 * gb + lr;
      f4 gacc = f4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) gacc = mfma16(va[4 * ks * RS], vb[4 * ks * RS], gacc);
#pragma unroll
      for (int q = 0; q < 4; ++q) gd[q] += (double)gacc[q];
    }

    // ---- pass 2: L_acc[chunk c rows] += X_c V; tile t = w + 8 k of the
    // chunk's 8 NR output tiles is (row tile t / NR, rank tile t % NR).  The
    // chunk loop runs at run time; the switch picks the chunk's accumulators
    // (register arrays need compile-time indices).
    auto lupd = [&](f4 (&acc)[NR]) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int t = w + NW * k;
        const int m = t / NR, n = t % NR;
        const float* xr = Xs + (16 * m + lr) * XLD + lk;
        const float* vb = Vf + lk * RS + 16 * n + lr;
        f4 ac = acc[k];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) ac = mfma16(xr[4 * ks], vb[4 * ks * RS], ac);
        acc[k] = ac;
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // (after pass 1 the chunks are read back last-loaded first: the freshest
    // lines are the likeliest still in L2, where a repeat of pass 1's order
    // would evict each chunk just before it is needed)
    auto ord = [&](int k) __attribute__((always_inline)) { return MODE == 0 ? NCH - 1 - k : k; };
    load_chunk<T, LAYOUT>(X, v, j0, ord(0), lane, w, pf, pf_ok);
    for (int k = 0; k < NCH; ++k) {
      const int c = ord(k);
      __syncthreads();
      if (MODE == 2 && want_norm)
        stash_chunk<T, LAYOUT, true>(v, j0, c, lane, w, pf, pf_ok, Xs, nsum);
      else stash_chunk<T, LAYOUT, false>(v, j0, c, lane, w, pf, pf_ok, Xs, nsum);
      __syncthreads();
      if (k + 1 < NCH) load_chunk<T, LAYOUT>(X, v, j0, ord(k + 1), lane, w, pf, pf_ok);
      switch (c) {
        case 0: lupd(lacc[0]); break;
        case 1: lupd(lacc[1]); break;
        case 2: lupd(lacc[2]); break;
        case 3: lupd(lacc[3]); break;
        case 4: lupd(lacc[4]); break;
        case 5: lupd(lacc[5]); break;
        case 6: lupd(lacc[6]); break;
        default: lupd(lacc[7]); break;
      }
    }
    __syncthreads();
  }

  // ---- per-workgroup outputs
  if (MODE == 3) return;
  const int wg = blockIdx.x;
  if (want_norm) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsum += __shfl_xor(nsum, off, 64);
    if (lane == 0) a.norm2_parts[wg * NW + w] = nsum;
  }
  float* lp = a.lacc_parts + (int64_t)wg * I * R;
#pragma unroll
  for (int c = 0; c < NCHM; ++c) {
    if (c < NCH) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int t = w + NW * k;
        const int m = t / NR, n = t % NR;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = CH * c + 16 * m + 4 * lk + q, r = 16 * n + lr;
          if (i < I && r < R) lp[i * R + r] = lacc[c][k][q];
        }
      }
    }
  }
  if (MODE == 0) {
    // wave w's partial is its block pair (upper triangle of a diagonal block
    // and its mirror, so it is exactly symmetric) and zero elsewhere
    double* gp = a.gv_parts + (int64_t)(wg * NW + w) * R * R;
    for (int e = lane; e < R * R; e += 64) gp[e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (w < NG) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * ga + 4 * lk + q, col = 16 * gb + lr;
        if (row < R && col < R && (ga < gb || row <= col)) {
          gp[row * R + col] = gd[q];
          gp[col * R + row] = gd[q];
        }
      }
    }
  }
}

template <typename T, int NR, int MODE>
void launch_l(const FusedArgs& a, int nwg, hipStream_t s) {
  const size_t bytes = (size_t)lds_big(NR, MODE).total * 4;
  if (a.v.Q != 1) {
    (void)hipFuncSetAttribute((const void*)k_fused_big<T, NR, MODE, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused_big<T, NR, MODE, 0>), dim3(nwg), dim3(NT), bytes, s, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k_fused_big<T, NR, MODE, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused_big<T, NR, MODE, 1>), dim3(nwg), dim3(NT), bytes, s, a);
  }
}

template <typename T, int NR>
void launch_m(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  if (mode == 0) launch_l<T, NR, 0>(a, nwg, s);
  else if (mode == 2) launch_l<T, NR, 2>(a, nwg, s);
  else launch_l<T, NR, 3>(a, nwg, s);
}

template <typename T>
void launch_t(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  switch ((a.R + 15) / 16) {
    case 1: launch_m<T, 1>(a, mode, nwg, s); break;
    case 2: launch_m<T, 2>(a, mode, nwg, s); break;
    case 3: launch_m<T, 3>(a, mode, nwg, s); break;
  }
}

}  // namespace

bool fused_big_shape(int x_dtype, const View& v, int64_t R, int mode) {
  if (x_dtype != TK_F32 && x_dtype != TK_BF16) return false;
  if (mode == 1) return false;
  return v.I > 256 && v.I <= (int64_t)CH * NCHM && R >= 1 && R <= 48;
}

int launch_fused_big(const FusedArgs& a, int mode, int nwg_max, hipStream_t s) {
  const int64_t ntiles = ceil_div(a.v.J(), TJ);
  int nwg = (int)(ntiles < NWG ? ntiles : NWG);
  if (nwg > nwg_max / NW) nwg = nwg_max / NW;
  if (a.x_dtype == TK_F32) launch_t<float>(a, mode, nwg, s);
  else launch_t<bf16_t>(a, mode, nwg, s);
  return nwg;
}

}  // namespace tk
