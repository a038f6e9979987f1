// Fused ALS sweep on the gfx950 matrix cores.
//
// One sweep of Algorithm 3.3 on the mode-n view [P, I, Q] reads every fibre
// a_j (a column of A_(n)) from HBM once and uses it twice (row-wise update
// rule of Section 3):
//    v_j   = Lq^T a_j                (row j of R_k; never written out)
//    G_V  += v_j v_j^T               (R_k^T R_k, FP32 per tile, FP64 across)
//    L_acc += a_j v_j^T              (A_(n) R_k, per-workgroup partial)
// and optionally the explicit residual sum_j ||a_j - L v_j||^2.  The init
// variant replaces v_j by row j of the Section 5 sketch S (and can add up
// ||A||^2 on the way); the TTM variant keeps only v_j = U^T a_j, which is
// fibre j of B x_n U^T, and writes it out.
//
// Work layout: a workgroup of 8 waves (two per SIMD) walks 64-fibre tiles
// (persistent grid, tile = blockIdx + k * gridDim).  The tile X (I x 64) is
// staged in LDS as FP32 from registers that were prefetched during the
// previous tile.  All three products use v_mfma_f32_16x16x4f32 (A 16x4,
// B 4x16, D 16x16):
//   R-update  16x16 output tiles (16 fibres x 16 ranks), K = I, dealt
//             round-robin over the waves: V = X^T Lq;
//   L-update  16x16 output tiles (16 mode rows x 16 ranks), K = 64 fibres,
//             dealt round-robin over the waves;
//   Gram      wave w: V^T V over fibres 8w..8w+7, upper block triangle.
// R is padded with zero columns to a multiple of 16, except that with
// 16 < R <= 20 the last four ranks take v_mfma_f32_4x4x1_16b_f32 instead
// (RM variant): 16 blocks of 4 x 4 outputs, so the four ranks
// cost a quarter of a padded 16-rank tile, on the waves that hold no other
// R-update tile.  Every reduction has a fixed order
// (deterministic, no atomics).
#include <type_traits>

#include "tk_kernels.h"

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 512;      // threads per workgroup
constexpr int NW = NT / 64;  // waves per workgroup
static_assert(NW == FUSED_WAVES, "partial buffers are sized for FUSED_WAVES waves");
constexpr int TJ = 64;       // fibres per tile
constexpr int XLD = 65;      // LDS row stride of the X tile
constexpr int NWG = 256;     // persistent workgroups (one per CU)

// D = A B + C with A 16x4 (lane l: row l%16, k l/16), B 4x16 (lane l:
// k l/16, column l%16), D 16x16 (lane l, element q: row 4(l/16)+q,
// column l%16).
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// 16 independent 4 x 4 products, K = 1: block b = lane / 4; lane 4b + i holds
// A_b[i], lane 4b + j holds B_b[j], and element i of lane 4b + j is
// D_b[i][j] = A_b[i] B_b[j] + C_b[i][j].
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ float to_f(T x);
template <> __device__ __forceinline__ float to_f<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f<bf16_t>(bf16_t x) { return bf16_to_f32(x); }

// Row stride of the rank-indexed LDS arrays: 16 mod 32 keeps the 16x16x4
// operand reads (two row offsets per half-wave) on distinct banks.
__host__ __device__ constexpr int rank_stride(int RP) { return (RP % 32 == 0) ? RP + 16 : RP; }

struct Lds {
  int xs, lq, lr, vf, vr, total;  // offsets in floats
};

__host__ __device__ constexpr int round4(int x) { return (x + 3) & ~3; }

// rm: room for the RM variant's final exchange of L-update sums ([4][64][4]).
// Lq, V and those partials start on 16-byte boundaries (4-float reads).
__host__ __device__ inline Lds lds_layout(int I, int NR, int mode, bool rm = false) {
  const int RP = 16 * NR;
  const int xrows = 16 * ((I + 15) / 16);
  const int RS = rank_stride(RP);
  Lds l;
  l.xs = 0;
  l.lq = round4(l.xs + (xrows + 1) * XLD);    // + spare row for the stash
  l.lr = l.lq + (mode != 2 ? xrows * RS : 0);
  l.vf = round4(l.lr + (mode == 1 ? xrows * (RP + 1) : 0));
  // TTM keeps V transposed ([RP][TJ + 1]) for coalesced, conflict-free writes
  l.total = l.vf + (mode == 3 && RP * (TJ + 1) > TJ * RS ? RP * (TJ + 1) : TJ * RS);
  l.vr = l.total;
  if (rm) l.total = l.vr + 4 * TJ * 4;
  return l;
}

// Prefetch of one tile into registers: a fixed number of unconditional
// loads per lane (IC = 8, 16, 26 or 32 row slots per wave, from the mode size
// class) whose row / fibre indices are clamped into the tensor, so the
// compiler issues them back to back without branches (duplicates of a
// clamped row hit the caches).
//  LAYOUT 0 (Q > 1): slot k is row ii = 8k + w of fibre j0 + lane
//          (coalesced along q); lanes past the last fibre read the last
//          fibre and are zeroed in the stash.
// Tiles past the end are fetched the same way (clamped), so that every
// prefetch is unconditional and the wait for one buffer never covers the
// loads of the other.
//  LAYOUT 1 (Q == 1): slot k = NC f + c is rows lane + 64c of fibre
//          j0 + w + 8f (NC = IC/8 chunks of 64 rows per fibre, 8 fibres).
//  LAYOUT 2 (FP32, Q a multiple of 4, 16-byte aligned tensor): 16-byte loads,
//          a quarter of the load instructions of LAYOUT 0 (issuing them is
//          what the slowest waves of a tile wait for): slot k holds rows
//          32k + 4w + lane / 16 (clamped), fibres j0 + 4 (lane % 16) .. + 3,
//          in pf[4k .. 4k + 3].
template <int LAYOUT, int IC>
__host__ __device__ constexpr int pf_slots() {
  return LAYOUT == 2 ? 4 * ((NW * IC + 31) / 32) : IC;
}

template <typename T, int LAYOUT, int IC>
__device__ __forceinline__ void prefetch(const T* __restrict__ X, const View& v, int64_t j0,
                                         int lane, int w, T* pf, bool& ok) {
  const int64_t J = v.J();
  const int I = (int)v.I;
  if constexpr (LAYOUT == 2) {
    constexpr int ICV = pf_slots<2, IC>() / 4;
    const int64_t j = j0 + 4 * (lane & 15);
    ok = j < J;
    const float4* b = (const float4*)(X + v.fibre_base(ok ? j : J - 4));
    const int64_t q4 = v.Q >> 2;
#pragma unroll
    for (int k = 0; k < ICV; ++k) {
      const int ii = min(32 * k + 4 * w + (lane >> 4), I - 1);
      const float4 x = b[(int64_t)ii * q4];
      pf[4 * k + 0] = x.x;
      pf[4 * k + 1] = x.y;
      pf[4 * k + 2] = x.z;
      pf[4 * k + 3] = x.w;
    }
  } else if (LAYOUT == 0) {
    const int64_t j = j0 + lane;
    ok = j < J;
    const T* b = X + v.fibre_base(ok ? j : J - 1);
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      const int ii = min(NW * k + w, I - 1);
      pf[k] = b[(int64_t)ii * v.Q];
    }
  } else {
    ok = true;
    constexpr int NC = IC / 8;              // 64-row chunks per fibre
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      const int f = k / NC, c = k % NC;
      const int64_t j = min(j0 + w + NW * f, J - 1);
      pf[k] = X[j * I + min(lane + 64 * c, I - 1)];
    }
  }
}

// Rows past I go to the spare row `xrows` of the X tile (no branches).
// With NORM the squares of the tile's elements are added to nsum (FP64).
template <typename T, int LAYOUT, int IC, bool NORM>
__device__ __forceinline__ void stash(const View& v, int64_t j0, int lane, int w, const T* pf,
                                      bool ok, int xrows, float* Xs, double& nsum) {
  const int I = (int)v.I;
  // (the masking of lanes past the last fibre is a bitwise and, not a
  // select: a branch here makes the compiler wait for every load in flight,
  // the next tile's included)
  // (the squares go to four partial sums: one FP64 chain would wait out the
  // FMA latency at every element)
  double ns[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (LAYOUT == 2) {
    constexpr int ICV = pf_slots<2, IC>() / 4;
    const uint32_t keep = ok ? 0xffffffffu : 0u;
#pragma unroll
    for (int k = 0; k < ICV; ++k) {
      const int ii = 32 * k + 4 * w + (lane >> 4);
      const int row = ii < I ? ii : xrows;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, pf[4 * k + e]) & keep);
        Xs[row * XLD + 4 * (lane & 15) + e] = x;
        if (NORM && ii < I) ns[e] += (double)x * (double)x;
      }
    }
  } else if (LAYOUT == 0) {
    const uint32_t keep = ok ? 0xffffffffu : 0u;
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      const int ii = NW * k + w;
      const int row = ii < I ? ii : xrows;
      const float x = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, to_f<T>(pf[k])) & keep);
      Xs[row * XLD + lane] = x;
      if (NORM && ii < I) ns[k & 3] += (double)x * (double)x;
    }
  } else {
    const int64_t J = v.J();
    constexpr int NC = IC / 8;
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      const int f = k / NC, c = k % NC;
      const uint32_t keep = (j0 + w + NW * f < J) ? 0xffffffffu : 0u;
      const int ii = lane + 64 * c;
      const int row = ii < I ? ii : xrows;
      const float x = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, to_f<T>(pf[k])) & keep);
      Xs[row * XLD + w + NW * f] = x;
      if (NORM && ii < I) ns[k & 3] += (double)x * (double)x;
    }
  }
  if (NORM) nsum += (ns[0] + ns[1]) + (ns[2] + ns[3]);
}

// MODE 0: sweep; 1: sweep + explicit residual; 2: init (sketch, no Gram);
// 3: TTM (R-update only, V written to Y).
template <typename T, int NR, int MODE, int LAYOUT, int IC, int RM>
__global__ void __launch_bounds__(NT, 1) k_fused(FusedArgs a) {
  extern __shared__ float smem[];
  static_assert(!RM || NR >= 2, "the RM variant keeps at least one 16-rank tile");
  constexpr int RP = 16 * NR;
  constexpr int RS = rank_stride(RP);        // Lq / Vf row stride
  constexpr int LRS = RP + 1;                // Lr row stride
  constexpr int NG = NR * (NR + 1) / 2;      // Gram output tiles
  constexpr int NRF = RM ? NR - 1 : NR;      // rank tiles on the matrix cores
  constexpr int U1 = (4 * NRF + NW - 1) / NW; // R-update tiles per wave (max)
  constexpr int RT = IC > 16 ? 2 : 1;        // L-update row tiles per wave (MT <= 8 RT)
  constexpr int U2 = RT * NRF;               // L-update tiles per wave
  constexpr int C0 = 16 * NRF;               // first rank of the RM columns
  constexpr int RMW = NW - 4 * NRF;          // RM: waves without an R-update tile
  static_assert(!RM || RMW == 4, "the RM variant's partial buffer holds four waves' sums");
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int MT = (I + 15) / 16;              // 16-row tiles of the mode
  const int xrows = 16 * MT;
  const Lds L = lds_layout(I, NR, MODE, RM != 0);
  float* Xs = smem + L.xs;
  float* Lq = smem + L.lq;
  float* Lr = smem + L.lr;
  float* Vf = smem + L.vf;
  float* Vr = smem + L.vr;

  // ---- once per kernel: zero the X tile (rows >= I stay zero), load Lq/Lr
  for (int e = threadIdx.x; e < (xrows + 1) * XLD; e += NT) Xs[e] = 0.0f;
  if (MODE != 2) {
    const int64_t ldi = a.lq_ldi ? a.lq_ldi : R, ldo = a.lq_ldi ? a.lq_ldo : 1;
    for (int e = threadIdx.x; e < xrows * RP; e += NT) {
      const int i = e / RP, r = e % RP;
      Lq[i * RS + r] = (i < I && r < R) ? a.Lq[i * ldi + r * ldo] : 0.0f;
    }
  }
  if (MODE == 1) {
    for (int e = threadIdx.x; e < xrows * RP; e += NT) {
      const int i = e / RP, r = e % RP;
      Lr[i * LRS + r] = (i < I && r < R) ? -a.Lr[i * R + r] : 0.0f;
    }
  }
  // RM: V columns past C0 + 3 are never written (they stay zero)
  if (RM)
    for (int e = threadIdx.x; e < L.vr - L.vf; e += NT) Vf[e] = 0.0f;

  // R-update tiles: t = w + NW u -> (fibre block t / NRF, rank tile t % NRF)
  const int cnt1 = 4 * NRF > w ? (4 * NRF - w + NW - 1) / NW : 0;
  f4 lacc[U2];
#pragma unroll
  for (int u = 0; u < U2; ++u) lacc[u] = f4{0, 0, 0, 0};
  f4 gacc[NG];
  double gd[NG][4];
#pragma unroll
  for (int p = 0; p < NG; ++p) {
    gacc[p] = f4{0, 0, 0, 0};
    gd[p][0] = gd[p][1] = gd[p][2] = gd[p][3] = 0.0;
  }
  double rsum = 0.0;
  const bool want_norm = MODE == 2 && a.norm2_parts != nullptr;
  // RM: L-update of the last four ranks, wave w: mode rows 64 (w % 4) ..
  // + 63 (block b: rows + 4b ..) over the fibre half w / 4 of every tile
  f4 racc = f4{0.0f, 0.0f, 0.0f, 0.0f}, racc1 = racc;
  const int rgrp = w & 3, rhalf = w >> 2;

  const T* X = (const T*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  const int nwg = gridDim.x;
  // Two register buffers: while a tile is processed from LDS the next two
  // are in flight (two tiles of loads per wave, under the 63-load limit).
  constexpr int PFN = pf_slots<LAYOUT, IC>();
  T pf0[PFN], pf1[PFN];
  bool ok0 = false, ok1 = false;
  int64_t tile = blockIdx.x;
  prefetch<T, LAYOUT, IC>(X, v, tile * TJ, lane, w, pf0, ok0);
  prefetch<T, LAYOUT, IC>(X, v, (tile + nwg) * TJ, lane, w, pf1, ok1);

  auto body = [&](const int64_t tile, T (&pf)[PFN], bool& pf_ok) __attribute__((always_inline)) {
    const int64_t j0 = tile * TJ;
    __syncthreads();
    if (MODE == 2 && want_norm) stash<T, LAYOUT, IC, true>(v, j0, lane, w, pf, pf_ok, xrows, Xs, rsum);
    else stash<T, LAYOUT, IC, false>(v, j0, lane, w, pf, pf_ok, xrows, Xs, rsum);
    __syncthreads();
    // This buffer now fetches the tile after the one the other buffer holds.
    // The older half of the waves issues its loads here; the younger half,
    // whose issue would queue behind theirs, issues after its part of the
    // R-update (the lighter one: with RM they take the four-rank remainder).
    const bool early = w < NW / 2;
    if (early) prefetch<T, LAYOUT, IC>(X, v, (tile + 2 * nwg) * TJ, lane, w, pf, pf_ok);

    if (MODE != 2) {
      // R-update: tile (fibre block f, rank tile n): A = X^T (16 fibres x
      // 4 rows), B = Lq (4 rows x 16 ranks), K = the MT 16-row stages of
      // the tile (rows I..16 MT - 1 of X and Lq are zero).  The operands of
      // the next stage are read before the four MFMAs of the current one.
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        if (u < cnt1) {
          const int t = w + NW * u;
          const int fb = t / NRF, n = t % NRF;
          const float* xa = Xs + lk * XLD + 16 * fb + lr;
          const float* lb = Lq + lk * RS + 16 * n + lr;
          // Two register sets of stage operands in ping-pong: the reads of
          // the next stage are in flight while the current one multiplies,
          // and no register copy forces a wait for them.  Four independent
          // accumulation chains (one per 4-row K step of a stage) are added
          // in a fixed order at the end.
          f4 vq[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) vq[q] = f4{0, 0, 0, 0};
          float a0[4], b0[4], a1[4], b1[4];
          auto ld = [&](float* ca, float* cb, int st) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              ca[q] = xa[(16 * st + 4 * q) * XLD];
              cb[q] = lb[(16 * st + 4 * q) * RS];
            }
          };
          auto mm = [&](const float* ca, const float* cb) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) vq[q] = mfma16(ca[q], cb[q], vq[q]);
          };
          ld(a0, b0, 0);
          int st = 0;
          // (scheduling barriers keep the reads ahead of the products)
          for (; st + 1 < MT; st += 2) {
            ld(a1, b1, st + 1);
            __builtin_amdgcn_sched_barrier(0);
            mm(a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            ld(a0, b0, st + 2 < MT ? st + 2 : MT - 1);
            __builtin_amdgcn_sched_barrier(0);
            mm(a1, b1);
            __builtin_amdgcn_sched_barrier(0);
          }
          if (st < MT) mm(a0, b0);
          const f4 vacc = (vq[0] + vq[1]) + (vq[2] + vq[3]);
          // V[16 fb + 4 lk + q][16 n + lr] = vacc[q]
          if (MODE == 3) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Vf[(16 * n + lr) * (TJ + 1) + 16 * fb + 4 * lk + q] = vacc[q];
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) Vf[(16 * fb + 4 * lk + q) * RS + 16 * n + lr] = vacc[q];
          }
        }
      }
      if (RM && w >= NW - RMW) {
        // the last four ranks on the waves without a 16-rank tile, wave w:
        // fibres 16 w0 .. + 15 (w0 = w - NW + RMW).  Block b = 4c + g: fibres
        // 16 w0 + 4g .. + 3 over the rows congruent to c mod 4, so lane l
        // takes A = X[4s + l / 16][16 w0 + l % 16] and B = Lq[4s + l / 16][C0
        // + l % 4]; the four row classes are added across lanes at the end.
        // Two accumulators take alternate steps (independent products).
        const int w0 = w - (NW - RMW);
        f4 sv0 = f4{0.0f, 0.0f, 0.0f, 0.0f}, sv1 = sv0;
        const float* xa = Xs + lk * XLD + 16 * w0 + lr;
        const float* lb = Lq + lk * RS + C0 + (lane & 3);
        // (xrows is a multiple of 16: a batch of four steps starting below
        // it lies inside it, and its loads go out together)
        for (int k = 0; k < xrows; k += 16) {
          float xv[4], lv[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            xv[b] = xa[(k + 4 * b) * XLD];
            lv[b] = lb[(k + 4 * b) * RS];
          }
          sv0 = mfma4(xv[0], lv[0], sv0);
          sv1 = mfma4(xv[1], lv[1], sv1);
          sv0 = mfma4(xv[2], lv[2], sv0);
          sv1 = mfma4(xv[3], lv[3], sv1);
        }
        f4 sv = sv0 + sv1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sv[q] += __shfl_xor(sv[q], 16, 64);
          sv[q] += __shfl_xor(sv[q], 32, 64);
        }
        // element q of lane l < 16: fibre 16 w0 + 4 (l / 4) + q, rank C0 + l % 4
        if (lane < 16) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int f = 16 * w0 + 4 * (lane >> 2) + q, r = C0 + (lane & 3);
            if (MODE == 3) Vf[r * (TJ + 1) + f] = sv[q];
            else Vf[f * RS + r] = sv[q];
          }
        }
      }
    } else {
      // init: V = the Section 5 sketch rows of this tile
      for (int e = threadIdx.x; e < TJ * RP; e += NT) {
        const int jl = e / RP, r = e % RP;
        const int64_t j = j0 + jl;
        float s = 0.0f;
        if (j < J && r < R)
          s = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        Vf[jl * RS + r] = s;
      }
    }
    if (!early) prefetch<T, LAYOUT, IC>(X, v, (tile + 2 * nwg) * TJ, lane, w, pf, pf_ok);
    __syncthreads();

    if (MODE == 3) {
      // fibre j of Y = B x_n U^T: Y[p, r, q] = V[j, r], coalesced along q
      float* Y = a.y;
      if (LAYOUT != 1) {
        const int64_t j = j0 + lane;
        if (j < J) {
          const int64_t p = j / v.Q, q = j - p * v.Q;
          float* yb = Y + p * (int64_t)R * v.Q + q;
          for (int r = w; r < R; r += NW) {
            yb[(int64_t)r * v.Q] = Vf[r * (TJ + 1) + lane];
          }
        }
      } else {
        for (int e = threadIdx.x; e < TJ * R; e += NT) {
          const int jl = e / R, r = e - jl * R;
          if (j0 + jl < J) Y[(j0 + jl) * R + r] = Vf[r * (TJ + 1) + jl];
        }
      }
      return;
    }

    // L-update: tile (m, n) += X[16m.., f] V[f, 16n..] over the 64 fibres.
    // Wave w owns the row tiles m = w + NW rt (rt < RT; clamped into the
    // mode, duplicates are never stored) for every rank tile n; the RT * NR
    // independent accumulations are interleaved per K step.
    {
      float vb[NRF][16];
#pragma unroll
      for (int n = 0; n < NRF; ++n)
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) vb[n][ks] = Vf[(4 * ks + lk) * RS + 16 * n + lr];
      const float* xr[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int m = min(w + NW * rt, MT - 1);
        xr[rt] = Xs + (16 * m + lr) * XLD + lk;
      }
      float ca[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) ca[rt] = xr[rt][0];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        float na[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) na[rt] = xr[rt][4 * (ks + 1 < 16 ? ks + 1 : ks)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int n = 0; n < NRF; ++n)
            lacc[rt * NRF + n] = mfma16(ca[rt], vb[n][ks], lacc[rt * NRF + n]);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) ca[rt] = na[rt];
      }
      if (RM && 64 * rgrp < xrows) {
        // A = X[64 g + lane][f] (rows past the tile read the spare row; their
        // sums are never stored), B = V[f][C0 + lane % 4]
        const float* xr = Xs + min(64 * rgrp + lane, xrows) * XLD + 32 * rhalf;
        const float* vr = Vf + 32 * rhalf * RS + C0 + (lane & 3);
#pragma unroll
        for (int f0 = 0; f0 < 32; f0 += 8) {
          float xv[8], vv[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            xv[b] = xr[f0 + b];
            vv[b] = vr[(f0 + b) * RS];
          }
#pragma unroll
          for (int b = 0; b < 8; b += 2) {
            racc = mfma4(xv[b], vv[b], racc);
            racc1 = mfma4(xv[b + 1], vv[b + 1], racc1);
          }
        }
      }

      if (MODE != 2) {
        // Gram over fibres 8w..8w+7 (2 K steps), upper block triangle.
        float g[2][NR];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
          for (int n = 0; n < NR; ++n) g[kk][n] = Vf[(8 * w + 4 * kk + lk) * RS + 16 * n + lr];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          int p = 0;
#pragma unroll
          for (int na = 0; na < NR; ++na)
#pragma unroll
            for (int nb = na; nb < NR; ++nb, ++p) gacc[p] = mfma16(g[kk][na], g[kk][nb], gacc[p]);
        }
#pragma unroll
        for (int p = 0; p < NG; ++p) {
#pragma unroll
          for (int q = 0; q < 4; ++q) gd[p][q] += (double)gacc[p][q];
          gacc[p] = f4{0, 0, 0, 0};
        }
      }
    }

    if (MODE == 1) {
      // explicit residual: D = X - L V^T per (16-row tile m, fibre block fb),
      // A = -L (16 rows x 4 ranks), B = V^T (4 ranks x 16 fibres); wave w
      // takes fibre block w % 4 and row tiles m = w / 4 + 2k.
      const int fb = w % 4;
      for (int m = w / 4; m < MT; m += 2) {
        f4 c;
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = Xs[(16 * m + 4 * lk + q) * XLD + 16 * fb + lr];
#pragma unroll
        for (int ks = 0; ks < RP / 4; ++ks)
          c = mfma16(Lr[(16 * m + lr) * LRS + 4 * ks + lk], Vf[(16 * fb + lr) * RS + 4 * ks + lk], c);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (16 * m + 4 * lk + q < I) rsum += (double)c[q] * (double)c[q];
      }
    }
  
  };

  for (; tile + nwg < ntiles; tile += 2 * nwg) {
    body(tile, pf0, ok0);
    body(tile + nwg, pf1, ok1);
  }
  if (tile < ntiles) body(tile, pf0, ok0);

  // ---- per-workgroup outputs
  const int wg = blockIdx.x;
  if (MODE == 3) return;
  if (want_norm) {
    // sum of squares of the tensor (init), one per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rsum += __shfl_xor(rsum, off, 64);
    if (lane == 0) a.norm2_parts[wg * NW + w] = rsum;
  }
  float* lp = a.lacc_parts + (int64_t)wg * I * R;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int m = w + NW * rt;
    if (m < MT) {
#pragma unroll
      for (int n = 0; n < NRF; ++n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * m + 4 * lk + q, r = 16 * n + lr;
          if (i < I && r < R) lp[i * R + r] = lacc[rt * NRF + n][q];
        }
      }
    }
  }
  if (RM) {
    // fibre half 1 (waves 4..7) hands its sums to half 0 through LDS
    racc += racc1;
    if (rhalf == 1) *(f4*)(Vr + (rgrp * 64 + lane) * 4) = racc;
    __syncthreads();
    if (rhalf == 0) {
      const f4 o = racc + *(const f4*)(Vr + (rgrp * 64 + lane) * 4);
      const int r = C0 + (lane & 3);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 64 * rgrp + 4 * (lane >> 2) + q;
        if (i < I && r < R) lp[i * R + r] = o[q];
      }
    }
  }
  if (MODE != 2) {
    // the upper triangle (of the diagonal blocks too) and its mirror cover
    // every entry once, so each partial is exactly symmetric
    double* gp = a.gv_parts + (int64_t)(wg * NW + w) * R * R;
    int p = 0;
#pragma unroll
    for (int na = 0; na < NR; ++na) {
#pragma unroll
      for (int nb = na; nb < NR; ++nb, ++p) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * na + 4 * lk + q, col = 16 * nb + lr;
          if (row < R && col < R && (na < nb || row <= col)) {
            gp[row * R + col] = gd[p][q];
            gp[col * R + row] = gd[p][q];
          }
        }
      }
    }
  }
  if (MODE == 1) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rsum += __shfl_xor(rsum, off, 64);
    if (lane == 0) a.resid_parts[wg * NW + w] = rsum;
  }
}

template <typename T, int NR, int MODE, int IC, int RM>
void launch_ic(const FusedArgs& a, int nwg, size_t bytes, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.v.Q % 4 == 0 && ((uintptr_t)a.X & 15) == 0) {
      (void)hipFuncSetAttribute((const void*)k_fused<T, NR, MODE, 2, IC, RM>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      hipLaunchKernelGGL((k_fused<T, NR, MODE, 2, IC, RM>), dim3(nwg), dim3(NT), bytes, s, a);
      return;
    }
  }
  if (a.v.Q != 1) {
    (void)hipFuncSetAttribute((const void*)k_fused<T, NR, MODE, 0, IC, RM>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused<T, NR, MODE, 0, IC, RM>), dim3(nwg), dim3(NT), bytes, s, a);
  } else if constexpr (IC % 8 == 0) {      // Q == 1 slots are 64-row chunks
    (void)hipFuncSetAttribute((const void*)k_fused<T, NR, MODE, 1, IC, RM>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused<T, NR, MODE, 1, IC, RM>), dim3(nwg), dim3(NT), bytes, s, a);
  }
}

// Row-slot class: 8, 16, 26 or 32 slots per wave (I <= 64, 128, 208, 256;
// the 26-slot class keeps two tiles of loads under the 63 outstanding loads
// of a wave, and is taken only for Q > 1, whose slots are single rows).
template <typename T, int NR, int MODE, int RM = 0>
void launch_mode(const FusedArgs& a, int nwg, size_t bytes, hipStream_t s) {
  if (a.v.I <= 64) launch_ic<T, NR, MODE, 8, RM>(a, nwg, bytes, s);
  else if (a.v.I <= 128) launch_ic<T, NR, MODE, 16, RM>(a, nwg, bytes, s);
  else if (a.v.I <= 208 && a.v.Q != 1) launch_ic<T, NR, MODE, 26, RM>(a, nwg, bytes, s);
  else launch_ic<T, NR, MODE, 32, RM>(a, nwg, bytes, s);
}

constexpr int LDS_MAX_BYTES = 160 * 1024;

// The RM variant: 16 < R <= 20, when its exchange buffer fits (with a third
// rank tile the kernel would spill registers).
bool use_rm(const FusedArgs& a, int NR, int mode) {
  return NR == 2 && a.R - 16 * (NR - 1) <= 4 &&
         (size_t)lds_layout((int)a.v.I, NR, mode, true).total * 4 <= (size_t)LDS_MAX_BYTES;
}

template <typename T, int NR>
int launch_nr(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  const bool rm = use_rm(a, NR, mode);
  const size_t bytes = (size_t)lds_layout((int)a.v.I, NR, mode, rm).total * 4;
  if constexpr (NR == 2) {
    if (rm) {
      if (mode == 0) launch_mode<T, NR, 0, 1>(a, nwg, bytes, s);
      else if (mode == 1) launch_mode<T, NR, 1, 1>(a, nwg, bytes, s);
      else if (mode == 2) launch_mode<T, NR, 2, 1>(a, nwg, bytes, s);
      else launch_mode<T, NR, 3, 1>(a, nwg, bytes, s);
      return nwg;
    }
  }
  if (mode == 0) launch_mode<T, NR, 0>(a, nwg, bytes, s);
  else if (mode == 1) launch_mode<T, NR, 1>(a, nwg, bytes, s);
  else if (mode == 2) launch_mode<T, NR, 2>(a, nwg, bytes, s);
  else launch_mode<T, NR, 3>(a, nwg, bytes, s);
  return nwg;
}

template <typename T>
int launch_t(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  switch ((a.R + 15) / 16) {
    case 1: return launch_nr<T, 1>(a, mode, nwg, s);
    case 2: return launch_nr<T, 2>(a, mode, nwg, s);
    case 3: return launch_nr<T, 3>(a, mode, nwg, s);
  }
  return 0;
}

}  // namespace

bool fused_supported(int x_dtype, const View& v, int R, int resid_mode) {
  if (x_dtype != TK_F32 && x_dtype != TK_BF16) return false;
  if (fused_big_shape(x_dtype, v, R, resid_mode == TK_RESID_EXPLICIT ? 1 : 0)) return true;
  if (v.I > 256 || v.I < 1 || R < 1 || R > 48) return false;
  const int NR = (R + 15) / 16;
  const int mode = resid_mode == TK_RESID_EXPLICIT ? 1 : 0;
  return (size_t)lds_layout((int)v.I, NR, mode).total * 4 <= (size_t)LDS_MAX_BYTES;
}

bool fused_ttm_supported(int x_dtype, const View& v, int64_t J) {
  if (x_dtype != TK_F32 && x_dtype != TK_BF16) return false;
  if (fused_big_shape(x_dtype, v, J, 3)) return true;
  if (v.I > 256 || v.I < 1 || J < 1 || J > 48) return false;
  const int NR = (int)((J + 15) / 16);
  return (size_t)lds_layout((int)v.I, NR, 3).total * 4 <= (size_t)LDS_MAX_BYTES;
}

int fused_workgroups(const View& v) {
  int64_t ntiles = ceil_div(v.J(), TJ);
  return (int)(ntiles < NWG ? ntiles : NWG);
}

int launch_fused(const FusedArgs& a, int nwg_max, hipStream_t s) {
  int nwg = fused_workgroups(a.v);
  if (nwg > nwg_max / NW) nwg = nwg_max / NW;
  const int mode = a.y ? 3 : a.sketch ? 2 : (a.Lr ? 1 : 0);
  if (fused_bf16_big_supported(a, mode)) return launch_fused_bf16_big(a, mode, nwg_max, s);
  if (fused_big_shape(a.x_dtype, a.v, a.R, mode)) return launch_fused_big(a, mode, nwg_max, s);
  if (fused_bf16_supported(a, mode)) return launch_fused_bf16(a, mode, nwg_max, s);
  if (a.x_dtype == TK_F32) return launch_t<float>(a, mode, nwg, s);
  return launch_t<bf16_t>(a, mode, nwg, s);
}

}  // namespace tk
