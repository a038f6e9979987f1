// Fused ALS sweep for BF16 storage on the gfx950 BF16 matrix cores.
//
// Same products as k_fused.hip (one read of every fibre a_j per sweep,
// row-wise rule of Section 3):  v_j = Lq^T a_j,  G_V += v_j v_j^T,
// L_acc += a_j v_j^T; the init variant uses the Section 5 sketch rows for
// v_j (and adds up ||A||^2), the TTM variant writes v_j out as fibre j of
// B x_n U^T.  The tensor is BF16, so its products with BF16 operands are
// exact in FP32.  The FP32 operands (Lq, V, the sketch) are split exactly
// into three BF16 terms (h + m + l equals the FP32 value: each split
// removes the leading 8 significant bits of a 24-bit significand), so every
// product is the exact FP32-operand product and only the order of the FP32
// accumulation differs from the FP32 matrix-core path.  G_V stays on the
// FP32 matrix cores from the FP32 V (the trace residual needs it).
//
// A sweep whose Lq is already rounded to BF16 precision (the drivers quantise
// L~ so for BF16 storage, the trace residual taking the Gram of the rounded
// values) multiplies by its single BF16 term instead of three.
//
// Work layout: 256 persistent workgroups of 8 waves walk tiles of TJ = 128
// fibres (view [P, I, Q] with Q even: each lane loads one dword holding two
// adjacent fibres of a row; the register-resident variant below loads
// eight adjacent fibres, 16 bytes, when Q is a multiple of 8).  The tile is
// kept in LDS as BF16 rows whose 16-byte chunks are XOR-swizzled by row;
// the L-update reads contiguous 16-byte runs of fibres.
//   R-update  wave w owns fibre block w (16 fibres) for every rank tile:
//             v_mfma_f32_16x16x32_bf16, A = X^T (16 fibres x 32 rows, two
//             transposing LDS reads per operand), B = Lq^T splits (32 rows x
//             16 ranks), K = 32-row stages;
//   L-update  wave w owns row tiles w + 8 rt for every rank tile:
//             v_mfma_f32_16x16x32_bf16, A = X (16 rows x 32 fibres), B = V
//             splits (32 fibres x 16 ranks), K = the 128 fibres;
//   Gram      v_mfma_f32_16x16x4f32 on the FP32 V, wave w: fibres 16w..16w+15.
// Every reduction has a fixed order (deterministic, no atomics).
#include "tk_kernels.h"

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s4 lds_s4;

namespace {

constexpr int NT = 512;
constexpr int NW = NT / 64;
static_assert(NW == FUSED_WAVES, "partial buffers are sized for FUSED_WAVES waves");
constexpr int TJ = 128;            // fibres per tile
constexpr int XS = TJ + 8;         // LDS row stride of the tile (BF16 elements)
constexpr int VS = TJ + 8;         // row stride of the V^T splits
constexpr int NWG = 256;

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// v = h + m + l exactly (three round-to-nearest BF16 terms).
__device__ __forceinline__ void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)v;
  const float r1 = v - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

__host__ __device__ constexpr int rank_stride(int RP) { return (RP % 32 == 0) ? RP + 16 : RP; }

// Element (row, fibre f) of the swizzled tile: 16-byte chunk f / 8 of the
// row is stored at chunk (f / 8) ^ (2 ((row / 8) & 3)).
__device__ __forceinline__ int xidx(int row, int f) {
  return row * XS + ((((f >> 3) ^ (((row >> 3) & 3) << 1))) << 3) + (f & 7);
}

// The R-update's A operand: rows row0 .. row0 + 7 (row0 a multiple of 8) of
// fibre f0 + j (j = lane % 16) of a tile, from two transposing LDS reads
// (ds_read_b64_tr_b16): lane j of each 16-lane group points at the four
// fibres f0 + 4 (j % 4) .. + 3 of row r0 + j / 4 and receives fibre f0 + j of
// rows r0 .. r0 + 3.  The swizzle moves whole 8-fibre chunks and is the same
// for the eight rows, so the four fibres stay contiguous and the second
// read is four rows on.
__device__ __forceinline__ bf8 rows8(const __bf16* x, int row0, int f0, int j) {
  const __bf16* p0 = x + xidx(row0 + (j >> 2), f0 + 4 * (j & 3));
  const s4 u0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(p0));
  const s4 u1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(p0 + 4 * XS));
  // (one whole-vector shuffle: element-wise inserts of these values are not
  // reliably compiled)
  return __builtin_bit_cast(bf8, __builtin_shufflevector(u0, u1, 0, 1, 2, 3, 4, 5, 6, 7));
}

struct LdsB {
  int xs, lq, vt, vf, total;  // offsets in bytes
};

__host__ __device__ inline LdsB lds_b16(int I, int NR, int mode) {
  const int RP = 16 * NR;
  const int XR = 32 * ((I + 31) / 32);
  const int LS = XR + 8;
  LdsB l;
  l.xs = 0;
  l.lq = l.xs + (XR + 1) * XS * 2;                        // + spare row
  l.vt = l.lq + (mode != 2 ? 3 * RP * LS * 2 : 0);
  l.vf = l.vt + (mode != 3 ? 3 * RP * VS * 2 : 0);
  const int vf_floats = mode == 0 ? TJ * rank_stride(RP) : (mode == 3 ? RP * (TJ + 1) : 0);
  l.total = l.vf + vf_floats * 4;
  return l;
}

// Prefetch: slot k is row 8k + w (clamped) of the fibre pair j0 + 2 lane,
// j0 + 2 lane + 1 (one dword; Q even keeps pairs inside one p and aligned).
// Lanes past the end read the last pair and are zeroed in the stash, so a
// tile wholly past the end is fetched (in bounds) and staged as zeros.
template <int IC>
__device__ __forceinline__ void prefetch(const uint32_t* __restrict__ X2, const View& v,
                                         int64_t j0, int lane, int w, uint32_t* pf, bool& ok) {
  const int64_t J = v.J();
  const int I = (int)v.I;
  const int64_t j = j0 + 2 * lane;
  ok = j < J;
  const uint32_t* b = X2 + (v.fibre_base(ok ? j : J - 2) >> 1);
  const int64_t q2 = v.Q >> 1;
#pragma unroll
  for (int k = 0; k < IC; ++k) {
    const int ii = min(NW * k + w, I - 1);
    pf[k] = b[(int64_t)ii * q2];
  }
}

template <int IC, bool NORM>
__device__ __forceinline__ void stash(const View& v, int lane, int w, const uint32_t* pf,
                                      bool ok, int XR, uint32_t* Xs32, double& nsum) {
  const int I = (int)v.I;
  // (the squares go to four partial sums: one FP64 chain would wait out the
  // FMA latency at every element)
  double ns[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < IC; ++k) {
    const int ii = NW * k + w;
    const int row = ii < I ? ii : XR;
    const uint32_t x = ok ? pf[k] : 0u;
    Xs32[xidx(row, 2 * lane) >> 1] = x;
    if (NORM && ii < I) {
      const float a = bf16_to_f32((bf16_t)(x & 0xffffu)), b = bf16_to_f32((bf16_t)(x >> 16));
      ns[k & 3] += (double)a * (double)a + (double)b * (double)b;
    }
  }
  if (NORM) nsum += (ns[0] + ns[1]) + (ns[2] + ns[3]);
}

// 16-byte form of the prefetch (Q a multiple of 8, 16-byte aligned tensor):
// slot k is row 32k + 4w + lane / 16 (clamped) of the eight fibres
// j0 + 8 (lane % 16) .. + 7, in pf[4k .. 4k + 3] (the same registers as the
// dword form's 4 NSL slots, with a quarter of its load instructions).  The
// eight never cross a row of the view, and a tile past the end is fetched in
// bounds and staged as zeros.
template <int NSL>
__device__ __forceinline__ void prefetch16(const uint4* __restrict__ X16, const View& v,
                                           int64_t j0, int lane, int w, uint32_t* pf, bool& ok) {
  const int64_t J = v.J();
  const int I = (int)v.I;
  const int64_t j = j0 + 8 * (lane & 15);
  ok = j < J;
  const uint4* b = X16 + (v.fibre_base(ok ? j : J - 8) >> 3);
  const int64_t q8 = v.Q >> 3;
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int ii = min(32 * k + 4 * w + (lane >> 4), I - 1);
    const uint4 x = b[(int64_t)ii * q8];
    pf[4 * k + 0] = x.x;
    pf[4 * k + 1] = x.y;
    pf[4 * k + 2] = x.z;
    pf[4 * k + 3] = x.w;
  }
}

// Stage the 16-byte slots: one 16-byte LDS store per slot (the swizzle moves
// whole 8-fibre chunks); rows past I go to the spare row XR.
template <int NSL, bool NORM>
__device__ __forceinline__ void stash16(const View& v, int lane, int w, const uint32_t* pf,
                                        bool ok, int XR, __bf16* Xb, double& nsum) {
  const int I = (int)v.I;
  const uint32_t keep = ok ? 0xffffffffu : 0u;
  double ns[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NSL; ++k) {
    const int ii = 32 * k + 4 * w + (lane >> 4);
    const int row = ii < I ? ii : XR;
    const uint4 x = make_uint4(pf[4 * k] & keep, pf[4 * k + 1] & keep, pf[4 * k + 2] & keep,
                               pf[4 * k + 3] & keep);
    *(uint4*)(Xb + xidx(row, 8 * (lane & 15))) = x;
    if (NORM && ii < I) {
      const uint32_t d[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float lo = bf16_to_f32((bf16_t)(d[e] & 0xffffu)), hi = bf16_to_f32((bf16_t)(d[e] >> 16));
        ns[e] += (double)lo * (double)lo + (double)hi * (double)hi;
      }
    }
  }
  if (NORM) nsum += (ns[0] + ns[1]) + (ns[2] + ns[3]);
}

// MODE 0: sweep; 2: init (sketch, norm, no Gram); 3: TTM.  NS: BF16 terms of
// Lq in the R-update (1 when the Lq values are BF16-representable, else 3).
template <int NR, int MODE, int IC, int NS>
__global__ void __launch_bounds__(NT, 1) k_fused_bf16(FusedArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int RP = 16 * NR;
  constexpr int RS = rank_stride(RP);
  constexpr int NG = NR * (NR + 1) / 2;
  constexpr int RT = IC == 32 ? 2 : 1;        // L-update row tiles per wave (MT <= 8 RT)
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int XR = 32 * ((I + 31) / 32);
  const int LS = XR + 8;
  const int MT = (I + 15) / 16;               // 16-row tiles of the mode (L-update)
  const int ST = XR / 32;                     // 32-row stages (R-update)
  const LdsB L = lds_b16(I, NR, MODE);
  __bf16* Xs = (__bf16*)(smem + L.xs);
  uint32_t* Xs32 = (uint32_t*)(smem + L.xs);
  __bf16* Lq = (__bf16*)(smem + L.lq);        // [3][RP][LS]: Lq^T splits
  __bf16* Vt = (__bf16*)(smem + L.vt);        // [3][RP][VS]: V^T splits
  float* Vf = (float*)(smem + L.vf);

  // ---- once per kernel: zero the tile (rows I..XR-1 stay zero), Lq splits
  for (int e = threadIdx.x; e < (XR + 1) * XS / 2; e += NT) Xs32[e] = 0u;
  if (MODE != 2) {
    const int64_t ldi = a.lq_ldi ? a.lq_ldi : R, ldo = a.lq_ldi ? a.lq_ldo : 1;
    for (int e = threadIdx.x; e < RP * LS; e += NT) {
      const int r = e / LS, i = e - r * LS;
      const float x = (i < I && r < R) ? a.Lq[i * ldi + r * ldo] : 0.0f;
      __bf16 h, m, l;
      split3(x, h, m, l);
      Lq[(0 * RP + r) * LS + i] = h;
      Lq[(1 * RP + r) * LS + i] = m;
      Lq[(2 * RP + r) * LS + i] = l;
    }
  }

  f4 lacc[RT][NR];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int n = 0; n < NR; ++n) lacc[rt][n] = f4{0, 0, 0, 0};
  f4 gacc[NG];
  double gd[NG][4];
#pragma unroll
  for (int p = 0; p < NG; ++p) {
    gacc[p] = f4{0, 0, 0, 0};
    gd[p][0] = gd[p][1] = gd[p][2] = gd[p][3] = 0.0;
  }
  double nsum = 0.0;
  const bool want_norm = MODE == 2 && a.norm2_parts != nullptr;

  const uint32_t* X2 = (const uint32_t*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  const int nwg = gridDim.x;
  uint32_t pf0[IC], pf1[IC];
  bool ok0 = false, ok1 = false;
  int64_t tile = blockIdx.x;
  if (tile < ntiles) prefetch<IC>(X2, v, tile * TJ, lane, w, pf0, ok0);
  if (tile + nwg < ntiles) prefetch<IC>(X2, v, (tile + nwg) * TJ, lane, w, pf1, ok1);

  auto body = [&](const int64_t tile, uint32_t (&pf)[IC], bool& pf_ok) __attribute__((always_inline)) {
    const int64_t j0 = tile * TJ;
    __syncthreads();
    if (MODE == 2 && want_norm) stash<IC, true>(v, lane, w, pf, pf_ok, XR, Xs32, nsum);
    else stash<IC, false>(v, lane, w, pf, pf_ok, XR, Xs32, nsum);
    __syncthreads();
    if (tile + 2 * nwg < ntiles) prefetch<IC>(X2, v, (tile + 2 * nwg) * TJ, lane, w, pf, pf_ok);

    if (MODE != 2) {
      // R-update: fibre block w, all rank tiles; A = the eight rows
      // 32 st + 8 lk + e of fibre 16 w + lr (one swizzled column), B = the
      // three Lq^T splits of rank 16 n + lr over the same rows.
      f4 vacc[NR];
#pragma unroll
      for (int n = 0; n < NR; ++n) vacc[n] = f4{0, 0, 0, 0};
      for (int st = 0; st < ST; ++st) {
        const int row0 = 32 * st + 8 * lk;
        const bf8 av = rows8(Xs, row0, 16 * w, lr);
#pragma unroll
        for (int n = 0; n < NR; ++n) {
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const bf8 bv = *(const bf8*)(Lq + (s * RP + 16 * n + lr) * LS + row0);
            vacc[n] = mfma_bf16(av, bv, vacc[n]);
          }
        }
      }
      // V[16 w + 4 lk + q][16 n + lr] = vacc[n][q]
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        if (MODE == 3) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Vf[(16 * n + lr) * (TJ + 1) + 16 * w + 4 * lk + q] = vacc[n][q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) Vf[(16 * w + 4 * lk + q) * RS + 16 * n + lr] = vacc[n][q];
          __bf16 h[4], m[4], l[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) split3(vacc[n][q], h[q], m[q], l[q]);
          const int o = (16 * n + lr) * VS + 16 * w + 4 * lk;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            Vt[0 * RP * VS + o + q] = h[q];
            Vt[1 * RP * VS + o + q] = m[q];
            Vt[2 * RP * VS + o + q] = l[q];
          }
        }
      }
    } else {
      // init: V = the Section 5 sketch rows of this tile (24-bit values,
      // split exactly)
      for (int e = threadIdx.x; e < TJ * RP; e += NT) {
        const int jl = e / RP, r = e - (e / RP) * RP;
        const int64_t j = j0 + jl;
        float s = 0.0f;
        if (j < J && r < R)
          s = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        __bf16 h, m, l;
        split3(s, h, m, l);
        Vt[(0 * RP + r) * VS + jl] = h;
        Vt[(1 * RP + r) * VS + jl] = m;
        Vt[(2 * RP + r) * VS + jl] = l;
      }
    }
    __syncthreads();

    if (MODE == 3) {
      // fibre j of Y = B x_n U^T: Y[p, r, q] = V[j, r], coalesced along q
      float* Y = a.y;
      for (int half = 0; half < 2; ++half) {
        const int jl = lane + 64 * half;
        const int64_t j = j0 + jl;
        if (j < J) {
          const int64_t p = j / v.Q, q = j - p * v.Q;
          float* yb = Y + p * (int64_t)R * v.Q + q;
          for (int r = w; r < R; r += NW) yb[(int64_t)r * v.Q] = Vf[r * (TJ + 1) + jl];
        }
      }
      return;
    }

    // L-update: row tiles m = w + 8 rt (clamped; duplicates never stored),
    // every rank tile, K = the 128 fibres in 4 steps of 32.
    {
      const __bf16* xr[RT];
      int rowm[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int m = min(w + NW * rt, MT - 1);
        rowm[rt] = 16 * m + lr;
        xr[rt] = Xs;
      }
#pragma unroll
      for (int ks = 0; ks < TJ / 32; ++ks) {
        bf8 av[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          av[rt] = *(const bf8*)(xr[rt] + xidx(rowm[rt], 32 * ks + 8 * lk));
#pragma unroll
        for (int n = 0; n < NR; ++n) {
#pragma unroll
          for (int s = 0; s < 3; ++s) {
            const bf8 bv = *(const bf8*)(Vt + (s * RP + 16 * n + lr) * VS + 32 * ks + 8 * lk);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) lacc[rt][n] = mfma_bf16(av[rt], bv, lacc[rt][n]);
          }
        }
      }
    }

    if (MODE == 0) {
      // Gram over fibres 16w..16w+15 (4 K steps), upper block triangle.
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        float g[NR];
#pragma unroll
        for (int n = 0; n < NR; ++n) g[n] = Vf[(16 * w + 4 * kk + lk) * RS + 16 * n + lr];
        int p = 0;
#pragma unroll
        for (int na = 0; na < NR; ++na)
#pragma unroll
          for (int nb = na; nb < NR; ++nb, ++p) gacc[p] = mfma_f32(g[na], g[nb], gacc[p]);
      }
#pragma unroll
      for (int p = 0; p < NG; ++p) {
#pragma unroll
        for (int q = 0; q < 4; ++q) gd[p][q] += (double)gacc[p][q];
        gacc[p] = f4{0, 0, 0, 0};
      }
    }
  };

  for (; tile < ntiles; tile += 2 * nwg) {
    body(tile, pf0, ok0);
    if (tile + nwg < ntiles) body(tile + nwg, pf1, ok1);
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
  for (int rt = 0; rt < RT; ++rt) {
    const int m = w + NW * rt;
    if (m < MT) {
#pragma unroll
      for (int n = 0; n < NR; ++n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * m + 4 * lk + q, r = 16 * n + lr;
          if (i < I && r < R) lp[i * R + r] = lacc[rt][n][q];
        }
      }
    }
  }
  if (MODE == 0) {
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
}

// ---------------------------------------------------------------------------
// Variant for R <= 32 (NR = 1, 2) and 32 * ceil(I / 32) <= 224: wave w owns
// rank tile n = w % NR and the fibre blocks w / NR + (8 / NR) b, b < NR, so
// its three Lq^T splits (the R-update B operands of every 32-row stage)
// stay in registers for the whole launch; G_V comes from the V splits on
// the BF16 matrix cores (the six products h h, h m, m h, h l, l h, m m: the
// three dropped ones are below FP32 rounding); and the tile is double
// buffered in LDS, so the stash of the next tile overlaps this tile's
// R-update.  Two barriers per tile.  The sweep's L-update multiplies by the
// two leading BF16 terms of V (16 significant bits: 2^-17 relative, far below
// the tensor's own BF16 rounding); the Gram keeps the six exact split
// products, which the trace residual needs.

constexpr int XR_MAX_R = 224;

// Tile rows of the size class: 64, 128 or 224 (I <= 64, 128, 224), the
// rows past I zero, so the R-update runs a fixed number of 32-row stages.
__host__ __device__ constexpr int xrows_r(int IC) { return IC == 32 ? XR_MAX_R : 4 * 8 * (IC / 4); }

__host__ __device__ inline LdsB lds_b16r(int IC, int NR, int mode) {
  const int RP = 16 * NR;
  const int XR = xrows_r(IC);
  LdsB l;
  l.xs = 0;
  l.lq = 2 * (XR + 1) * XS * 2;            // end of the two tile buffers
  l.vt = l.lq;
  l.vf = l.vt + (mode != 3 ? 3 * RP * VS * 2 : 0);
  l.total = l.vf + (mode == 3 ? RP * (TJ + 1) * 4 : 0);
  return l;
}

// V16: the 16-byte prefetch form (else one dword of two fibres per slot).
template <int NR, int MODE, int IC, int NS, bool V16>
__global__ void __launch_bounds__(NT, 1) k_fused_bf16r(FusedArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int RP = 16 * NR;
  constexpr int NG = NR * (NR + 1) / 2;
  constexpr int RT = IC == 32 ? 2 : 1;        // L-update row tiles per wave
  // row slots per wave and 32-row stages of the size class
  constexpr int XR = xrows_r(IC);
  constexpr int ICR = XR / NW;
  constexpr int STM = XR / 32;
  // a second register buffer of tile loads, where the registers allow it
  constexpr bool DB = !(MODE == 0 && NS == 3 && IC == 32);
  // BF16 terms of V in the L-update: the sweep takes V to 16 significant
  // bits (h + m; 2^-17 relative, far below the tensor's own BF16 rounding),
  // the init pass the exact three terms of the sketch
  constexpr int NSV = MODE == 2 ? 3 : 2;
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int MT = (I + 15) / 16;
  const int nw = w % NR;                      // rank tile of this wave (R-update)
  const LdsB L = lds_b16r(IC, NR, MODE);
  const int xbuf = (XR + 1) * XS;             // elements per tile buffer
  __bf16* Xs = (__bf16*)(smem + L.xs);
  uint32_t* Xs32 = (uint32_t*)(smem + L.xs);
  __bf16* Vt = (__bf16*)(smem + L.vt);        // [3][RP][VS]
  float* Vf = (float*)(smem + L.vf);          // TTM: [RP][TJ + 1]

  for (int e = threadIdx.x; e < xbuf; e += NT) Xs32[e] = 0u;   // both buffers

  // Lq^T splits of rank 16 nw + lr, rows 32 st + 8 lk + e, as B operands (the
  // first NS of the three)
  bf8 bq[STM][NS];
  if (MODE != 2) {
    const int64_t ldi = a.lq_ldi ? a.lq_ldi : R, ldo = a.lq_ldi ? a.lq_ldo : 1;
    const int r = 16 * nw + lr;
#pragma unroll
    for (int st = 0; st < STM; ++st) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 32 * st + 8 * lk + e;
        const float x = (row < I && r < R) ? a.Lq[row * ldi + r * ldo] : 0.0f;
        __bf16 sp[3];
        split3(x, sp[0], sp[1], sp[2]);
#pragma unroll
        for (int s3 = 0; s3 < NS; ++s3) bq[st][s3][e] = sp[s3];
      }
    }
  }

  f4 lacc[RT][NR];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int n = 0; n < NR; ++n) lacc[rt][n] = f4{0, 0, 0, 0};
  // G_V: unit w < 2 NG of wave w is block pair w / 2 = (gna, gnb), 32-fibre
  // K step w % 2 of every tile
  static_assert(2 * NG <= NW, "one G_V unit per wave");
  const bool gown = w < 2 * NG;
  int gna = 0, gnb = 0;
  for (int x = 0, q = 0; x < NR; ++x)
    for (int y = x; y < NR; ++y, ++q)
      if (q == (w >> 1)) { gna = x; gnb = y; }
  double gd[4] = {0.0, 0.0, 0.0, 0.0};
  double nsum = 0.0;
  const bool want_norm = MODE == 2 && a.norm2_parts != nullptr;

  const uint32_t* X2 = (const uint32_t*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  const int nwg = gridDim.x;
  // Two register buffers (DB) keep the loads of two tiles in flight: the
  // buffer stashed for tile t + nwg then fetches tile t + 3 nwg.  Every
  // prefetch and stash is unconditional (tiles past the end are fetched in
  // bounds and staged as zeros, so they add nothing), and the loop has one
  // shape, so the wait before a stash leaves the other buffer's loads in
  // flight.  Without DB (register budget) one buffer fetches t + 2 nwg.
  constexpr int NB = DB ? 2 : 1;
  uint32_t pf0[ICR], pf1[ICR];
  bool ok0 = false, ok1 = false;
  int64_t tile = blockIdx.x;
  int cur = 0;
  auto fetch = [&](int64_t j0, uint32_t (&pf)[ICR], bool& ok) __attribute__((always_inline)) {
    if constexpr (V16) prefetch16<XR / 32>((const uint4*)a.X, v, j0, lane, w, pf, ok);
    else prefetch<ICR>(X2, v, j0, lane, w, pf, ok);
  };
  // stage a register buffer into tile buffer `buf`
  auto put = [&](const uint32_t (&pf)[ICR], bool ok, int buf) __attribute__((always_inline)) {
    if constexpr (V16) {
      __bf16* Xb = Xs + buf * xbuf;
      if (want_norm) stash16<XR / 32, true>(v, lane, w, pf, ok, XR, Xb, nsum);
      else stash16<XR / 32, false>(v, lane, w, pf, ok, XR, Xb, nsum);
    } else {
      uint32_t* Xb32 = Xs32 + buf * (xbuf >> 1);
      if (want_norm) stash<ICR, true>(v, lane, w, pf, ok, XR, Xb32, nsum);
      else stash<ICR, false>(v, lane, w, pf, ok, XR, Xb32, nsum);
    }
  };
  __syncthreads();
  if (tile < ntiles) {
    fetch(tile * TJ, pf0, ok0);
    put(pf0, ok0, 0);
    fetch((tile + nwg) * TJ, pf0, ok0);
    if (DB) fetch((tile + 2 * nwg) * TJ, pf1, ok1);
  }
  __syncthreads();

  auto body = [&](const int64_t tile, uint32_t (&pf)[ICR], bool& pf_ok)
                  __attribute__((always_inline)) {
    const int64_t j0 = tile * TJ;
    const __bf16* Xc = Xs + cur * xbuf;

    // ---- phase A: R-update (or sketch rows) of this tile; stash the next
    if (MODE != 2) {
      f4 vacc[NR];
#pragma unroll
      for (int b = 0; b < NR; ++b) vacc[b] = f4{0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < STM; ++st) {
        const int row0 = 32 * st + 8 * lk;
#pragma unroll
        for (int b = 0; b < NR; ++b) {
          const bf8 av = rows8(Xc, row0, 16 * (w / NR + (NW / NR) * b), lr);
#pragma unroll
          for (int s3 = 0; s3 < NS; ++s3) vacc[b] = mfma_bf16(av, bq[st][s3], vacc[b]);
        }
      }
      // V[16 fb + 4 lk + q][16 nw + lr] = vacc[b][q]
#pragma unroll
      for (int b = 0; b < NR; ++b) {
        const int fq = 16 * (w / NR + (NW / NR) * b) + 4 * lk;
        if (MODE == 3) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Vf[(16 * nw + lr) * (TJ + 1) + fq + q] = vacc[b][q];
        } else {
          bf16_t hs[4], ms[4], ls[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            __bf16 h, m, l;
            split3(vacc[b][q], h, m, l);
            hs[q] = __builtin_bit_cast(bf16_t, h);
            ms[q] = __builtin_bit_cast(bf16_t, m);
            ls[q] = __builtin_bit_cast(bf16_t, l);
          }
          const int o = (16 * nw + lr) * VS + fq;          // 8-byte aligned
          uint2* d0 = (uint2*)(Vt + 0 * RP * VS + o);
          uint2* d1 = (uint2*)(Vt + 1 * RP * VS + o);
          uint2* d2 = (uint2*)(Vt + 2 * RP * VS + o);
          *d0 = make_uint2(hs[0] | ((uint32_t)hs[1] << 16), hs[2] | ((uint32_t)hs[3] << 16));
          *d1 = make_uint2(ms[0] | ((uint32_t)ms[1] << 16), ms[2] | ((uint32_t)ms[3] << 16));
          *d2 = make_uint2(ls[0] | ((uint32_t)ls[1] << 16), ls[2] | ((uint32_t)ls[3] << 16));
        }
      }
    } else {
      for (int e = threadIdx.x; e < TJ * RP; e += NT) {
        const int jl = e / RP, r = e - (e / RP) * RP;
        const int64_t j = j0 + jl;
        float sv = 0.0f;
        if (j < J && r < R)
          sv = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
        __bf16 h, m, l;
        split3(sv, h, m, l);
        Vt[(0 * RP + r) * VS + jl] = h;
        Vt[(1 * RP + r) * VS + jl] = m;
        Vt[(2 * RP + r) * VS + jl] = l;
      }
    }
    {
      // the next tile (zeros past the end; a duplicate norm term cannot
      // arise: lanes past the end add nothing)
      put(pf, pf_ok, cur ^ 1);
    }
    // The buffer just staged fetches the tile NB + 1 steps ahead (past the
    // end of the tensor by at most (NB + 1) nwg tiles: the clamp keeps the
    // fibre index valid).  The older half of the waves issues its loads
    // here; in the sweep and the TTM the younger half, whose issue would
    // queue behind theirs, issues at the end of phase B (the buffer is next
    // staged NB tiles later).  The init pass's phase B is the same L-update
    // on every wave, so there all waves issue here.
    const int64_t ahead = tile + (NB + 1) * (int64_t)nwg;
    const bool early = MODE == 2 || w < NW / 2;
    if (early) fetch((ahead < ntiles ? ahead : ntiles) * TJ, pf, pf_ok);
    __syncthreads();

    // ---- phase B
    if (MODE == 3) {
      float* Y = a.y;
      for (int half = 0; half < 2; ++half) {
        const int jl = lane + 64 * half;
        const int64_t j = j0 + jl;
        if (j < J) {
          const int64_t p = j / v.Q, q = j - p * v.Q;
          float* yb = Y + p * (int64_t)R * v.Q + q;
          for (int r = w; r < R; r += NW) yb[(int64_t)r * v.Q] = Vf[r * (TJ + 1) + jl];
        }
      }
    } else {
      // L-update: row tiles m = w + 8 rt (clamped; duplicates never stored)
      int rowm[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) rowm[rt] = 16 * min(w + NW * rt, MT - 1) + lr;
#pragma unroll
      for (int ks = 0; ks < TJ / 32; ++ks) {
        bf8 av[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) av[rt] = *(const bf8*)(Xc + xidx(rowm[rt], 32 * ks + 8 * lk));
#pragma unroll
        for (int n = 0; n < NR; ++n) {
#pragma unroll
          for (int s3 = 0; s3 < NSV; ++s3) {
            const bf8 bv = *(const bf8*)(Vt + (s3 * RP + 16 * n + lr) * VS + 32 * ks + 8 * lk);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) lacc[rt][n] = mfma_bf16(av[rt], bv, lacc[rt][n]);
          }
        }
      }
      if (MODE == 0 && gown) {
        // this wave's G_V unit: the six split products above FP32 rounding
        // (K step (w % 2) of the tile's fibres: two 32-fibre halves of the
        // 128, i.e. fibres 64 (w % 2) .. + 63 in two 32-fibre steps)
        f4 g = f4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < TJ / 64; ++kk) {
          const int ko = 64 * (w & 1) + 32 * kk + 8 * lk;
          const bf8 ah = *(const bf8*)(Vt + (0 * RP + 16 * gna + lr) * VS + ko);
          const bf8 am = *(const bf8*)(Vt + (1 * RP + 16 * gna + lr) * VS + ko);
          const bf8 al = *(const bf8*)(Vt + (2 * RP + 16 * gna + lr) * VS + ko);
          const bf8 bh = *(const bf8*)(Vt + (0 * RP + 16 * gnb + lr) * VS + ko);
          const bf8 bm = *(const bf8*)(Vt + (1 * RP + 16 * gnb + lr) * VS + ko);
          const bf8 bl = *(const bf8*)(Vt + (2 * RP + 16 * gnb + lr) * VS + ko);
          g = mfma_bf16(ah, bh, g);
          g = mfma_bf16(ah, bm, g);
          g = mfma_bf16(am, bh, g);
          g = mfma_bf16(ah, bl, g);
          g = mfma_bf16(al, bh, g);
          g = mfma_bf16(am, bm, g);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) gd[q] += (double)g[q];
      }
    }
    if (!early) fetch((ahead < ntiles ? ahead : ntiles) * TJ, pf, pf_ok);
    __syncthreads();
    cur ^= 1;
  };
  if (DB) {
    for (; tile < ntiles; tile += 2 * nwg) {
      body(tile, pf0, ok0);
      body(tile + nwg, pf1, ok1);
    }
  } else {
    for (; tile < ntiles; tile += nwg) body(tile, pf0, ok0);
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
  for (int rt = 0; rt < RT; ++rt) {
    const int m = w + NW * rt;
    if (m < MT) {
#pragma unroll
      for (int n = 0; n < NR; ++n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * m + 4 * lk + q, r = 16 * n + lr;
          if (i < I && r < R) lp[i * R + r] = lacc[rt][n][q];
        }
      }
    }
  }
  if (MODE == 0) {
    // this wave's G_V partial: its block pair (each diagonal block's upper
    // triangle and its mirror, so it is exactly symmetric), zero elsewhere
    double* gp = a.gv_parts + (int64_t)(wg * NW + w) * R * R;
    for (int e = lane; e < R * R; e += 64) gp[e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (gown) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * gna + 4 * lk + q, col = 16 * gnb + lr;
        if (row < R && col < R && (gna < gnb || row <= col)) {
          gp[row * R + col] = gd[q];
          gp[col * R + row] = gd[q];
        }
      }
    }
  }
}

template <int NR, int MODE, int IC, int NS>
void launch3r(const FusedArgs& a, int nwg, hipStream_t s) {
  const size_t bytes = (size_t)lds_b16r(IC, NR, MODE).total;
  if (a.v.Q % 8 == 0 && ((uintptr_t)a.X & 15) == 0) {
    (void)hipFuncSetAttribute((const void*)k_fused_bf16r<NR, MODE, IC, NS, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_fused_bf16r<NR, MODE, IC, NS, true>), dim3(nwg), dim3(NT), bytes, s, a);
    return;
  }
  (void)hipFuncSetAttribute((const void*)k_fused_bf16r<NR, MODE, IC, NS, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  hipLaunchKernelGGL((k_fused_bf16r<NR, MODE, IC, NS, false>), dim3(nwg), dim3(NT), bytes, s, a);
}

template <int NR, int MODE, int IC, int NS>
void launch3(const FusedArgs& a, int nwg, hipStream_t s) {
  const size_t bytes = (size_t)lds_b16((int)a.v.I, NR, MODE).total;
  (void)hipFuncSetAttribute((const void*)k_fused_bf16<NR, MODE, IC, NS>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  hipLaunchKernelGGL((k_fused_bf16<NR, MODE, IC, NS>), dim3(nwg), dim3(NT), bytes, s, a);
}

// NS = 1 for sweeps whose Lq is BF16-representable (the drivers round it so);
// the TTM and other callers pass FP32 operands, split in three.
template <int NR, int MODE, int NS>
void launch2s(const FusedArgs& a, int nwg, hipStream_t s) {
  if (NR <= 2 && a.v.I <= XR_MAX_R) {
    if (a.v.I <= 64) launch3r<NR <= 2 ? NR : 2, MODE, 8, NS>(a, nwg, s);
    else if (a.v.I <= 128) launch3r<NR <= 2 ? NR : 2, MODE, 16, NS>(a, nwg, s);
    else launch3r<NR <= 2 ? NR : 2, MODE, 32, NS>(a, nwg, s);
    return;
  }
  if (a.v.I <= 64) launch3<NR, MODE, 8, NS>(a, nwg, s);
  else if (a.v.I <= 128) launch3<NR, MODE, 16, NS>(a, nwg, s);
  else launch3<NR, MODE, 32, NS>(a, nwg, s);
}

template <int NR, int MODE>
void launch2(const FusedArgs& a, int nwg, hipStream_t s) {
  if (MODE == 0 && a.lq_bf16) launch2s<NR, MODE, 1>(a, nwg, s);
  else launch2s<NR, MODE, 3>(a, nwg, s);
}

template <int NR>
void launch1(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  if (mode == 0) launch2<NR, 0>(a, nwg, s);
  else if (mode == 2) launch2<NR, 2>(a, nwg, s);
  else launch2<NR, 3>(a, nwg, s);
}

}  // namespace

constexpr int LDS_MAX_BYTES_B16 = 160 * 1024;

bool fused_bf16_supported(const FusedArgs& a, int mode) {
  const View& v = a.v;
  if (a.x_dtype != TK_BF16 || mode == 1) return false;
  if (v.Q < 2 || (v.Q & 1) || ((uintptr_t)a.X & 3)) return false;
  if (v.I < 1 || v.I > 256 || a.R < 1 || a.R > 48) return false;
  const int NR = (a.R + 15) / 16;
  if (NR <= 2 && v.I <= XR_MAX_R)
    return (size_t)lds_b16r(v.I <= 64 ? 8 : v.I <= 128 ? 16 : 32, NR, mode).total <=
           (size_t)LDS_MAX_BYTES_B16;
  return (size_t)lds_b16((int)v.I, NR, mode).total <= (size_t)LDS_MAX_BYTES_B16;
}

int launch_fused_bf16(const FusedArgs& a, int mode, int nwg_max, hipStream_t s) {
  int64_t ntiles = ceil_div(a.v.J(), TJ);
  int nwg = (int)(ntiles < NWG ? ntiles : NWG);
  if (nwg > nwg_max / NW) nwg = nwg_max / NW;
  switch ((a.R + 15) / 16) {
    case 1: launch1<1>(a, mode, nwg, s); break;
    case 2: launch1<2>(a, mode, nwg, s); break;
    case 3: launch1<3>(a, mode, nwg, s); break;
  }
  return nwg;
}

}  // namespace tk
