// Fused ALS sweep for BF16 storage and large modes (256 < I_n <= 1024, R <= 48)
// on the gfx950 BF16 matrix cores, and the initial sketch pass of the same
// shapes (MODE 2).
//
// The products are those of the other sweep kernels (one HBM read of every
// fibre a_j per sweep, row-wise rule of Section 3): v_j = Lq^T a_j,
// G_V += v_j v_j^T, L_acc += a_j v_j^T.  The tensor is BF16 and the sweep's
// Lq = L (L^T L)^{-1} arrives rounded to BF16 precision (the quantised L~ whose
// Gram the trace residual uses), so the R-update is one BF16 product per term,
// exact in FP32.  V is split exactly into three BF16 terms (h + m + l = v): the
// Gram takes the six split products above FP32 rounding (exact products of
// the FP32 V, which the trace residual needs), the L-update the two leading
// terms (V to 16 significant bits, 2^-17 relative, far below the tensor's own
// BF16 rounding).
//
// The sketch pass (Section 5 initial guess): L_acc = B_(n) S for the sketch S
// whose rows are generated in the kernel, with ||B||^2 from the staged values.
// It is pass 2 alone; the sketch values are 24-bit multiples of 2^-24, so
// their three BF16 terms are exact and the L-update takes all three (the
// product is that of the FP32 sketch, up to FP32 accumulation).  The next
// tile's sketch rows are split into the other of two V buffers during the
// last step of a tile.
//
// Work layout: 256 persistent workgroups of NWK = 8 waves.  Lq^T stays in LDS for the
// whole launch.  A tile of 64 fibres is streamed in chunks of 128 rows through
// two LDS chunk buffers, twice: pass 1 forms V over the chunks, pass 2 forms
// L_acc chunk by chunk (its reads of the tile are served by the L2: a tile is
// 128 KiB).  The chunk of the step after next is loaded into registers while
// a step works, and each step ends in one barrier (the next chunk is stashed
// into the other LDS buffer while this one is used).  At R = 48 the L_acc
// tiles take 96 of a wave's 256 registers, so operands are read a few at a
// time (scheduling barriers) and one chunk of loads is in flight per wave.
//   R-update  output tiles (fibre block fb of 16, rank tile n) t = w + NWK u,
//             fb = t % 4, n = t / 4 (per SIMD three tiles at R = 48):
//             v_mfma_f32_16x16x32_bf16, A = 16 fibres x 32 rows of the chunk,
//             B = Lq^T (32 rows x 16 ranks);
//   L-update  wave w: row tiles w + NWK i of every chunk, all rank tiles,
//             K = the 64 fibres, two V terms;
//   Gram      wave w < NR (NR + 1) / 2: block pair w (na <= nb), the six split
//             products above FP32 rounding.
// LAYOUT 0 (Q > 1): the chunk is kept as [row][fibre]; the R-update gathers
// eight rows of a fibre.  LAYOUT 1 (Q == 1, a fibre is a contiguous row of the
// tensor): the chunk is kept as [fibre][row]; the L-update gathers eight
// fibres of a row.  16-byte chunks are XOR-swizzled so that both access
// directions spread over the LDS banks.  Every reduction has a fixed order.
#include "tk_kernels.h"

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s4 lds_s4;

namespace {

constexpr int TJ = 64;             // fibres per tile
constexpr int CH = 128;            // rows per chunk
constexpr int NCHM = 8;            // chunks per mode, at most (I <= 1024)
constexpr int NWG = 256;
constexpr int RS0 = TJ + 8;        // LAYOUT 0: row stride (BF16 elements)
constexpr int RS1 = CH + 8;        // LAYOUT 1: fibre stride
constexpr int VS = TJ + 8;         // row stride of the V^T splits

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// v = h + m + l exactly (three round-to-nearest BF16 terms).
__device__ __forceinline__ void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)v;
  const float r1 = v - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// Element offsets in a chunk buffer.  LAYOUT 0: (row, fibre) at row * RS0 +
// fibre, its 16-byte chunk f / 8 moved to (f / 8) ^ 2 ((row / 8) & 3).
// LAYOUT 1: at fibre * RS1 + row, chunk row / 8 moved to
// (row / 8) ^ 2 ((fibre / 8) & 3).
template <int LAYOUT>
__device__ __forceinline__ int cidx(int row, int f) {
  if (LAYOUT == 0) return row * RS0 + ((((f >> 3) ^ (((row >> 3) & 3) << 1))) << 3) + (f & 7);
  return f * RS1 + ((((row >> 3) ^ (((f >> 3) & 3) << 1))) << 3) + (row & 7);
}

template <int LAYOUT>
__host__ __device__ constexpr int chunk_elems() { return LAYOUT == 0 ? CH * RS0 : TJ * RS1; }

struct LdsBB {
  int lq, xs, vt, total;  // byte offsets
};

// MODE 0: Lq^T, two chunk buffers, the three V^T splits; MODE 2: two chunk
// buffers and two sets of V^T splits (this tile's and the next one's).
__host__ __device__ inline LdsBB lds_bb(int I, int NR, int LAYOUT, int MODE) {
  const int RP = 16 * NR;
  const int KP = CH * ((I + CH - 1) / CH);   // rows padded to whole chunks
  LdsBB l;
  l.lq = 0;
  l.xs = l.lq + (MODE == 0 ? RP * (KP + 8) * 2 : 0);
  l.vt = l.xs + 2 * (LAYOUT == 0 ? CH * RS0 : TJ * RS1) * 2;
  l.total = l.vt + (MODE == 0 ? 1 : 2) * 3 * RP * VS * 2;
  return l;
}

// A chunk of the step (tile, chunk c) into registers: SL = 16 / NWK 16-byte
// slots per thread (a chunk is 1024 of them), eight BF16 values each.
// LAYOUT 0: slot k holds row 128 c + 8 w + lane / 8 + 8 NWK k, fibres
// j0 + 8 (lane % 8) .. + 7 (Q a multiple of 8: the eight never cross a row of
// the view).  LAYOUT 1: slot k holds fibre j0 + 4 w + lane / 16 + 4 NWK k, rows
// 128 c + 8 (lane % 16) .. + 7 (I a multiple of 8).  Indices are clamped into the
// tensor (the values outside are zeroed when stashed).
template <int LAYOUT, int NWK>
__device__ __forceinline__ void load_chunk(const uint4* __restrict__ X16, const View& v,
                                           int64_t j0, int c, int lane, int w,
                                           uint4 (&rb)[16 / NWK]) {
  constexpr int SL = 16 / NWK;
  const int64_t J = v.J();
  const int I = (int)v.I;
  if (LAYOUT == 0) {
    const int64_t j = min(j0 + 8 * (lane & 7), J - 8);
    const uint4* b = X16 + (v.fibre_base(j) >> 3);
    const int64_t q8 = v.Q >> 3;
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int row = min(CH * c + 8 * w + (lane >> 3) + 8 * NWK * k, I - 1);
      rb[k] = b[(int64_t)row * q8];
    }
  } else {
    const int row = min(CH * c + 8 * (lane & 15), I - 8);
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int64_t j = min(j0 + 4 * w + (lane >> 4) + 4 * NWK * k, J - 1);
      rb[k] = X16[(j * I + row) >> 3];
    }
  }
}

// With NORM the squares of the staged values (zeros outside the tensor) are
// added to ns (four FP64 partial sums).
template <int LAYOUT, int NWK, bool NORM>
__device__ __forceinline__ void stash_chunk(const View& v, int64_t j0, int c, int lane, int w,
                                            const uint4 (&rb)[16 / NWK], __bf16* Xb,
                                            double (&ns)[4]) {
  constexpr int SL = 16 / NWK;
  const int64_t J = v.J();
  const int I = (int)v.I;
  // (values outside the tensor are masked with a bitwise and per dword: a
  // select of whole vectors would go through memory)
  auto masked = [](const uint4& x, bool keep) __attribute__((always_inline)) {
    const uint32_t m = keep ? 0xffffffffu : 0u;
    return make_uint4(x.x & m, x.y & m, x.z & m, x.w & m);
  };
  auto sq = [&](const uint4& x) __attribute__((always_inline)) {
    const uint32_t d[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double lo = (double)__uint_as_float(d[e] << 16);
      const double hi = (double)__uint_as_float(d[e] & 0xffff0000u);
      ns[e] += lo * lo + hi * hi;
    }
  };
  if (LAYOUT == 0) {
    const bool fok = j0 + 8 * (lane & 7) < J;
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int r = 8 * w + (lane >> 3) + 8 * NWK * k;
      const uint4 x = masked(rb[k], fok && CH * c + r < I);
      *(uint4*)(Xb + cidx<0>(r, 8 * (lane & 7))) = x;
      if (NORM) sq(x);
    }
  } else {
    const int r = 8 * (lane & 15);
    const bool rok = CH * c + r < I;
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int f = 4 * w + (lane >> 4) + 4 * NWK * k;
      const uint4 x = masked(rb[k], rok && j0 + f < J);
      *(uint4*)(Xb + cidx<1>(r, f)) = x;
      if (NORM) sq(x);
    }
  }
}

// Eight BF16 values across the stored order, from two transposing LDS reads
// (ds_read_b64_tr_b16).  The 16 lanes of a group cover four consecutive
// lines of the buffer (rows in LAYOUT 0, fibres in LAYOUT 1) by 16 elements
// along them: lane j points at elements 4 (j % 4) .. + 3 of line j / 4, and
// receives element j of the four lines.  The second read is four lines on.
// The chunk swizzle moves whole 8-element runs and is the same for eight
// lines that start at a multiple of 8, so each lane's four elements are
// contiguous.
__device__ __forceinline__ bf8 tr8(const __bf16* p, int step) {
  const s4 u0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(p));
  const s4 u1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(p + step));
  // (one whole-vector shuffle: element-wise inserts of these values are not
  // reliably compiled)
  return __builtin_bit_cast(bf8, __builtin_shufflevector(u0, u1, 0, 1, 2, 3, 4, 5, 6, 7));
}

// A operand of the R-update: rows row0..row0+7 (row0 a multiple of 8) of
// fibre f0 + j, j = lane % 16.
template <int LAYOUT>
__device__ __forceinline__ bf8 rupd_a(const __bf16* Xb, int row0, int f0, int j) {
  if (LAYOUT == 1) return *(const bf8*)(Xb + cidx<1>(row0, f0 + j));
  return tr8(Xb + cidx<0>(row0 + (j >> 2), f0 + 4 * (j & 3)), 4 * RS0);
}

// A operand of the L-update: fibres f0..f0+7 (f0 a multiple of 8) of row
// r0 + j, j = lane % 16.
template <int LAYOUT>
__device__ __forceinline__ bf8 lupd_a(const __bf16* Xb, int r0, int j, int f0) {
  if (LAYOUT == 0) return *(const bf8*)(Xb + cidx<0>(r0 + j, f0));
  return tr8(Xb + cidx<1>(r0 + 4 * (j & 3), f0 + (j >> 2)), 4 * RS1);
}

template <int NR, int LAYOUT, int NWK, int MODE>
__global__ void __launch_bounds__(64 * NWK, 1) k_fused_bf16_big(FusedArgs a) {
  static_assert(MODE == 0 || MODE == 2, "sweep or sketch pass");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int NT = 64 * NWK;
  constexpr int SL = 16 / NWK;               // 16-byte load slots per thread and chunk
  constexpr int RP = 16 * NR;
  constexpr int NG = NR * (NR + 1) / 2;      // G_V block pairs
  constexpr int NU = (4 * NR + NWK - 1) / NWK;    // R-update tiles per wave (max)
  constexpr int RTW = 8 / NWK;               // L-update row tiles per wave and chunk
  constexpr int CE = chunk_elems<LAYOUT>();
  const View v = a.v;
  const int I = (int)v.I, R = a.R;
  const int64_t J = v.J();
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int NCH = (I + CH - 1) / CH;
  const int KP = CH * NCH;
  const int LS = KP + 8;                     // Lq^T row stride
  const LdsBB L = lds_bb(I, NR, LAYOUT, MODE);
  __bf16* Lq = (__bf16*)(smem + L.lq);       // [RP][LS]: Lq^T
  __bf16* Xs = (__bf16*)(smem + L.xs);       // two chunk buffers
  __bf16* Vt = (__bf16*)(smem + L.vt);       // [3][RP][VS]: V^T splits (MODE 2: two sets)
  constexpr int NTERM = MODE == 2 ? 3 : 2;   // V terms in the L-update
  const bool want_norm = MODE == 2 && a.norm2_parts != nullptr;
  double ns[4] = {0.0, 0.0, 0.0, 0.0};

  // ---- once per kernel: Lq^T (rows past I and ranks past R zero)
  if (MODE == 0) {
    const int64_t ldi = a.lq_ldi ? a.lq_ldi : R, ldo = a.lq_ldi ? a.lq_ldo : 1;
    for (int e = threadIdx.x; e < RP * KP; e += NT) {
      const int r = e / KP, i = e - r * KP;
      const float x = (i < I && r < R) ? a.Lq[i * ldi + r * ldo] : 0.0f;
      Lq[r * LS + i] = (__bf16)x;              // exact: x is BF16-representable
    }
  }

  f4 lacc[NCHM][RTW][NR];
#pragma unroll
  for (int c = 0; c < NCHM; ++c)
#pragma unroll
    for (int i = 0; i < RTW; ++i)
#pragma unroll
      for (int n = 0; n < NR; ++n) lacc[c][i][n] = f4{0, 0, 0, 0};
  // G_V: wave w < NG owns block pair w = (gna, gnb), gna <= gnb, over both
  // 32-fibre K steps of every tile
  static_assert(NG <= NWK, "one G_V block pair per wave");
  const bool gown = w < NG;
  int gna = 0, gnb = 0;
  for (int x = 0, q = 0; x < NR; ++x)
    for (int y = x; y < NR; ++y, ++q)
      if (q == w) { gna = x; gnb = y; }
  double gd[4] = {0.0, 0.0, 0.0, 0.0};
  // R-update tiles of this wave: t = w + NWK u < 4 NR, fb = t % 4, n = t / 4
  const int nu = 4 * NR > w ? (4 * NR - w + NWK - 1) / NWK : 0;
  f4 vacc[NU];

  const uint4* X16 = (const uint4*)a.X;
  const int64_t ntiles = ceil_div(J, TJ);
  const int64_t my_tiles = (int64_t)blockIdx.x < ntiles
                               ? (ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int spt = MODE == 0 ? 2 * NCH : NCH;   // steps per tile
  const int64_t total = my_tiles * spt;
  // Step s works on tile blockIdx.x + (s / spt) gridDim.x, pass (s % spt) /
  // NCH, chunk (s % spt) % NCH (MODE 2: pass 2, chunk s % spt).  The positions (tile, step in the tile) of
  // steps s, s + 1 and s + 2 are advanced by increments: no 64-bit division
  // in the loop.
  auto advance = [&](int64_t& t, int& st) __attribute__((always_inline)) {
    if (++st == spt) {
      st = 0;
      t += gridDim.x;
    }
  };
  const int64_t t_last = blockIdx.x + (my_tiles - 1) * gridDim.x;
  // (steps past the end load the last chunk again, so every load is
  // unconditional)
  auto step_load = [&](int64_t s, int64_t t, int st, uint4 (&rb)[SL]) __attribute__((always_inline)) {
    const int64_t tt = s < total ? t : t_last;
    const int sst = s < total ? st : spt - 1;
    load_chunk<LAYOUT, NWK>(X16, v, tt * TJ, sst < NCH ? sst : sst - NCH, lane, w, rb);
  };
  auto step_stash = [&](int64_t s, int64_t t, int st, const uint4 (&rb)[SL])
                        __attribute__((always_inline)) {
    if (MODE == 2 && want_norm)
      stash_chunk<LAYOUT, NWK, true>(v, t * TJ, st, lane, w, rb, Xs + (s & 1) * CE, ns);
    else
      stash_chunk<LAYOUT, NWK, false>(v, t * TJ, st < NCH ? st : st - NCH, lane, w, rb,
                                      Xs + (s & 1) * CE, ns);
  };
  // MODE 2: the three BF16 terms of the sketch rows of tile t (zero past J
  // and R) into V^T split set `set`
  auto sketch_tile = [&](int64_t t, int set) __attribute__((always_inline)) {
    __bf16* Vd = Vt + set * 3 * RP * VS;
    for (int e = threadIdx.x; e < RP * TJ; e += NT) {
      const int r = e / TJ, jl = e - (e / TJ) * TJ;
      const int64_t j = t * TJ + jl;
      float x = 0.0f;
      if (j < J && r < R) x = sketch_value(a.seed, ((uint64_t)a.mode << 48) + (uint64_t)(j * R + r));
      __bf16 h, m, l;
      split3(x, h, m, l);
      Vd[(0 * RP + r) * VS + jl] = h;
      Vd[(1 * RP + r) * VS + jl] = m;
      Vd[(2 * RP + r) * VS + jl] = l;
    }
  };

  // the work of step s (position st in its tile) on its chunk buffer; MODE 2
  // reads the V^T split set vset
  auto step_work = [&](int64_t s, int st, int vset) __attribute__((always_inline)) {
    const __bf16* Xb = Xs + (s & 1) * CE;
    const __bf16* Vw = Vt + (MODE == 2 ? vset * 3 * RP * VS : 0);
    if (MODE == 0 && st < NCH) {
      // ---- pass 1: V += X_c^T Lq_c
      const int c = st;
      if (c == 0) {
#pragma unroll
        for (int u = 0; u < NU; ++u) vacc[u] = f4{0, 0, 0, 0};
      }
      // (the wave's tiles t = w + NWK u share the fibre block w % 4; the
      // operands of the next 32-row block are read while this one's products
      // run)
      static_assert(NWK % 4 == 0, "a wave's R-update tiles share one fibre block");
      const int fb0 = 16 * (w & 3);
      bf8 av[2], bv[2][NU];
      auto rread = [&](int kb, int sl) __attribute__((always_inline)) {
        const int row0 = 32 * kb + 8 * lk;
        av[sl] = rupd_a<LAYOUT>(Xb, row0, fb0, lr);
#pragma unroll
        for (int u = 0; u < NU; ++u)
          if (u < nu)
            bv[sl][u] = *(const bf8*)(Lq + (16 * ((w + NWK * u) >> 2) + lr) * LS + CH * c + row0);
      };
      rread(0, 0);
#pragma unroll
      for (int kb = 0; kb < CH / 32; ++kb) {
        if (kb + 1 < CH / 32) rread(kb + 1, (kb + 1) & 1);
#pragma unroll
        for (int u = 0; u < NU; ++u)
          if (u < nu) vacc[u] = mfma_bf16(av[kb & 1], bv[kb & 1][u], vacc[u]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (c == NCH - 1) {
        // V^T splits: V[16 fb + 4 lk + q][16 n + lr] = vacc[u][q]
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (u < nu) {
            const int t = w + NWK * u;
            const int fb = t & 3, n = t >> 2;
            bf16_t hs[4], ms[4], ls[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              __bf16 h, m, l;
              split3(vacc[u][q], h, m, l);
              hs[q] = __builtin_bit_cast(bf16_t, h);
              ms[q] = __builtin_bit_cast(bf16_t, m);
              ls[q] = __builtin_bit_cast(bf16_t, l);
            }
            const int o = (16 * n + lr) * VS + 16 * fb + 4 * lk;   // 8-byte aligned
            *(uint2*)(Vt + 0 * RP * VS + o) =
                make_uint2(hs[0] | ((uint32_t)hs[1] << 16), hs[2] | ((uint32_t)hs[3] << 16));
            *(uint2*)(Vt + 1 * RP * VS + o) =
                make_uint2(ms[0] | ((uint32_t)ms[1] << 16), ms[2] | ((uint32_t)ms[3] << 16));
            *(uint2*)(Vt + 2 * RP * VS + o) =
                make_uint2(ls[0] | ((uint32_t)ls[1] << 16), ls[2] | ((uint32_t)ls[3] << 16));
          }
        }
      }
    } else {
      // ---- pass 2: L_acc[chunk rows] += X_c V (row tiles w + NWK i of the chunk)
      const int c = MODE == 0 ? st - NCH : st;
      if (MODE == 0 && c == 0 && gown) {
        // G_V block pair (gna, gnb) from the V splits: the six split products
        // above FP32 rounding, the operands read a few at a time
        const int ra = 16 * gna + lr, rb = 16 * gnb + lr;
        f4 g = f4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < TJ / 32; ++ks) {
          const int ko = 32 * ks + 8 * lk;
          const bf8 ah = *(const bf8*)(Vt + (0 * RP + ra) * VS + ko);
          const bf8 bh = *(const bf8*)(Vt + (0 * RP + rb) * VS + ko);
          const bf8 am = *(const bf8*)(Vt + (1 * RP + ra) * VS + ko);
          const bf8 bm = *(const bf8*)(Vt + (1 * RP + rb) * VS + ko);
          g = mfma_bf16(ah, bh, g);
          g = mfma_bf16(ah, bm, g);
          g = mfma_bf16(am, bh, g);
          g = mfma_bf16(am, bm, g);
          __builtin_amdgcn_sched_barrier(0);
          const bf8 al = *(const bf8*)(Vt + (2 * RP + ra) * VS + ko);
          const bf8 bl = *(const bf8*)(Vt + (2 * RP + rb) * VS + ko);
          g = mfma_bf16(ah, bl, g);
          g = mfma_bf16(al, bh, g);
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) gd[q] += (double)g[q];
      }
      // (in the sweep V enters as its two leading BF16 terms, h + m: 2^-17
      // relative, far below the tensor's own BF16 rounding; the Gram above
      // keeps all six products the trace residual needs.  The sketch takes
      // its three exact terms.)
      auto lupd = [&](f4 (&acc)[RTW][NR]) __attribute__((always_inline)) {
#pragma unroll
        for (int ks = 0; ks < TJ / 32; ++ks) {
          bf8 av[RTW];
#pragma unroll
          for (int i = 0; i < RTW; ++i)
            av[i] = lupd_a<LAYOUT>(Xb, 16 * (w + NWK * i), lr, 32 * ks + 8 * lk);
#pragma unroll
          for (int n = 0; n < NR; ++n) {
#pragma unroll
            for (int s3 = 0; s3 < NTERM; ++s3) {
              const bf8 bv = *(const bf8*)(Vw + (s3 * RP + 16 * n + lr) * VS + 32 * ks + 8 * lk);
#pragma unroll
              for (int i = 0; i < RTW; ++i) acc[i][n] = mfma_bf16(av[i], bv, acc[i][n]);
              // (one operand read in flight at a time: the registers go to L_acc)
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      };
      // (register arrays need compile-time indices: the chunk picks them)
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
  };

  // ---- the step loop: one register buffer, two LDS chunk buffers
  uint4 rb0[SL];
  int64_t t0 = blockIdx.x, t1 = t0, t2;
  int st0 = 0, st1 = 0, st2;
  advance(t1, st1);
  t2 = t1;
  st2 = st1;
  advance(t2, st2);
  int vset = 0;                               // MODE 2: split set of tile t0
  if (total > 0) {
    step_load(0, t0, st0, rb0);
    __syncthreads();
    if (MODE == 2) sketch_tile(t0, 0);
    step_stash(0, t0, st0, rb0);
    step_load(1, t1, st1, rb0);
    __syncthreads();
  }
  for (int64_t s = 0; s < total; ++s) {
    step_work(s, st0, vset);
    if (MODE == 2 && st0 == spt - 1) {
      // the next tile's sketch rows into the other set (its previous tile
      // finished with it before the last barrier)
      vset ^= 1;
      if (s + 1 < total) sketch_tile(t1, vset);
    }
    if (s + 1 < total) step_stash(s + 1, t1, st1, rb0);
    step_load(s + 2, t2, st2, rb0);
    __syncthreads();
    t0 = t1;
    st0 = st1;
    t1 = t2;
    st1 = st2;
    advance(t2, st2);
  }

  // ---- per-workgroup outputs
  const int wg = blockIdx.x;
  if (want_norm) {
    double nsum = (ns[0] + ns[1]) + (ns[2] + ns[3]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nsum += __shfl_xor(nsum, off, 64);
    static_assert(NWK == FUSED_WAVES, "one norm partial per wave");
    if (lane == 0) a.norm2_parts[wg * FUSED_WAVES + w] = nsum;
  }
  float* lp = a.lacc_parts + (int64_t)wg * I * R;
#pragma unroll
  for (int c = 0; c < NCHM; ++c) {
    if (c < NCH) {
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
#pragma unroll
        for (int n = 0; n < NR; ++n) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = CH * c + 16 * (w + NWK * i) + 4 * lk + q, r = 16 * n + lr;
            if (row < I && r < R) lp[row * R + r] = lacc[c][i][n][q];
          }
        }
      }
    }
  }
  if (MODE == 2) return;
  // G_V partials, FUSED_WAVES slots per workgroup: wave w fills slots
  // w + NWK k, its block pair in the first (each diagonal block's upper triangle
  // and its mirror, so it is exactly symmetric), zero elsewhere
  for (int sl = w; sl < FUSED_WAVES; sl += NWK) {
    double* gz = a.gv_parts + (int64_t)(wg * FUSED_WAVES + sl) * R * R;
    for (int e = lane; e < R * R; e += 64) gz[e] = 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (gown) {
    double* gp = a.gv_parts + (int64_t)(wg * FUSED_WAVES + w) * R * R;
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

template <int NR, int LAYOUT, int MODE>
void launch_bb(const FusedArgs& a, int nwg, hipStream_t s) {
  constexpr int NWK = 8;
  const size_t bytes = (size_t)lds_bb((int)a.v.I, NR, LAYOUT, MODE).total;
  (void)hipFuncSetAttribute((const void*)k_fused_bf16_big<NR, LAYOUT, NWK, MODE>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  hipLaunchKernelGGL((k_fused_bf16_big<NR, LAYOUT, NWK, MODE>), dim3(nwg), dim3(64 * NWK),
                     bytes, s, a);
}

template <int NR>
void launch_bb_nr(const FusedArgs& a, int mode, int nwg, hipStream_t s) {
  if (mode == 2) {
    if (a.v.Q == 1) launch_bb<NR, 1, 2>(a, nwg, s);
    else launch_bb<NR, 0, 2>(a, nwg, s);
  } else {
    if (a.v.Q == 1) launch_bb<NR, 1, 0>(a, nwg, s);
    else launch_bb<NR, 0, 0>(a, nwg, s);
  }
}

}  // namespace

constexpr int LDS_MAX_BYTES_BB = 160 * 1024;

bool fused_bf16_big_supported(const FusedArgs& a, int mode) {
  const View& v = a.v;
  if (a.x_dtype != TK_BF16) return false;
  if (!(mode == 0 && a.lq_bf16) && mode != 2) return false;
  if (v.I <= 256 || v.I > (int64_t)CH * NCHM || a.R < 1 || a.R > 48) return false;
  if ((uintptr_t)a.X & 15) return false;
  // LAYOUT 0 loads eight fibres of a row (Q a multiple of 8), LAYOUT 1 eight
  // rows of a fibre (I a multiple of 8), 16 bytes at a time
  if (v.Q == 1 ? (v.I & 7) : (v.Q & 7)) return false;
  if (v.J() < 8) return false;
  const int NR = (a.R + 15) / 16;
  return (size_t)lds_bb((int)v.I, NR, v.Q == 1 ? 1 : 0, mode).total <= (size_t)LDS_MAX_BYTES_BB;
}

int launch_fused_bf16_big(const FusedArgs& a, int mode, int nwg_max, hipStream_t s) {
  const int64_t ntiles = ceil_div(a.v.J(), TJ);
  int nwg = (int)(ntiles < NWG ? ntiles : NWG);
  if (nwg > nwg_max / FUSED_WAVES) nwg = nwg_max / FUSED_WAVES;
  switch ((a.R + 15) / 16) {
    case 1: launch_bb_nr<1>(a, mode, nwg, s); break;
    case 2: launch_bb_nr<2>(a, mode, nwg, s); break;
    case 3: launch_bb_nr<3>(a, mode, nwg, s); break;
  }
  return nwg;
}

}  // namespace tk
