// Internal interface between the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tk_device.h"
#include "../../include/tucker_als.h"

namespace tk {

// A Gram is declared singular when a squared Cholesky pivot drops to
// PIVOT_TOL times its largest diagonal entry (Remark 3).
constexpr double PIVOT_TOL = 1e-13;

template <typename T> struct Store;
template <> struct Store<double> {
  __host__ __device__ static double cvt(double x) { return x; }
};
template <> struct Store<float> {
  __host__ __device__ static float cvt(double x) { return (float)x; }
};
template <> struct Store<bf16_t> {
  __host__ __device__ static bf16_t cvt(double x) { return f32_to_bf16((float)x); }
};

// ---------------------------------------------------------------- small LA
// out[e] = sum_w in[w*stride + e] in FP64, fixed order.  With tmp (room for
// REDUCE_GROUPS / 4 * n doubles) the sum runs in two stages over up to
// REDUCE_GROUPS interleaved part groups; without it, in one.
constexpr int REDUCE_GROUPS = 256;
template <typename T>
void launch_reduce_parts(const T* in, int parts, int64_t n, int64_t stride, double* out,
                         double* tmp, hipStream_t s);
template <typename T>
void launch_identity(T* U, int64_t n, hipStream_t s);
template <typename T>
void launch_convert(const double* in, int64_t n, T* out, hipStream_t s);
template <typename T>
void launch_widen(const T* in, int64_t n, double* out, hipStream_t s);

// Singular vectors within an orthonormal basis (Section 3, after Algorithm 3.4).
// launch_sym_eig: eigenvectors W (r x r row-major, descending eigenvalues, each column's
// largest-magnitude entry positive) and eigenvalues of the symmetric FP64 r x r matrix M,
// r <= 64, by cyclic Jacobi in one workgroup; *status = TK_ERR_NONFINITE on Inf/NaN.
// launch_rotate: out = Q W, Q m x r, W r x r, out m x r, all FP64 row-major.
void launch_sym_eig(const double* M, int r, double* W, double* evals, int* status,
                    hipStream_t s);
void launch_rotate(const double* Q, int64_t m, int r, const double* W, double* out,
                   hipStream_t s);

// ---------------------------------------------------------------- streaming
// Contraction over the mode index (generic VALU path):
//   out(j, o) = sum_i W(i, o) X[p, i, q],  j = p*Q + q,  0 <= o < O
// W(i, o) = W[i*w_ldi + o*w_ldo] (compute type C).
// out_kind 0: row-major matrix out[j*O + o] (type C)
// out_kind 1: tensor out[(p*O + o)*Q + q]   (type C)
// resid (optional, FP64 per workgroup): sum_j ||x_j - Lr v_j||^2 where
//   Lr(i, o) = Lr[i*O + o] (type C) and v_j = out(j, :).
struct VpassArgs {
  const void* X; int x_dtype; View v;
  const void* W; int64_t w_ldi, w_ldo; int64_t O;
  void* out; int out_kind;
  const void* Lr; double* resid_parts;
};
int launch_vpass(const VpassArgs& a, int nwg_max, int* nwg_used, hipStream_t s);

// Contraction over fibres (generic VALU path):
//   L(i, r) = sum_j X[p, i, q] V(j, r)
// v_kind 0: V(j, r) = V[j*R + r]                   (type C)
// v_kind 1: V(j, r) = sketch(seed, mode, j*R + r)  (Section 5 initial guess)
// v_kind 2: V(j, r) = Y[p, r, q]                   (tensor, x_dtype)
// Per-workgroup partials parts[c*I*R + i*R + r] (type C) for fibre chunk c;
// norm2_parts (optional) receives per-chunk sums of X^2 (FP64).
struct LpassArgs {
  const void* X; int x_dtype; View v;
  int v_kind; const void* V; int64_t R; uint64_t seed; int mode;
  void* parts; double* norm2_parts;
};
int lpass_chunks(const View& v, int64_t R, int nwg_max);
// Workgroups of an L-pass over `chunks` fibre chunks (one norm2 partial each).
int lpass_blocks(const View& v, int chunks);
void launch_lpass(const LpassArgs& a, int chunks, hipStream_t s);

// G = V^T V partials over row chunks: parts[c*R*R + a*R + b] (FP64).
void launch_gram_parts(const void* V, int c_dtype, int64_t J, int64_t R, int chunks,
                       double* parts, hipStream_t s);

// Sum of squares partials (FP64) over `chunks` workgroups.
void launch_norm2_parts(const void* X, int x_dtype, int64_t n, int chunks, double* parts,
                        hipStream_t s);

// Fused ALS sweep on the matrix cores (FP32/BF16 storage, I <= 256, R <= 64):
// one read of every fibre a_j gives v_j = Lq^T a_j, G_V += v_j v_j^T and
// L_acc += a_j v_j^T (and, with resid, sum ||a_j - Lr v_j||^2).
// TTM variant (y != null): Y[p, r, q] = sum_i Lq(i, r) X[p, i, q] with
// Lq(i, r) = Lq[i*lq_ldi + r*lq_ldo] (lq_ldi == 0: row-major I x R).
struct FusedArgs {
  const void* X; int x_dtype; View v; int R;
  const float* Lq;       // I x R, quantised L~ (compute type float)
  const float* Lr;       // I x R, factor for the explicit residual (or null)
  float* lacc_parts;     // [nwg][I][R]
  double* gv_parts;      // [FUSED_WAVES * nwg][R][R]
  double* resid_parts;   // [FUSED_WAVES * nwg] (explicit residual)
  int sketch; uint64_t seed; int mode;  // init variant: V = sketch, no G_V
  int lq_bf16;           // the Lq values are BF16-representable (BF16 sweeps
                         // multiply by them as one BF16 term)
  double* norm2_parts;   // [FUSED_WAVES * nwg] sums of X^2 (init variant, optional)
  float* y;              // TTM output (or null)
  int64_t lq_ldi, lq_ldo;
};
// Shapes the fused kernel takes (LDS budget), for the given residual mode.
bool fused_supported(int x_dtype, const View& v, int R, int resid_mode);
// Shapes its TTM variant takes (J output rows of the mode).
bool fused_ttm_supported(int x_dtype, const View& v, int64_t J);
// Launches and returns the number of workgroups W; L_acc partials are
// [W][I][R], Gram and residual partials [FUSED_WAVES * W] (one per wave).
constexpr int FUSED_WAVES = 8;
int launch_fused(const FusedArgs& a, int nwg_max, hipStream_t s);
// BF16 storage on the BF16 matrix cores (sweep, init, TTM; Q even): used by
// launch_fused when it takes the shape; same partial-buffer layout.
bool fused_bf16_supported(const FusedArgs& a, int mode);
int launch_fused_bf16(const FusedArgs& a, int mode, int nwg_max, hipStream_t s);
// BF16 storage, modes of 256 < I <= 1024 rows, R <= 48, sweep with
// BF16-representable Lq (Lq resident in LDS) or the initial sketch pass: on
// the BF16 matrix cores, the fibres streamed in chunks of rows; used by
// launch_fused when it takes the shape.
bool fused_bf16_big_supported(const FusedArgs& a, int mode);
int launch_fused_bf16_big(const FusedArgs& a, int mode, int nwg_max, hipStream_t s);
// Rounds n FP32 values to BF16 precision in place (round to nearest even).
void launch_round_bf16(float* x, int64_t n, hipStream_t s);
// Modes of 256 < I <= 1024 rows (R <= 48; sweep, init, TTM), streamed in
// chunks of rows: used by launch_fused when it takes the shape.
bool fused_big_shape(int x_dtype, const View& v, int64_t R, int mode);
int launch_fused_big(const FusedArgs& a, int mode, int nwg_max, hipStream_t s);

// One-workgroup FP64 steps of the mode solve (see k_mode_step.hip).
enum { STEP_SOLVE = 1, STEP_QR = 2, STEP_PREP = 4, STEP_PREP_SPECULATIVE = 8 };
struct StepArgs {
  int64_t m; int r; int ops;
  // SOLVE: Lnext = Lacc GV^{-1}; res2[0] = rsum ? *rsum : norm2 - tr(Gq^-1 GV),
  // res2[1] = tr(Gq^-1 GV) with Gq^-1 = Wq^T Wq (Wq as left by the last PREP)
  const double* Lacc; const double* GV; double* Lnext;
  double norm2; const double* rsum; double* res2;
  const double* norm2p;  // when non-null, replaces norm2 (read on the device)
  // QR: Qout = Q of the reduced QR of Qin (Q1: m x r scratch)
  const double* Qin; double* Q1; double* Qout;
  // PREP from Lnext (SOLVE) or Qout (QR): Lq = L (L^T L)^{-1} in the compute
  // type (rounded to BF16 precision when lq_bf16), Wq = chol(Lq^T Lq)^{-1}
  // (r x r lower, row-major, of the rounded Lq), Lr = L in the compute type
  // (if non-null)
  void* Lq; void* Lr; double* Wq; int lq_bf16;
  int* status;        // failures of SOLVE / QR / non-speculative PREP
  int* prep_status;   // failures of a speculative PREP
  // optional FP64 buffer of gpart_cap doubles for the Gram partials of a
  // cooperative multi-workgroup launch (null: one workgroup)
  double* gpart; int64_t gpart_cap;
  int tr;             // rows per staged tile (set by launch_mode_step)
};
void launch_mode_step(const StepArgs& a, int q_dtype, hipStream_t s);

// Batched st-HOSVD-ALS of small order-3 FP32 tensors (I_n <= 128,
// R_n <= 16): one persistent launch, one tensor per workgroup at a time.
struct BatchLaunch {
  const float* A; const void* desc; int count;
  float* U; float* G;
  int32_t* status; int32_t* iters; int* queue;
  char* scratch; int64_t slot_bytes, belems;
  double tol; int max_iters; int resid_mode; uint64_t seed;
  int nwg;
};
constexpr int BATCHED_CONFIGS = 4;
int batched_slot_bytes(int64_t belems);
bool batched_shape_ok(const int32_t* dims, const int32_t* ranks);
void launch_batched(const BatchLaunch& L, int cfg, hipStream_t s);
size_t batched_desc_bytes();
void fill_desc(void* host_desc, int t, int orig, int64_t a_off, int64_t g_off,
               const int64_t* u_off, const int64_t* dims, const int32_t* ranks);

}  // namespace tk
