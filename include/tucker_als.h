/*
 * tucker_als.h -- C ABI of libtucker_als.so, ALS-based truncated HOSVD on
 * MI355X (gfx950).
 *
 * Method: Xiao, Yang & Li, "Efficient Alternating Least Squares Algorithms
 * for Low Multilinear Rank Approximation of Tensors" (arXiv 2004.02583).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Tensors are dense and row-major (C order, last mode fastest).  The
 *    mode-n view of an order-N tensor with dims I_1..I_N is the 3-D array
 *    [P, I_n, Q] with P = prod_{k<n} I_k and Q = prod_{k>n} I_k; the mode-n
 *    unfolding A_(n) (Section 2) is never materialised.  Its columns are
 *    the fibres j = p*Q + q (C order over the other modes).
 *  - Modes are 0-based.  1 <= N <= TK_MAX_ORDER.  dims are int64 > 0.
 *  - Matrices (factors U_n, TTM operands) are row-major: U_n is I_n x R_n.
 *  - Pointers documented "device" are device pointers (hipMalloc / torch
 *    CUDA tensors); "host" pointers are ordinary host memory.
 *  - Ownership: the caller owns every buffer.  The library never allocates
 *    device memory; scratch comes from the caller's workspace `ws` of at
 *    least the size returned by the matching *_workspace_bytes query.
 *    Inputs are only read; outputs are overwritten entirely.
 *  - All device work is enqueued on `stream`.  als_* calls block until their
 *    work on `stream` is done (the convergence loop reads a small status
 *    block back to the host each sweep); ttm, tucker_reconstruct and
 *    contract_allbut are asynchronous.
 *  - Argument validation happens before any HIP call, so every negative
 *    status other than TK_ERR_HIP / TK_ERR_RANK_DEFICIENT / TK_ERR_NONFINITE
 *    can be produced on a machine without a GPU.
 */
#ifndef TUCKER_ALS_H
#define TUCKER_ALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define TK_API __attribute__((visibility("default")))
#else
#define TK_API
#endif

#define TK_MAX_ORDER 8

/* Element types.  FP64 storage computes in FP64; FP32 and BF16 storage
 * contract on the matrix cores with FP32 accumulation.  Grams, Cholesky,
 * solves and QR are always FP64. */
typedef enum {
  TK_F64 = 0,
  TK_F32 = 1,
  TK_BF16 = 2
} tk_dtype;

/* Status codes. */
typedef enum {
  TK_OK = 0,
  TK_NOT_CONVERGED = 1,            /* results valid; some mode hit max_iters */
  TK_SKIPPED = 2,                  /* per-mode report only: the mode was not
                                      processed because an earlier one failed */
  TK_ERR_INVALID_ARG = -1,         /* null pointer, bad N/dims/ranks/order   */
  TK_ERR_UNSUPPORTED_DTYPE = -2,   /* dtype combination not provided         */
  TK_ERR_WORKSPACE_TOO_SMALL = -3, /* ws_bytes below the query's value       */
  TK_ERR_RANK_DEFICIENT = -4,      /* a Gram failed the FP64 Cholesky pivot
                                      test: R_n exceeds the numerical rank
                                      (Remark 3)                              */
  TK_ERR_NONFINITE = -5,           /* the input holds Inf/NaN                */
  TK_ERR_HIP = -6                  /* a HIP runtime call failed              */
} tk_status;

/* Residual evaluation inside the ALS sweep (stop test, eq. E5.01).
 * TK_RESID_TRACE: res^2 = ||B||^2 - tr(G_L'^{-1} G_V) from FP64 Grams, where B
 *   is the tensor being swept (A, or the truncated tensor of st-HOSVD), G_V =
 *   R^T R and G_L' is the Gram of the quantised L (L^T L)^{-1} the sweep
 *   actually used (no extra tensor work; ||B||^2 comes from the initial pass).
 *   The subtraction cancels: with FP32 accumulation its absolute error is a
 *   few 2^-24 ||B||^2 / sqrt(J / I_n) in res^2, which decides the stop test
 *   when the residual is small and eta tight.
 * TK_RESID_EXPLICIT: res^2 = sum_j ||a_j - L v_j||^2 accumulated during the
 *   sweep from the fibres themselves (one more small contraction per fibre;
 *   no extra HBM traffic; free of that cancellation).
 * TK_RESID_AUTO (default): per mode, TRACE for FP64 storage; for FP32 and BF16
 *   storage EXPLICIT when the trace form cannot resolve the stop test at a
 *   relative residual of 1e-4, i.e. when 4 * 2^-24 * sqrt((I_n + 64) / J)
 *   exceeds 1e-4 * eta (J = prod_{k != n} of the swept tensor's dims), TRACE
 *   otherwise (and when eta == 0).  tk_als_info.resid_form reports the choice. */
typedef enum {
  TK_RESID_AUTO = 0,
  TK_RESID_TRACE = 1,
  TK_RESID_EXPLICIT = 2
} tk_resid_mode;

/* Arithmetic of the tensor contractions.  Only TK_COMPUTE_AS_STORAGE exists:
 * FP64 data contracts in FP64, FP32 and BF16 data on the matrix cores with
 * FP32 accumulation (FP32 operands of BF16 products split exactly into BF16
 * terms).  Other values are rejected with TK_ERR_UNSUPPORTED_DTYPE. */
typedef enum {
  TK_COMPUTE_AS_STORAGE = 0
} tk_compute;

/* Options of the ALS drivers.  Zero-initialise, set struct_size =
 * sizeof(tk_als_opts), then override fields; NULL opts means defaults. */
typedef struct {
  size_t struct_size;      /* sizeof(tk_als_opts)                           */
  double tol;              /* eta of eq. E5.01 (default 1e-4, Section 6)     */
  int32_t max_iters;       /* max L-updates per mode (default 50, Section 6) */
  int32_t resid_mode;      /* tk_resid_mode (default TK_RESID_AUTO)           */
  uint64_t seed;           /* seed of the initial sketch S (Section 5)        */
  const int32_t* order;    /* host; st-HOSVD processing order, a permutation
                              of 0..N-1 (Algorithm 3.5); NULL = 0..N-1      */
  int32_t singular_vectors; /* als_thosvd only: nonzero replaces each factor
                              by the singular vectors of A_(n) within its
                              span (Section 3, after Algorithm 3.4); 0 keeps
                              the QR basis (default)                        */
  int32_t compute;         /* tk_compute (default TK_COMPUTE_AS_STORAGE)      */
  const void* const* init_U; /* host array of N device pointers or NULL: the
                              initial guess L_0 of Algorithm 3.3 per mode
                              (I_n x R_n row-major, full column rank, FP64
                              when a_dtype == TK_F64 else FP32), used instead
                              of the Section 5 sketch (a warm start); a NULL
                              entry keeps the sketch for that mode.  Only its
                              span matters: the iteration is started from
                              the Q of its reduced QR.  With a warm start of
                              the first processed mode ||A|| takes one pass
                              of its own.                                   */
} tk_als_opts;

/* Per-call report. */
typedef struct {
  int32_t iters[TK_MAX_ORDER];     /* L-updates performed for mode n        */
  int32_t converged[TK_MAX_ORDER]; /* 1 if eq. E5.01 fired for mode n        */
  double resid[TK_MAX_ORDER];      /* final ALS residual ||B_(n)-L R^T||_F   */
  double norm_a;                   /* ||A||_F of the input                   */
  int32_t sweeps;                  /* tensor sweeps executed in total        */
  int32_t status;                  /* same as the return value               */
  int32_t mode_status[TK_MAX_ORDER]; /* per mode: TK_OK, TK_NOT_CONVERGED, the
                                      failure of that mode (negative; a final
                                      QR's rank deficiency counts for its
                                      mode), or TK_SKIPPED                    */
  int32_t resid_form[TK_MAX_ORDER];  /* TK_RESID_TRACE or TK_RESID_EXPLICIT:
                                      the form mode n's stop test used        */
} tk_als_info;

/* --------------------------------------------------------------------------
 * als_sthosvd -- Algorithm 3.5 (st-HOSVD-ALS).
 *
 * For each mode n in opts->order: ALS (Algorithm 3.3) on the current B_(n)
 * with the initial guess of Section 5 (L_0 = Q of the QR of B_(n) S, S with
 * U[0,1) entries from the counter-based SplitMix64 generator, entry (j, r)
 * of mode n at counter n*2^48 + j*R_n + r of the stream seeded with
 * opts->seed, value (output >> 40) * 2^-24) and the stop test of eq. E5.01
 * against ||A||_F of the input; U_n = Q of the reduced QR of the returned L
 * (diag(R_hat) > 0); then B <- B x_n U_n^T, which equals Algorithm 3.5's
 * R_hat R^T because R is the least-squares solution for that L.  G is the
 * final B.  R_n == I_n yields U_n = identity with no iterations.
 *
 *  A      device, input tensor, dtype a_dtype, dims[0..N-1] row-major.
 *  dims   host, int64[N].        ranks  host, int32[N], 1 <= R_n <= I_n,
 *                                       R_n <= 64 (the r x r small linear
 *                                       algebra runs in one workgroup's LDS)
 *                                       and R_n <= prod_{k != n} R_k.
 *  opts   host or NULL.
 *  U      host array of N device pointers; U[n] receives I_n x R_n
 *         row-major, FP64 when a_dtype == TK_F64, else FP32.
 *  G      device, R_1 x ... x R_N row-major, same dtype as U.
 *  ws     device workspace of ws_bytes >= als_workspace_bytes(1, ...).
 *  info   host or NULL.
 * Returns TK_OK, TK_NOT_CONVERGED or a negative tk_status. */
TK_API int als_sthosvd(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                const int32_t* ranks, const tk_als_opts* opts, void* const* U,
                void* G, void* ws, size_t ws_bytes, tk_als_info* info,
                void* stream);

/* als_sthosvd_noalloc -- als_sthosvd for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation, kernels and results, with the
 * workspace taken from a device array inside the library instead of `ws`.
 * That array holds als_sthosvd_noalloc_max_bytes() bytes (64 MiB) per GPU,
 * exists on every GPU the library runs on until the process ends, and is
 * found on the current device (`stream` must belong to it).  The call
 * allocates nothing (no hipMalloc, hipFree, pinned host buffer or library
 * routine that allocates) and reads its status block through pageable host
 * memory unless this thread already holds the pinned buffer of an earlier
 * als_* call.  Shapes whose als_workspace_bytes(1, ...) exceeds the array
 * return TK_ERR_WORKSPACE_TOO_SMALL before any device work.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * host threads, or work still running on another stream) race and must be
 * serialised by the caller.  Arguments and return values otherwise as for
 * als_sthosvd. */
TK_API int als_sthosvd_noalloc(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                               const int32_t* ranks, const tk_als_opts* opts, void* const* U,
                               void* G, tk_als_info* info, void* stream);

/* Size in bytes of the device array als_sthosvd_noalloc works in. */
TK_API size_t als_sthosvd_noalloc_max_bytes(void);

/* als_thosvd -- Algorithm 3.4 (t-HOSVD-ALS): the per-mode ALS + QR of
 * als_sthosvd on the unchanged A for every mode, then
 * G = A x_1 U_1^T ... x_N U_N^T (Section 2, eq. best).  Arguments as for
 * als_sthosvd; opts->order is ignored.
 * With opts->singular_vectors != 0 each factor is replaced, before the core
 * is formed, by the singular vectors of A_(n) inside the span of the QR basis
 * Q (Section 3, after Algorithm 3.4): U_n = Q W with W the eigenvectors of
 * the FP64 R_n x R_n Gram Q^T A_(n) A_(n)^T Q of C = Q^T A_(n) (one more pass
 * over A per mode; Q enters that pass in the compute dtype), columns in
 * descending order of the singular values, each column of W signed so that
 * its entry of largest magnitude is positive.  The core is then the one of
 * these factors.  Singular vectors are unique up to sign only where the
 * singular values are distinct. */
TK_API int als_thosvd(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
               const int32_t* ranks, const tk_als_opts* opts, void* const* U,
               void* G, void* ws, size_t ws_bytes, tk_als_info* info,
               void* stream);

/* Workspace bytes of als_thosvd (which = 0) or als_sthosvd (which = 1) for
 * the given shape, dtype and ranks; 0 for invalid arguments. */
TK_API size_t als_workspace_bytes(int32_t which, int32_t a_dtype, int32_t N,
                           const int64_t* dims, const int32_t* ranks);

/* --------------------------------------------------------------------------
 * ttm -- mode-n tensor-times-matrix (Section 2):
 *   Y = X x_mode op(M),  Y[..., j, ...] = sum_i X[..., i, ...] op(M)[j, i],
 * op(M) of size J x I_mode.  trans_m == 0: M is stored J x I_mode
 * row-major; trans_m == 1: M is stored I_mode x J row-major (so U^T is used
 * without being materialised).  Y has dims with dims[mode] replaced by J.
 * Supported (x_dtype, m_dtype, y_dtype): (F64, F64, F64), (F32, F32, F32),
 * (BF16, F32, F32).  Asynchronous on `stream`. */
TK_API int ttm(const void* X, int32_t x_dtype, int32_t N, const int64_t* dims,
        int32_t mode, const void* M, int32_t m_dtype, int64_t J,
        int32_t trans_m, void* Y, int32_t y_dtype, void* stream);

/* tucker_reconstruct -- A_hat = G x_1 U_1 x_2 ... x_N U_N (Section 2).
 * G device R_1 x ... x R_N; U host array of N device pointers, U[n] is
 * I_n x R_n row-major; out device I_1 x ... x I_N.  dtype is TK_F64 or
 * TK_F32 for G, U and out alike.  ws: device, >= the query's bytes (holds
 * the intermediate expansions).  Asynchronous on `stream`. */
TK_API int tucker_reconstruct(const void* G, int32_t dtype, int32_t N,
                       const int32_t* ranks, const int64_t* dims,
                       const void* const* U, void* out, void* ws,
                       size_t ws_bytes, void* stream);

TK_API size_t tucker_reconstruct_workspace_bytes(int32_t dtype, int32_t N,
                                          const int32_t* ranks,
                                          const int64_t* dims);

/* --------------------------------------------------------------------------
 * contract_allbut -- K = X_(mode) Y_(mode)^T, the contraction of two tensors
 * over every mode except `mode`.  X has dims xdims (I_mode = xdims[mode]),
 * Y has the same dims except ydims[mode] = J.  K is I_mode x J row-major,
 * FP64 when the inputs are FP64, else FP32.  This is the gradient of a
 * mode-n product with respect to its matrix: for Y = X x_n M,
 * dL/dM = (dL/dY)_(n) X_(n)^T (adjoint of the Section 2 definition).
 * Inputs (F64, F64) or (F32, F32); 1 <= J <= 64 (TK_ERR_INVALID_ARG
 * otherwise).  ws >= contract_allbut_workspace_bytes.
 * Asynchronous on `stream`. */
TK_API int contract_allbut(const void* X, const void* Y, int32_t dtype, int32_t N,
                    const int64_t* xdims, int32_t mode, int64_t J, void* K,
                    void* ws, size_t ws_bytes, void* stream);

TK_API size_t contract_allbut_workspace_bytes(int32_t dtype, int32_t N,
                                       const int64_t* xdims, int32_t mode,
                                       int64_t J);

/* --------------------------------------------------------------------------
 * Single steps of the ALS mode solve, exposed for step-by-step checking.
 *
 * als_init_step: Section 5 initial guess on the mode-`mode` view of A.
 *   Y = A_(mode) S (I_mode x R, FP64 out, device) with S as in als_sthosvd,
 *   then L0 = Q of the reduced QR of Y (FP64, device, may alias nothing);
 *   *norm2 (host) receives ||A||_F^2.  1 <= R <= min(I_mode, 64).
 *   ws >= als_workspace_bytes(1, ...) for a tensor of these dims with all
 *   ranks equal to R.
 *
 * als_sweep_step: one sweep of Algorithm 3.3 from L_k (FP64 I_mode x R,
 *   device): R_k = A_(mode)^T L_k (L_k^T L_k)^{-1} (never stored),
 *   L_{k+1} = A_(mode) R_k (R_k^T R_k)^{-1} written to L_next (FP64,
 *   device), *res2 (host) receives ||A_(mode) - L_k R_k^T||_F^2 computed as
 *   selected by resid_mode (TK_RESID_TRACE or TK_RESID_EXPLICIT; AUTO is
 *   rejected here) with norm2 = ||A||_F^2.  1 <= R <= min(I_mode, 64).
 *
 * qr_f64: reduced QR of the FP64 m x r (row-major, device) matrix L into
 *   Q (m x r, device) with diag(R_hat) > 0 (CholeskyQR2 in FP64),
 *   1 <= r <= min(m, 64).  R_hat is not returned: Rhat is reserved and must
 *   be NULL (TK_ERR_INVALID_ARG otherwise).  ws: device, at least
 *   m*r*8 + 3*65536 bytes.  Blocks until done.  Returns
 *   TK_ERR_RANK_DEFICIENT when the Gram fails the pivot test. */
TK_API int als_init_step(const void* A, int32_t a_dtype, int32_t N,
                  const int64_t* dims, int32_t mode, int32_t R, uint64_t seed,
                  void* Y, void* L0, double* norm2, void* ws, size_t ws_bytes,
                  void* stream);

TK_API int als_sweep_step(const void* A, int32_t a_dtype, int32_t N,
                   const int64_t* dims, int32_t mode, int32_t R,
                   const void* L, void* L_next, double norm2,
                   int32_t resid_mode, double* res2, void* ws,
                   size_t ws_bytes, void* stream);

TK_API int qr_f64(const void* L, int64_t m, int32_t r, void* Q, void* Rhat,
           void* ws, size_t ws_bytes, void* stream);

/* als_sweep_kernel: the tensor-streaming part of one ALS sweep alone
 * (the R- and L-updates of Algorithm 3.3 without their small solves), for
 * timing and step checking.  With Lq = L_k (L_k^T L_k)^{-1} (FP32, I_mode x R,
 * device): V = A_(mode)^T Lq (never stored), GV = V^T V (FP64 R x R) and
 * Lacc = A_(mode) V (FP64 I_mode x R).  When `reduce` is 0 only the
 * streaming kernel runs and leaves per-workgroup partials in ws (Lacc and
 * GV are untouched); with 1 the partials are summed in a fixed order into
 * Lacc and GV.  For BF16 storage Lq is first rounded to BF16 precision
 * (round to nearest even), as the drivers quantise L~ for BF16 sweeps with
 * the trace residual (which uses the Gram of the rounded values):
 * V = A^T round(Lq).
 * Shapes outside the fused kernels' range (FP64 storage, I_mode > 1024,
 * R > 48) use the two-pass kernels.  a_dtype F32 or BF16.
 * ws >= als_workspace_bytes(1, ...) for a tensor of these dims with all
 * ranks equal to R.  Asynchronous on `stream`. */
TK_API int als_sweep_kernel(const void* A, int32_t a_dtype, int32_t N,
                            const int64_t* dims, int32_t mode, int32_t R,
                            const float* Lq, double* Lacc, double* GV,
                            int32_t reduce, void* ws, size_t ws_bytes,
                            void* stream);

/* --------------------------------------------------------------------------
 * als_sthosvd_batched -- Algorithm 3.5 for `count` independent order-3
 * tensors in one persistent device launch sequence captured in a HIP graph.
 *
 *  A_packed  device; tensor t occupies A_packed[a_off[t] ...] (elements),
 *            row-major with dims dims3[3t..3t+2].
 *  dims3     host int64[3*count];  ranks3 host int32[3*count].
 *  a_off     host int64[count] element offsets into A_packed.
 *  U_packed  device FP32; factor n of tensor t at u_off[3t+n], I_n x R_n.
 *  G_packed  device FP32; core of tensor t at g_off[t].
 *  u_off     host int64[3*count];  g_off host int64[count].
 *  opts      host or NULL (order ignored: natural order).
 *  iters     host int32[3*count] or NULL: L-updates per (tensor, mode).
 *  status    host int32[count] or NULL: per-tensor tk_status.
 * a_dtype must be TK_F32.  Returns the worst status over the batch. */
TK_API int als_sthosvd_batched(const void* A_packed, int32_t a_dtype, int32_t count,
                        const int64_t* dims3, const int32_t* ranks3,
                        const int64_t* a_off, const tk_als_opts* opts,
                        void* U_packed, const int64_t* u_off, void* G_packed,
                        const int64_t* g_off, int32_t* iters, int32_t* status,
                        void* ws, size_t ws_bytes, void* stream);

TK_API size_t als_sthosvd_batched_workspace_bytes(int32_t count, const int64_t* dims3,
                                           const int32_t* ranks3);

/* --------------------------------------------------------------------------
 * hooi_refine -- HOOI (higher-order orthogonal iteration) started from the
 * caller's factors, the refinement the paper applies to t-/st-HOSVD results
 * (Section 6.3, Table 6.3-2).  One outer iteration updates, for n = 0..N-1
 * in turn, U_n to an orthonormal basis of the dominant R_n-dimensional left
 * subspace of Y_(n), Y = A x_{k != n} U_k^T: ALS (Algorithm 3.3, options from
 * opts: tol, max_iters, resid_mode; the E5.01 test against ||A||_F) on Y_(n),
 * warm-started from the current U_n, then the reduced QR (diag(R_hat) > 0).
 * After the last mode G = Y x_{N-1} U_{N-1}^T and the error
 * e = sqrt(||A||^2 - ||G||^2) / ||A|| (orthonormal factors); the iteration
 * stops when |e_prev - e| <= tol, e_prev starting at the error of the given
 * factors.  With FP32/BF16 storage ||G||^2 comes from the FP32 core, whose
 * rounding leaves an absolute error of a few 1e-9 on e^2: e is meaningful
 * down to about 3e-4, and below that tol should not be relied on (use
 * max_iters, and measure the error by reconstruction).
 *  A      device, input tensor (dtype a_dtype), as for als_thosvd.
 *  U      host array of N device pointers, in/out: I_n x R_n row-major with
 *         orthonormal columns on entry (FP64 when a_dtype == TK_F64, else
 *         FP32), overwritten by the refined factors.
 *  G      device, R_1 x ... x R_N, same dtype as U: the core of the result.
 *  tol    >= 0, stop tolerance on the change of e.  max_iters >= 0 outer
 *         iterations (0: only the error of the given factors and their core).
 *  ws     device workspace of ws_bytes >= hooi_workspace_bytes(...).
 *  info   host or NULL.
 * Returns TK_OK, TK_NOT_CONVERGED (max_iters reached) or a negative
 * tk_status. */
typedef struct {
  int32_t iters;       /* outer iterations performed                        */
  int32_t converged;   /* 1 if |e_prev - e| <= tol was reached               */
  double relerr_init;  /* e of the given factors                             */
  double relerr;       /* e of the returned factors                          */
  double norm_a;       /* ||A||_F                                           */
  int32_t sweeps;      /* ALS sweeps over all inner solves                   */
  int32_t status;      /* same as the return value                          */
} tk_hooi_info;

TK_API int hooi_refine(const void* A, int32_t a_dtype, int32_t N, const int64_t* dims,
                       const int32_t* ranks, const tk_als_opts* opts, double tol,
                       int32_t max_iters, void* const* U, void* G, void* ws,
                       size_t ws_bytes, tk_hooi_info* info, void* stream);

TK_API size_t hooi_workspace_bytes(int32_t a_dtype, int32_t N, const int64_t* dims,
                                   const int32_t* ranks);

/* --------------------------------------------------------------------------
 * st_order_auto -- a processing order for als_sthosvd chosen by the cost
 * model in the proof of Prop. 1 (eq. 2.2): the permutation (i_1, ..., i_N)
 * minimising sum_n R_{i_1} ... R_{i_n} * I_{i_n} ... I_{i_N} over all N!
 * orders (exact integer arithmetic), the first in lexicographic order among
 * equal costs.  With equal dimensions this is the order of ascending ranks
 * (Prop. 1).  Host only: touches no device and needs no GPU.
 *  dims   host, int64[N];  ranks host, int32[N] (as for als_sthosvd).
 *  order  host, int32[N] receives the permutation.
 * Returns TK_OK or TK_ERR_INVALID_ARG. */
TK_API int st_order_auto(int32_t N, const int64_t* dims, const int32_t* ranks, int32_t* order);

/* Human-readable name of a tk_status value (static storage). */
TK_API const char* tk_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_ALS_H */
