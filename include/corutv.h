/*
 * corutv.h -- C ABI of libcorutv, an MI355X (gfx950) implementation of
 * Compressed Randomized UTV (CoR-UTV) and of ALM-CoRUTV robust PCA.
 *
 * Method (Kaloorazi & de Lamare, "Study of Compressed Randomized UTV
 * Decompositions for Low-Rank Matrix Approximations in Data Science"):
 *   Sec. 3.1, eqs. 4-9 and Algorithm 1: for A (m x n), l = k + p and q power
 *   iterations, draw a standard Gaussian test matrix Omega (n x l), sketch
 *   C1 = A Omega and C2 = A^T C1 (repeated q + 1 times), take thin QR bases
 *   Q1, Q2, compress D = Q1^T A Q2 (l x l), factor D P = Qt R by column-pivoted
 *   QR and return A ~ U T V^T with U = Q1 Qt, T = R, V = Q2 P.
 *   Sec. 4, Algorithm 2 with eq. 12: robust PCA M = L + S by the inexact
 *   augmented Lagrange multiplier method with CoR-UTV thresholding.
 *
 * Conventions shared by every entry point
 *   - All matrix pointers are DEVICE pointers on the context's device; the
 *     caller owns and allocates them.  The library never allocates device
 *     memory: every scratch buffer is carved from the workspace handed to
 *     corutv_create.
 *   - Host pointers are marked "host".  Nothing is retained after a call
 *     returns, except for corutv_submit (see there).
 *   - Integer sizes are int64_t; element types are given by corutv_dtype.
 *   - Return value: CORUTV_OK (0) or a negative error code; CORUTV_PENDING (1)
 *     only from corutv_poll.  No C++ exception crosses this boundary.  After
 *     CORUTV_E_INVAL no output has been touched; after other errors outputs
 *     are unspecified.  CORUTV_E_DEVICE poisons the context (destroy it).
 *   - Blocking calls enqueue on the context's first stream and synchronize it
 *     before returning.
 *   - Workspace: blocking calls and serving requests take their scratch
 *     ranges from one first-fit arena over the workspace, under the context's
 *     lock, so they never overlap.  A blocking call made while requests are
 *     in flight waits until its range is free (new admissions pause until
 *     it has one) and then runs beside them.
 */
#ifndef CORUTV_H
#define CORUTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define CORUTV_OK 0
#define CORUTV_PENDING 1      /* corutv_poll: request queued or running       */
#define CORUTV_E_INVAL -1     /* bad argument: sizes, pointers, layout, enums */
#define CORUTV_E_NOMEM -2     /* workspace too small for the request          */
#define CORUTV_E_BUSY -3      /* serving queue full                           */
#define CORUTV_E_NUMERIC -4   /* NaN/Inf in the input or an unrecoverable QR  */
#define CORUTV_E_DEVICE -5    /* HIP runtime error; context is poisoned       */
#define CORUTV_E_NOTFOUND -6  /* unknown ticket                               */

/* ---- enums -------------------------------------------------------------- */
enum corutv_dtype { CORUTV_F64 = 0, CORUTV_F32 = 1 };
enum corutv_layout { CORUTV_COL_MAJOR = 0, CORUTV_ROW_MAJOR = 1 };
/* Arithmetic of the passes over A (sketches, power products, core pass).
 * F64: double operands on FP64 matrix cores.  F32: float operands on FP32
 * matrix cores.  BF16: float A and operands rounded to nearest-even bfloat16
 * in the tile loader, FP32 accumulation, for the first sketch and the power
 * iterations; the second sketch Z = A^T Q1 and the core pass A Q2, which give
 * the returned factors directly, run in the BF16X3 form.  BF16X3: every pass
 * splits x = hi + lo into two bfloat16 parts and accumulates
 * lo*hi + hi*lo + hi*hi in FP32.  In every form
 * the Gram matrices, Cholesky factors, the l x l core and its QRCP are FP64.
 * F64 needs an F64 A; F32/BF16/BF16X3 need an F32 A.
 * The thin QRs of the sketches are CholeskyQR2 (two CholeskyQR steps).  In
 * the F32/BF16/BF16X3 forms, whose bases are stored in FP32, a QR stops after
 * the first step when u l (||R1||_F ||R1^-1||_F)^2 <= 2^-24 (u = 2^-53): the
 * first step's loss of orthogonality, of order u cond(sketch)^2, is then
 * below FP32 rounding. */
enum corutv_prec { CORUTV_PREC_F64 = 0, CORUTV_PREC_F32 = 1, CORUTV_PREC_BF16 = 2, CORUTV_PREC_BF16X3 = 3 };
/* Triangle of T.  AUTO follows Sec. 3: upper for m >= n, and for m < n the
 * method runs on A^T and returns a lower T.  UPPER/LOWER force the triangle
 * (LOWER on m >= n factors D^T by QRCP: U = Q1 P, T = R^T, V = Q2 Qt). */
enum corutv_tri { CORUTV_TRI_AUTO = 0, CORUTV_TRI_UPPER = 1, CORUTV_TRI_LOWER = 2 };

/* Dense matrix descriptor: element (i, j) lives at
 *   ptr[i + j*ld]  (COL_MAJOR, ld >= rows)   or   ptr[i*ld + j]  (ROW_MAJOR, ld >= cols). */
typedef struct corutv_mat {
  void* ptr;       /* device pointer                                   */
  int64_t rows;
  int64_t cols;
  int64_t ld;
  int32_t dtype;   /* enum corutv_dtype                                */
  int32_t layout;  /* enum corutv_layout                               */
} corutv_mat;

typedef struct corutv_opts {
  int32_t prec;      /* enum corutv_prec                                     */
  int32_t tri;       /* enum corutv_tri                                      */
  int32_t want_err;  /* nonzero: compute ||A - U T V^T||_F / ||A||_F (one    */
                     /* extra pass over A, not part of the method)           */
  int32_t flags;     /* CORUTV_FLAG_* bits; other bits must be 0             */
  int32_t panel_rows; /* CORUTV_FLAG_A_HOST: storage rows of A per staged    */
                      /* panel (rows if ROW_MAJOR, columns if COL_MAJOR);    */
                      /* 0 selects 4096. Ignored otherwise                   */
} corutv_opts;

/* corutv_opts.flags: form the core from the R factor of the second sketch
 * instead of a third pass over A.  With Q2 R_Z = Z = A^T Q1 the core is
 * D = Q1^T A Q2 = R_Z^T exactly (Sec. 3.1, eqs. 5-7), so the decomposition
 * needs 2q + 2 passes instead of 2q + 3 and returns the same factors in exact
 * arithmetic (in floating point D differs at the rounding level of the passes).
 * This is also the paper's single-revisit core Q1^T C1 (Q2^T Psi)^+ (Sec. 3.1,
 * Algorithm 1): since Q1^T A = R_Z^T Q2^T, that expression equals R_Z^T
 * whenever Q2^T Psi has full rank. */
#define CORUTV_FLAG_CORE_FROM_RZ 1
/* corutv_opts.flags: A->ptr is a host pointer.  The method only reads A in
 * whole passes (Sec. 3.1 counts its cost in passes over data stored
 * externally), so each pass streams A through the device in panels of
 * panel_rows storage rows, two staging panels in the workspace, the copy of
 * one panel overlapping the products of the other.  Pinned host memory
 * (hipHostMalloc) is needed for the overlap; pageable memory works, slower.
 * F64 and F32 forms only, want_err must be 0, blocking corutv_decompose
 * only (not the serving queue).  The workspace must hold the staging panels:
 * size it with corutv_workspace_bytes_host. */
#define CORUTV_FLAG_A_HOST 2

typedef struct corutv_info {
  double rel_err;        /* relative Frobenius error if want_err, else -1       */
  double a_fro;          /* ||A||_F if want_err, else -1                        */
  double gpu_ms;         /* device time of the whole decomposition              */
  int32_t ell;           /* l = k + p                                           */
  int32_t transposed;    /* 1 when the wide problem was solved on A^T           */
  int32_t tri;           /* CORUTV_TRI_UPPER or CORUTV_TRI_LOWER returned       */
  int32_t qr_fallbacks;  /* tall-skinny QRs that fell back to Householder       */
  int32_t passes;        /* passes over A: 2q + 3 (+1 with want_err)            */
  int32_t qr_one_step;   /* tall-skinny QRs that stopped after one CholeskyQR   */
                         /* step (F32/BF16/BF16X3 only; see corutv_prec)       */
} corutv_info;

typedef struct corutv_config {
  int32_t device;            /* HIP device ordinal                                   */
  int32_t n_streams;         /* >= 1; streams[0] is the context stream, the rest     */
                             /* are serving slots                                    */
  void* const* streams;      /* host array of hipStream_t (may hold 0 = null stream) */
  void* workspace;           /* device buffer, 256-byte aligned                      */
  uint64_t workspace_bytes;
  int32_t max_queue;         /* serving queue capacity (0 -> 4096)                   */
  uint32_t flags;            /* reserved, 0                                          */
} corutv_config;

typedef struct corutv_ctx corutv_ctx;

/* Create a context bound to cfg->device, its streams and workspace.  The
 * workspace and streams must stay valid until corutv_destroy.  Returns
 * E_INVAL for an unaligned workspace, a null one with nonzero
 * workspace_bytes, or n_streams < 1.  A null workspace with zero bytes makes
 * a context for corutv_decompose_noalloc (every other call then returns
 * E_NOMEM).  Creation also looks up, once per device, the device address of
 * the library's fixed scratch array used by corutv_decompose_noalloc. */
int corutv_create(corutv_ctx** out, const corutv_config* cfg);

/* Drain (finish) every queued or running request, stop the serving thread
 * and free host-side state.  Device memory is the caller's. */
int corutv_destroy(corutv_ctx* ctx);

/* Workspace bytes one decomposition of an m x n matrix needs (closed form,
 * independent of the data).  Returns 0 for invalid sizes. */
uint64_t corutv_workspace_bytes(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q, int32_t prec);
/* Workspace for corutv_decompose with CORUTV_FLAG_A_HOST: the bytes of
 * corutv_workspace_bytes plus two staging panels of panel_rows (0: 4096)
 * storage rows of an m x n A of the given layout (enum corutv_layout) in the
 * dtype of prec.  Returns 0 for invalid arguments or a BF16 form. */
uint64_t corutv_workspace_bytes_host(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q, int32_t prec,
                                     int32_t layout, int32_t panel_rows);

/* Rank-l CoR-UTV of A (Sec. 3.1, eqs. 4-9; Algorithm 1 with q power steps).
 *   A     m x n, F64 or F32 as opts->prec requires, either layout; read only.
 *   k, p  target rank and oversampling, l = k + p; need k >= 1, p >= 0,
 *         l <= min(m, n), l <= 256.  q >= 0 power iterations.
 *   seed  key of the Philox4x64-10 stream of Omega; entry (i, j) of Omega is
 *         the Box-Muller normal of the block at counter (i, j, 0, 0), key
 *         (seed, 0): words w0, w1 give u1 = ((w0 >> 11) + 1) 2^-53 and
 *         u2 = (w1 >> 11) 2^-53, z = sqrt(-2 ln u1) cos(2 pi u2), with ln
 *         and cos fixed as truncated series evaluated without fused
 *         multiply-add (12-term atanh series for ln, exact quadrant
 *         reduction and degree-18 Taylor polynomials for cos), so the
 *         stream is reproducible bit for bit (see corutv_omega).
 *   U     m x l, V  n x l: outputs, F64 or F32, either layout.
 *   T     l x l FP64 output, column-major with leading dimension ldt >= l;
 *         the other triangle is stored as exact zeros.
 *   piv   nullable, l int32 device entries: the column permutation of the
 *         QRCP (UPPER: D[:, piv] = Qt R; LOWER: D^T[:, piv] = Qt R).
 *   info  nullable host struct.
 * Blocking.  E_NUMERIC if A holds NaN/Inf. */
int corutv_decompose(corutv_ctx* ctx, const corutv_mat* A, int32_t k, int32_t p, int32_t q,
                     uint64_t seed, const corutv_opts* opts, corutv_mat* U, double* T,
                     int64_t ldt, corutv_mat* V, int32_t* piv, corutv_info* info);

/* corutv_decompose for callers that cannot allocate device memory, e.g.
 * code under HIP graph capture, tight serving loops, or hosts that forbid
 * hipMalloc.  Same arguments, validation, kernels and results (bit for bit)
 * as corutv_decompose; CORUTV_FLAG_A_HOST is rejected (E_INVAL).  Its
 * scratch is not carved from the context's workspace but from a fixed array
 * of 64 MiB inside the library's device memory, one per device, held until
 * the process ends; the call itself allocates nothing (no hipMalloc,
 * hipFree, event or stream creation).  A decomposition whose workspace
 * (corutv_workspace_bytes) exceeds 64 MiB returns E_NOMEM -- e.g. a
 * 2000 x 1500 F64 matrix at l = 30 needs 35 MiB, a 20000 x 15000 one at
 * l = 110 needs 450 MiB.  Every call on one device shares that device's
 * array and leaves its contents behind; the call clears what must start at
 * zero itself.  Calls that overlapped on one device would race on the
 * array, so within a process each call holds a per-device lock for its whole
 * (blocking) duration and calls run one after another; other processes have
 * their own copy.  Blocking, on the context stream. */
int corutv_decompose_noalloc(corutv_ctx* ctx, const corutv_mat* A, int32_t k, int32_t p, int32_t q,
                             uint64_t seed, const corutv_opts* opts, corutv_mat* U, double* T,
                             int64_t ldt, corutv_mat* V, int32_t* piv, corutv_info* info);

/* ALM-CoRUTV robust PCA (Sec. 4, Algorithm 2; operators of eq. 12).
 *   M      m x n F32 input (read only).  S: m x n F32 output (the sparse part).
 *          The iteration state (multiplier, next CoR-UTV input) and every
 *          CoR-UTV of the loop are FP64 (opts->prec is ignored): the shrink
 *          threshold lambda/mu falls below FP32 resolution late in the run.
 *   L      nullable m x n F32 output (the low-rank part, formed densely).
 *   lambda <= 0 selects 1/sqrt(max(m, n)).
 *   k, p, q: the CoR-UTV of every iteration (l = k + p <= 256).
 *   max_iter iterations, stopping early once ||M-L-S||_F < tol ||M||_F if tol > 0.
 *   Iteration j draws its test matrix with counter word 3 = j; mu_0 =
 *   1.25 / T[0,0] of a CoR-UTV of M (word 3 = 0xFFFF), mu_{j+1} =
 *   min(1.5 mu_j, 1e7 mu_0); Y_0 = S_0 = 0.
 *   info   nullable host struct. */
typedef struct corutv_rpca_info {
  int32_t iters;
  int32_t final_rank;   /* r of the last thresholding                        */
  double zeta;          /* ||M - L - S||_F / ||M||_F after the last iteration */
  double mu0;
  double mu;            /* mu after the last update                           */
  double gpu_ms;
  double step_ms;       /* summed duration of the fused elementwise kernel over
                           the iterations when pass timing is on, else 0     */
} corutv_rpca_info;
int corutv_rpca(corutv_ctx* ctx, const corutv_mat* M, double lambda, int32_t k, int32_t p,
                int32_t q, int32_t max_iter, double tol, uint64_t seed, const corutv_opts* opts,
                corutv_mat* L, corutv_mat* S, corutv_rpca_info* info);
/* Workspace bytes corutv_rpca needs for an m x n input (0 for invalid sizes). */
uint64_t corutv_rpca_workspace_bytes(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q);
/* The rank history of the last successful corutv_rpca call on ctx (Sec. 4,
 * Algorithm 2, eq. 12): r_j, the number of diagonal entries of T_j above
 * 1/mu_j that iteration j kept, for the first min(iterations, 4096)
 * iterations.  Writes min(n, that count) entries to ranks (host memory,
 * nullable when n = 0) and the count to *count (nullable).  Returns E_INVAL
 * for a null ctx or n < 0. */
int corutv_rpca_ranks(corutv_ctx* ctx, int32_t* ranks, int32_t n, int32_t* count);

/* ---- serving ------------------------------------------------------------
 * Non-blocking decompositions with continuous batching: requests queue on the
 * host, a scheduler thread admits each one as soon as a serving slot (stream)
 * and enough workspace are free, and several admitted requests run
 * concurrently on different streams.  Kernel configurations depend only on
 * the request's shape, so a result is bit-identical alone and in a mix.
 * The request descriptor is copied; A, U, T, V and piv must stay valid and
 * unmodified until the ticket completes.  The request is ordered after the
 * work queued on the context stream (streams[0]) when corutv_submit is
 * called: an event recorded there is waited for before its first kernel. */
typedef struct corutv_request {
  corutv_mat A;
  corutv_mat U;
  corutv_mat V;
  double* T;
  int64_t ldt;
  int32_t* piv;     /* nullable */
  int32_t k, p, q;
  int32_t priority; /* reserved, 0 */
  uint64_t seed;
  corutv_opts opts;
} corutv_request;

/* Returns OK (admitted or queued), E_BUSY (queue full: max_queue requests
 * waiting for admission), E_NOMEM (footprint larger than the whole
 * workspace: can never run) or E_INVAL. */
int corutv_submit(corutv_ctx* ctx, const corutv_request* req, uint64_t* ticket);
/* PENDING while queued or running; OK once outputs are valid (info filled,
 * ticket retired); otherwise the request's error code (ticket retired).
 * E_NOTFOUND for unknown or retired tickets.  Thread safe. */
int corutv_poll(corutv_ctx* ctx, uint64_t ticket, corutv_info* info);
/* Cancel a request that has not started (OK) -- running ones finish. */
int corutv_cancel(corutv_ctx* ctx, uint64_t ticket);
/* Block until the ticket completes; same results as corutv_poll. */
int corutv_wait(corutv_ctx* ctx, uint64_t ticket, corutv_info* info);

const char* corutv_strerror(int code);

/* ---- measurement ---------------------------------------------------------
 * When enabled, corutv_decompose records HIP events on its stream around
 * every pass over A (the sketch kernels of eqs. 4, 5 and 7 and the power
 * products of Algorithm 1) and accumulates their device time; the residual
 * pass of want_err is not included.  Disabled by default; enabling or
 * reading clears nothing else. */
typedef struct corutv_pass_stats {
  int64_t passes;      /* passes timed since the last reset               */
  double total_ms;     /* summed device time of those passes              */
  double min_ms;       /* fastest single pass                             */
  double max_ms;       /* slowest single pass                             */
} corutv_pass_stats;
int corutv_pass_timing(corutv_ctx* ctx, int32_t enable, int32_t reset);
/* Test hook for the error path: the after_checks-th next launch check of a
 * call on this context (counting from 1) reports a HIP error, as a failed
 * launch would: that call returns CORUTV_E_DEVICE and poisons the context
 * (every later call returns CORUTV_E_DEVICE, queued requests complete with
 * it).  No device fault is caused; kernels already queued run normally.
 * 0 disarms. */
int corutv_debug_inject_failure(corutv_ctx* ctx, int32_t after_checks);
int corutv_get_pass_stats(corutv_ctx* ctx, corutv_pass_stats* out);

/* ---- single steps (parity checks and diagnostics) -----------------------
 * Each runs one stage of the pipeline on caller buffers, blocking. */

/* Omega (n x l) of the Gaussian stream above with counter word 3 = sub,
 * written column-major with leading dimension ld >= n as F64 or F32 (F32 is
 * the round-to-nearest-even of the F64 value). */
int corutv_omega(corutv_ctx* ctx, int64_t n, int32_t ell, uint64_t seed, uint32_t sub,
                 int32_t dtype, void* out, int64_t ld);

/* One pass over A: Y = A X (trans = 0, X n x l, Y m x l) or Y = A^T X
 * (trans = 1, X m x l, Y n x l) in the arithmetic prec; X, Y column-major F64
 * (prec F64) or F32 (other precs); Y holds the FP32/FP64 accumulation. */
int corutv_sketch(corutv_ctx* ctx, const corutv_mat* A, int32_t trans, int32_t prec,
                  const void* X, int64_t ldx, int32_t ell, void* Y, int64_t ldy);

/* Thin QR of an F64 column-major X (rows x l, rows >= l) by CholeskyQR2 with
 * FP64 Gram and Cholesky, falling back to Householder QR when a Cholesky
 * factor breaks down (eq. 6).  Q (rows x l, F64, ldq) with diag(R) >= 0;
 * R nullable (l x l upper, column-major, ldr).  *fallback (host, nullable)
 * is set to 1 when the Householder path ran. */
int corutv_tsqr(corutv_ctx* ctx, const double* X, int64_t rows, int32_t ell, int64_t ldx,
                double* Q, int64_t ldq, double* R, int64_t ldr, int32_t* fallback);

/* Column-pivoted QR of a square l x l FP64 matrix D (eq. 8), column-major
 * with leading dimension ldd:  D[:, piv] = Qt R, diag(R) >= 0.  Pivot rule:
 * largest trailing column norm, recomputed from scratch at every step (no
 * downdating); ties to the lowest column position.  The norms are reduced in
 * the kernel's own fixed order (per-lane partial sums and fused
 * multiply-adds), so the result is a deterministic function of the input
 * bits; another summation order changes a norm only by rounding, so the
 * pivot differs from a sequential-order QRCP only where the two largest
 * trailing norms lie within that rounding of each other.  Qt, R column-major
 * with leading dimension l. */
int corutv_qrcp(corutv_ctx* ctx, int32_t ell, const double* D, int64_t ldd, double* Qt,
                double* R, int32_t* piv);

#ifdef __cplusplus
}
#endif
#endif /* CORUTV_H */
