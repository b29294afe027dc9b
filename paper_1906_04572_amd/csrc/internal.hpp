// Internal declarations of libcorutv (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

#include "../../include/corutv.h"

namespace corutv {

// Skinny matrices (m x l, n x l) live column-major as [ellp][ld] with the
// column count padded to a multiple of 16 (MFMA tile) and zero padding.
constexpr int kPadL = 16;
__host__ __device__ inline int pad_ell(int ell) { return (ell + kPadL - 1) / kPadL * kPadL; }
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Arithmetic of one pass over A.
enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 };

// Geometry of the partial tiles a stream-K sketch pass writes.  The pass
// splits the reduction into 8 chunks (one per XCD); inside a chunk the
// (tile, k-block) units are divided evenly over gx workgroups.  Partial tile
// (x, j, slot) holds workgroup j of chunk x's contribution to output tile
// (first tile of j) + slot, laid out [ellp][tw].
struct Partials {
  void* ptr = nullptr;    // float (F32/BF16 forms) or double (F64)
  int elem = 4;           // bytes per element
  int ellp = 0;
  int tw = 0;             // output rows per tile
  int tiles = 0;
  int nchunk = 8;         // K chunks: 8 (chunk x on XCD x) or 1 (short K)
  int nkx = 0;            // k-blocks per chunk
  int gx = 0;             // workgroups per chunk
  int maxslot = 0;
  int64_t n = 0;          // output length
  bool direct = false;    // the pass wrote its output itself (nothing to sum)
};


// ---- launchers (return hipError_t) ----------------------------------------
hipError_t launch_omega(int64_t n, int ell, int ellp, uint64_t seed, uint32_t sub, double* out64,
                        float* out32, int64_t ld, hipStream_t st);

// One pass over a row-major R x C matrix: trans = 0 -> out (R x l) = A S^T-operand,
// i.e. Y = A W with W (C x l) stored as S[c*lds + j]; trans = 1 -> Z (C x l) = A^T Q
// with Q (R x l) stored as S[c*lds + i].  Writes partial tiles into `part`
// (whose geometry is filled in here).
// part_elems: capacity of part_buf in elements; the grid shrinks to fit.
// sbf: for the bf16 forms, scratch of sketch_bf16_bytes(ellp, lds) bytes that
// receives the bf16 hi/lo split of S (unused otherwise, may be null).
// out (optional): where launch_sum_partials(part, ell, ellp, out, nullptr,
// ldo) would put the result.  When the reduction is short (one K chunk) and
// the output has at least num_cu tiles, each workgroup then takes one whole
// tile and writes it there (FP64, columns ell..ellp-1 zero); part->direct
// is set and launch_sum_partials does nothing.
hipError_t launch_sketch(int prec, int trans, const void* A, int64_t lda, int64_t R, int64_t C,
                         const void* S, int64_t lds, int ellp, void* part_buf, int64_t part_elems,
                         Partials* part, int num_cu, hipStream_t st, void* sbf, double* out = nullptr,
                         int64_t ldo = 0, int ell = 0);
inline size_t sketch_bf16_bytes(int ellp, int64_t lds) { return 2 * (size_t)ellp * lds * 2; }
// Capacity (elements) that covers every grid launch_sketch may pick on a
// 256-CU device.
int64_t partials_capacity(int64_t n_out, int64_t k_len, int ellp, int prec);

// y[c*ld + i] += x[c*ld + i] for i < rows, c < cols (FP64, column-major).
hipError_t launch_add_cols(double* y, const double* x, int64_t rows, int cols, int64_t ld, hipStream_t st);

// out64[c*ld + i] = sum of the partial tiles for row i (i < n, c < ell); zero for
// ell <= c < ncols.  Optionally also out32 (float copy).
hipError_t launch_sum_partials(const Partials& p, int ell, int ncols, double* out64, float* out32,
                               int64_t ld, hipStream_t st);

// Row-block products.  xty: part[b] = sum over the rows of split b of
// Xa[i,:]^T Xb[i,:] (ell x ell, column-major); the splits are summed in order
// by launch_reduce.  Xa, Xb column-major FP64 with leading dims.
int xty_splits(int64_t rows, int ell);
hipError_t launch_xty(const double* Xa, int64_t lda, const double* Xb, int64_t ldb, int64_t rows,
                      int ell, double* part, int splits, const int* skip, hipStream_t st);
hipError_t launch_reduce(const double* part, int splits, int64_t elems, double* out,
                         const int* skip, hipStream_t st);

// Dense output descriptor used by the row-matrix kernel.
struct MatOut {
  void* ptr = nullptr;
  int64_t ld = 0;
  int dtype = CORUTV_F64;
  int layout = CORUTV_COL_MAJOR;
};
// Y[i, :] = X[i, :] B (rows x ell times ell x ell, B column-major FP64 with
// ldb; X column-major FP64).  When `perm` is given, Y[:, j] = X[:, perm[j]]
// instead (B unused).  Outputs: up to two destinations (may be null).  Rows
// >= rows are not written; columns ell..ellp-1 of FP64 skinny destinations
// (dtype F64/F32 column-major with pad = 1) are zero-filled.  b_upper: B is
// upper triangular (entries below the diagonal are zero and are skipped).
// Runs only when *skip == run_val (skip may be null); when *skip == alt_val
// instead (product only, no perm) it writes the single destination oa (pad
// pada) in place of o1 and o2: one launch for the two outcomes of a status.
hipError_t launch_rowmat(const double* X, int64_t ldx, int64_t rows, int ell, const double* B,
                         int64_t ldb, const int32_t* perm, MatOut o1, int pad1, MatOut o2, int pad2,
                         const int* skip, hipStream_t st, bool b_upper = false, int run_val = 0,
                         MatOut oa = MatOut(), int pada = 0, int alt_val = -1);

// Cholesky G = R^T R of an SPD ell x ell FP64 matrix (column-major, ld ell)
// and the inverse of R, both written column-major (ld ell).  status gets
// bit 1 on breakdown (non-positive or non-finite pivot) and bit 2 when the
// input holds NaN/Inf.  Runs only when *skip == 0 (skip may be null).
// work: chol_work_bytes(ell) bytes of device scratch (0 for ell <= 128).
// single_thr > 0: on success, status also gets bit 3 (value 4) when
// u * ell * ||R||_F^2 * ||R^-1||_F^2 <= single_thr, i.e. when one CholeskyQR
// step already leaves an orthogonality loss below that level.
size_t chol_work_bytes(int ell);
hipError_t launch_chol(const double* G, int ell, double* R, double* Rinv, int* status,
                       const int* skip, double* work, hipStream_t st, double single_thr = 0.0);

// R = R2 R1 (upper triangular, column-major ld ell) when *status shows the
// Cholesky route was taken; otherwise does nothing.
hipError_t launch_trprod(const double* R2, const double* R1, int ell, double* R, const int* status,
                         hipStream_t st);

// CholeskyQR2 of X (rows x ell, ell <= 16, column-major FP64, ld) in three
// launches, or one when rows <= 1024: Q (FP64, columns ell..15 zero;
// optional float copy), R (nullable, ell x ell column-major: R2 R1, or R1
// when one step suffices), status bits as launch_chol (1: breakdown, the
// caller's Householder fallback runs; 2: non-finite data; 4: one step,
// allowed when single_thr > 0).  work: qr16_work_bytes() bytes whose last 256
// bytes (the block counter) must be zero before the first use; the kernels
// leave them zero.
// covered (nullable): when given, the launches also run the Householder
// fallback after a breakdown where its register-resident form fits (W: rows
// x ell scratch with ld ldw for the panel reflectors; hw: the tree's
// workspace as for launch_householder_qr), and *covered tells whether they
// did; if not, the caller runs launch_householder_qr as before.
size_t qr16_work_bytes();
hipError_t launch_qr16(const double* X, int64_t ld, int64_t rows, int ell, double* Q, float* Q32,
                       double* R, int* status, double* work, double single_thr, hipStream_t st,
                       double* W = nullptr, int64_t ldw = 0, double* hw = nullptr, bool* covered = nullptr);

// Householder thin QR of X (rows x ell, column-major FP64) -> Q (diag R >= 0,
// FP64 and optionally a float copy), R (nullable); runs only when
// (*status & 3) == 1 (a Cholesky breakdown on finite data).  work: rows x ell
// (must not overlap X or Q); hw: hh_work_bytes(rows, ell) bytes for the
// two-level tree of a tall X (nullable when that is 0).
hipError_t launch_householder_qr(const double* X, int64_t ldx, int64_t rows, int ell, double* work,
                                 int64_t ldw, double* Q, int64_t ldq, float* Q32, int64_t ldq32,
                                 double* R, const int* status, double* hw, hipStream_t st);
int hh_panels(int64_t rows, int ell);
size_t hh_work_bytes(int64_t rows, int ell);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);

// Up to kZeroRanges device ranges to clear in one launch: ptr[r] 16-byte
// aligned, words[r] 16-byte words (bytes / 16).  A fill kernel rather than
// hipMemsetAsync: one launch for all ranges, and safe under graph capture.
constexpr int kZeroRanges = 6;
struct ZeroRanges {
  void* ptr[kZeroRanges];
  int64_t words[kZeroRanges];
  int count;
};
hipError_t launch_zero_ranges(const ZeroRanges& z, hipStream_t st);

// Column-pivoted QR of an ell x ell FP64 matrix (column-major, ldd; trans
// reads D^T).  Qt, R column-major ld ell; piv int32.  work: 2*ell*ell + 2*ell doubles.
hipError_t launch_qrcp(const double* D, int64_t ldd, int trans, int ell, double* Qt, double* R,
                       int32_t* piv, double* work, hipStream_t st);

// Copy an ell x ell FP64 column-major matrix (optionally transposed, with
// zeroed strict lower (upper=1) or strict upper (upper=0) part) to dst.
hipError_t launch_copy_tri(const double* src, int ell, int trans, int upper, double* dst, int64_t ldd,
                           hipStream_t st);
// n (1..3) chained copies in one launch: stage 0 is launch_copy_tri(src,
// ell, trans[0], upper[0], dst[0], ld[0]); stage k the same copy of stage
// k - 1's result into dst[k].
hipError_t launch_copy_tri_chain(const double* src, int ell, int n, double* const* dst, const int64_t* ld,
                                 const int* trans, const int* upper, hipStream_t st);

// Residual: part[b] = { sum (A - B V^T)^2, sum A^2 } over row block b, with
// A row-major R x C (dtype F64/F32), B (R x ell) and V (C x ell) column-major
// FP64 skinny matrices.  Then summed in order.
int residual_blocks(int64_t R);
hipError_t launch_residual(const void* A, int dtype, int64_t lda, int64_t R, int64_t C,
                           const double* B, int64_t ldb, const double* V, int64_t ldv, int ell,
                           double* part, hipStream_t st);

// RPCA elementwise step (rpca.hip): S, Y (and B for the next iteration, L if
// non-null) from M and the rank-r factors P (m x ell), Q (n x ell) with r the
// number of diagonal entries of T above 1/mu (written to *rank_out when that
// is non-null); per-block sums of the squared residual M - L - S go to
// part[rpca_partial_blocks()].  The nstatus status words of the iteration's
// decomposition are OR-ed into *sticky (nullable).
int rpca_partial_blocks();
hipError_t launch_rpca_elementwise(const float* M, int lay_m, int64_t ldm, float* S, int lay_s,
                                   int64_t lds, double* Y, int64_t ldy, double* B, int64_t ldb, float* L,
                                   int lay_l, int64_t ldl, int64_t m, int64_t n, const double* P,
                                   int64_t ldp, const double* Q, int64_t ldq, const double* T,
                                   int64_t ldt, int ell, double mu, double mu_next, double lambda,
                                   double* part, const int* status, int nstatus, int* sticky,
                                   int* rank_out, hipStream_t st);
hipError_t launch_sumsq(const float* X, int lay, int64_t ld, int64_t m, int64_t n, double* part,
                        hipStream_t st);
hipError_t launch_widen(const float* X, int lay, int64_t ld, int64_t m, int64_t n, double* B, int64_t ldb,
                        hipStream_t st);

}  // namespace corutv
