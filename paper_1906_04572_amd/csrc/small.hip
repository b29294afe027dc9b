// The small steps around the passes over A (Sec. 3.1 eqs. 6-9, Algorithm 1):
// thin QR of the sketches (CholeskyQR2 with FP64 Gram and Cholesky, and a
// Householder fallback), the l x l core reduction, the lifts U = Q1 Qt and
// V = Q2 P, and the optional residual ||A - U T V^T||_F.
//
// All arithmetic here is FP64.  Skinny matrices (rows x l) are column-major.
// Reductions over rows are split into a fixed number of row blocks whose
// partial sums are added in block order, so results are deterministic.
#include <cmath>

#include "internal.hpp"

namespace corutv {
namespace {

// ---------------------------------------------------------------------------
// Sum of the stream-K partial tiles.  One block per (output tile, column
// group): the tile's contributing partial slots are listed once in LDS in the
// fixed order (chunk x ascending, workgroup ascending), then every thread sums
// its (column, row) entries over that list.
constexpr int kSegMax = 2048;
constexpr int kSumCols = 16;  // columns per block

template <typename T>
__global__ void __launch_bounds__(256) sum_partials_kernel(Partials p, const T* __restrict__ P, int ell,
                                                           int ncols, double* __restrict__ out64,
                                                           float* __restrict__ out32, int64_t ld) {
  __shared__ int seg[kSegMax];
  __shared__ int nseg;
  const int t = blockIdx.x;
  const int c0 = blockIdx.y * kSumCols;
  if (threadIdx.x == 0) {
    const int64_t U = (int64_t)p.tiles * p.nkx;
    const int64_t lo = (int64_t)t * p.nkx, hi = lo + p.nkx;
    int n = 0;
    for (int x = 0; x < 8; ++x) {
      for (int j = (int)(lo * p.gx / U); j < p.gx; ++j) {
        const int64_t u0 = (int64_t)j * U / p.gx;
        if (u0 >= hi) break;
        const int64_t u1 = (int64_t)(j + 1) * U / p.gx;
        if ((u0 > lo ? u0 : lo) >= (u1 < hi ? u1 : hi)) continue;
        if (n < kSegMax) seg[n] = (x * p.gx + j) * p.maxslot + (t - (int)(u0 / p.nkx));
        ++n;
      }
    }
    nseg = n;
  }
  __syncthreads();
  const int ns = nseg < kSegMax ? nseg : kSegMax;
  const int64_t tile_elems = (int64_t)p.ellp * p.tw;
  for (int e = threadIdx.x; e < kSumCols * p.tw; e += blockDim.x) {
    const int nl = e % p.tw;
    const int c = c0 + e / p.tw;
    const int64_t n = (int64_t)t * p.tw + nl;
    if (c >= ncols || n >= p.n) continue;
    double v = 0.0;
    if (c < ell) {
      const T* src = P + (int64_t)c * p.tw + nl;
      for (int k = 0; k < ns; ++k) v += (double)src[(int64_t)seg[k] * tile_elems];
    }
    if (out64) out64[(int64_t)c * ld + n] = v;
    if (out32) out32[(int64_t)c * ld + n] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// Xa^T Xb over row splits.  Block: 64 x 64 output tile, 4 x 4 per thread.
constexpr int XT = 64, XR = 32;

__global__ void __launch_bounds__(256) xty_kernel(const double* __restrict__ Xa, int64_t lda,
                                                  const double* __restrict__ Xb, int64_t ldb,
                                                  int64_t rows, int ell, double* __restrict__ part,
                                                  int splits, const int* skip) {
  if (skip && *skip) return;
  __shared__ double sa[XR][XT + 1];
  __shared__ double sb[XR][XT + 1];
  const int ntile = (ell + XT - 1) / XT;
  const int tile = blockIdx.x % (ntile * ntile);
  const int split = blockIdx.x / (ntile * ntile);
  const int a0 = (tile % ntile) * XT, b0 = (tile / ntile) * XT;
  const int tid = threadIdx.x, ta = tid >> 4, tb = tid & 15;
  const int64_t per = (rows + splits - 1) / splits;
  const int64_t r0 = (int64_t)split * per;
  const int64_t r1 = r0 + per < rows ? r0 + per : rows;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += XR) {
    // stage XR rows x 64 columns of each operand (coalesced along rows)
    for (int e = tid; e < XR * XT; e += 256) {
      const int r = e % XR, c = e / XR;
      const int64_t row = rb + r;
      const bool ok = row < r1;
      sa[r][c] = (ok && a0 + c < ell) ? Xa[(int64_t)(a0 + c) * lda + row] : 0.0;
      sb[r][c] = (ok && b0 + c < ell) ? Xb[(int64_t)(b0 + c) * ldb + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < XR; ++r) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sa[r][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sb[r][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)split * ell * ell;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ta + 16 * i, b = b0 + tb + 16 * j;
      if (a < ell && b < ell) out[(int64_t)b * ell + a] = acc[i][j];
    }
}

// out[e] = sum over k of part[k * elems + e], in a fixed order: thread group
// g (0..3) sums splits g, g+4, ...; the four group sums are added in order.
__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ part, int splits,
                                                     int64_t elems, double* __restrict__ out,
                                                     const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[4][64];
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  double s = 0.0;
  if (e < elems)
    for (int k = grp; k < splits; k += 4) s += part[(int64_t)k * elems + e];
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < elems) out[e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
}

// ---------------------------------------------------------------------------
// Y = X B (or column gather).  Block: 64 rows x 64 columns, 4 x 4 per thread.
__device__ __forceinline__ void store_out(const MatOut& o, int64_t i, int c, double v) {
  const int64_t off = o.layout == CORUTV_COL_MAJOR ? (int64_t)c * o.ld + i : i * o.ld + c;
  if (o.dtype == CORUTV_F64)
    ((double*)o.ptr)[off] = v;
  else
    ((float*)o.ptr)[off] = (float)v;
}

__global__ void __launch_bounds__(256) rowmat_kernel(const double* __restrict__ X, int64_t ldx,
                                                     int64_t rows, int ell, const double* __restrict__ B,
                                                     int64_t ldb, const int32_t* __restrict__ perm,
                                                     MatOut o1, int pad1, MatOut o2, int pad2,
                                                     const int* skip) {
  if (skip && *skip) return;
  constexpr int KB = 32;
  __shared__ double sx[64][KB + 1];
  __shared__ double sbm[KB][64 + 1];
  const int tid = threadIdx.x, ta = tid >> 4, tb = tid & 15;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int ellp = pad_ell(ell);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  if (perm) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = i0 + ta + 16 * i;
        const int c = c0 + tb + 16 * j;
        if (r < rows && c < ell) acc[i][j] = X[(int64_t)perm[c] * ldx + r];
      }
  } else {
    for (int k0 = 0; k0 < ell; k0 += KB) {
      for (int e = tid; e < 64 * KB; e += 256) {
        const int r = e % 64, k = e / 64;
        const int64_t row = i0 + r;
        sx[r][k] = (row < rows && k0 + k < ell) ? X[(int64_t)(k0 + k) * ldx + row] : 0.0;
      }
      for (int e = tid; e < 64 * KB; e += 256) {
        const int k = e % KB, c = e / KB;
        sbm[k][c] = (k0 + k < ell && c0 + c < ell) ? B[(int64_t)(c0 + c) * ldb + k0 + k] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int k = 0; k < KB; ++k) {
        double xv[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = sx[ta + 16 * i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = sbm[k][tb + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(xv[i], bv[j], acc[i][j]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = i0 + ta + 16 * i;
      const int c = c0 + tb + 16 * j;
      if (r >= rows) continue;
      if (c < ell) {
        if (o1.ptr) store_out(o1, r, c, acc[i][j]);
        if (o2.ptr) store_out(o2, r, c, acc[i][j]);
      } else if (c < ellp) {
        if (o1.ptr && pad1) store_out(o1, r, c, 0.0);
        if (o2.ptr && pad2) store_out(o2, r, c, 0.0);
      }
    }
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R fused with the inverse of R, one workgroup of 1024
// threads.  Element (r, c) of the working matrix lives in a register of
// thread (r mod 32, c mod 32) (block-cyclic).  The upper triangle holds the
// matrix being factored, the strict lower triangle the rows of Z = R^{-T}
// (L = R^T, Z = L^{-1}); rows are kept unscaled and scaled at the end.
// Step s: the owners of row s publish it (double-buffered LDS vector), every
// thread reads the pivot d = W[s,s] and computes iv = 1/sqrt(d), then
//   W[r,c] -= (W[s,r] iv^2) W[s,c]   for r > s and (c >= r or c < s)
//   W[r,s] -= W[s,r] iv^2            for r > s (the Z diagonal iv enters)
// which is the rank-1 update of the trailing matrix and the forward
// substitution step of L Z = I.  One barrier per step.
template <int NPT>
__device__ __forceinline__ void chol_reg_body(const double* __restrict__ G, int ell,
                                              double* __restrict__ R, double* __restrict__ Rinv,
                                              int* status, double* rowbuf, double* inv,
                                              double* sh) {
  const int tid = threadIdx.x;
  const int tr = tid & 31, tc = tid >> 5;
  double w[NPT][NPT];
#pragma unroll
  for (int a = 0; a < NPT; ++a)
#pragma unroll
    for (int b = 0; b < NPT; ++b) {
      const int r = tr + 32 * a, c = tc + 32 * b;
      w[a][b] = (r < ell && c < ell && r <= c) ? G[(int64_t)c * ell + r] : 0.0;
    }
  if (tid == 0) {
    double dmax = 0.0;
    int bad = 0;
    for (int i = 0; i < ell; ++i) {
      const double d = G[(int64_t)i * ell + i];
      if (!isfinite(d)) bad = 1;
      if (d > dmax) dmax = d;
    }
    // a pivot below 4 l u max_i G_ii means the sketch's condition number is
    // beyond ~ (4 l u)^(-1/2): CholeskyQR is not reliable, fall back
    sh[0] = bad ? -1.0 : 4.0 * ell * 2.220446049250313e-16 * dmax;
  }
  __syncthreads();
  const double thr = sh[0];
  if (thr < 0.0) {
    if (tid == 0) atomicOr(status, 2);
    return;
  }
  for (int s = 0; s < ell; ++s) {
    double* row = rowbuf + (s & 1) * 256;
#pragma unroll
    for (int a = 0; a < NPT; ++a) {
      if (tr + 32 * a != s) continue;
#pragma unroll
      for (int b = 0; b < NPT; ++b) {
        const int c = tc + 32 * b;
        if (c < ell) row[c] = w[a][b];
      }
    }
    __syncthreads();
    const double d = row[s];
    if (!(d > thr) || !isfinite(d)) {
      if (tid == 0) atomicOr(status, 1);
      return;  // uniform: every thread read the same d
    }
    // 1/sqrt(d): hardware estimate refined by two Newton steps
    double iv = __builtin_amdgcn_rsq(d);
    iv = iv * (1.5 - 0.5 * d * iv * iv);
    iv = iv * (1.5 - 0.5 * d * iv * iv);
    const double iv2 = iv * iv;
    if (tid == 0) inv[s] = iv;
    double rc[NPT];
#pragma unroll
    for (int b = 0; b < NPT; ++b) {
      const int c = tc + 32 * b;
      rc[b] = c < ell ? row[c] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < NPT; ++a) {
      if (32 * a + 31 <= s) continue;  // whole row block finished: uniform skip
      const int r = tr + 32 * a;
      if (r <= s || r >= ell) continue;
      const double t = row[r] * iv2;
#pragma unroll
      for (int b = 0; b < NPT; ++b) {
        const int c = tc + 32 * b;
        if (c >= ell) continue;
        if (c >= r || c < s)
          w[a][b] -= t * rc[b];
        else if (c == s)
          w[a][b] -= t;
      }
    }
  }
  __syncthreads();
  // outputs: element (r, c) of W gives
  //   r < c : R[r,c] = W[r,c] iv_r
  //   r = c : R[r,r] = sqrt(W[r,r]), Rinv[r,r] = iv_r
  //   r > c : Rinv[c,r] = Z[r,c] = W[r,c] iv_r  (and zeros in the lower parts)
#pragma unroll
  for (int a = 0; a < NPT; ++a)
#pragma unroll
    for (int b = 0; b < NPT; ++b) {
      const int r = tr + 32 * a, c = tc + 32 * b;
      if (r >= ell || c >= ell) continue;
      const int64_t rc_ = (int64_t)c * ell + r, cr = (int64_t)r * ell + c;
      if (r < c) {
        R[rc_] = w[a][b] * inv[r];
      } else if (r == c) {
        R[rc_] = sqrt(w[a][b]);
        Rinv[rc_] = inv[r];
      } else {
        R[rc_] = 0.0;
        Rinv[rc_] = 0.0;
        Rinv[cr] = w[a][b] * inv[r];
      }
    }
}

template <int NPT>
__global__ void __launch_bounds__(1024) chol_kernel(const double* G, int ell, double* R, double* Rinv,
                                                    int* status, const int* skip) {
  if (skip && *skip) return;
  __shared__ double rowbuf[512];
  __shared__ double inv[256];
  __shared__ double sh[2];
  chol_reg_body<NPT>(G, ell, R, Rinv, status, rowbuf, inv, sh);
}

// ---------------------------------------------------------------------------
// Householder thin QR (fallback).  One workgroup of 1024 threads; each wave
// owns columns j = wave (mod 16) for the dot products and updates.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(1024) householder_kernel(const double* __restrict__ X,
                                                           int64_t ldx, int64_t rows, int ell,
                                                           double* __restrict__ W, int64_t ldw,
                                                           double* __restrict__ Q, int64_t ldq,
                                                           float* __restrict__ Q32, int64_t ldq32,
                                                           double* __restrict__ R,
                                                           const int* status) {
  if ((*status & 3) != 1) return;  // only after a Cholesky breakdown
  __shared__ double tau[256], alpha[256], vhead[256];
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = 16;
  for (int64_t e = tid; e < rows * ell; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    W[(int64_t)j * ldw + i] = X[(int64_t)j * ldx + i];
  }
  __syncthreads();
  for (int s = 0; s < ell; ++s) {
    // norm of W[s:, s]
    double part = 0.0;
    for (int64_t i = s + tid; i < rows; i += 1024) {
      const double v = W[(int64_t)s * ldw + i];
      part += v * v;
    }
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      double nrm2 = 0.0;
      for (int w = 0; w < nw; ++w) nrm2 += red[w];
      const double x0 = W[(int64_t)s * ldw + s];
      const double nrm = sqrt(nrm2);
      if (nrm == 0.0) {
        tau[s] = 0.0;
        alpha[s] = 0.0;
        vhead[s] = 0.0;
      } else {
        const double a = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - a;
        const double vtv = nrm2 - x0 * x0 + v0 * v0;
        tau[s] = 2.0 / vtv;
        alpha[s] = a;
        vhead[s] = v0;
      }
    }
    __syncthreads();
    const double ts = tau[s], v0 = vhead[s];
    if (ts != 0.0) {
      for (int j = s + 1 + wave; j < ell; j += nw) {
        double d = 0.0;
        for (int64_t i = s + lane; i < rows; i += 64) {
          const double vi = i == s ? v0 : W[(int64_t)s * ldw + i];
          d += vi * W[(int64_t)j * ldw + i];
        }
        d = wave_sum(d) * ts;
        for (int64_t i = s + lane; i < rows; i += 64) {
          const double vi = i == s ? v0 : W[(int64_t)s * ldw + i];
          W[(int64_t)j * ldw + i] -= d * vi;
        }
      }
    }
    __syncthreads();
  }
  // R (upper, ell x ell, column-major ld ell) with diag >= 0
  if (R) {
    for (int e = tid; e < ell * ell; e += 1024) {
      const int i = e % ell, j = e / ell;
      double v = i < j ? W[(int64_t)j * ldw + i] : (i == j ? alpha[i] : 0.0);
      if (alpha[i] < 0.0) v = -v;
      R[e] = v;
    }
  }
  __syncthreads();
  // Q = H_0 ... H_{ell-1} [I; 0], accumulated backwards into Q's columns.
  for (int64_t e = tid; e < rows * ell; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    Q[(int64_t)j * ldq + i] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int s = ell - 1; s >= 0; --s) {
    const double ts = tau[s], v0 = vhead[s];
    if (ts != 0.0) {
      for (int j = s + wave; j < ell; j += nw) {
        double d = 0.0;
        for (int64_t i = s + lane; i < rows; i += 64) {
          const double vi = i == s ? v0 : W[(int64_t)s * ldw + i];
          d += vi * Q[(int64_t)j * ldq + i];
        }
        d = wave_sum(d) * ts;
        for (int64_t i = s + lane; i < rows; i += 64) {
          const double vi = i == s ? v0 : W[(int64_t)s * ldw + i];
          Q[(int64_t)j * ldq + i] -= d * vi;
        }
      }
    }
    __syncthreads();
  }
  // sign normalisation diag(R) >= 0: flip the columns of Q with alpha < 0
  for (int64_t e = tid; e < rows * ell; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    double v = Q[(int64_t)j * ldq + i];
    if (alpha[j] < 0.0) {
      v = -v;
      Q[(int64_t)j * ldq + i] = v;
    }
    if (Q32) Q32[(int64_t)j * ldq32 + i] = (float)v;
  }
}

// ---------------------------------------------------------------------------
__global__ void copy_tri_kernel(const double* __restrict__ src, int ell, int trans, int upper,
                                double* __restrict__ dst, int64_t ldd) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ell * ell) return;
  const int i = e % ell, j = e / ell;
  double v = trans ? src[(int64_t)i * ell + j] : src[(int64_t)j * ell + i];
  if (upper ? (i > j) : (i < j)) v = 0.0;
  dst[(int64_t)j * ldd + i] = v;
}

// ---------------------------------------------------------------------------
// residual: sum over A tiles of (a - (B V^T)_ij)^2 and a^2 (FP64).
constexpr int kResBlocks = 1024;

template <typename TA>
__global__ void __launch_bounds__(256) residual_kernel(const TA* __restrict__ A, int64_t lda,
                                                       int64_t R, int64_t C,
                                                       const double* __restrict__ B, int64_t ldb,
                                                       const double* __restrict__ V, int64_t ldv,
                                                       int ell, double* __restrict__ part) {
  constexpr int KB = 16;
  __shared__ double sb[64][KB + 1];
  __shared__ double sv[KB][64 + 1];
  __shared__ double red[2][256];
  const int tid = threadIdx.x, ta = tid >> 4, tb = tid & 15;
  const int64_t tr = (R + 63) / 64, tc = (C + 63) / 64;
  double e2 = 0.0, a2 = 0.0;
  for (int64_t tile = blockIdx.x; tile < tr * tc; tile += gridDim.x) {
    const int64_t i0 = (tile / tc) * 64, j0 = (tile % tc) * 64;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < ell; k0 += KB) {
      for (int e = tid; e < 64 * KB; e += 256) {
        const int r = e % 64, k = e / 64;
        sb[r][k] = (i0 + r < R && k0 + k < ell) ? B[(int64_t)(k0 + k) * ldb + i0 + r] : 0.0;
        sv[k][r] = (j0 + r < C && k0 + k < ell) ? V[(int64_t)(k0 + k) * ldv + j0 + r] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        double bv[4], vv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = sb[ta * 4 + i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) vv[j] = sv[k][tb + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(bv[i], vv[j], acc[i][j]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = i0 + ta * 4 + i, c = j0 + tb + 16 * j;
        if (r < R && c < C) {
          const double a = (double)A[r * lda + c];
          const double d = a - acc[i][j];
          e2 += d * d;
          a2 += a * a;
        }
      }
  }
  red[0][tid] = e2;
  red[1][tid] = a2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red[0][tid] += red[0][tid + off];
      red[1][tid] += red[1][tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_sum_partials(const Partials& p, int ell, int ncols, double* out64, float* out32,
                               int64_t ld, hipStream_t st) {
  if (p.n == 0 || ncols == 0) return hipSuccess;
  // every segment list must fit: at most 8 * (gx + 1) entries per tile
  if (8 * (p.gx + 1) > kSegMax) return hipErrorInvalidValue;
  dim3 grid((unsigned)p.tiles, (unsigned)((ncols + kSumCols - 1) / kSumCols));
  if (p.elem == 8)
    sum_partials_kernel<double><<<grid, dim3(256), 0, st>>>(p, (const double*)p.ptr, ell, ncols, out64,
                                                            out32, ld);
  else
    sum_partials_kernel<float><<<grid, dim3(256), 0, st>>>(p, (const float*)p.ptr, ell, ncols, out64,
                                                           out32, ld);
  return hipGetLastError();
}

int xty_splits(int64_t rows, int ell) {
  const int nt = (ell + XT - 1) / XT;
  int s = 512 / (nt * nt);
  const int64_t maxs = (rows + XR - 1) / XR;
  if (s > maxs) s = (int)maxs;
  return s < 1 ? 1 : s;
}

hipError_t launch_xty(const double* Xa, int64_t lda, const double* Xb, int64_t ldb, int64_t rows,
                      int ell, double* part, int splits, const int* skip, hipStream_t st) {
  const int nt = (ell + XT - 1) / XT;
  xty_kernel<<<dim3(nt * nt * splits), dim3(256), 0, st>>>(Xa, lda, Xb, ldb, rows, ell, part, splits,
                                                          skip);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int splits, int64_t elems, double* out, const int* skip,
                         hipStream_t st) {
  reduce_kernel<<<dim3((unsigned)((elems + 63) / 64)), dim3(256), 0, st>>>(part, splits, elems, out, skip);
  return hipGetLastError();
}

hipError_t launch_rowmat(const double* X, int64_t ldx, int64_t rows, int ell, const double* B,
                         int64_t ldb, const int32_t* perm, MatOut o1, int pad1, MatOut o2, int pad2,
                         const int* skip, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  const int ellp = pad_ell(ell);
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((ellp + 63) / 64));
  rowmat_kernel<<<grid, dim3(256), 0, st>>>(X, ldx, rows, ell, B, ldb, perm, o1, pad1, o2, pad2, skip);
  return hipGetLastError();
}

hipError_t launch_chol(const double* G, int ell, double* R, double* Rinv, int* status,
                       const int* skip, hipStream_t st) {
  const int npt = (ell + 31) / 32;
  if (npt <= 4)
    chol_kernel<4><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip);
  else if (npt == 5)
    chol_kernel<5><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip);
  else if (npt == 6)
    chol_kernel<6><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip);
  else if (npt == 7)
    chol_kernel<7><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip);
  else
    chol_kernel<8><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip);
  return hipGetLastError();
}

hipError_t launch_householder_qr(const double* X, int64_t ldx, int64_t rows, int ell, double* work,
                                 int64_t ldw, double* Q, int64_t ldq, float* Q32, int64_t ldq32,
                                 double* R, const int* status, hipStream_t st) {
  householder_kernel<<<dim3(1), dim3(1024), 0, st>>>(X, ldx, rows, ell, work, ldw, Q, ldq, Q32, ldq32,
                                                     R, status);
  return hipGetLastError();
}

hipError_t launch_copy_tri(const double* src, int ell, int trans, int upper, double* dst, int64_t ldd,
                           hipStream_t st) {
  const int n = ell * ell;
  copy_tri_kernel<<<dim3((n + 255) / 256), dim3(256), 0, st>>>(src, ell, trans, upper, dst, ldd);
  return hipGetLastError();
}

int residual_blocks(int64_t R) {
  (void)R;
  return kResBlocks;
}

hipError_t launch_residual(const void* A, int dtype, int64_t lda, int64_t R, int64_t C,
                           const double* B, int64_t ldb, const double* V, int64_t ldv, int ell,
                           double* part, hipStream_t st) {
  if (dtype == CORUTV_F64)
    residual_kernel<double><<<dim3(kResBlocks), dim3(256), 0, st>>>((const double*)A, lda, R, C, B, ldb,
                                                                    V, ldv, ell, part);
  else
    residual_kernel<float><<<dim3(kResBlocks), dim3(256), 0, st>>>((const float*)A, lda, R, C, B, ldb,
                                                                   V, ldv, ell, part);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st) {
  fill_int_kernel<<<dim3((n + 255) / 256), dim3(256), 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace corutv
