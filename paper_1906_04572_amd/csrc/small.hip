// The small steps around the passes over A (Sec. 3.1 eqs. 6-9, Algorithm 1):
// thin QR of the sketches (CholeskyQR2 with FP64 Gram and Cholesky, and a
// Householder fallback), the l x l core reduction, the lifts U = Q1 Qt and
// V = Q2 P, and the optional residual ||A - U T V^T||_F.
//
// All arithmetic here is FP64.  Skinny matrices (rows x l) are column-major.
// Reductions over rows are split into a fixed number of row blocks whose
// partial sums are added in block order, so results are deterministic.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace corutv {
namespace {

// ---------------------------------------------------------------------------
// Sum of the stream-K partial tiles.  The workgroups of every K chunk split
// the units identically, so a tile's contributing partial slots are chunk x
// (0..nchunk-1) times the same list of workgroups; the list is built once in LDS and
// the slots are taken in the fixed order (chunk x ascending, workgroup
// ascending).  A block covers reps x 256 / tpe entries of one output tile;
// with tpe > 1 (a tile fed by many slots: a short output, a long contraction) tpe
// threads share an entry, each summing a contiguous part of the slot list,
// and the parts are added in order.
constexpr int kSegMax = 2048;

template <typename T>
__global__ void __launch_bounds__(256) sum_partials_kernel(Partials p, const T* __restrict__ P, int ell,
                                                           int ncols, double* __restrict__ out64,
                                                           float* __restrict__ out32, int64_t ld, int tpe,
                                                           int reps) {
  __shared__ int wg[kSegMax], wslot[kSegMax], seg[kSegMax];
  __shared__ int wcount[4];
  __shared__ double acc[256];
  const int t = blockIdx.x;
  // the workgroups whose unit ranges meet this tile's units, in ascending
  // order: 256 candidates at a time, one per thread, placed by a prefix
  // count (ballot within a wave, then the waves in order)
  {
    const int64_t U = (int64_t)p.tiles * p.nkx;
    const int64_t lo = (int64_t)t * p.nkx, hi = lo + p.nkx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int base = 0;
    for (int64_t jb = lo * p.gx / U; jb < p.gx; jb += 256) {
      const int64_t j = jb + threadIdx.x;
      bool valid = false, past = false;
      int slot = 0;
      if (j < p.gx) {
        const int64_t u0 = j * U / p.gx;
        if (u0 >= hi) {
          past = true;
        } else {
          const int64_t u1 = (j + 1) * U / p.gx;
          valid = (u0 > lo ? u0 : lo) < (u1 < hi ? u1 : hi);
          slot = t - (int)(u0 / p.nkx);
        }
      }
      const unsigned long long m = __ballot(valid);
      const int pos = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[wave] = __popcll(m);
      __syncthreads();
      int off = base;
      for (int w = 0; w < wave; ++w) off += wcount[w];
      if (valid && off + pos < kSegMax) {
        wg[off + pos] = (int)j;
        wslot[off + pos] = slot;
      }
      base += wcount[0] + wcount[1] + wcount[2] + wcount[3];
      const int any_past = __syncthreads_or(past);  // also orders the wcount reuse
      if (any_past) break;  // every later candidate starts past this tile
    }
    if (threadIdx.x == 0) wcount[0] = base < kSegMax ? base : kSegMax;
  }
  __syncthreads();
  const int nwg = wcount[0];
  const int nw = nwg, ns = p.nchunk * nw;
  for (int k = threadIdx.x; k < ns; k += blockDim.x) {
    const int x = k / nw, q = k - x * nw;
    seg[k] = (x * p.gx + wg[q]) * p.maxslot + wslot[q];
  }
  __syncthreads();
  const int epb = 256 / tpe;
  const int el = threadIdx.x % epb, part = threadIdx.x / epb;
  const int64_t tile_elems = (int64_t)p.ellp * p.tw;
  const int k0 = part * ns / tpe, k1 = (part + 1) * ns / tpe;
  for (int r = 0; r < reps; ++r) {
    // entry of the tile: column e / tw, row e % tw
    const int e = (blockIdx.y * reps + r) * epb + el;
    const int nl = e % p.tw;
    const int c = e / p.tw;
    const int64_t n = (int64_t)t * p.tw + nl;
    double v = 0.0;
    if (c < ell && n < p.n) {
      const T* src = P + (int64_t)c * p.tw + nl;
      // loads in groups of eight so their latencies overlap; the sum still
      // runs over the slots in list order
      int k = k0;
      for (; k + 8 <= k1; k += 8) {
        T l[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) l[j] = src[(int64_t)seg[k + j] * tile_elems];
#pragma unroll
        for (int j = 0; j < 8; ++j) v += (double)l[j];
      }
      for (; k < k1; ++k) v += (double)src[(int64_t)seg[k] * tile_elems];
    }
    if (tpe > 1) {
      acc[threadIdx.x] = v;
      __syncthreads();
      if (part == 0)
        for (int q = 1; q < tpe; ++q) v += acc[q * epb + el];
      __syncthreads();
    }
    if (part == 0 && c < ncols && n < p.n) {
      if (out64) out64[(int64_t)c * ld + n] = v;
      if (out32) out32[(int64_t)c * ld + n] = (float)v;
    }
  }
}

// ---------------------------------------------------------------------------
// Xa^T Xb over row splits on FP64 matrix cores.  A workgroup (4 waves) owns a
// 64 x 64 region of the l x l result and the rows of one split; rows are
// staged through LDS in chunks of 32 (column-major, padded stride), the next
// chunk prefetched into registers while the current one is multiplied.  Wave
// w computes the 32 x 32 block (w & 1, w >> 1) of the region as 2 x 2 tiles
// of v_mfma_f64_16x16x4f64 (lane l: A(l%16, k), B(k, l%16), k = l/16 + 4 kstep;
// accumulator slot s = element (l/16 + 4s, l%16)).  For a Gram matrix
// (Xa == Xb) only regions on or above the diagonal are computed and the
// off-diagonal ones are written twice.  Each split writes its own l x l
// partial (column-major); reduce_kernel adds them in a fixed order.
typedef double d4x __attribute__((ext_vector_type(4)));
constexpr int XT = 64, XR = 32, XSP = XR + 1;

__host__ __device__ inline int xty_regions(int ell, int sym) {
  const int nr = (ell + XT - 1) / XT;
  return sym ? nr * (nr + 1) / 2 : nr * nr;
}

__global__ void __launch_bounds__(256) xty_kernel(const double* __restrict__ Xa, int64_t lda,
                                                  const double* __restrict__ Xb, int64_t ldb,
                                                  int64_t rows, int ell, double* __restrict__ part,
                                                  int splits, int sym, const int* skip) {
  if (skip && *skip) return;
  __shared__ double sa[XT * XSP];
  __shared__ double sb[XT * XSP];
  const int nr = (ell + XT - 1) / XT;
  const int nreg = xty_regions(ell, sym);
  int reg = blockIdx.x % nreg;
  const int split = blockIdx.x / nreg;
  int ra = 0, rb = 0;
  if (sym) {
    int len = nr;
    while (reg >= len) {
      reg -= len;
      ++ra;
      --len;
    }
    rb = ra + reg;
  } else {
    ra = reg % nr;
    rb = reg / nr;
  }
  const int a0 = ra * XT, b0 = rb * XT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int wa = (w & 1) * 32, wb = (w >> 1) * 32;
  const int64_t per = (rows + splits - 1) / splits;
  const int64_t r0 = (int64_t)split * per;
  const int64_t r1 = r0 + per < rows ? r0 + per : rows;
  // loader: thread covers column tid / 32 + 8 e, row tid % 32 of a chunk.
  // Loads use clamped (always valid) addresses and are unconditional; the
  // mask is applied when the values are stored to LDS, one iteration later,
  // so the compiler cannot turn a masked load into a branch that waits for it.
  const int lr = tid & (XR - 1), lc = tid >> 5;
  double va[8], vb[8];
  auto fetch = [&](int64_t rb0) {
    const int64_t row = rb0 + lr;
    const int64_t rr = row < r1 ? row : r0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = lc + 8 * e;
      const int ca = a0 + c < ell ? a0 + c : ell - 1;
      const int cb = b0 + c < ell ? b0 + c : ell - 1;
      va[e] = Xa[(int64_t)ca * lda + rr];
      vb[e] = Xb[(int64_t)cb * ldb + rr];
    }
  };
  d4x acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (d4x){0.0, 0.0, 0.0, 0.0};
  if (r0 < r1) fetch(r0);
  for (int64_t rb0 = r0; rb0 < r1; rb0 += XR) {
    const bool rok = rb0 + lr < r1;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = lc + 8 * e;
      sa[c * XSP + lr] = (rok && a0 + c < ell) ? va[e] : 0.0;
      sb[c * XSP + lr] = (rok && b0 + c < ell) ? vb[e] : 0.0;
    }
    __syncthreads();
    if (rb0 + XR < r1) fetch(rb0 + XR);
#pragma unroll
    for (int ks = 0; ks < XR / 4; ++ks) {
      const int k = 4 * ks + g;
      const double a0f = sa[(wa + i) * XSP + k], a1f = sa[(wa + 16 + i) * XSP + k];
      const double b0f = sb[(wb + i) * XSP + k], b1f = sb[(wb + 16 + i) * XSP + k];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0f, b0f, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0f, b1f, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1f, b0f, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1f, b1f, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)split * ell * ell;
  const bool mirror = sym && ra != rb;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int a = a0 + wa + 16 * x + g + 4 * s, b = b0 + wb + 16 * y + i;
        if (a < ell && b < ell) {
          out[(int64_t)b * ell + a] = acc[x][y][s];
          if (mirror) out[(int64_t)a * ell + b] = acc[x][y][s];
        }
      }
}

// out[e] = sum over k of part[k * elems + e], in a fixed order: thread group
// q (0..15) sums splits q, q+16, ... in order; the sixteen group sums are
// added in group order.
__global__ void __launch_bounds__(1024) reduce_kernel(const double* __restrict__ part, int splits,
                                                      int64_t elems, double* __restrict__ out,
                                                      const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[16][64];
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  double s = 0.0;
  if (e < elems)
    for (int k = grp; k < splits; k += 16) s += part[(int64_t)k * elems + e];
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < elems) {
    double t = red[0][el];
#pragma unroll
    for (int q = 1; q < 16; ++q) t += red[q][el];
    out[e] = t;
  }
}

// ---------------------------------------------------------------------------
// Output helpers and the column gather Y[:, j] = X[:, perm[j]].
__device__ __forceinline__ void store_out(const MatOut& o, int64_t i, int c, double v) {
  const int64_t off = o.layout == CORUTV_COL_MAJOR ? (int64_t)c * o.ld + i : i * o.ld + c;
  if (o.dtype == CORUTV_F64)
    ((double*)o.ptr)[off] = v;
  else
    ((float*)o.ptr)[off] = (float)v;
}

// The same with streaming (non-temporal) stores: results that the next
// kernel reads anyway come from memory (each XCD's L2 is written back and
// invalidated between kernels), so they need not stay dirty in L2 until the
// end of the kernel.
__device__ __forceinline__ void store_out_nt(const MatOut& o, int64_t i, int c, double v) {
  const int64_t off = o.layout == CORUTV_COL_MAJOR ? (int64_t)c * o.ld + i : i * o.ld + c;
  if (o.dtype == CORUTV_F64)
    __builtin_nontemporal_store(v, (double*)o.ptr + off);
  else
    __builtin_nontemporal_store((float)v, (float*)o.ptr + off);
}

// One thread per row, one block row per output column: loads and column-major
// stores both run along rows.
__global__ void __launch_bounds__(256) gather_cols_kernel(const double* __restrict__ X, int64_t ldx,
                                                          int64_t rows, int ell,
                                                          const int32_t* __restrict__ perm, MatOut o1,
                                                          int pad1, MatOut o2, int pad2, const int* skip,
                                                          int run_val) {
  if (skip && *skip != run_val) return;
  const int c = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  if (c < ell) {
    const double v = X[(int64_t)perm[c] * ldx + r];
    if (o1.ptr) store_out(o1, r, c, v);
    if (o2.ptr) store_out(o2, r, c, v);
  } else {
    if (o1.ptr && pad1) store_out(o1, r, c, 0.0);
    if (o2.ptr && pad2) store_out(o2, r, c, 0.0);
  }
}

// Y = X B for l <= 16: one thread per row, B (zero outside l x l) in LDS
// where every thread reads the same entry at a time; y_c accumulates its
// terms in increasing k (with b_upper, k <= c only).  Same outputs, padding
// and status gate as rowmat_mfma_kernel.
__global__ void __launch_bounds__(256) rowmat16_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                       int ell, const double* __restrict__ B, int64_t ldb,
                                                       MatOut o1, int pad1, MatOut o2, int pad2, int b_upper,
                                                       const int* skip, int run_val, MatOut oa, int pada,
                                                       int alt_val) {
  if (skip) {
    const int sv = *skip;
    if (sv == alt_val) {
      o1 = oa;
      pad1 = pada;
      o2 = MatOut();
      pad2 = 0;
    } else if (sv != run_val) {
      return;
    }
  }
  __shared__ double sb[256];  // sb[k * 16 + c] = B[k][c]
  const int tid = threadIdx.x;
  {
    const int k = tid >> 4, c = tid & 15;
    sb[tid] = (k < ell && c < ell) ? B[(int64_t)c * ldb + k] : 0.0;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + tid;
  if (r >= rows) return;
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = k < ell ? X[(int64_t)k * ldx + r] : 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c < ell) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < ell && (!b_upper || k <= c)) v = fma(x[k], sb[k * 16 + c], v);
      if (o1.ptr) store_out(o1, r, c, v);
      if (o2.ptr) store_out(o2, r, c, v);
    } else {
      if (o1.ptr && pad1) store_out(o1, r, c, 0.0);
      if (o2.ptr && pad2) store_out(o2, r, c, 0.0);
    }
  }
}

// Y = X B on FP64 matrix cores, computed as Y^T = B^T X^T so that the
// accumulator lanes run along rows of Y (coalesced column-major stores).  A
// workgroup (4 waves) owns 32 rows x 128 columns of Y; wave w computes rows
// 16 (w & 1) .. + 15 for the four 16-column tiles of column half w >> 1, with
// X read straight from global memory (16 consecutive rows per lane group).
// B^T is staged through LDS in chunks of 32 of the contraction index (two
// buffers, one barrier per chunk).  The next chunk's loads go to a second
// register set before the current chunk's products.  Addresses past the ends
// are clamped to valid entries, so every load is unconditional; only the
// contraction indices past the end of a ragged last chunk are masked (X set
// to zero there; B is finite, and columns past ell are never stored).  With
// b_upper (B upper triangular) a tile skips the chunks that lie below its
// diagonal.  32-row blocks keep the work per CU even at a few hundred blocks.
__global__ void __launch_bounds__(256) rowmat_mfma_kernel(const double* __restrict__ X, int64_t ldx,
                                                          int64_t rows, int ell,
                                                          const double* __restrict__ B, int64_t ldb,
                                                          MatOut o1, int pad1, MatOut o2, int pad2,
                                                          int b_upper, const int* skip, int run_val,
                                                          MatOut oa, int pada, int alt_val) {
  if (skip) {
    const int sv = *skip;
    if (sv == alt_val) {
      o1 = oa;
      pad1 = pada;
      o2 = MatOut();
      pad2 = 0;
    } else if (sv != run_val) {
      return;
    }
  }
  constexpr int KB = 32, SP = KB + 1, KS = KB / 4, NT = 4, CW = 128;
  constexpr int BPT = KB * CW / 256;  // B values staged per thread and chunk
  __shared__ double sbt[2][CW * SP];  // sbt[buf][c * SP + k] = B[k0 + k][c0 + c]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * CW;
  const int cw0 = 64 * (w >> 1);  // this wave's first column within the block
  const int ellp = pad_ell(ell);
  const int ntw = (ellp - c0 - cw0) / 16;  // this wave's column tiles (may be <= 0)
  const int nt = ntw < NT ? ntw : NT;
  const int kend = b_upper ? (c0 + CW < ell ? c0 + CW : ell) : ell;
  const int nchunk = (kend + KB - 1) / KB, nfull = kend / KB;
  const int64_t rw = r0 + 16 * (w & 1) + i;
  const bool rok = rw < rows;
  const int64_t rr = rok ? rw : rows - 1;
  // two register sets, used alternately, so the loads for chunk ci + 1 land
  // in registers that the products of chunk ci do not read
  double bq0[BPT], xq0[KS], bq1[BPT], xq1[KS];
  auto fetch = [&](int k0, double (&bq)[BPT], double (&xq)[KS]) {
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int e = tid + 256 * j, k = e % KB, c = e / KB;
      const int kk = k0 + k < ell ? k0 + k : ell - 1;
      const int cc = c0 + c < ell ? c0 + c : ell - 1;
      bq[j] = B[(int64_t)cc * ldb + kk];
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = k0 + 4 * ks + g;
      xq[ks] = X[(int64_t)(k < ell ? k : ell - 1) * ldx + rr];
    }
  };
  d4x acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (d4x){0.0, 0.0, 0.0, 0.0};
  auto chunk = [&](int ci, double (&bq)[BPT], double (&xq)[KS], double (&bn)[BPT], double (&xn)[KS]) {
    const int k0 = ci * KB;
    double* sb = sbt[ci & 1];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int e = tid + 256 * j, k = e % KB, c = e / KB;
      sb[c * SP + k] = bq[j];
    }
    if (ci >= nfull) {  // ragged last chunk (uniform)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) xq[ks] = k0 + 4 * ks + g < kend ? xq[ks] : 0.0;
    }
    __syncthreads();
    // unconditional, so that the wait counts are the same on every path (the
    // last chunk reloads itself into the idle set)
    fetch(ci + 1 < nchunk ? k0 + KB : k0, bn, xn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int ct = cw0 + 16 * t;  // tile's first column within the block
      // tile t needs this chunk unless all of it lies below B's diagonal
      if (t < nt && (!b_upper || k0 <= c0 + ct + 15)) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const double bf = sb[(ct + i) * SP + 4 * ks + g];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, xq[ks], acc[t], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  fetch(0, bq0, xq0);
  for (int ci = 0; ci < nchunk; ci += 2) {
    chunk(ci, bq0, xq0, bq1, xq1);
    if (ci + 1 < nchunk) chunk(ci + 1, bq1, xq1, bq0, xq0);
  }
  if (!rok) return;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= nt) break;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int c = c0 + cw0 + 16 * t + g + 4 * s;
      if (c < ell) {
        if (o1.ptr) store_out_nt(o1, rr, c, acc[t][s]);
        if (o2.ptr) store_out_nt(o2, rr, c, acc[t][s]);
      } else if (c < ellp) {
        if (o1.ptr && pad1) store_out_nt(o1, rr, c, 0.0);
        if (o2.ptr && pad2) store_out_nt(o2, rr, c, 0.0);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R fused with R^{-1}, blocked, one workgroup of 1024
// threads (16 waves).  The l x l matrix is cut into nb = ceil(l/16) block
// rows and columns (padding: identity).  Tiles are 16 x 16 row-major:
//   W(I, K), I <= K : the matrix being factored; ends as R(I, K)
//   E(I, K), I >= K : Z = L^{-1} (L = R^T), built by the same row operations
//   X               : U^{-1} of the current diagonal block (row-major)
// Block step J:
//   1. one wave factors the diagonal block D = U^T U (unblocked, in registers
//      with lane shuffles) and writes U to W(J, J), U^{-T} to E(J, J) and
//      U^{-1} to X;
//   2. block row J: W(J, K) <- U^{-T} W(J, K) for K > J (rows of R) and
//      E(J, M) <- U^{-T} E(J, M) for M < J (rows of Z);
//   3. trailing update W(K, K2) -= R(J, K)^T R(J, K2) for J < K <= K2 and
//      E(K, M) -= R(J, K)^T E(J, M) for K > J, M <= J.  Wave 0 takes the
//      update of W(J+1, J+1) and goes straight on to step 1 of J + 1, so
//      each block step costs two barriers.
// Steps 2 and 3 are 16 x 16 x 16 products on FP64 matrix cores
// (v_mfma_f64_16x16x4f64, lane l holds A(l%16, k), B(k, l%16) with
// k = l/16 + 4 kstep; accumulator slot s is element (l/16 + 4s, l%16)).
// A pivot <= 4 l u max_i G_ii (or not finite) is a breakdown: status bit 1,
// and the caller's Householder fallback takes over.
typedef double d4c __attribute__((ext_vector_type(4)));

constexpr int kCholLdsNb = 8;  // tiles in LDS up to l = 128

__device__ __forceinline__ d4c tile_acc_load(const double* t, int lane) {
  const int g = lane >> 4, j = lane & 15;
  d4c r;
  r[0] = t[g * 16 + j];
  r[1] = t[(g + 4) * 16 + j];
  r[2] = t[(g + 8) * 16 + j];
  r[3] = t[(g + 12) * 16 + j];
  return r;
}

__device__ __forceinline__ void tile_acc_store(double* t, d4c v, int lane) {
  const int g = lane >> 4, j = lane & 15;
  t[g * 16 + j] = v[0];
  t[(g + 4) * 16 + j] = v[1];
  t[(g + 8) * 16 + j] = v[2];
  t[(g + 12) * 16 + j] = v[3];
}

// acc + sgn * A^T B for row-major 16 x 16 tiles A, B
__device__ __forceinline__ d4c tile_atb(const double* A, const double* B, d4c acc, double sgn,
                                        int lane) {
  const int g = lane >> 4, i = lane & 15;
  double a[4], b[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + g;
    a[ks] = sgn * A[k * 16 + i];
    b[ks] = B[k * 16 + i];
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One wave: D (16 x 16, symmetric, row-major at src) = U^T U.  Lane c < 32
// holds column c of [D | I] in registers (x[r] = row r).  Step s needs the
// pivot d_s and the multipliers D[r][s]/d_s of the rows below: column s,
// broadcast from lane s with v_readlane (a uniform lane index); the pivot
// row is each lane's own x[s], so rows r > s update as
// x[r] -= D[r][s] (x[s]/d_s).  The row scaling by 1/sqrt(d_r) that turns
// [L D' | L^-1] into [U | U^{-T}] is done once at the end.  Returns false on
// breakdown (the same on every lane: the pivot is a broadcast).
__device__ __forceinline__ bool chol_diag16(const double* src, int base, int ell, double thr,
                                            double* u_out, double* e_out, double* x_out, int lane) {
  const int c = lane & 31;
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = c < 16 ? src[r * 16 + c] : (r == c - 16 ? 1.0 : 0.0);
  double dd[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const double d = readlane_f64(x[s], s);
    if (base + s < ell && (!(d > thr) || !isfinite(d))) return false;
    dd[s] = d;
    // 1/d: hardware estimate refined by two Newton steps
    double rd = __builtin_amdgcn_rcp(d);
    rd = fma(rd, fma(-d, rd, 1.0), rd);
    rd = fma(rd, fma(-d, rd, 1.0), rd);
    // x[r] -= (D[r][s] / d_s) x[s], with x[s] / d_s formed once per lane
    const double piv_row = x[s] * rd;
#pragma unroll
    for (int r = s + 1; r < 16; ++r) x[r] = fma(-readlane_f64(x[r], s), piv_row, x[r]);
  }
  if (lane < 32) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      // 1/sqrt(d_r): hardware estimate refined by two Newton steps
      double iv = __builtin_amdgcn_rsq(dd[r]);
      iv = iv * (1.5 - 0.5 * dd[r] * iv * iv);
      iv = iv * (1.5 - 0.5 * dd[r] * iv * iv);
      const double v = x[r] * iv;
      if (c < 16) {
        u_out[r * 16 + c] = c >= r ? v : 0.0;
      } else {
        e_out[r * 16 + (c - 16)] = v;
        x_out[(c - 16) * 16 + r] = v;
      }
    }
  }
  return true;
}

__device__ __forceinline__ int chol_widx(int nb, int I, int K) { return I * nb - I * (I - 1) / 2 + (K - I); }
__device__ __forceinline__ int chol_eidx(int I, int K) { return I * (I + 1) / 2 + K; }

template <bool kLds>
__global__ void __launch_bounds__(1024) chol_kernel(const double* __restrict__ G, int ell,
                                                    double* __restrict__ R, double* __restrict__ Rinv,
                                                    int* status, const int* skip, double* work,
                                                    double single_thr) {
  if (skip && *skip) return;
  constexpr int kLdsTiles = kLds ? kCholLdsNb * (kCholLdsNb + 1) : 1;
  __shared__ double lds_tiles[kLdsTiles * 256];
  __shared__ double xt[256], dbuf[256];
  __shared__ double red[8];
  __shared__ double red_r[16], red_i[16];
  __shared__ double thr_s;
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int nb = (ell + 15) / 16;
  const int nw = nb * (nb + 1) / 2;
  double* wt = kLds ? lds_tiles : work;  // W tiles, then E tiles
  double* et = wt + (size_t)nw * 256;
  auto W = [&](int I, int K) { return wt + (size_t)chol_widx(nb, I, K) * 256; };
  auto E = [&](int I, int K) { return et + (size_t)chol_eidx(I, K) * 256; };

  // largest diagonal entry (and whether any is not finite)
  if (tid < 256) {
    const double d = tid < ell ? G[(int64_t)tid * ell + tid] : 0.0;
    double mx = isfinite(d) ? d : -1.0;
    double bad = isfinite(d) ? 0.0 : 1.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mx = fmax(mx, __shfl_xor(mx, off, 64));
      bad = fmax(bad, __shfl_xor(bad, off, 64));
    }
    if (lane == 0) {
      red[wave] = mx;
      red[4 + wave] = bad;
    }
  }
  // tiles: W from G (identity in the padding); consecutive threads read
  // consecutive entries of a column of G
  for (int e = tid; e < nb * nb * 256; e += blockDim.x) {
    const int tt = e >> 8, tI = tt / nb, tK = tt - tI * nb;
    if (tI > tK) continue;
    const int cc = e & 15, rr = (e >> 4) & 15;
    const int gi = 16 * tI + cc, gj = 16 * tK + rr;  // tile element (cc, rr) = G(gi, gj)
    W(tI, tK)[cc * 16 + rr] = (gi < ell && gj < ell) ? G[(int64_t)gj * ell + gi] : (gi == gj ? 1.0 : 0.0);
  }
  for (int e = tid; e < nw * 256; e += blockDim.x) et[e] = 0.0;
  if (tid == 0) {
    const double dmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double bad = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
    // a pivot below 4 l u max_i G_ii means the sketch's condition number is
    // beyond ~ (4 l u)^(-1/2): CholeskyQR is not reliable, fall back
    thr_s = bad != 0.0 ? -1.0 : 4.0 * ell * 2.220446049250313e-16 * dmax;
    flag = 0;
  }
  __syncthreads();
  const double thr = thr_s;
  if (thr < 0.0) {
    if (tid == 0) atomicOr(status, 2);
    return;
  }
  if (wave == 0 && !chol_diag16(W(0, 0), 0, ell, thr, W(0, 0), E(0, 0), xt, lane) && lane == 0) flag = 1;
  __syncthreads();
  if (flag) {
    if (tid == 0) atomicOr(status, 1);
    return;
  }
  for (int J = 0; J < nb; ++J) {
    // 2. block row J
    const int nW = nb - 1 - J;
    for (int o = wave; o < nW + J; o += nwaves) {
      double* T = o < nW ? W(J, J + 1 + o) : E(J, o - nW);
      d4c acc = {0.0, 0.0, 0.0, 0.0};
      acc = tile_atb(xt, T, acc, 1.0, lane);
      tile_acc_store(T, acc, lane);
    }
    __syncthreads();
    if (nW == 0) break;
    // 3. trailing update; wave 0: W(J+1, J+1), then the next diagonal block
    if (wave == 0) {
      d4c acc = tile_acc_load(W(J + 1, J + 1), lane);
      acc = tile_atb(W(J, J + 1), W(J, J + 1), acc, -1.0, lane);
      tile_acc_store(dbuf, acc, lane);
      if (!chol_diag16(dbuf, 16 * (J + 1), ell, thr, W(J + 1, J + 1), E(J + 1, J + 1), xt, lane) &&
          lane == 0)
        flag = 1;
    } else {
      const int nWops = nW * (nW + 1) / 2;
      const int nops = nWops - 1 + nW * (J + 1);
      for (int o = wave - 1; o < nops; o += nwaves - 1) {
        int q = o + 1;  // index 0 of the W list is W(J+1, J+1)
        if (q < nWops) {
          int a = 0, len = nW;
          while (q >= len) {
            q -= len;
            ++a;
            --len;
          }
          const int K = J + 1 + a, K2 = K + q;
          double* T = W(K, K2);
          d4c acc = tile_acc_load(T, lane);
          acc = tile_atb(W(J, K), W(J, K2), acc, -1.0, lane);
          tile_acc_store(T, acc, lane);
        } else {
          q -= nWops;
          const int K = J + 1 + q / (J + 1), M = q % (J + 1);
          double* T = E(K, M);
          d4c acc = tile_acc_load(T, lane);
          acc = tile_atb(W(J, K), E(J, M), acc, -1.0, lane);
          tile_acc_store(T, acc, lane);
        }
      }
    }
    __syncthreads();
    if (flag) {
      if (tid == 0) atomicOr(status, 1);
      return;
    }
  }
  // R (upper, zeros below) and R^{-1} = Z^T, column-major; one 16 x 16
  // block per wave at a time, 16 lanes writing 16 consecutive rows.  The
  // squared Frobenius norms of both are summed on the way.
  double ssr = 0.0, ssi = 0.0;
  for (int tt = wave; tt < nb * nb; tt += nwaves) {
    const int I = tt % nb, K = tt / nb;  // row block, column block
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = lane & 15, cc = (lane >> 4) + 4 * u;
      const int r = 16 * I + rr, c = 16 * K + cc;
      if (r >= ell || c >= ell) continue;
      double vr = 0.0, vi = 0.0;
      if (I <= K) {
        vr = W(I, K)[rr * 16 + cc];
        if (r <= c) vi = E(K, I)[cc * 16 + rr];
        if (r > c) vr = 0.0;
      }
      R[(int64_t)c * ell + r] = vr;
      Rinv[(int64_t)c * ell + r] = vi;
      ssr += vr * vr;
      ssi += vi * vi;
    }
  }
  if (single_thr > 0.0) {
    // One CholeskyQR step leaves Q^T Q - I of order u kappa(X)^2, and
    // kappa_2(R) <= ||R||_F ||R^-1||_F.  When u l (||R||_F ||R^-1||_F)^2 is at
    // most single_thr, the second step is not needed: status bit 3.
    ssr = wave_sum_f64(ssr);
    ssi = wave_sum_f64(ssi);
    if (lane == 0) {
      red_r[wave] = ssr;
      red_i[wave] = ssi;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int q = 0; q < nwaves; ++q) {
        a += red_r[q];
        b += red_i[q];
      }
      if (2.220446049250313e-16 * ell * a * b <= single_thr) atomicOr(status, 4);
    }
  }
}

// ---------------------------------------------------------------------------
// CholeskyQR2 of a sketch with l <= 16 columns (eq. 6), in three launches:
//   step 0: Gram of X;                      last block: R1, R1^-1 = chol(G)
//   step 1: X1 = X R1^-1 and the Gram of X1; last block: R2, R2^-1, R = R2 R1
//           (when the first step already suffices, status 4: Q = X R1^-1)
//   step 2: Q = X1 R2^-1, with X1 recomputed from X (the same operations in
//           the same order as in step 1, so the same values)
// or, when one workgroup holds every row (at most 1024), in one launch that
// runs the three steps back to back.  The rows are split into nblk row
// blocks of 1024-row chunks; each thread holds one row of a chunk in
// registers, the chunk goes to LDS and its Gram accumulates on FP64 matrix
// cores (v_mfma_f64_16x16x4f64: lane l feeds row 4t + l/16, column l%16 as
// both operands, 64 rows per wave); the 16 waves' sums are added in wave
// order and written as the block's partial.  The last block to finish (a
// counter in device memory, agent-scope fences on both sides) adds the
// partials in block order (four quarters of the blocks in parallel, the
// quarters then added in order) and factors the Gram with the same one-wave
// 16 x 16 kernel, breakdown rule and one-step rule as chol_kernel.  No block
// waits for another.  Status bits as for chol_kernel; after bit 1 the
// Householder fallback takes over from X.
constexpr int kQ16Rows = 1024;      // rows of a chunk (one per thread)
constexpr int kQ16MaxBlocks = 256;
constexpr int kQ16Pad = 17;         // LDS row stride of a chunk (doubles)

struct Q16Args {
  const double* x0;   // the sketch X (rows x l, column-major, ld)
  int64_t ld, rows;
  int ell, nblk;
  double* gpart;      // nblk x 256 partial Grams (row-major 16 x 16)
  double* tiles;      // 4 x 256: R1, R1^-1, R2, R2^-1 (row-major 16 x 16)
  double* rfac;       // nullable: R (l x l, column-major)
  double* q64;        // Q (rows x 16, ld; columns l..15 zero)
  float* q32;         // nullable float copy of Q (ld)
  int* status;
  int* counter;
  double single_thr;
};

struct Q16Lds {
  double tile[kQ16Rows * kQ16Pad];  // a chunk, then the waves' Gram sums
  double ra[256], rb[256];          // R^-1 factors the launch applies
  double gm[256], ex[256], xs[256];
  double red[8];
  int flag;
};

// row i of X (zeros beyond l and for rows not in the block); every load
// unconditional, from a clamped address (ic: a row of the block)
__device__ __forceinline__ void q16_row(const Q16Args& a, int64_t i, int64_t ic, bool in, double (&x)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double v = a.x0[(int64_t)(k < a.ell ? k : a.ell - 1) * a.ld + ic];
    x[k] = (in && k < a.ell) ? v : 0.0;
  }
}

// The chunk in LDS (row-major, stride kQ16Pad): each thread writes and reads
// its own row; a wave's matrix-core products touch only its 64 rows, so
// these steps need no barrier between them.
__device__ __forceinline__ void q16_put(Q16Lds& sh, const double (&x)[16]) {
#pragma unroll
  for (int j = 0; j < 16; ++j) sh.tile[threadIdx.x * kQ16Pad + j] = x[j];
}

__device__ __forceinline__ void q16_get(const Q16Lds& sh, double (&y)[16]) {
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j] = sh.tile[threadIdx.x * kQ16Pad + j];
}

// the wave's rows <- rows x M (M row-major 16 x 16 in LDS: an upper
// triangular R^-1 with the identity in the padding, so columns >= l stay
// zero), 16 rows at a time on FP64 matrix cores (operand A: lane l feeds row
// l%16, column 4s + l/16; operand B: row 4s + l/16 of M, column l%16)
__device__ __forceinline__ void q16_tile_mul(Q16Lds& sh, const double* M, int64_t nvalid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  if (wave * 64 >= nvalid) return;  // the wave's rows are all padding (zeros)
  double b[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) b[ks] = M[(4 * ks + g) * 16 + c];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int row0 = wave * 64 + rb * 16;
    d4c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sh.tile[(row0 + c) * kQ16Pad + 4 * ks + g], b[ks], acc, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) sh.tile[(row0 + g + 4 * q) * kQ16Pad + c] = acc[q];
  }
}

// the Gram of the wave's 64 rows into its accumulator (lane l feeds row
// 4t + l/16, column l%16 as both operands); nvalid: rows of the chunk that
// hold data (the others are zeros and add nothing)
__device__ __forceinline__ void q16_tile_gram(const Q16Lds& sh, d4c& acc, int64_t nvalid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave * 64 >= nvalid) return;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const double v = sh.tile[(wave * 64 + 4 * t + (lane >> 4)) * kQ16Pad + (lane & 15)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
  }
}

// the 16 waves' accumulators added in wave order: entry e of the block's
// Gram for threads e < 256 (ends with a barrier)
__device__ __forceinline__ double q16_gram_block(Q16Lds& sh, const d4c& acc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __syncthreads();  // every wave is done with its rows of the chunk
#pragma unroll
  for (int q = 0; q < 4; ++q) sh.tile[wave * 256 + ((lane >> 4) + 4 * q) * 16 + (lane & 15)] = acc[q];
  __syncthreads();
  double g = 0.0;
  if (tid < 256) {
#pragma unroll
    for (int w = 0; w < 16; ++w) g += sh.tile[w * 256 + tid];
  }
  __syncthreads();
  return g;
}

// Cholesky of the Gram in sh.gm (identity in the padding) by wave 0: R to
// sh.gm (row-major, upper), R^-1 to sh.xs (row-major).  Returns, for wave 0,
// the status bits: 1 breakdown, 2 non-finite data, 4 one step suffices
// (when one_thr > 0).  The caller's barrier publishes the results.
__device__ __forceinline__ int q16_chol(Q16Lds& sh, int ell, double one_thr) {
  const int lane = threadIdx.x & 63;
  const double d = lane < ell ? sh.gm[lane * 17] : 0.0;
  double mx = isfinite(d) ? d : -1.0;
  double bad = isfinite(d) ? 0.0 : 1.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    bad = fmax(bad, __shfl_xor(bad, off, 64));
  }
  if (bad != 0.0) return 2;
  // breakdown threshold 4 l u max_i G_ii
  const double thr = 4.0 * ell * 2.220446049250313e-16 * mx;
  if (!chol_diag16(sh.gm, 0, ell, thr, sh.gm, sh.ex, sh.xs, lane)) return 1;
  if (one_thr > 0.0) {
    // one CholeskyQR step leaves Q^T Q - I of order u kappa(X)^2, and
    // kappa_2(R) <= ||R||_F ||R^-1||_F
    double ssr = 0.0, ssi = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = lane + 64 * q, r = e >> 4, c = e & 15;
      if (r < ell && c < ell) {
        ssr += sh.gm[e] * sh.gm[e];
        ssi += sh.xs[e] * sh.xs[e];
      }
    }
    ssr = wave_sum_f64(ssr);
    ssi = wave_sum_f64(ssi);
    if (2.220446049250313e-16 * ell * ssr * ssi <= one_thr) return 4;
  }
  return 0;
}

// Q rows from the thread's row y (already the basis), FP64 and float copy
__device__ __forceinline__ void q16_store(const Q16Args& a, int64_t i, bool in, const double (&y)[16]) {
  if (!in) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    a.q64[(int64_t)j * a.ld + i] = y[j];
    if (a.q32) a.q32[(int64_t)j * a.ld + i] = (float)y[j];
  }
}

// R = R2 R1 (column-major l x l) from row-major R2 (r2) and R1 (r1)
__device__ __forceinline__ void q16_rfac(double* out, const double* r2, const double* r1, int ell, int from,
                                         int step) {
  for (int e = from; e < ell * ell; e += step) {
    const int i = e % ell, j = e / ell;
    double v = 0.0;
    for (int t = i; t <= j; ++t) v = fma(r2[i * 16 + t], r1[t * 16 + j], v);
    out[e] = i <= j ? v : 0.0;
  }
}

// The Gram held by threads e < 256 into sh.gm with the identity in the
// padding, then factored by wave 0.  Returns the status bits to every
// thread (sh.flag); R and R^-1 stay in sh.gm / sh.xs.
__device__ __forceinline__ int q16_factor(Q16Lds& sh, double g, int ell, double one_thr) {
  const int tid = threadIdx.x;
  if (tid < 256) {
    const int r = tid >> 4, c = tid & 15;
    sh.gm[tid] = (r < ell && c < ell) ? g : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < 64) {
    const int f = q16_chol(sh, ell, one_thr);
    if (tid == 0) sh.flag = f;
  }
  __syncthreads();
  return sh.flag;
}

// steps 0 and 1 of the three-launch form, and step 2 (sw: the status word
// as the launch found it)
template <int STEP>
__device__ __forceinline__ void q16_body(const Q16Args& a, Q16Lds& sh, int sw) {
  if (STEP >= 1 && (sw & 3)) return;  // breakdown or non-finite data: nothing to do here
  if (STEP == 2 && (sw & 4)) return;  // the first step already wrote Q
  const bool final1 = STEP == 1 && (sw & 4);
  const int tid = threadIdx.x;
  const int ell = a.ell;
  if (STEP >= 1 && tid < 256) {
    sh.ra[tid] = a.tiles[256 + tid];                // R1^-1
    if (STEP == 2) sh.rb[tid] = a.tiles[768 + tid];  // R2^-1
  }
  if (final1 && blockIdx.x == 0 && a.rfac && tid < ell * ell) {  // R = R1
    const int i = tid % ell, j = tid / ell;
    a.rfac[tid] = a.tiles[i * 16 + j];
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * a.rows / a.nblk;
  const int64_t r1 = (int64_t)(blockIdx.x + 1) * a.rows / a.nblk;
  const bool gram = !(STEP == 2 || final1);
  d4c acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = r0; c0 < r1; c0 += kQ16Rows) {
    const int64_t i = c0 + tid;
    const bool in = i < r1;
    double x[16];
    q16_row(a, i, in ? i : r1 - 1, in, x);
    q16_put(sh, x);
    const int64_t nv = r1 - c0;
    if (STEP >= 1) q16_tile_mul(sh, sh.ra, nv);  // X1 (or Q when one step suffices)
    if (STEP == 2) q16_tile_mul(sh, sh.rb, nv);  // Q
    if (gram) {
      q16_tile_gram(sh, acc, nv);
    } else {
      q16_get(sh, x);
      q16_store(a, i, in, x);
    }
  }
  if (!gram) return;
  const double g = q16_gram_block(sh, acc);
  if (tid == 0) sh.flag = 0;
  if (tid < 256) {
    a.gpart[(int64_t)blockIdx.x * 256 + tid] = g;
    __threadfence();  // the partial is visible device-wide before the count
  }
  __syncthreads();
  if (tid == 0) sh.flag = atomicAdd(a.counter, 1) == a.nblk - 1;
  __syncthreads();
  if (!sh.flag) return;
  __threadfence();  // every other block's partial is visible from here on
  // the partials in block order: quarter u = tid / 256 adds blocks
  // [u nq, (u + 1) nq) of entry tid % 256, its loads in flight in groups of
  // 16 (clamped addresses; the clamped terms are not added); then the
  // quarters in order
  const int e = tid & 255, u = tid >> 8;
  const int nq = (a.nblk + 3) / 4;
  const int b0 = u * nq, b1 = min(a.nblk, b0 + nq);
  double gq = 0.0;
  for (int bb = b0; bb < b1; bb += 16) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = a.gpart[(int64_t)min(bb + k, b1 - 1) * 256 + e];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (bb + k < b1) gq += v[k];
  }
  sh.tile[u * 256 + e] = gq;
  __syncthreads();
  const double gt = ((sh.tile[e] + sh.tile[256 + e]) + sh.tile[512 + e]) + sh.tile[768 + e];
  const int f = q16_factor(sh, gt, ell, STEP == 0 ? a.single_thr : 0.0);
  if (tid == 0) {
    if (f & 3) atomicOr(a.status, f & 3);
    if (f == 4) atomicOr(a.status, 4);
  }
  if (!(f & 3) && tid < 256) {
    // R (upper, row-major) and R^-1 for the next launch
    a.tiles[(STEP == 0 ? 0 : 512) + tid] = sh.gm[tid];
    a.tiles[(STEP == 0 ? 256 : 768) + tid] = sh.xs[tid];
  }
  if (STEP == 1 && !(f & 3) && a.rfac) q16_rfac(a.rfac, sh.gm, a.tiles, ell, tid, 1024);
  if (tid == 0) atomicExch(a.counter, 0);  // ready for the next launch
}

template <int STEP>
__global__ void __launch_bounds__(1024) q16_kernel(Q16Args a) {
  __shared__ Q16Lds sh;
  q16_body<STEP>(a, sh, *a.status);
}

// The three steps in one workgroup (rows <= 1024, X kept in registers).
// Returns the status bits of the factorization that ended it (bit 1
// breakdown and bit 2 non-finite data, already recorded; else 0 or 4).
__device__ __forceinline__ int q16_one_body(const Q16Args& a, Q16Lds& sh) {
  const int tid = threadIdx.x, ell = a.ell;
  const bool in = tid < a.rows;
  double x[16];
  q16_row(a, tid, in ? tid : a.rows - 1, in, x);
  q16_put(sh, x);
  d4c acc = {0.0, 0.0, 0.0, 0.0};
  q16_tile_gram(sh, acc, a.rows);
  int f = q16_factor(sh, q16_gram_block(sh, acc), ell, a.single_thr);
  if (f & 3) {
    if (tid == 0) atomicOr(a.status, f & 3);
    return f & 3;
  }
  if (tid < 256) {
    sh.ra[tid] = sh.xs[tid];  // R1^-1
    sh.rb[tid] = sh.gm[tid];  // R1
  }
  q16_put(sh, x);  // the Gram sums used the tile
  __syncthreads();
  q16_tile_mul(sh, sh.ra, a.rows);  // X1
  if (f == 4) {  // one step suffices: Q = X R1^-1, R = R1
    if (tid == 0) atomicOr(a.status, 4);
    q16_get(sh, x);
    q16_store(a, tid, in, x);
    if (a.rfac && tid < ell * ell) {
      const int i = tid % ell, j = tid / ell;
      a.rfac[tid] = sh.rb[i * 16 + j];
    }
    return 4;
  }
  acc = d4c{0.0, 0.0, 0.0, 0.0};
  q16_tile_gram(sh, acc, a.rows);
  f = q16_factor(sh, q16_gram_block(sh, acc), ell, 0.0);
  if (f & 3) {
    if (tid == 0) atomicOr(a.status, f & 3);
    return f & 3;
  }
  // X1 again (the Gram sums used the tile), then Q = X1 R2^-1
  q16_put(sh, x);
  q16_tile_mul(sh, sh.ra, a.rows);
  q16_tile_mul(sh, sh.xs, a.rows);
  q16_get(sh, x);
  q16_store(a, tid, in, x);
  if (a.rfac) q16_rfac(a.rfac, sh.gm, sh.rb, ell, tid, 1024);
  return 0;
}

__global__ void __launch_bounds__(1024) q16_one_kernel(Q16Args a) {
  __shared__ Q16Lds sh;
  q16_one_body(a, sh);
}

// ---------------------------------------------------------------------------
// Householder thin QR (fallback after a Cholesky breakdown).  A tall X is
// factored as a two-level tree (TSQR, Demmel, Grigori, Hoemmen and Langou):
// each of P row panels is reduced by Householder reflections in its own
// workgroup, the P stacked ell x ell triangles are reduced by one workgroup,
// and each panel's reflectors are applied to its ell x ell block of the root
// Q.  The product is X = Q R with Q orthonormal for any X, rank-deficient
// ones included.  A short X (fewer than two panels) is one workgroup's job.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over i = s, s + 64, ... < rows (lane offsets added by the caller) of
// v_i w_i, with v_s replaced by v0; four loads of each column in flight, the
// terms still added in ascending i
__device__ __forceinline__ double hh_dot(const double* __restrict__ v, const double* __restrict__ w,
                                         int64_t i, int64_t s, int64_t rows, double v0) {
  double d = 0.0;
  for (; i + 192 < rows; i += 256) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = v[i + 64 * u];
      b[u] = w[i + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) d += (i + 64 * u == s ? v0 : a[u]) * b[u];
  }
  for (; i < rows; i += 64) d += (i == s ? v0 : v[i]) * w[i];
  return d;
}

// w_i -= d v_i over the same index set
__device__ __forceinline__ void hh_axpy(const double* __restrict__ v, double* __restrict__ w, int64_t i,
                                        int64_t s, int64_t rows, double v0, double d) {
  for (; i + 192 < rows; i += 256) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = v[i + 64 * u];
      b[u] = w[i + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) w[i + 64 * u] = b[u] - d * (i + 64 * u == s ? v0 : a[u]);
  }
  for (; i < rows; i += 64) w[i] -= d * (i == s ? v0 : v[i]);
}

// Householder reduction of the rows x ell column-major W in place (NT
// threads; waves own columns j = wave mod NT/64).  On return the part of
// column s below row s holds the tail of reflector s (its head is vhead[s]),
// the strict upper part holds R's off-diagonal entries, R[s,s] = alpha[s] and
// H_s = I - tau[s] v v^T (tau = 0 for a zero column).
template <int NT>
__device__ void hh_factor(double* __restrict__ W, int64_t ldw, int64_t rows, int ell, double* tau,
                          double* alpha, double* vhead, double* red) {
  constexpr int nw = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int s = 0; s < ell; ++s) {
    double part = 0.0;
    for (int64_t i = s + tid; i < rows; i += NT) {
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
      const double* vs = W + (int64_t)s * ldw;
      for (int j = s + 1 + wave; j < ell; j += nw) {
        double* wj = W + (int64_t)j * ldw;
        const double d = wave_sum(hh_dot(vs, wj, s + lane, s, rows, v0)) * ts;
        hh_axpy(vs, wj, s + lane, s, rows, v0, d);
      }
    }
    __syncthreads();
  }
}

// Q <- H_0 ... H_{ell-1} Q for the rows x ell Q, with the reflectors left in W
// by hh_factor.  Columns below jmin are not touched (Q = [I; 0] needs only
// j >= s at step s: earlier columns are unit vectors zero from row s on).
template <int NT>
__device__ void hh_apply(const double* __restrict__ W, int64_t ldw, int64_t rows, int ell,
                         const double* tau, const double* vhead, double* __restrict__ Q, int64_t ldq,
                         bool identity) {
  constexpr int nw = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int s = ell - 1; s >= 0; --s) {
    const double ts = tau[s], v0 = vhead[s];
    if (ts != 0.0) {
      const double* vs = W + (int64_t)s * ldw;
      for (int j = (identity ? s : 0) + wave; j < ell; j += nw) {
        double* qj = Q + (int64_t)j * ldq;
        const double d = wave_sum(hh_dot(vs, qj, s + lane, s, rows, v0)) * ts;
        hh_axpy(vs, qj, s + lane, s, rows, v0, d);
      }
    }
    __syncthreads();
  }
}

constexpr int kHhLds = 7168;       // doubles of a panel reduced in LDS (56 KB)
constexpr int kHhRootLds = 18432;  // doubles of LDS of the one-workgroup QR (144 KB)

// One workgroup: X (rows x ell) -> Q (diag R >= 0), R (nullable, ld ell).
// The working copy of X and then Q are kept in LDS when both fit, else the
// working copy alone, else both live in device memory (W and Q).
__global__ void __launch_bounds__(1024) householder_kernel(const double* __restrict__ X,
                                                           int64_t ldx, int64_t rows, int ell,
                                                           double* __restrict__ W, int64_t ldw,
                                                           double* __restrict__ Q, int64_t ldq,
                                                           float* __restrict__ Q32, int64_t ldq32,
                                                           double* __restrict__ R,
                                                           const int* status) {
  if ((*status & 3) != 1) return;  // only after a Cholesky breakdown
  __shared__ double sw[kHhRootLds];
  __shared__ double tau[256], alpha[256], vhead[256];
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const int64_t n = rows * ell;
  const bool lds = n <= kHhRootLds;
  const bool qlds = 2 * n <= kHhRootLds;
  double* Wp = lds ? sw : W;
  const int64_t ldp = lds ? rows : ldw;
  double* Qp = qlds ? sw + n : Q;
  const int64_t ldqp = qlds ? rows : ldq;
  for (int64_t e = tid; e < n; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    Wp[(int64_t)j * ldp + i] = X[(int64_t)j * ldx + i];
  }
  __syncthreads();
  hh_factor<1024>(Wp, ldp, rows, ell, tau, alpha, vhead, red);
  // R (upper, ell x ell, column-major ld ell) with diag >= 0
  if (R) {
    for (int e = tid; e < ell * ell; e += 1024) {
      const int i = e % ell, j = e / ell;
      double v = i < j ? Wp[(int64_t)j * ldp + i] : (i == j ? alpha[i] : 0.0);
      if (alpha[i] < 0.0) v = -v;
      R[e] = v;
    }
  }
  // Q = H_0 ... H_{ell-1} [I; 0]
  for (int64_t e = tid; e < n; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    Qp[(int64_t)j * ldqp + i] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  hh_apply<1024>(Wp, ldp, rows, ell, tau, vhead, Qp, ldqp, true);
  // sign normalisation diag(R) >= 0: flip the columns of Q with alpha < 0
  for (int64_t e = tid; e < n; e += 1024) {
    const int64_t i = e % rows;
    const int j = (int)(e / rows);
    double v = Qp[(int64_t)j * ldqp + i];
    if (alpha[j] < 0.0) v = -v;
    if (qlds || alpha[j] < 0.0) Q[(int64_t)j * ldq + i] = v;
    if (Q32) Q32[(int64_t)j * ldq32 + i] = (float)v;
  }
}

// Panels of the tree.  A panel of at most kHhLds entries is factored in LDS
// (panels then split the rows evenly: panel b is rows [b rows / P,
// (b + 1) rows / P)); otherwise panel b is rows [b h, b h + h) of the
// workspace copy, the last one taking the remainder.  Either way the
// reflectors end in W (rows of the panel), where the expand step reads them.
__device__ __forceinline__ void hh_panel_range(int b, int64_t rows, int64_t h, int P, int lds, int64_t& r0,
                                               int64_t& hb) {
  if (lds) {
    r0 = (int64_t)b * rows / P;
    hb = (int64_t)(b + 1) * rows / P - r0;
  } else {
    r0 = (int64_t)b * h;
    hb = b == P - 1 ? rows - r0 : h;
  }
}

// Tree level 1: panel b is reduced (in LDS or in W); its triangle goes to
// rows [b ell, (b + 1) ell) of the stacked Rs (ld P ell), its tau and
// reflector heads to tv[b * 2 ell ...].
__global__ void __launch_bounds__(256) hh_panel_kernel(const double* __restrict__ X, int64_t ldx,
                                                       int64_t rows, int ell, int64_t h, int P, int lds,
                                                       double* __restrict__ W, int64_t ldw,
                                                       double* __restrict__ Rs, double* __restrict__ tv,
                                                       const int* status) {
  if ((*status & 3) != 1) return;
  __shared__ double sw[kHhLds];
  __shared__ double tau[256], alpha[256], vhead[256];
  __shared__ double red[4];
  const int tid = threadIdx.x, b = blockIdx.x;
  int64_t r0, hb;
  hh_panel_range(b, rows, h, P, lds, r0, hb);
  double* Wp = lds ? sw : W + r0;
  const int64_t ldp = lds ? hb : ldw;
  for (int64_t e = tid; e < hb * ell; e += 256) {
    const int64_t i = e % hb;
    const int j = (int)(e / hb);
    Wp[(int64_t)j * ldp + i] = X[(int64_t)j * ldx + r0 + i];
  }
  __syncthreads();
  hh_factor<256>(Wp, ldp, hb, ell, tau, alpha, vhead, red);
  const int64_t ldr = (int64_t)P * ell;
  for (int e = tid; e < ell * ell; e += 256) {
    const int i = e % ell, j = e / ell;
    Rs[(int64_t)j * ldr + (int64_t)b * ell + i] =
        i < j ? Wp[(int64_t)j * ldp + i] : (i == j ? alpha[i] : 0.0);
  }
  for (int s = tid; s < ell; s += 256) {
    tv[(int64_t)b * 2 * ell + s] = tau[s];
    tv[(int64_t)b * 2 * ell + ell + s] = vhead[s];
  }
  if (lds) {
    for (int64_t e = tid; e < hb * ell; e += 256) {
      const int64_t i = e % hb;
      const int j = (int)(e / hb);
      W[(int64_t)j * ldw + r0 + i] = sw[(int64_t)j * hb + i];
    }
  }
}

// Tree level 2 (after the root's Householder QR of Rs gave Qr, ld P ell):
// panel b of Q is its reflectors applied to [Qr rows b ell ... ; 0].
__global__ void __launch_bounds__(256) hh_expand_kernel(const double* __restrict__ W, int64_t ldw,
                                                        int64_t rows, int ell, int64_t h, int P, int lds,
                                                        const double* __restrict__ Qr,
                                                        const double* __restrict__ tv,
                                                        double* __restrict__ Q, int64_t ldq,
                                                        float* __restrict__ Q32, int64_t ldq32,
                                                        const int* status) {
  if ((*status & 3) != 1) return;
  // LDS panels: the reflectors and the panel of Q both in LDS
  __shared__ double sw[kHhLds], sq[kHhLds];
  __shared__ double tau[256], vhead[256];
  const int tid = threadIdx.x, b = blockIdx.x;
  int64_t r0, hb;
  hh_panel_range(b, rows, h, P, lds, r0, hb);
  const int64_t ldr = (int64_t)P * ell;
  for (int s = tid; s < ell; s += 256) {
    tau[s] = tv[(int64_t)b * 2 * ell + s];
    vhead[s] = tv[(int64_t)b * 2 * ell + ell + s];
  }
  double* Qp = lds ? sq : Q + r0;
  const int64_t ldqp = lds ? hb : ldq;
  for (int64_t e = tid; e < hb * ell; e += 256) {
    const int64_t i = e % hb;
    const int j = (int)(e / hb);
    Qp[(int64_t)j * ldqp + i] = i < ell ? Qr[(int64_t)j * ldr + (int64_t)b * ell + i] : 0.0;
    if (lds) sw[(int64_t)j * hb + i] = W[(int64_t)j * ldw + r0 + i];
  }
  __syncthreads();
  if (lds)
    hh_apply<256>(sw, hb, hb, ell, tau, vhead, sq, hb, false);
  else
    hh_apply<256>(W + r0, ldw, hb, ell, tau, vhead, Q + r0, ldq, false);
  if (lds || Q32) {
    for (int64_t e = tid; e < hb * ell; e += 256) {
      const int64_t i = e % hb;
      const int j = (int)(e / hb);
      const double v = Qp[(int64_t)j * ldqp + i];
      if (lds) Q[(int64_t)j * ldq + r0 + i] = v;
      if (Q32) Q32[(int64_t)j * ldq32 + r0 + i] = (float)v;
    }
  }
}

// ---------------------------------------------------------------------------
// The same three Householder steps for l <= 64, organised for small l: thread
// t serves column j = t % L (L = 16, 32 or 64 >= l) and the rows
// i = t / L + G q (G = NT / L row groups), so every column operation of a
// step (the norm, the dot products with the reflector, the update) runs for
// all columns at once.  A sum over the rows adds each thread's partial sum
// (its rows in increasing order) over the row groups: the lanes of a wave by
// a butterfly over the group bits of the lane index, then the waves in wave
// order through LDS (double-buffered: one barrier per sum); every thread
// reads the column's total with the same bits.  Working copies in LDS are
// row-major with row stride L + 1.
template <bool RowMajor>
struct HhMat {
  double* p;
  int64_t ld;
  __device__ __forceinline__ double& at(int64_t i, int j) const { return RowMajor ? p[i * ld + j] : p[(int64_t)j * ld + i]; }
};

template <int NT, int L>
__device__ __forceinline__ double col_sum_at(double part, double* red, int buf, int col) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = L; off < 64; off <<= 1) part = part + __shfl_xor(part, off, 64);
  double* rb = red + buf * (NT / 64) * L;
  if (lane < L) rb[wave * L + lane] = part;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) tot += rb[w * L + col];
  return tot;
}

// Own rows i >= s of thread row group r: r + G q, the first one at or after s.
template <int G>
__device__ __forceinline__ int64_t hh_first_row(int r, int s) {
  const int d = s - r;
  return d <= 0 ? (int64_t)r : r + (int64_t)((d + G - 1) / G) * G;
}

// sum over own rows i >= s of v_i B(i, j), v_i = (i == s ? v0 : W(i, s)):
// four rows in flight, four partial sums added as (a0 + a1) + (a2 + a3)
template <int G, typename MB>
__device__ __forceinline__ double hh_rows_dot(HhMat<true> W, MB B, int64_t rows, int r, int s, int j, double v0) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t i = hh_first_row<G>(r, s);
  for (; i + 3 * G < rows; i += 4 * G) {
    const double x0 = i == s ? v0 : W.at(i, s), x1 = W.at(i + G, s), x2 = W.at(i + 2 * G, s),
                 x3 = W.at(i + 3 * G, s);
    const double y0 = B.at(i, j), y1 = B.at(i + G, j), y2 = B.at(i + 2 * G, j), y3 = B.at(i + 3 * G, j);
    a0 = fma(x0, y0, a0);
    a1 = fma(x1, y1, a1);
    a2 = fma(x2, y2, a2);
    a3 = fma(x3, y3, a3);
  }
  for (; i < rows; i += G) a0 = fma(i == s ? v0 : W.at(i, s), B.at(i, j), a0);
  return (a0 + a1) + (a2 + a3);
}

// B(i, j) -= d v_i over own rows i >= s
template <int G, typename MB>
__device__ __forceinline__ void hh_rows_axpy(HhMat<true> W, MB B, int64_t rows, int r, int s, int j, double v0,
                                             double d) {
  int64_t i = hh_first_row<G>(r, s);
  if (i == s && i < rows) {
    B.at(i, j) -= d * v0;
    i += G;
  }
  for (; i + 3 * G < rows; i += 4 * G) {
    const double x0 = W.at(i, s), x1 = W.at(i + G, s), x2 = W.at(i + 2 * G, s), x3 = W.at(i + 3 * G, s);
    B.at(i, j) -= d * x0;
    B.at(i + G, j) -= d * x1;
    B.at(i + 2 * G, j) -= d * x2;
    B.at(i + 3 * G, j) -= d * x3;
  }
  for (; i < rows; i += G) B.at(i, j) -= d * W.at(i, s);
}

// Householder reduction of the rows x ell matrix W (LDS, row-major) in place;
// the same outputs as hh_factor.  red: 2 (NT/64) L doubles of LDS.
template <int NT, int L>
__device__ void hh_factor_s(HhMat<true> W, int64_t rows, int ell, double* tau, double* alpha, double* vhead,
                            double* red) {
  constexpr int G = NT / L;
  const int t = threadIdx.x, j = t % L, r = t / L;
  int buf = 0;  // consecutive sums use alternate halves of red
  for (int s = 0; s < ell; ++s) {
    // squared norm of column s over rows >= s (threads of column s)
    double p = 0.0;
    if (j == s) p = hh_rows_dot<G>(W, W, rows, r, s, s, W.at(s, s) /* v_s = x_s here */);
    const double nrm2 = col_sum_at<NT, L>(p, red, buf, s);
    buf ^= 1;
    const double x0 = W.at(s, s);
    const double nrm = sqrt(nrm2);
    double ts = 0.0, v0 = 0.0, a = 0.0;
    if (nrm != 0.0) {
      a = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - a;
      ts = 2.0 / (nrm2 - x0 * x0 + v0 * v0);
    }
    if (t == 0) {
      tau[s] = ts;
      alpha[s] = a;
      vhead[s] = v0;
    }
    if (ts == 0.0) continue;  // uniform: a zero column needs no reflector
    // d_j = tau v^T W[:, j] for the columns right of s, then the update
    const bool act = j > s && j < ell;
    double d = act ? hh_rows_dot<G>(W, W, rows, r, s, j, v0) : 0.0;
    d = col_sum_at<NT, L>(d, red, buf, j) * ts;
    buf ^= 1;
    if (act) hh_rows_axpy<G>(W, W, rows, r, s, j, v0, d);
  }
  __syncthreads();
}

// Q <- H_0 ... H_{ell-1} Q with the reflectors of hh_factor_s in W (LDS,
// row-major); identity: Q starts as [I; 0] (columns j < s untouched at s).
template <int NT, int L, bool QRow>
__device__ void hh_apply_s(HhMat<true> W, int64_t rows, int ell, const double* tau, const double* vhead,
                           HhMat<QRow> Q, bool identity, double* red) {
  constexpr int G = NT / L;
  const int t = threadIdx.x, j = t % L, r = t / L;
  int buf = 0;
  for (int s = ell - 1; s >= 0; --s) {
    const double ts = tau[s], v0 = vhead[s];
    if (ts == 0.0) continue;
    const bool act = j < ell && (!identity || j >= s);
    double d = act ? hh_rows_dot<G>(W, Q, rows, r, s, j, v0) : 0.0;
    d = col_sum_at<NT, L>(d, red, buf, j) * ts;
    buf ^= 1;
    if (act) hh_rows_axpy<G>(W, Q, rows, r, s, j, v0, d);
  }
  __syncthreads();
}

constexpr int kHhSmallLds = 17920;  // doubles of working copies in LDS (140 KB)

// One workgroup (the root of the tree, or a whole short X): X (rows x ell,
// column-major) -> Q (diag R >= 0), R (nullable).  W in LDS; Q in LDS when
// both fit, else in device memory.
template <int L, bool QInLds>
__global__ void __launch_bounds__(1024) householder_s_kernel(const double* __restrict__ X, int64_t ldx,
                                                             int64_t rows, int ell, double* __restrict__ Q,
                                                             int64_t ldq, float* __restrict__ Q32, int64_t ldq32,
                                                             double* __restrict__ R, const int* status) {
  if ((*status & 3) != 1) return;
  __shared__ double sw[kHhSmallLds];
  __shared__ double tau[L], alpha[L], vhead[L];
  __shared__ double red[2 * 16 * L];
  const int tid = threadIdx.x;
  // row stride L + 1 (no two rows of a column in one bank) when it fits, else L
  const int64_t LS = (QInLds ? 2 : 1) * rows * (L + 1) <= kHhSmallLds ? L + 1 : L;
  HhMat<true> W{sw, LS};
  for (int64_t e = tid; e < rows * L; e += 1024) {
    const int64_t i = e / L;
    const int j = (int)(e % L);
    W.at(i, j) = j < ell ? X[(int64_t)j * ldx + i] : 0.0;
  }
  __syncthreads();
  hh_factor_s<1024, L>(W, rows, ell, tau, alpha, vhead, red);
  if (R) {
    for (int e = tid; e < ell * ell; e += 1024) {
      const int i = e % ell, j = e / ell;
      double v = i < j ? W.at(i, j) : (i == j ? alpha[i] : 0.0);
      if (alpha[i] < 0.0) v = -v;
      R[e] = v;
    }
  }
  auto run = [&](auto Qm) {
    for (int64_t e = tid; e < rows * L; e += 1024) {
      const int64_t i = e / L;
      const int j = (int)(e % L);
      if (j < ell) Qm.at(i, j) = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    hh_apply_s<1024, L>(W, rows, ell, tau, vhead, Qm, true, red);
    for (int64_t e = tid; e < rows * L; e += 1024) {
      const int64_t i = e / L;
      const int j = (int)(e % L);
      if (j >= ell) continue;
      double v = Qm.at(i, j);
      if (alpha[j] < 0.0) v = -v;
      Q[(int64_t)j * ldq + i] = v;
      if (Q32) Q32[(int64_t)j * ldq32 + i] = (float)v;
    }
  };
  if constexpr (QInLds)
    run(HhMat<true>{sw + rows * LS, LS});
  else
    run(HhMat<false>{Q, ldq});
}

// Tree level 1 for l <= 64: panel b (rows split evenly) reduced in LDS.
template <int L>
__global__ void __launch_bounds__(1024) hh_panel_s_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                         int ell, int P, double* __restrict__ W, int64_t ldw,
                                                         double* __restrict__ Rs, double* __restrict__ tv,
                                                         const int* status) {
  if ((*status & 3) != 1) return;
  constexpr int LS = L + 1;
  __shared__ double sw[kHhSmallLds];
  __shared__ double tau[L], alpha[L], vhead[L];
  __shared__ double red[2 * 16 * L];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int64_t r0 = (int64_t)b * rows / P, hb = (int64_t)(b + 1) * rows / P - r0;
  HhMat<true> Wm{sw, LS};
  for (int64_t e = tid; e < hb * L; e += 1024) {
    const int64_t i = e / L;
    const int j = (int)(e % L);
    Wm.at(i, j) = j < ell ? X[(int64_t)j * ldx + r0 + i] : 0.0;
  }
  __syncthreads();
  hh_factor_s<1024, L>(Wm, hb, ell, tau, alpha, vhead, red);
  const int64_t ldr = (int64_t)P * ell;
  for (int e = tid; e < ell * ell; e += 1024) {
    const int i = e % ell, j = e / ell;
    Rs[(int64_t)j * ldr + (int64_t)b * ell + i] = i < j ? Wm.at(i, j) : (i == j ? alpha[i] : 0.0);
  }
  for (int q = tid; q < ell; q += 1024) {
    tv[(int64_t)b * 2 * ell + q] = tau[q];
    tv[(int64_t)b * 2 * ell + ell + q] = vhead[q];
  }
  // the reflectors (and R's entries above them) to W, column-major
  for (int64_t e = tid; e < hb * ell; e += 1024) {
    const int64_t i = e % hb;
    const int j = (int)(e / hb);
    W[(int64_t)j * ldw + r0 + i] = Wm.at(i, j);
  }
}

// Tree level 2 for l <= 64: panel b of Q is its reflectors (staged in LDS)
// applied to [Qr rows b ell ... ; 0]; the panel of Q in LDS when both fit.
template <int L, bool QInLds>
__global__ void __launch_bounds__(1024) hh_expand_s_kernel(const double* __restrict__ W, int64_t ldw, int64_t rows,
                                                          int ell, int P, const double* __restrict__ Qr,
                                                          const double* __restrict__ tv, double* __restrict__ Q,
                                                          int64_t ldq, float* __restrict__ Q32, int64_t ldq32,
                                                          const int* status) {
  if ((*status & 3) != 1) return;
  constexpr int LS = L + 1;
  __shared__ double sw[kHhSmallLds];
  __shared__ double tau[L], vhead[L];
  __shared__ double red[2 * 16 * L];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int64_t r0 = (int64_t)b * rows / P, hb = (int64_t)(b + 1) * rows / P - r0;
  const int64_t ldr = (int64_t)P * ell;
  for (int q = tid; q < ell; q += 1024) {
    tau[q] = tv[(int64_t)b * 2 * ell + q];
    vhead[q] = tv[(int64_t)b * 2 * ell + ell + q];
  }
  HhMat<true> Wm{sw, LS};
  for (int64_t e = tid; e < hb * L; e += 1024) {
    const int64_t i = e / L;
    const int j = (int)(e % L);
    Wm.at(i, j) = j < ell ? W[(int64_t)j * ldw + r0 + i] : 0.0;
  }
  auto run = [&](auto Qm) {
    for (int64_t e = tid; e < hb * L; e += 1024) {
      const int64_t i = e / L;
      const int j = (int)(e % L);
      if (j < ell) Qm.at(i, j) = i < ell ? Qr[(int64_t)j * ldr + (int64_t)b * ell + i] : 0.0;
    }
    __syncthreads();
    hh_apply_s<1024, L>(Wm, hb, ell, tau, vhead, Qm, false, red);
    for (int64_t e = tid; e < hb * L; e += 1024) {
      const int64_t i = e / L;
      const int j = (int)(e % L);
      if (j >= ell) continue;
      const double v = Qm.at(i, j);
      if (QInLds) Q[(int64_t)j * ldq + r0 + i] = v;
      if (Q32) Q32[(int64_t)j * ldq32 + r0 + i] = (float)v;
    }
  };
  if constexpr (QInLds)
    run(HhMat<true>{sw + hb * LS, LS});
  else
    run(HhMat<false>{Q + r0, ldq});
}

// ---------------------------------------------------------------------------
// Householder QR with the working matrix in registers (l <= 64, panels of at
// most 1024 / M rows).  The columns are taken in M sets of 16 (M = 1, 2, 4),
// the rows in G = 4 NW row groups (NW waves, G >= 16 M):
// thread t serves columns c + 16 m (c = t % 16, m < M) of the rows
// i = r + G q (r = t / 16, q < R), holding W(i, c + 16 m) in w[m][q], so
// the 16 lanes of a row group (one DPP row) hold one row.  A step s needs
// column s at every thread of a row group: a DPP row broadcast (row_newbcast,
// an immediate lane, hence one code path per s % 16) from set s / 16.  Each
// step takes a single sum over the rows: p_j = x^T W(:, j) over rows >= s,
// x = column s, gives both ||x||^2 (j = s) and, with the pivot row W(s, :),
// the reflector products v^T W(:, j) = p_j - alpha W(s, j)
// (v = x - alpha e_s).  A sum over the rows adds each thread's partial sum
// (rows in increasing order, in four partial sums) over the four row groups
// of a wave by two v_permlane swaps, then the first wave adds the waves'
// sums in wave order and publishes the column totals (two barriers; every
// thread reading all the waves' sums would cost more LDS bandwidth than the
// second barrier).  Rows below s occur only among the first G (s < l <= G),
// and rows at or beyond the panel's height hold zeros, so only q = 0 takes a
// mask.  Fewer waves (a short panel or root) make the two barriers and the
// sum over the waves of each step cheaper.
template <int S>
__device__ __forceinline__ double hhr_bc16_one(double v) {
  // v_mov_b64_dpp row_newbcast:S
  return __longlong_as_double(__builtin_amdgcn_update_dpp(0LL, __double_as_longlong(v), 0x150 + S, 0xF, 0xF, false));
}

template <int S, int M, int R>
__device__ __forceinline__ void hhr_bcm(const double (&w)[M][R], double (&x)[R], int ms) {
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (m == ms) {  // uniform
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = hhr_bc16_one<S>(w[m][q]);
    }
}

// x[q] = the value of column s (uniform) in row q of the thread's row group
template <int M, int R>
__device__ __forceinline__ void hhr_col(const double (&w)[M][R], double (&x)[R], int s) {
  const int ms = s >> 4;
  switch (s & 15) {
    case 0: hhr_bcm<0, M, R>(w, x, ms); break;
    case 1: hhr_bcm<1, M, R>(w, x, ms); break;
    case 2: hhr_bcm<2, M, R>(w, x, ms); break;
    case 3: hhr_bcm<3, M, R>(w, x, ms); break;
    case 4: hhr_bcm<4, M, R>(w, x, ms); break;
    case 5: hhr_bcm<5, M, R>(w, x, ms); break;
    case 6: hhr_bcm<6, M, R>(w, x, ms); break;
    case 7: hhr_bcm<7, M, R>(w, x, ms); break;
    case 8: hhr_bcm<8, M, R>(w, x, ms); break;
    case 9: hhr_bcm<9, M, R>(w, x, ms); break;
    case 10: hhr_bcm<10, M, R>(w, x, ms); break;
    case 11: hhr_bcm<11, M, R>(w, x, ms); break;
    case 12: hhr_bcm<12, M, R>(w, x, ms); break;
    case 13: hhr_bcm<13, M, R>(w, x, ms); break;
    case 14: hhr_bcm<14, M, R>(w, x, ms); break;
    default: hhr_bcm<15, M, R>(w, x, ms); break;
  }
}

// The reflector's entry in the thread's row q: x, with v0 at row s and zero
// above it (only q = 0 can hold rows <= s)
template <int R>
__device__ __forceinline__ double hhr_v(const double (&x)[R], int q, int r, int s, double v0) {
  if (q > 0) return x[q];
  return r == s ? v0 : (r > s ? x[0] : 0.0);
}

// a + b with a, b the two halves that v_permlane16_swap (rows of 16 lanes)
// or v_permlane32_swap (halves of 32 lanes) hand out for the operand pair
// (v, v): every lane gets the same sum of its row and the paired row
template <bool k32>
__device__ __forceinline__ double hhr_swap_add(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  unsigned a0, a1, b0, b1;
  if constexpr (k32) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
  }
  const double x = __longlong_as_double(((long long)a1 << 32) | a0);
  const double y = __longlong_as_double(((long long)b1 << 32) | b0);
  return x + y;  // (even row or lower half) + (odd row or upper half)
}

// LDS of the register-resident kernels (L = 16 M columns)
template <int M>
struct HhrLds {
  double part[16 * 16 * M], tot[16 * M], prow[2 * 16 * M];
  double tau[16 * M], alpha[16 * M], vhead[16 * M];
};

// Column totals of the per-thread partial sums p[m] (column c + 16 m): the
// row groups of each wave, then (first wave) the 16 waves in order.  Barrier
// 1 publishes the waves' sums (and whatever the caller wrote before it),
// barrier 2 the totals in sh.tot.
template <int M, int NW>
__device__ __forceinline__ void hhr_totals(const double (&p)[M], HhrLds<M>& sh) {
  constexpr int L = 16 * M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double v = hhr_swap_add<true>(hhr_swap_add<false>(p[m]));
    if (lane < 16) sh.part[wave * L + 16 * m + lane] = v;
  }
  __syncthreads();
  if (wave == 0 && lane < L) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) a += sh.part[w * L + lane];
    sh.tot[lane] = a;
  }
  __syncthreads();
}

// Householder reduction of the nr x ell panel held in w (zeros outside it).
// Afterwards w holds R above the diagonal, the reflector tails below it and
// the original x_s on the diagonal; tau, alpha (R's diagonal) and vhead (the
// first entry of each reflector) go to LDS.  Ends with a barrier.
template <int M, int R, int NW>
__device__ void hhr_factor(double (&w)[M][R], int ell, HhrLds<M>& sh) {
  const int t = threadIdx.x, c = t & 15, r = t >> 4;
  for (int s = 0; s < ell; ++s) {
    double x[R];
    hhr_col<M, R>(w, x, s);
    double p[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double xv = (q == 0 && r < s) ? 0.0 : x[q];
        a[q & 3] = fma(xv, w[m][q], a[q & 3]);
      }
      p[m] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    double* prow = sh.prow + (s & 1) * 16 * M;
    if (r == s) {  // this row group holds the pivot row s (in q = 0)
#pragma unroll
      for (int m = 0; m < M; ++m) prow[c + 16 * m] = w[m][0];
    }
    hhr_totals<M, NW>(p, sh);
    const double ts = sh.tot[s], x0 = prow[s];
    const double nrm = sqrt(ts);
    double tv = 0.0, v0 = 0.0, a = 0.0;
    if (nrm != 0.0) {
      a = x0 >= 0.0 ? -nrm : nrm;
      v0 = x0 - a;
      tv = 2.0 / (ts - x0 * x0 + v0 * v0);
    }
    if (t == 0) {
      sh.tau[s] = tv;
      sh.alpha[s] = a;
      sh.vhead[s] = v0;
    }
    // columns at or left of s are left as they are: d = 0 there
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int j = c + 16 * m;
      const double d = (tv != 0.0 && j > s && j < ell) ? tv * (sh.tot[j] - a * prow[j]) : 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q) w[m][q] = fma(-d, hhr_v(x, q, r, s, v0), w[m][q]);
    }
  }
  __syncthreads();
}

// One reflector of hhr_apply for one set of 16 columns with the broadcast
// taken row by row instead of into a register array (R = 16: the apply
// holds two arrays already): MODE 0 returns the partial sum of v_i y_i,
// MODE 1 applies y_i -= d v_i.
template <int S, int R, int MODE>
__device__ __forceinline__ double hhr_refl_s(const double (&w)[R], double (&y)[R], int r, int s, double v0, double d) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double v = hhr_bc16_one<S>(w[q]);
    if (q == 0) v = r == s ? v0 : (r > s ? v : 0.0);
    if (MODE == 0) a[q & 3] = fma(v, y[q], a[q & 3]);
    else y[q] = fma(-d, v, y[q]);
  }
  return (a[0] + a[1]) + (a[2] + a[3]);
}

template <int R, int MODE>
__device__ __forceinline__ double hhr_refl(const double (&w)[R], double (&y)[R], int r, int s, double v0, double d) {
  switch (s & 15) {
#define CORUTV_RF(S) \
  case S:            \
    return hhr_refl_s<S, R, MODE>(w, y, r, s, v0, d);
    CORUTV_RF(0) CORUTV_RF(1) CORUTV_RF(2) CORUTV_RF(3) CORUTV_RF(4) CORUTV_RF(5) CORUTV_RF(6) CORUTV_RF(7)
    CORUTV_RF(8) CORUTV_RF(9) CORUTV_RF(10) CORUTV_RF(11) CORUTV_RF(12) CORUTV_RF(13) CORUTV_RF(14)
#undef CORUTV_RF
    default:
      return hhr_refl_s<15, R, MODE>(w, y, r, s, v0, d);
  }
}

// qv <- H_0 ... H_{ell-1} qv with the reflectors of hhr_factor (w and the
// tau, vhead in sh).
template <int M, int R, int NW>
__device__ void hhr_apply(const double (&w)[M][R], double (&qv)[M][R], int ell, HhrLds<M>& sh) {
  const int t = threadIdx.x, c = t & 15, r = t >> 4;
  for (int s = ell - 1; s >= 0; --s) {
    const double tv = sh.tau[s];
    if (tv == 0.0) continue;  // uniform
    const double v0 = sh.vhead[s];
    if constexpr (R == 16) {  // one set of columns (M R <= 16)
      static_assert(M == 1, "16 rows per thread with one set of columns only");
      double p[1] = {hhr_refl<R, 0>(w[0], qv[0], r, s, v0, 0.0)};
      hhr_totals<M, NW>(p, sh);
      const double d = c < ell ? tv * sh.tot[c] : 0.0;
      hhr_refl<R, 1>(w[0], qv[0], r, s, v0, d);
      continue;
    }
    double x[R];
    hhr_col<M, R>(w, x, s);
    double p[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < R; ++q) a[q & 3] = fma(hhr_v(x, q, r, s, v0), qv[m][q], a[q & 3]);
      p[m] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    hhr_totals<M, NW>(p, sh);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const double d = c + 16 * m < ell ? tv * sh.tot[c + 16 * m] : 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q) qv[m][q] = fma(-d, hhr_v(x, q, r, s, v0), qv[m][q]);
    }
  }
}

// w[m][q] = X(r0 + i, c + 16 m) for own rows i < nr and columns < ell, else
// 0.  Every load is unconditional, from a clamped address, and masked
// afterwards: loads under per-lane branches are waited for one by one.
template <int M, int R, int NW>
__device__ __forceinline__ void hhr_load(double (&w)[M][R], const double* __restrict__ X, int64_t ldx, int64_t r0,
                                         int nr, int ell) {
  constexpr int G = 4 * NW;  // row groups
  const int c = threadIdx.x & 15, r = threadIdx.x >> 4;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = r + G * q, j = c + 16 * m;
      const int ic = i < nr ? i : nr - 1, jc = j < ell ? j : ell - 1;
      w[m][q] = X[(int64_t)jc * ldx + r0 + ic];
    }
  // every load issued first; each value made opaque before its mask (a
  // select between a loaded value and a constant is otherwise turned into a
  // branch around the load, which then waits for each load in turn)
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = r + G * q, j = c + 16 * m;
      double v = w[m][q];
      asm volatile("" : "+v"(v));
      w[m][q] = (i < nr && j < ell) ? v : 0.0;
    }
}

// The kernels of a QR run after a Cholesky breakdown on finite data.
__device__ __forceinline__ bool hhr_runs(const int* status) { return (*status & 3) == 1; }

// One workgroup: X (rows x ell, column-major) -> Q (diag R >= 0, FP64 and
// optionally a float copy), R (nullable, ell x ell column-major).
template <int M, int R, int NW>
__device__ __forceinline__ void hhr_one_body(HhrLds<M>& sh, const double* __restrict__ X, int64_t ldx,
                                             int64_t rows, int ell, double* __restrict__ Q, int64_t ldq,
                                             float* __restrict__ Q32, int64_t ldq32, double* __restrict__ Rout) {
  const int t = threadIdx.x, c = t & 15, r = t >> 4;
  double w[M][R];
  hhr_load<M, R, NW>(w, X, ldx, 0, (int)rows, ell);
  hhr_factor<M, R, NW>(w, ell, sh);
  if (Rout && r < ell) {  // rows i < ell are the first 4 NW (q = 0)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int j = c + 16 * m;
      if (j < ell) {
        double v = r < j ? w[m][0] : (r == j ? sh.alpha[r] : 0.0);
        if (sh.alpha[r] < 0.0) v = -v;
        Rout[(int64_t)j * ell + r] = v;
      }
    }
  }
  double qv[M][R];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int q = 0; q < R; ++q) qv[m][q] = (q == 0 && r == c + 16 * m && r < ell) ? 1.0 : 0.0;
  hhr_apply<M, R, NW>(w, qv, ell, sh);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = c + 16 * m;
    if (j >= ell) continue;
    const bool flip = sh.alpha[j] < 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = r + 4 * NW * q;
      if (i < rows) {
        const double v = flip ? -qv[m][q] : qv[m][q];
        Q[(int64_t)j * ldq + i] = v;
        if (Q32) Q32[(int64_t)j * ldq32 + i] = (float)v;
      }
    }
  }
}

template <int M, int R, int NW>
__global__ void __launch_bounds__(64 * NW) hhr_one_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                       int ell, double* __restrict__ Q, int64_t ldq,
                                                       float* __restrict__ Q32, int64_t ldq32,
                                                       double* __restrict__ Rout, const int* status) {
  if (!hhr_runs(status)) return;
  __shared__ HhrLds<M> sh;
  hhr_one_body<M, R, NW>(sh, X, ldx, rows, ell, Q, ldq, Q32, ldq32, Rout);
}

// Tree level 1: panel b (rows split evenly over P panels) reduced; its
// reflectors (and R's entries above them) to W, its triangle to rows
// b ell .. of Rs (ld P ell), tau and vhead to tv.
template <int M, int R, int NW>
__device__ __forceinline__ void hhr_panel_body(HhrLds<M>& sh, const double* __restrict__ X, int64_t ldx,
                                               int64_t rows, int ell, int P, int b, double* __restrict__ W,
                                               int64_t ldw, double* __restrict__ Rs, double* __restrict__ tv) {
  const int t = threadIdx.x, c = t & 15, r = t >> 4;
  const int64_t r0 = (int64_t)b * rows / P, hb = (int64_t)(b + 1) * rows / P - r0;
  double w[M][R];
  hhr_load<M, R, NW>(w, X, ldx, r0, (int)hb, ell);
  hhr_factor<M, R, NW>(w, ell, sh);
  const int64_t ldr = (int64_t)P * ell;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = c + 16 * m;
    if (j >= ell) continue;
    if (r < ell) Rs[(int64_t)j * ldr + (int64_t)b * ell + r] = r < j ? w[m][0] : (r == j ? sh.alpha[r] : 0.0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = r + 4 * NW * q;
      if (i < hb) W[(int64_t)j * ldw + r0 + i] = w[m][q];
    }
  }
  if (t < ell) {
    tv[(int64_t)b * 2 * ell + t] = sh.tau[t];
    tv[(int64_t)b * 2 * ell + ell + t] = sh.vhead[t];
  }
}

template <int M, int R, int NW>
__global__ void __launch_bounds__(64 * NW) hhr_panel_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                         int ell, int P, double* __restrict__ W, int64_t ldw,
                                                         double* __restrict__ Rs, double* __restrict__ tv,
                                                         const int* status) {
  if (!hhr_runs(status)) return;
  __shared__ HhrLds<M> sh;
  hhr_panel_body<M, R, NW>(sh, X, ldx, rows, ell, P, blockIdx.x, W, ldw, Rs, tv);
}

// Tree level 2: panel b of Q = its reflectors applied to [Qr rows b ell ..; 0].
template <int M, int R, int NW>
__device__ __forceinline__ void hhr_expand_body(HhrLds<M>& sh, const double* __restrict__ W, int64_t ldw,
                                                int64_t rows, int ell, int P, int b,
                                                const double* __restrict__ Qr, const double* __restrict__ tv,
                                                double* __restrict__ Q, int64_t ldq, float* __restrict__ Q32,
                                                int64_t ldq32) {
  const int t = threadIdx.x, c = t & 15, r = t >> 4;
  const int64_t r0 = (int64_t)b * rows / P, hb = (int64_t)(b + 1) * rows / P - r0;
  const int64_t ldr = (int64_t)P * ell;
  if (t < ell) {
    sh.tau[t] = tv[(int64_t)b * 2 * ell + t];
    sh.vhead[t] = tv[(int64_t)b * 2 * ell + ell + t];
  }
  double w[M][R], qv[M][R];
  hhr_load<M, R, NW>(w, W, ldw, r0, (int)hb, ell);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = c + 16 * m;
    const int jc = j < ell ? j : ell - 1, rc = r < ell ? r : ell - 1;
    const double v = Qr[(int64_t)jc * ldr + (int64_t)b * ell + rc];  // unconditional, as in hhr_load
#pragma unroll
    for (int q = 0; q < R; ++q) qv[m][q] = (q == 0 && r < ell && j < ell) ? v : 0.0;
  }
  __syncthreads();
  hhr_apply<M, R, NW>(w, qv, ell, sh);
  // the output addresses are formed here, not kept in registers across the
  // loop above (the empty asm hides where the bases come from)
  double* Qo = Q + r0;
  float* Q32o = Q32 ? Q32 + r0 : nullptr;
  asm volatile("" : "+s"(Qo), "+s"(Q32o));
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = c + 16 * m;
    if (j >= ell) continue;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = r + 4 * NW * q;
      if (i < hb) {
        Qo[(int64_t)j * ldq + i] = qv[m][q];
        if (Q32o) Q32o[(int64_t)j * ldq32 + i] = (float)qv[m][q];
      }
    }
  }
}

template <int M, int R, int NW>
__global__ void __launch_bounds__(64 * NW) hhr_expand_kernel(const double* __restrict__ W, int64_t ldw, int64_t rows,
                                                          int ell, int P, const double* __restrict__ Qr,
                                                          const double* __restrict__ tv, double* __restrict__ Q,
                                                          int64_t ldq, float* __restrict__ Q32, int64_t ldq32,
                                                          const int* status) {
  if (!hhr_runs(status)) return;
  __shared__ HhrLds<M> sh;
  hhr_expand_body<M, R, NW>(sh, W, ldw, rows, ell, P, blockIdx.x, Qr, tv, Q, ldq, Q32, ldq32);
}

// ---------------------------------------------------------------------------
// A chain of up to three triangle copies in one launch: stage k copies stage
// k - 1's result (stage 0 copies src) as copy_tri_kernel would; every entry
// of every stage is traced back to src through the stages' transposes and
// masks.
struct TriChain {
  double* dst[3];
  int64_t ld[3];
  int trans[3], upper[3];
  int n;
};

__global__ void copy_tri_chain_kernel(const double* __restrict__ src, int ell, TriChain c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ell * ell) return;
  const int i0 = e % ell, j0 = e / ell;
  for (int k = 0; k < c.n; ++k) {
    int i = i0, j = j0;
    bool zero = false;
    for (int t = k; t >= 0; --t) {
      if (c.upper[t] ? (i > j) : (i < j)) zero = true;
      if (c.trans[t]) {
        const int x = i;
        i = j;
        j = x;
      }
    }
    c.dst[k][(int64_t)j0 * c.ld[k] + i0] = zero ? 0.0 : src[(int64_t)j * ell + i];
  }
}

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

// y[c * ld + i] += x[c * ld + i] for i < rows, c < cols
__global__ void add_cols_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t rows, int cols,
                                int64_t ld) {
  const int c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    y[(int64_t)c * ld + i] += x[(int64_t)c * ld + i];
}

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Zero up to kZeroRanges device ranges (16-byte aligned, whole 16-byte
// words) in one launch.
__global__ void __launch_bounds__(256) zero_ranges_kernel(ZeroRanges z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < z.count; ++r) {
    uint4* p = (uint4*)z.ptr[r];
    const int64_t n = z.words[r];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      p[i] = uint4{0u, 0u, 0u, 0u};
  }
}

// R = R2 R1 for two upper triangular l x l factors (column-major, ld l):
// the R factor of CholeskyQR2 (X = Q' R1, Q' = Q R2); R = R1 when the QR
// stopped after one step (status 4).  After a breakdown the Householder
// fallback writes R itself.
__global__ void __launch_bounds__(256) trprod_kernel(const double* __restrict__ R2,
                                                     const double* __restrict__ R1, int ell,
                                                     double* __restrict__ R, const int* status) {
  const int sw = *status & 7;
  if (sw != 0 && sw != 4) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ell * ell) return;
  const int i = e % ell, j = e / ell;
  if (sw == 4) {  // one CholeskyQR step: R = R1
    R[e] = R1[e];
    return;
  }
  double v = 0.0;
  for (int t = i; t <= j; ++t) v = fma(R2[(int64_t)t * ell + i], R1[(int64_t)j * ell + t], v);
  R[e] = i <= j ? v : 0.0;
}

}  // namespace

hipError_t launch_add_cols(double* y, const double* x, int64_t rows, int cols, int64_t ld, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  const int64_t bx = std::min<int64_t>((rows + 255) / 256, 64);
  add_cols_kernel<<<dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, st>>>(y, x, rows, cols, ld);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholeskyQR2 for at most 16 columns with the Householder fallback in the
// same launches: after a breakdown (status bit 1 alone) the launch that
// would have run the next CholeskyQR step runs the register-resident
// Householder QR of X instead, so no launch is spent on a fallback that is
// not needed.
//   one workgroup (rows <= 1024): q16h_one_kernel<HR> factors X by
//     Householder right after the failed Cholesky (HR rows per thread);
//   tall (rows in nblk blocks of at most 1024, nblk l <= 1024): step 1
//     factors each block as a panel of the two-level tree, the root (the
//     stacked triangles) is reduced by hhr_one_kernel in a launch of its own
//     between the steps (in the same launch, its registers would spill
//     those of the others), and step 2 expands each panel's Q.
namespace {

struct Q16Hh {
  double* W;    // panel reflectors (rows x l, ld ldw)
  int64_t ldw;
  double* Rs;   // stacked triangles (nblk l x l)
  double* Qr;   // the root's Q
  double* tv;   // per panel: tau[l], vhead[l]
};

template <int HR>
__global__ void __launch_bounds__(1024) q16h_one_kernel(Q16Args a) {
  __shared__ Q16Lds sh;
  __shared__ HhrLds<1> hs;
  if (q16_one_body(a, sh) == 1)
    hhr_one_body<1, HR, 16>(hs, a.x0, a.ld, a.rows, a.ell, a.q64, a.ld, a.q32, a.ld, a.rfac);
}

template <int STEP>
__global__ void __launch_bounds__(1024) q16h_kernel(Q16Args a, Q16Hh h) {
  __shared__ Q16Lds sh;
  __shared__ HhrLds<1> hs;
  const int sw = *a.status;
  if ((sw & 3) != 1) {
    q16_body<STEP>(a, sh, sw);
    return;
  }
  if (STEP == 1)
    hhr_panel_body<1, 16, 16>(hs, a.x0, a.ld, a.rows, a.ell, a.nblk, blockIdx.x, h.W, h.ldw, h.Rs, h.tv);
  else
    hhr_expand_body<1, 16, 16>(hs, h.W, h.ldw, a.rows, a.ell, a.nblk, blockIdx.x, h.Qr, h.tv, a.q64, a.ld, a.q32,
                           a.ld);
}

}  // namespace

int qr16_blocks(int64_t rows) {
  const int64_t b = (rows + kQ16Rows - 1) / kQ16Rows;
  return (int)std::max<int64_t>(1, std::min<int64_t>(kQ16MaxBlocks, b));
}

size_t qr16_work_bytes() { return ((size_t)kQ16MaxBlocks * 256 + 4 * 256) * 8 + 256; }

static int hhr_rows_per_thread(int M, int64_t nr);

hipError_t launch_qr16(const double* X, int64_t ld, int64_t rows, int ell, double* Q, float* Q32, double* R,
                       int* status, double* work, double single_thr, hipStream_t st, double* W, int64_t ldw,
                       double* hw, bool* covered) {
  if (covered) *covered = false;
  if (ell < 1 || ell > 16 || rows < ell) return hipErrorInvalidValue;
  Q16Args a;
  a.x0 = X;
  a.ld = ld;
  a.rows = rows;
  a.ell = ell;
  a.nblk = qr16_blocks(rows);
  a.gpart = work;
  a.tiles = work + (size_t)kQ16MaxBlocks * 256;
  a.counter = (int*)(a.tiles + 4 * 256);
  a.rfac = R;
  a.q64 = Q;
  a.q32 = Q32;
  a.status = status;
  a.single_thr = single_thr;
  if (rows <= kQ16Rows) {
    if (covered) {
      const int hr = hhr_rows_per_thread(1, rows);
      if (hr == 4) q16h_one_kernel<4><<<dim3(1), dim3(1024), 0, st>>>(a);
      else if (hr == 8) q16h_one_kernel<8><<<dim3(1), dim3(1024), 0, st>>>(a);
      else q16h_one_kernel<16><<<dim3(1), dim3(1024), 0, st>>>(a);
      *covered = true;
    } else {
      q16_one_kernel<<<dim3(1), dim3(1024), 0, st>>>(a);
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)a.nblk);
  // the merged fallback: blocks of at most 1024 rows (the panels), their
  // stacked triangles at most 1024 rows (the root)
  const int64_t pe = (int64_t)a.nblk * ell;
  const int hr = hhr_rows_per_thread(1, pe);
  if (covered && W && hw && (rows + a.nblk - 1) / a.nblk <= kQ16Rows && pe <= kQ16Rows && hr > 0) {
    Q16Hh h;
    h.W = W;
    h.ldw = ldw;
    h.Rs = hw;  // the same layout as the separate tree's
    h.Qr = hw + 2 * pe * ell;
    h.tv = h.Qr + pe * ell;
    q16_kernel<0><<<grid, dim3(1024), 0, st>>>(a);
    q16h_kernel<1><<<grid, dim3(1024), 0, st>>>(a, h);
    if (hr == 4)
      hhr_one_kernel<1, 4, 16><<<dim3(1), dim3(1024), 0, st>>>(h.Rs, pe, pe, ell, h.Qr, pe, nullptr, 0, R, status);
    else if (hr == 8)
      hhr_one_kernel<1, 8, 16><<<dim3(1), dim3(1024), 0, st>>>(h.Rs, pe, pe, ell, h.Qr, pe, nullptr, 0, R, status);
    else
      hhr_one_kernel<1, 16, 16><<<dim3(1), dim3(1024), 0, st>>>(h.Rs, pe, pe, ell, h.Qr, pe, nullptr, 0, R, status);
    q16h_kernel<2><<<grid, dim3(1024), 0, st>>>(a, h);
    *covered = true;
    return hipGetLastError();
  }
  q16_kernel<0><<<grid, dim3(1024), 0, st>>>(a);
  q16_kernel<1><<<grid, dim3(1024), 0, st>>>(a);
  q16_kernel<2><<<grid, dim3(1024), 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_trprod(const double* R2, const double* R1, int ell, double* R, const int* status,
                         hipStream_t st) {
  trprod_kernel<<<dim3((ell * ell + 255) / 256), dim3(256), 0, st>>>(R2, R1, ell, R, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_sum_partials(const Partials& p, int ell, int ncols, double* out64, float* out32,
                               int64_t ld, hipStream_t st) {
  if (p.direct || p.n == 0 || ncols == 0) return hipSuccess;
  // every segment list must fit: at most 8 * (gx + 1) entries per tile
  if (p.nchunk < 1 || (int64_t)p.nchunk * (p.gx + 1) > kSegMax) return hipErrorInvalidValue;
  // about nchunk (gx / tiles + 1) slots feed a tile; give each thread at least 8
  const int64_t slots = p.nchunk * ((int64_t)p.gx / p.tiles + 1);
  int tpe = 1;
  while (tpe < 16 && slots / (2 * tpe) >= 8) tpe *= 2;
  // a block covers reps x 256 / tpe entries (16 columns when one thread sums
  // each entry and the output has tiles enough to fill the device: the slot
  // list is built once per block; a short output takes one block per 256
  // entries instead, so its slot sums spread over more CUs)
  const int epb = 256 / tpe;
  const int64_t blocks1 = (int64_t)p.tiles * (((int64_t)ncols * p.tw + epb - 1) / epb);
  const int reps = (tpe == 1 && blocks1 >= 1024) ? 16 * p.tw / 256 : 1;
  dim3 grid((unsigned)p.tiles, (unsigned)(((int64_t)ncols * p.tw + epb * reps - 1) / (epb * reps)));
  if (p.elem == 8)
    sum_partials_kernel<double><<<grid, dim3(256), 0, st>>>(p, (const double*)p.ptr, ell, ncols, out64,
                                                            out32, ld, tpe, reps);
  else
    sum_partials_kernel<float><<<grid, dim3(256), 0, st>>>(p, (const float*)p.ptr, ell, ncols, out64,
                                                           out32, ld, tpe, reps);
  return hipGetLastError();
}

int xty_splits(int64_t rows, int ell) {
  // about 512 workgroups for a Gram matrix, at least 64 rows per split
  int s = 512 / xty_regions(ell, 1);
  const int64_t maxs = (rows + 63) / 64;
  if (s > maxs) s = (int)maxs;
  return s < 1 ? 1 : s;
}

hipError_t launch_xty(const double* Xa, int64_t lda, const double* Xb, int64_t ldb, int64_t rows,
                      int ell, double* part, int splits, const int* skip, hipStream_t st) {
  const int sym = (Xa == Xb && lda == ldb) ? 1 : 0;
  xty_kernel<<<dim3(xty_regions(ell, sym) * splits), dim3(256), 0, st>>>(Xa, lda, Xb, ldb, rows, ell, part,
                                                                         splits, sym, skip);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int splits, int64_t elems, double* out, const int* skip,
                         hipStream_t st) {
  reduce_kernel<<<dim3((unsigned)((elems + 63) / 64)), dim3(1024), 0, st>>>(part, splits, elems, out, skip);
  return hipGetLastError();
}

hipError_t launch_rowmat(const double* X, int64_t ldx, int64_t rows, int ell, const double* B,
                         int64_t ldb, const int32_t* perm, MatOut o1, int pad1, MatOut o2, int pad2,
                         const int* skip, hipStream_t st, bool b_upper, int run_val, MatOut oa, int pada,
                         int alt_val) {
  if (rows == 0) return hipSuccess;
  const int ellp = pad_ell(ell);
  if (oa.ptr && (perm || !skip || alt_val == run_val)) return hipErrorInvalidValue;
  if (!oa.ptr) alt_val = -1;
  if (perm) {
    const dim3 grid((unsigned)((rows + 255) / 256), (unsigned)ellp);
    gather_cols_kernel<<<grid, dim3(256), 0, st>>>(X, ldx, rows, ell, perm, o1, pad1, o2, pad2, skip,
                                                   run_val);
  } else if (ell <= 16) {
    rowmat16_kernel<<<dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st>>>(
        X, ldx, rows, ell, B, ldb, o1, pad1, o2, pad2, b_upper ? 1 : 0, skip, run_val, oa, pada, alt_val);
  } else {
    const dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((ellp + 127) / 128));
    rowmat_mfma_kernel<<<grid, dim3(256), 0, st>>>(X, ldx, rows, ell, B, ldb, o1, pad1, o2, pad2,
                                                   b_upper ? 1 : 0, skip, run_val, oa, pada, alt_val);
  }
  return hipGetLastError();
}

size_t chol_work_bytes(int ell) {
  const int nb = (ell + 15) / 16;
  return nb <= kCholLdsNb ? 0 : (size_t)nb * (nb + 1) * 256 * sizeof(double);
}

hipError_t launch_chol(const double* G, int ell, double* R, double* Rinv, int* status,
                       const int* skip, double* work, hipStream_t st, double single_thr) {
  if ((ell + 15) / 16 <= kCholLdsNb)
    chol_kernel<true><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip, nullptr, single_thr);
  else
    chol_kernel<false><<<dim3(1), dim3(1024), 0, st>>>(G, ell, R, Rinv, status, skip, work, single_thr);
  return hipGetLastError();
}

// Panel height of the Householder tree when panels do not fit LDS: about
// sqrt(rows ell), so a panel and the stacked triangles (P ell rows) are of
// similar height; at least four triangles' worth of rows and at least 256.
static int64_t hh_panel_rows(int64_t rows, int ell) {
  const int64_t bal = (int64_t)std::sqrt((double)rows * ell);
  return std::max<int64_t>(std::max<int64_t>(256, 4 * (int64_t)ell), bal);
}

struct HhTree {
  int P = 1;       // panels (1: one workgroup does the whole QR)
  int64_t h = 0;   // panel height (device-memory panels)
  int lds = 0;     // panels in LDS, rows split evenly
};

// LDS panels when a panel of at least 2 ell rows fits and the stacked
// triangles stay at most 4096 rows; else the device-memory tree.
static HhTree hh_tree(int64_t rows, int ell) {
  HhTree t;
  const int64_t hl = kHhLds / ell;
  if (hl >= 2 * (int64_t)ell && hl >= 64) {
    const int64_t P = (rows + hl - 1) / hl;
    if (P < 2) return t;
    if (P * ell <= 4096) {
      t.P = (int)P;
      t.lds = 1;
      return t;
    }
  }
  const int64_t h = hh_panel_rows(rows, ell);
  const int64_t P = rows / h;
  if (P >= 2) {
    t.P = (int)P;
    t.h = h;
  }
  return t;
}

int hh_panels(int64_t rows, int ell) { return hh_tree(rows, ell).P; }

// The register-resident kernels: M sets of 16 columns (1, 2 or 4) and R rows
// per thread (4, 8, 16 with M R <= 16) for a panel of nr rows; 0 when they
// do not apply.
static int hhr_sets(int ell) { return ell <= 16 ? 1 : (ell <= 32 ? 2 : (ell <= 64 ? 4 : 0)); }
static int hhr_rows_per_thread(int M, int64_t nr) {
  const int64_t q = (nr + 63) / 64;
  const int r = q <= 4 ? 4 : (q <= 8 ? 8 : (q <= 16 ? 16 : 0));
  return M * r <= 16 ? r : 0;
}
struct HhrShape {
  int R = 0, NW = 0;
};
static HhrShape hhr_shape(int M, int64_t nr);

// Panels of the register-resident tree: 1 (one workgroup), P >= 2, or 0
// when rows is too large for two levels.  Within panel rows <= 1024 / M,
// stacked triangles P ell <= 1024 / M and panel rows >= ell, the P whose
// launches (panels and expansion with the panel's shape, the root with its
// own) need the fewest waves plus rows per thread in all (a step's cost
// grows with both), the smallest such P.
static int hhr_panels(int64_t rows, int ell) {
  const int M = hhr_sets(ell);
  if (M == 0) return 0;
  const int64_t cap = 1024 / M;
  if (rows <= cap) return 1;
  const int64_t pmin = (rows + cap - 1) / cap, pmax = std::min<int64_t>(cap / ell, rows / ell);
  if (pmin > pmax) return 0;
  int64_t best = pmin;
  int best_cost = 1 << 30;
  for (int64_t P = pmin; P <= pmax; ++P) {
    const HhrShape a = hhr_shape(M, (rows + P - 1) / P), b = hhr_shape(M, P * ell);
    const int cost = 2 * (a.NW + a.R) + b.NW + b.R;
    if (cost < best_cost) {
      best_cost = cost;
      best = P;
    }
  }
  return (int)best;
}

size_t hh_work_bytes(int64_t rows, int ell) {
  const int P = std::max(hh_panels(rows, ell), hhr_panels(rows, ell));
  if (P < 2) return 0;
  const size_t pe = (size_t)P * ell;
  return (3 * pe * ell + 2 * pe) * 8;
}

// Householder QR by the register-resident kernels (one workgroup, or the
// two-level tree); false when they do not apply.
// Rows per thread and waves of one register-resident launch over nr rows:
// the fewest waves (at least 4 M, so that the first row groups hold every
// row above the diagonal) that hold the rows with at most 16 / M rows per
// thread, then the fewest rows per thread.
static HhrShape hhr_shape(int M, int64_t nr) {
  HhrShape sh;
  for (const int nw : {4, 8, 16}) {
    if (4 * nw < 16 * M) continue;
    for (const int r : {4, 8, 16}) {
      if (M * r > 16) break;
      if ((int64_t)4 * nw * r >= nr) {
        sh.R = r;
        sh.NW = nw;
        return sh;
      }
    }
  }
  return sh;
}

// the launch shapes hhr_shape picks
#define CORUTV_HHR_SHAPES(X) X(1, 4, 4) X(1, 8, 4) X(1, 16, 4) X(1, 16, 8) X(1, 16, 16) X(2, 4, 8) X(2, 8, 8) \
  X(2, 8, 16) X(4, 4, 16)

static bool launch_hhr(const double* X, int64_t ldx, int64_t rows, int ell, double* work, int64_t ldw, double* Q,
                       int64_t ldq, float* Q32, int64_t ldq32, double* R, const int* status, double* hw,
                       hipStream_t st) {
  const int P = hhr_panels(rows, ell);
  const int M = hhr_sets(ell);
  if (P == 0) return false;
  auto one = [&](const double* x, int64_t ldxx, int64_t nr, double* q, int64_t ldqq, float* q32, int64_t ldq32x,
                 double* rr) {
    const HhrShape h = hhr_shape(M, nr);
#define CORUTV_HHR_ONE(MM, RR, NWW)                                                                            \
  if (M == MM && h.R == RR && h.NW == NWW)                                                                     \
    hhr_one_kernel<MM, RR, NWW><<<dim3(1), dim3(64 * NWW), 0, st>>>(x, ldxx, nr, ell, q, ldqq, q32, ldq32x, rr, \
                                                                    status);
    CORUTV_HHR_SHAPES(CORUTV_HHR_ONE)
#undef CORUTV_HHR_ONE
  };
  if (P == 1) {
    one(X, ldx, rows, Q, ldq, Q32, ldq32, R);
    return true;
  }
  if (!hw) return false;
  const int64_t pe = (int64_t)P * ell;
  double* Rs = hw;                  // stacked triangles, pe x ell
  double* Qr = Rs + 2 * pe * ell;   // the root's Q
  double* tv = Qr + pe * ell;       // per panel: tau[ell], vhead[ell]
  const HhrShape h = hhr_shape(M, (rows + P - 1) / P);
#define CORUTV_HHR_PANEL(MM, RR, NWW)                                                                            \
  if (M == MM && h.R == RR && h.NW == NWW)                                                                       \
    hhr_panel_kernel<MM, RR, NWW><<<dim3(P), dim3(64 * NWW), 0, st>>>(X, ldx, rows, ell, P, work, ldw, Rs, tv, \
                                                                      status);
#define CORUTV_HHR_EXPAND(MM, RR, NWW)                                                                           \
  if (M == MM && h.R == RR && h.NW == NWW)                                                                       \
    hhr_expand_kernel<MM, RR, NWW><<<dim3(P), dim3(64 * NWW), 0, st>>>(work, ldw, rows, ell, P, Qr, tv, Q, ldq, \
                                                                       Q32, ldq32, status);
  CORUTV_HHR_SHAPES(CORUTV_HHR_PANEL)
  one(Rs, pe, pe, Qr, pe, nullptr, 0, R);
  CORUTV_HHR_SHAPES(CORUTV_HHR_EXPAND)
#undef CORUTV_HHR_PANEL
#undef CORUTV_HHR_EXPAND
  return true;
}
#undef CORUTV_HHR_SHAPES

hipError_t launch_householder_qr(const double* X, int64_t ldx, int64_t rows, int ell, double* work,
                                 int64_t ldw, double* Q, int64_t ldq, float* Q32, int64_t ldq32,
                                 double* R, const int* status, double* hw, hipStream_t st) {
  if (launch_hhr(X, ldx, rows, ell, work, ldw, Q, ldq, Q32, ldq32, R, status, hw, st)) return hipGetLastError();
  const HhTree tr = hh_tree(rows, ell);
  const int P = tr.P;
  // l <= 64: the kernels that work on all columns at once, where their LDS
  // copies fit
  const int L = ell <= 16 ? 16 : (ell <= 32 ? 32 : (ell <= 64 ? 64 : 0));
  auto fits = [&](int64_t r, int copies) { return L > 0 && copies * r * L <= kHhSmallLds; };
  auto fits_padded = [&](int64_t r, int copies) { return L > 0 && copies * r * (L + 1) <= kHhSmallLds; };
  auto one_wg = [&](const double* x, int64_t ldxx, int64_t r, double* q, int64_t ldqq, float* q32, int64_t ldq32x,
                    double* wk, int64_t ldwk) {
    // (with Q in device memory the older kernel is the faster one)
    if (!fits(r, 2)) {
      householder_kernel<<<dim3(1), dim3(1024), 0, st>>>(x, ldxx, r, ell, wk, ldwk, q, ldqq, q32, ldq32x, R,
                                                         status);
      return;
    }
    const bool ql = true;
#define CORUTV_HH_ONE(LL)                                                                                  \
  if (L == LL) {                                                                                             \
    if (ql)                                                                                                  \
      householder_s_kernel<LL, true><<<dim3(1), dim3(1024), 0, st>>>(x, ldxx, r, ell, q, ldqq, q32, ldq32x, R, \
                                                                    status);                                \
    else                                                                                                     \
      householder_s_kernel<LL, false><<<dim3(1), dim3(1024), 0, st>>>(x, ldxx, r, ell, q, ldqq, q32, ldq32x, R,\
                                                                     status);                               \
  }
    CORUTV_HH_ONE(16)
    CORUTV_HH_ONE(32)
    CORUTV_HH_ONE(64)
#undef CORUTV_HH_ONE
  };
  if (P < 2) {
    one_wg(X, ldx, rows, Q, ldq, Q32, ldq32, work, ldw);
    return hipGetLastError();
  }
  if (!hw) return hipErrorInvalidValue;
  const int64_t pe = (int64_t)P * ell;
  double* Rs = hw;             // stacked triangles, pe x ell
  double* Rw = Rs + pe * ell;  // the root's working copy
  double* Qr = Rw + pe * ell;  // the root's Q
  double* tv = Qr + pe * ell;  // per panel: tau[ell], vhead[ell]
  const int64_t hb = (rows + P - 1) / P;  // rows of the largest LDS panel
  if (tr.lds && fits_padded(hb, 1)) {
    const bool ql = fits_padded(hb, 2);
#define CORUTV_HH_TREE(LL)                                                                                      \
  if (L == LL) {                                                                                                  \
    hh_panel_s_kernel<LL><<<dim3(P), dim3(1024), 0, st>>>(X, ldx, rows, ell, P, work, ldw, Rs, tv, status);        \
    one_wg(Rs, pe, pe, Qr, pe, nullptr, 0, Rw, pe);                                                               \
    if (ql)                                                                                                       \
      hh_expand_s_kernel<LL, true><<<dim3(P), dim3(1024), 0, st>>>(work, ldw, rows, ell, P, Qr, tv, Q, ldq, Q32,   \
                                                                 ldq32, status);                                 \
    else                                                                                                          \
      hh_expand_kernel<<<dim3(P), dim3(256), 0, st>>>(work, ldw, rows, ell, tr.h, P, tr.lds, Qr, tv, Q, ldq, Q32,  \
                                                      ldq32, status);                                            \
  }
    CORUTV_HH_TREE(16)
    CORUTV_HH_TREE(32)
    CORUTV_HH_TREE(64)
#undef CORUTV_HH_TREE
    return hipGetLastError();
  }
  hh_panel_kernel<<<dim3(P), dim3(256), 0, st>>>(X, ldx, rows, ell, tr.h, P, tr.lds, work, ldw, Rs, tv,
                                                 status);
  householder_kernel<<<dim3(1), dim3(1024), 0, st>>>(Rs, pe, pe, ell, Rw, pe, Qr, pe, nullptr, 0, R,
                                                     status);
  hh_expand_kernel<<<dim3(P), dim3(256), 0, st>>>(work, ldw, rows, ell, tr.h, P, tr.lds, Qr, tv, Q, ldq,
                                                  Q32, ldq32, status);
  return hipGetLastError();
}

hipError_t launch_copy_tri(const double* src, int ell, int trans, int upper, double* dst, int64_t ldd,
                           hipStream_t st) {
  const int n = ell * ell;
  copy_tri_kernel<<<dim3((n + 255) / 256), dim3(256), 0, st>>>(src, ell, trans, upper, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_copy_tri_chain(const double* src, int ell, int n, double* const* dst, const int64_t* ld,
                                 const int* trans, const int* upper, hipStream_t st) {
  if (n < 1 || n > 3) return hipErrorInvalidValue;
  TriChain c;
  c.n = n;
  for (int k = 0; k < 3; ++k) {
    c.dst[k] = k < n ? dst[k] : nullptr;
    c.ld[k] = k < n ? ld[k] : 0;
    c.trans[k] = k < n ? trans[k] : 0;
    c.upper[k] = k < n ? upper[k] : 0;
  }
  const int e = ell * ell;
  copy_tri_chain_kernel<<<dim3((e + 255) / 256), dim3(256), 0, st>>>(src, ell, c);
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

hipError_t launch_zero_ranges(const ZeroRanges& z, hipStream_t st) {
  if (z.count < 0 || z.count > kZeroRanges) return hipErrorInvalidValue;
  int64_t most = 0;
  for (int r = 0; r < z.count; ++r) {
    if (((uintptr_t)z.ptr[r] & 15) != 0 || z.words[r] < 0) return hipErrorInvalidValue;
    most = std::max(most, z.words[r]);
  }
  if (most == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(1024, (most + 255) / 256);
  zero_ranges_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(z);
  return hipGetLastError();
}

}  // namespace corutv
