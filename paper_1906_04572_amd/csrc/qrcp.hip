// Column-pivoted QR of the l x l core (Sec. 3.1 eq. 8; Algorithm 1 QRCP step):
// D P = Qt R by Businger-Golub pivoting and Householder reflectors.
//
// Pivot loop: one workgroup; four threads serve each column.  Columns are
// never moved: a logical position -> original column map is permuted
// instead.  Every wave redundantly finds the pivot and the reflector from
// the shared norms (no serial phase), then every owner updates its own
// column and computes its next trailing norm.
//   l <= 128: qrcp_reg_kernel, 512 threads, each column in the registers of
//             its four owners (thread k holds rows k, k+4, ...) and mirrored
//             in LDS for the pivot broadcast; one barrier per step (the norm
//             arrays are double-buffered); Qt formed in the same launch;
//   l <= 192: qrcp_big_kernel, the same register layout (768 threads at
//             most), pivot column broadcast through LDS, reflectors staged
//             through device memory for Qt;
//   l <= 224: qrcp_bigl_kernel, the same with the top rows of every column
//             in LDS, then qrcp_formq_cols_kernel (one wave per column of Qt);
//   l <= 256: qrcp_pivot_global + qrcp_formq_cols_kernel, 1024 threads, the
//             working matrix in device memory (column-major), two barriers
//             per step.
//
// Every reduction has a fixed order (so the factorization is a deterministic
// function of the input bits), chosen for speed rather than to match any
// other implementation: a lane sums its own rows into four independent
// partial sums (row blocks q taken in increasing order, block q into partial
// q mod 4, fused multiply-adds), adds them as (p0 + p1) + (p2 + p3), and the
// four lanes of a column add their results by a butterfly (every lane ends
// with the same bits).  Another order changes a norm only by rounding, so the
// pivot agrees with any other QRCP of the same matrix except where the two
// largest trailing norms lie within that rounding of each other.
//   norms   acc_j = W[s,j]^2 + t_j, t_j = sum over rows i > s of W[i,j]^2
//   pivot   first logical position j >= s with the largest acc_j
//   reflector  nrm = sqrt(acc_p); alpha = -nrm if x0 >= 0 else nrm;
//           v = W[s:, p] with v_0 = x0 - alpha; vtv = v0*v0 + t_p; tau = 2/vtv
//   update  d_j = sum over rows i >= s of v_i W[i,j]; W[i,j] -= (d_j tau) v_i
// Qt = H_0 H_1 ... H_{l-1} is formed afterwards (backward accumulation); it
// does not influence the pivots.
// diag(R) is made non-negative by flipping rows of R and columns of Qt.
#include "internal.hpp"

namespace corutv {
namespace {

constexpr int kQrcpRegMax = 128;  // columns in registers up to this size

// W: column-major l x l (element (i, c) at W[c*l + i], c = original column).
// 1024 threads: thread t serves logical column t/4 and the residue class
// k = t%4 of the sum4 partial sums (positions k, k+4, ... of each ordered
// term list).  The four lanes of a column are adjacent, so the combination
// (a0 + a1) + (a2 + a3) is done with two lane exchanges and every lane ends
// with the same bits.
// Outputs: R (column-major, ld l), piv, and for the Q kernel the reflector
// matrix V (column-major: V[s*l + i] = v_s[i], zero above s), tau, sign.
__device__ __forceinline__ double combine4(double a) {
  // lanes 4j..4j+3 hold a0..a3; returns (a0 + a1) + (a2 + a3) on all four
  const double b = __shfl_xor(a, 1, 64);
  const int k = threadIdx.x & 3;
  const double pair = (k & 1) ? (b + a) : (a + b);  // (a0 + a1) or (a2 + a3)
  const double other = __shfl_xor(pair, 2, 64);
  return (k & 2) ? (other + pair) : (pair + other);
}

__device__ __forceinline__ void qrcp_pivot_body(double* __restrict__ W, double* __restrict__ nrm,
                                                double* __restrict__ tl, int* __restrict__ pv,
                                                double* __restrict__ alph,
                                                const double* __restrict__ D, int64_t ldd, int trans,
                                                int ell, double* __restrict__ Rout,
                                                int32_t* __restrict__ piv, double* __restrict__ Vout,
                                                double* __restrict__ tauout) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int e = tid; e < ell * ell; e += nt) {
    const int i = e / ell, c = e % ell;
    W[(int64_t)c * ell + i] = trans ? D[(int64_t)i * ldd + c] : D[(int64_t)c * ldd + i];
  }
  if (tid < ell) pv[tid] = tid;  // buffer 0
  __syncthreads();
  const int j = tid >> 2, k = tid & 3;
  int cur = 0;  // parity of the piv buffer holding the current map
  for (int s = 0; s < ell; ++s) {
    const int* pin = pv + cur * 256;
    int* pout = pv + (cur ^ 1) * 256;
    // (A) tails and norms of the trailing logical columns
    if (j >= s && j < ell) {
      const int c = pin[j];
      double a = 0.0;
      for (int i = s + 1 + k; i < ell; i += 4) {
        const double w = W[(int64_t)c * ell + i];
        a = a + w * w;
      }
      const double t = combine4(a);
      if (k == 0) {
        const double h = W[(int64_t)c * ell + s];
        tl[j] = t;
        nrm[j] = h * h + t;
      }
    }
    __syncthreads();
    // (B) pivot and reflector, computed identically by every wave; the
    // argmax (largest value, lowest position on ties) is exact in any
    // reduction order
    int p = ell;
    double best = -1.0;
    const int lane = tid & 63;
    for (int c = s + lane; c < ell; c += 64) {
      const double v = nrm[c];
      if (v > best) {  // c increases, so ties keep the lower position
        best = v;
        p = c;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int op = __shfl_xor(p, off, 64);
      if (ov > best || (ov == best && op < p)) {
        best = ov;
        p = op;
      }
    }
    if (p >= ell) {  // only NaN norms: keep the current column
      p = s;
      best = nrm[s];
    }
    const int cp = pin[p];  // original column of the pivot
    const double nr = sqrt(best);
    double tau = 0.0, alpha = 0.0, v0 = 0.0;
    if (nr != 0.0) {
      const double x0 = W[(int64_t)cp * ell + s];
      alpha = x0 >= 0.0 ? -nr : nr;
      v0 = x0 - alpha;
      const double vtv = v0 * v0 + tl[p];
      tau = 2.0 / vtv;
    }
    // logical map after swapping positions s and p
    if (tid < ell) pout[tid] = tid == s ? cp : (tid == p ? pin[s] : pin[tid]);
    if (tid == 0) alph[s] = alpha;
    if (tid == 0) tauout[s] = tau;
    if (tau != 0.0 && j > s && j < ell) {
      const int c = j == p ? pin[s] : pin[j];
      // terms at positions q = i - s: q = 0 -> v0 W[s,c]; q > 0 -> W[i,cp] W[i,c]
      double a = 0.0;
      if (k == 0) a = a + v0 * W[(int64_t)c * ell + s];
      for (int i = s + (k == 0 ? 4 : k); i < ell; i += 4) a = a + W[(int64_t)cp * ell + i] * W[(int64_t)c * ell + i];
      const double d = combine4(a);
      const double f = d * tau;
      if (k == 0) W[(int64_t)c * ell + s] = W[(int64_t)c * ell + s] - f * v0;
      for (int i = s + (k == 0 ? 4 : k); i < ell; i += 4)
        W[(int64_t)c * ell + i] = W[(int64_t)c * ell + i] - f * W[(int64_t)cp * ell + i];
    }
    // reflector of step s: v_s = (v0, W[s+1:, cp]); column cp is not touched
    // by later steps (its logical position s < every later trailing column)
    if (tid < ell) Vout[(int64_t)s * ell + tid] = tid < s ? 0.0 : (tid == s ? v0 : W[(int64_t)cp * ell + tid]);
    cur ^= 1;
    __syncthreads();
  }
  // R[s][j] = W[s][piv[j]] for j > s, alpha_s on the diagonal; rows with a
  // negative diagonal are flipped.
  const int* pfin = pv + cur * 256;
  for (int e = tid; e < ell * ell; e += nt) {
    const int r = e % ell, jj = e / ell;  // column-major: row r, column jj
    double v = 0.0;
    if (jj > r)
      v = W[(int64_t)pfin[jj] * ell + r];
    else if (jj == r)
      v = alph[r];
    if (alph[r] < 0.0) v = -v;
    Rout[(int64_t)jj * ell + r] = v;
  }
  if (tid < ell) piv[tid] = pfin[tid];
}

__global__ void __launch_bounds__(1024) qrcp_pivot_global(const double* D, int64_t ldd, int trans,
                                                         int ell, double* Rout, int32_t* piv,
                                                         double* Vout, double* tauout,
                                                         double* signout, double* work) {
  __shared__ double nrm[256], tl[256], alph[256];
  __shared__ int pv[512];
  qrcp_pivot_body(work, nrm, tl, pv, alph, D, ldd, trans, ell, Rout, piv, Vout, tauout);
  __syncthreads();
  if ((int)threadIdx.x < ell) signout[threadIdx.x] = alph[threadIdx.x] < 0.0 ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// l <= 128.  Thread t serves column c = t/4 and holds w[q] = W[4q + k, c]
// (k = t%4).  A sum4 over rows r0, r0+1, ... is then, on each lane, a
// sequential sum over its own rows in increasing order: lane k holds the
// chain of positions congruent to (k - r0) mod 4.  Terms of rows before r0
// enter as exact zeros (adding +-0 leaves the bits of a sum unchanged).
// Cross-lane steps use DPP (quad permutes inside a column's four lanes, a
// row-broadcast reduction for the pivot) rather than LDS permutes.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double uniform_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of a lane's four partial sums, then over the four lanes of a column
// (lanes 4j..4j+3): a butterfly whose additions are commutative pairs, so all
// four lanes end with the same bits.
__device__ __forceinline__ double lane4_sum(const double (&a)[4]) {
  const double t = (a[0] + a[1]) + (a[2] + a[3]);
  const double u = t + dpp_f64<0xB1, 0xF>(t);  // lanes k, k ^ 1
  return u + dpp_f64<0x4E, 0xF>(u);            // pairs k, k ^ 2
}

// largest value over the wave (NaN-free input), the same on every lane
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1, 0xF>(v));   // quad_perm xor 1
  v = fmax(v, dpp_f64<0x4E, 0xF>(v));   // quad_perm xor 2
  v = fmax(v, dpp_f64<0x141, 0xF>(v));  // row_half_mirror
  v = fmax(v, dpp_f64<0x140, 0xF>(v));  // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v));  // row_bcast:15
  v = fmax(v, dpp_f64<0x143, 0xC>(v));  // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int kMirrorLd = 132;  // LDS column stride of the mirror (doubles, >= 128)
constexpr int kSeg = 8;         // row blocks per uniformly skipped segment

// The reflector a column would get as the pivot of a step: from its squared
// norm acc = x0*x0 + tail (x0 the head entry), nr = sqrt(acc),
// alpha = -sign(x0) nr, v0 = x0 - alpha, tau = 2 / (v0*v0 + tail).  Each
// owner evaluates this for its own column when it publishes its norm, so the
// pivot step only has to look the winner's values up.
__device__ __forceinline__ void reflector_of(double acc, double x0, double tail, double& alpha, double& v0,
                                             double& tau) {
  const double nr = sqrt(acc);
  alpha = 0.0;
  v0 = 0.0;
  tau = 0.0;
  if (nr != 0.0) {
    alpha = x0 >= 0.0 ? -nr : nr;
    v0 = x0 - alpha;
    const double vtv = v0 * v0 + tail;
    tau = 2.0 / vtv;
  }
}

template <int NR>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
qrcp_reg_kernel(const double* __restrict__ D, int64_t ldd, int trans, int ell, double* __restrict__ Qout,
                double* __restrict__ Rout, int32_t* __restrict__ piv) {
  // M[c * kMirrorLd + i] = W[i, c] (rows l..127 zero), refreshed by each
  // owner after its update; after the loop the mirror of the pivot column of
  // step s is turned into the reflector v_s (0 above row s, v0 at s)
  __shared__ double M[kQrcpRegMax * kMirrorLd];
  // per logical position, double-buffered: norm, and the reflector the
  // column there would give; original column index
  __shared__ double nrm[2][kQrcpRegMax], ralpha[2][kQrcpRegMax], rv0[2][kQrcpRegMax],
      rtau[2][kQrcpRegMax];
  __shared__ int colat[2][kQrcpRegMax];
  __shared__ double alph[kQrcpRegMax], taus[kQrcpRegMax], v0s[kQrcpRegMax];
  __shared__ int pcol[kQrcpRegMax];
  constexpr int NS = (NR + kSeg - 1) / kSeg;
  const int tid = threadIdx.x, lane = tid & 63;
  const int c = tid >> 2, k = tid & 3;
  const bool col_ok = c < ell;
  const int cl = col_ok ? c : ell - 1;
  double* mc = M + c * kMirrorLd;
  double w[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int row = 4 * q + k;
    const int rl = row < ell ? row : ell - 1;
    const double v = trans ? D[(int64_t)rl * ldd + cl] : D[(int64_t)cl * ldd + rl];
    w[q] = (row < ell && col_ok) ? v : 0.0;
    mc[row] = w[q];
  }
  int mypos = c;
  // norms of step 0: head row 0, tail rows 1..
  if (col_ok) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NR; ++q) a[q & 3] = (q > 0 || k >= 1) ? fma(w[q], w[q], a[q & 3]) : a[q & 3];
    const double tail = lane4_sum(a);
    if (k == 0) {
      const double acc = w[0] * w[0] + tail;
      double al, v0, ta;
      reflector_of(acc, w[0], tail, al, v0, ta);
      nrm[0][c] = acc;
      ralpha[0][c] = al;
      rv0[0][c] = v0;
      rtau[0][c] = ta;
      colat[0][c] = c;
    }
  }
  __syncthreads();
  for (int s = 0; s < ell; s = __builtin_amdgcn_readfirstlane(s + 1)) {
    const int b = s & 1;
    // pivot: largest norm (NaN never wins), lowest position on ties
    const int j0 = s + lane, j1 = j0 + 64;
    double c0 = j0 < ell ? nrm[b][j0] : -1.0;
    double c1 = j1 < ell ? nrm[b][j1] : -1.0;
    c0 = c0 >= 0.0 ? c0 : -1.0;
    c1 = c1 >= 0.0 ? c1 : -1.0;
    const double gm = wave_max(fmax(c0, c1));
    int p = s;  // only NaN norms: keep the current column
    if (gm >= 0.0) {
      const unsigned long long m0 = __ballot(c0 == gm);
      p = m0 ? s + __ffsll((long long)m0) - 1 : s + 64 + __ffsll((long long)__ballot(c1 == gm)) - 1;
    }
    p = __builtin_amdgcn_readfirstlane(p);
    const int cp = __builtin_amdgcn_readfirstlane(colat[b][p]);
    const double alpha = uniform_f64(ralpha[b][p]);
    const double v0 = uniform_f64(rv0[b][p]);
    const double tau = uniform_f64(rtau[b][p]);
    if (tid == 0) {
      alph[s] = alpha;
      taus[s] = tau;
      v0s[s] = v0;
      pcol[s] = cp;
    }
    if (c == cp)
      mypos = s;
    else if (mypos == s)
      mypos = p;
    const bool act = col_ok && mypos > s;
    const int qs = s >> 2, gs = qs / kSeg;
    // v = (0 above row s, v0, W[s+1:, cp]) from the mirror of column cp: the
    // segment holding row s is masked, earlier segments hold only rows < s
    if (act && tau != 0.0) {
      const double* mp = M + cp * kMirrorLd;
      double vv[NR];
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        if (g > gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) vv[q] = mp[4 * q + k];
        } else if (g == gs) {
          // All loads first, each made opaque before the masking: a select
          // between a loaded value and a constant is otherwise turned into a
          // branch around the load, which then waits for every load in turn.
          double xs[kSeg];
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) xs[q - g * kSeg] = mp[4 * q + k];
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) {
            double x = xs[q - g * kSeg];
            asm volatile("" : "+v"(x));
            const int row = 4 * q + k;
            vv[q] = row < s ? 0.0 : (row == s ? v0 : x);
          }
        }
      }
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) a[q & 3] = fma(vv[q], w[q], a[q & 3]);
        }
      const double f = lane4_sum(a) * tau;
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) {
            w[q] = w[q] - f * vv[q];
            mc[4 * q + k] = w[q];
          }
        }
    }
    if (act && s + 1 < ell) {
      // norm of step s + 1 (head row s + 1, tail rows s + 2..) and the
      // reflector this column would give
      const int qh = (s + 1) >> 2;
      const int gt = ((s + 2) >> 2) / kSeg;
      double a[4] = {0.0, 0.0, 0.0, 0.0}, hv = 0.0;
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        if (g > gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) a[q & 3] = fma(w[q], w[q], a[q & 3]);
        } else if (g == gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[q & 3] = 4 * q + k >= s + 2 ? fma(w[q], w[q], a[q & 3]) : a[q & 3];
        }
      }
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g == qh / kSeg) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) hv = q == qh ? w[q] : hv;
        }
      const double tail = lane4_sum(a);
      if (k == ((s + 1) & 3)) {
        const double acc = hv * hv + tail;
        double al, rv, ta;
        reflector_of(acc, hv, tail, al, rv, ta);
        nrm[b ^ 1][mypos] = acc;
        ralpha[b ^ 1][mypos] = al;
        rv0[b ^ 1][mypos] = rv;
        rtau[b ^ 1][mypos] = ta;
        colat[b ^ 1][mypos] = c;
      }
    }
    __syncthreads();
  }
  // R[r][j] = W[r][piv[j]] above the diagonal, alpha_j on it; rows with a
  // negative diagonal flipped.  Column-major.  The mirror of each column
  // becomes the reflector of the step that chose it.
  if (col_ok) {
    const int jj = mypos;
    const double v0 = v0s[jj];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = 4 * q + k;
      if (r < ell) {
        double v = r < jj ? w[q] : (r == jj ? alph[jj] : 0.0);
        if (alph[r] < 0.0) v = -v;
        Rout[(int64_t)jj * ell + r] = v;
        if (r <= jj) mc[r] = r == jj ? v0 : 0.0;
      }
    }
    if (k == 0) piv[jj] = c;
  }
  __syncthreads();
  // Qt = H_0 (H_1 (... H_{l-1} I)): every column is independent, so each
  // group of four lanes runs the backward loop on its own (no barriers)
#pragma unroll
  for (int q = 0; q < NR; ++q) w[q] = (4 * q + k == c) ? 1.0 : 0.0;
  for (int s = ell - 1; s >= 0; s = __builtin_amdgcn_readfirstlane(s - 1)) {
    const double ts = taus[s];
    if (col_ok && c >= s && ts != 0.0) {
      const double* mp = M + pcol[s] * kMirrorLd;
      const int gs = (s >> 2) / kSeg;
      double vv[NR];
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) vv[q] = mp[4 * q + k];
        }
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) a[q & 3] = fma(vv[q], w[q], a[q & 3]);
        }
      const double dd = lane4_sum(a) * ts;
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) w[q] -= dd * vv[q];
        }
    }
  }
  if (col_ok) {
    const double sg = alph[c] < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int row = 4 * q + k;
      if (row < ell) Qout[(int64_t)c * ell + row] = sg * w[q];
    }
  }
}

// ---------------------------------------------------------------------------
// 128 < l <= 192: the same per-column register layout with 4 * ceil(l/4)
// rows per column (NR = 40 or 48 per thread), 16 NR threads (at most 12
// waves, so a thread may hold 96 registers of column data).  The l x l
// mirror would not fit in LDS, so the pivot column is broadcast through a
// zero-padded LDS vector written by its owners after the pivot search (two
// barriers per step), and each reflector is also written to device memory;
// Qt is then formed from chunks of reflectors staged through LDS.
constexpr int kBigMax = 192;
constexpr int kVChunk = 64;

template <int NR>
__global__ void __launch_bounds__(16 * NR)
qrcp_big_kernel(const double* __restrict__ D, int64_t ldd, int trans, int ell, double* __restrict__ Qout,
                double* __restrict__ Rout, int32_t* __restrict__ piv, double* __restrict__ Vg) {
  constexpr int LP = 4 * NR;              // padded rows and columns
  constexpr int NC = (LP + 63) / 64;      // pivot candidates per lane
  constexpr int NS = (NR + kSeg - 1) / kSeg;
  __shared__ double nrm[2][LP], ralpha[2][LP], rv0[2][LP], rtau[2][LP];
  __shared__ int colat[2][LP];
  __shared__ double vcol[LP];
  __shared__ double alph[LP], taus[LP];
  __shared__ double vch[kVChunk * LP];
  const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
  const int c = tid >> 2, k = tid & 3;
  const bool col_ok = c < ell;
  const int cl = col_ok ? c : ell - 1;
  double w[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int row = 4 * q + k;
    const int rl = row < ell ? row : ell - 1;
    const double v = trans ? D[(int64_t)rl * ldd + cl] : D[(int64_t)cl * ldd + rl];
    w[q] = (row < ell && col_ok) ? v : 0.0;
  }
  for (int i = tid; i < LP; i += nt) vcol[i] = 0.0;
  int mypos = c;
  if (col_ok) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NR; ++q) a[q & 3] = (q > 0 || k >= 1) ? fma(w[q], w[q], a[q & 3]) : a[q & 3];
    const double tail = lane4_sum(a);
    if (k == 0) {
      const double acc = w[0] * w[0] + tail;
      double al, v0, ta;
      reflector_of(acc, w[0], tail, al, v0, ta);
      nrm[0][c] = acc;
      ralpha[0][c] = al;
      rv0[0][c] = v0;
      rtau[0][c] = ta;
      colat[0][c] = c;
    }
  }
  __syncthreads();
  for (int s = 0; s < ell; s = __builtin_amdgcn_readfirstlane(s + 1)) {
    const int b = s & 1;
    // pivot: largest norm (NaN never wins), lowest position on ties; the
    // candidates of round h are positions s + 64h + lane, so the first
    // round holding the maximum gives the lowest position
    double cand[NC];
    double cb = -1.0;
#pragma unroll
    for (int h = 0; h < NC; ++h) {
      const int j = s + lane + 64 * h;
      const double v = j < ell ? nrm[b][j] : -1.0;
      cand[h] = v >= 0.0 ? v : -1.0;
      cb = fmax(cb, cand[h]);
    }
    const double gm = wave_max(cb);
    int p = s;  // only NaN norms: keep the current column
    if (gm >= 0.0) {
#pragma unroll
      for (int h = NC - 1; h >= 0; --h) {
        const unsigned long long m = __ballot(cand[h] == gm);
        if (m) p = s + 64 * h + __ffsll((long long)m) - 1;
      }
    }
    p = __builtin_amdgcn_readfirstlane(p);
    const int cp = __builtin_amdgcn_readfirstlane(colat[b][p]);
    const double alpha = uniform_f64(ralpha[b][p]);
    const double v0 = uniform_f64(rv0[b][p]);
    const double tau = uniform_f64(rtau[b][p]);
    if (c == cp) {  // reflector v_s = (0 above row s, v0, W[s+1:, cp])
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int row = 4 * q + k;
        if (row < ell) {
          const double v = row < s ? 0.0 : (row == s ? v0 : w[q]);
          vcol[row] = v;
          Vg[(int64_t)s * ell + row] = v;
        }
      }
    }
    if (tid == 0) {
      alph[s] = alpha;
      taus[s] = tau;
    }
    if (c == cp)
      mypos = s;
    else if (mypos == s)
      mypos = p;
    const bool act = col_ok && mypos > s;
    __syncthreads();
    const int gs = (s >> 2) / kSeg;
    if (act && tau != 0.0) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[q & 3] = fma(vcol[4 * q + k], w[q], a[q & 3]);
        }
      const double f = lane4_sum(a) * tau;
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) w[q] = w[q] - f * vcol[4 * q + k];
        }
    }
    if (act && s + 1 < ell) {
      const int qh = (s + 1) >> 2;
      const int gt = ((s + 2) >> 2) / kSeg;
      double a[4] = {0.0, 0.0, 0.0, 0.0}, hv = 0.0;
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        if (g > gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) a[q & 3] = fma(w[q], w[q], a[q & 3]);
        } else if (g == gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[q & 3] = 4 * q + k >= s + 2 ? fma(w[q], w[q], a[q & 3]) : a[q & 3];
        }
      }
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g == qh / kSeg) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) hv = q == qh ? w[q] : hv;
        }
      const double tail = lane4_sum(a);
      if (k == ((s + 1) & 3)) {
        const double acc = hv * hv + tail;
        double al, rv, ta;
        reflector_of(acc, hv, tail, al, rv, ta);
        nrm[b ^ 1][mypos] = acc;
        ralpha[b ^ 1][mypos] = al;
        rv0[b ^ 1][mypos] = rv;
        rtau[b ^ 1][mypos] = ta;
        colat[b ^ 1][mypos] = c;
      }
    }
    __syncthreads();
  }
  if (col_ok) {
    const int jj = mypos;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = 4 * q + k;
      if (r < ell) {
        double v = r < jj ? w[q] : (r == jj ? alph[jj] : 0.0);
        if (alph[r] < 0.0) v = -v;
        Rout[(int64_t)jj * ell + r] = v;
      }
    }
    if (k == 0) piv[jj] = c;
  }
  // Qt = H_0 (H_1 (... H_{l-1} I)), reflectors staged through LDS in chunks
  // of kVChunk (last chunk first); within a chunk every column runs on its
  // own (no barriers)
#pragma unroll
  for (int q = 0; q < NR; ++q) w[q] = (4 * q + k == c) ? 1.0 : 0.0;
  for (int end = ell; end > 0; end -= kVChunk) {
    const int lo = end > kVChunk ? end - kVChunk : 0;
    __syncthreads();
    for (int e = tid; e < (end - lo) * LP; e += nt) {
      const int si = e / LP, i = e % LP;
      vch[e] = i < ell ? Vg[(int64_t)(lo + si) * ell + i] : 0.0;
    }
    __syncthreads();
    for (int s = end - 1; s >= lo; s = __builtin_amdgcn_readfirstlane(s - 1)) {
      const double ts = taus[s];
      if (col_ok && c >= s && ts != 0.0) {
        const double* v = vch + (s - lo) * LP;
        const int gs = (s >> 2) / kSeg;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int g = 0; g < NS; ++g)
          if (g >= gs) {
#pragma unroll
            for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) a[q & 3] = fma(v[4 * q + k], w[q], a[q & 3]);
          }
        const double dd = lane4_sum(a) * ts;
#pragma unroll
        for (int g = 0; g < NS; ++g)
          if (g >= gs) {
#pragma unroll
            for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) w[q] -= dd * v[4 * q + k];
          }
      }
    }
  }
  if (col_ok) {
    const double sg = alph[c] < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int row = 4 * q + k;
      if (row < ell) Qout[(int64_t)c * ell + row] = sg * w[q];
    }
  }
}

// ---------------------------------------------------------------------------
// 192 < l <= 224: the layout of qrcp_big_kernel, with the top rows of every
// column (blocks q < NL: rows 4q + k) in LDS and the others in registers.
// The top rows leave the active trailing block first, so after the first 4 NL
// steps only registers are touched.  Qt is formed afterwards by
// qrcp_formq_cols_kernel from the reflectors, taus and signs written here.
constexpr int kBigLMax = 224;

template <int NR, int NL>
__global__ void __launch_bounds__(16 * (NR + NL))
qrcp_bigl_kernel(const double* __restrict__ D, int64_t ldd, int trans, int ell, double* __restrict__ Rout,
                 int32_t* __restrict__ piv, double* __restrict__ Vg, double* __restrict__ taug,
                 double* __restrict__ signg) {
  constexpr int LP = 4 * (NR + NL);       // padded rows and columns
  constexpr int NC = (LP + 63) / 64;      // pivot candidates per lane
  constexpr int NS = (NR + kSeg - 1) / kSeg;
  __shared__ double nrm[2][LP], ralpha[2][LP], rv0[2][LP], rtau[2][LP];
  __shared__ int colat[2][LP];
  __shared__ double vcol[LP];
  __shared__ double alph[LP];
  __shared__ double wl[NL * LP * 4];  // row 4q + k (q < NL) of column c at wl[(q LP + c) 4 + k]
  const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
  const int c = tid >> 2, k = tid & 3;
  const bool col_ok = c < ell;
  const int cl = col_ok ? c : ell - 1;
  double* wc = wl + c * 4 + k;  // + q LP 4
  double w[NR];                 // row 4 (NL + q) + k
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int row = 4 * q + k;
    const int rl = row < ell ? row : ell - 1;
    const double v = trans ? D[(int64_t)rl * ldd + cl] : D[(int64_t)cl * ldd + rl];
    wc[q * LP * 4] = (row < ell && col_ok) ? v : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int row = 4 * (NL + q) + k;
    const int rl = row < ell ? row : ell - 1;
    const double v = trans ? D[(int64_t)rl * ldd + cl] : D[(int64_t)cl * ldd + rl];
    w[q] = (row < ell && col_ok) ? v : 0.0;
  }
  for (int i = tid; i < LP; i += nt) vcol[i] = 0.0;
  int mypos = c;
  if (col_ok) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const double x = wc[q * LP * 4];
      a[q & 3] = (q > 0 || k >= 1) ? fma(x, x, a[q & 3]) : a[q & 3];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) a[(NL + q) & 3] = fma(w[q], w[q], a[(NL + q) & 3]);
    const double tail = lane4_sum(a);
    if (k == 0) {
      const double x0 = wc[0];
      const double acc = x0 * x0 + tail;
      double al, v0, ta;
      reflector_of(acc, x0, tail, al, v0, ta);
      nrm[0][c] = acc;
      ralpha[0][c] = al;
      rv0[0][c] = v0;
      rtau[0][c] = ta;
      colat[0][c] = c;
    }
  }
  __syncthreads();
  for (int s = 0; s < ell; s = __builtin_amdgcn_readfirstlane(s + 1)) {
    const int b = s & 1;
    double cand[NC];
    double cb = -1.0;
#pragma unroll
    for (int h = 0; h < NC; ++h) {
      const int j = s + lane + 64 * h;
      const double v = j < ell ? nrm[b][j] : -1.0;
      cand[h] = v >= 0.0 ? v : -1.0;
      cb = fmax(cb, cand[h]);
    }
    const double gm = wave_max(cb);
    int p = s;  // only NaN norms: keep the current column
    if (gm >= 0.0) {
#pragma unroll
      for (int h = NC - 1; h >= 0; --h) {
        const unsigned long long m = __ballot(cand[h] == gm);
        if (m) p = s + 64 * h + __ffsll((long long)m) - 1;
      }
    }
    p = __builtin_amdgcn_readfirstlane(p);
    const int cp = __builtin_amdgcn_readfirstlane(colat[b][p]);
    const double alpha = uniform_f64(ralpha[b][p]);
    const double v0 = uniform_f64(rv0[b][p]);
    const double tau = uniform_f64(rtau[b][p]);
    const int qs = s >> 2;
    if (c == cp) {  // reflector v_s = (0 above row s, v0, W[s+1:, cp])
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int row = 4 * q + k;
        if (q >= qs && row < ell) {
          const double v = row < s ? 0.0 : (row == s ? v0 : wc[q * LP * 4]);
          vcol[row] = v;
          Vg[(int64_t)s * ell + row] = v;
        } else if (row < ell) {
          Vg[(int64_t)s * ell + row] = 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int row = 4 * (NL + q) + k;
        if (row < ell) {
          const double v = row < s ? 0.0 : (row == s ? v0 : w[q]);
          vcol[row] = v;
          Vg[(int64_t)s * ell + row] = v;
        }
      }
    }
    if (tid == 0) {
      alph[s] = alpha;
      taug[s] = tau;
    }
    if (c == cp)
      mypos = s;
    else if (mypos == s)
      mypos = p;
    const bool act = col_ok && mypos > s;
    __syncthreads();
    // register segments g < gs hold only rows < s
    const int gs = qs > NL ? (qs - NL) / kSeg : 0;
    if (act && tau != 0.0) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q >= qs) a[q & 3] = fma(vcol[4 * q + k], wc[q * LP * 4], a[q & 3]);
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[(NL + q) & 3] = fma(vcol[4 * (NL + q) + k], w[q], a[(NL + q) & 3]);
        }
      const double f = lane4_sum(a) * tau;
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q >= qs) wc[q * LP * 4] = wc[q * LP * 4] - f * vcol[4 * q + k];
#pragma unroll
      for (int g = 0; g < NS; ++g)
        if (g >= gs) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) w[q] = w[q] - f * vcol[4 * (NL + q) + k];
        }
    }
    if (act && s + 1 < ell) {
      // norm of step s + 1 (head row s + 1, tail rows s + 2..)
      const int qt2 = (s + 2) >> 2, qh = (s + 1) >> 2;
      const int gt = qt2 > NL ? (qt2 - NL) / kSeg : 0;
      double a[4] = {0.0, 0.0, 0.0, 0.0}, hv = 0.0;
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q >= qt2) {
          const double x = wc[q * LP * 4];
          a[q & 3] = 4 * q + k >= s + 2 ? fma(x, x, a[q & 3]) : a[q & 3];
        }
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        if (g > gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[(NL + q) & 3] = fma(w[q], w[q], a[(NL + q) & 3]);
        } else if (g == gt) {
#pragma unroll
          for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q)
            a[(NL + q) & 3] = 4 * (NL + q) + k >= s + 2 ? fma(w[q], w[q], a[(NL + q) & 3]) : a[(NL + q) & 3];
        }
      }
      if (qh < NL) {
        hv = wl[(qh * LP + c) * 4 + k];
      } else {
#pragma unroll
        for (int g = 0; g < NS; ++g)
          if (g == (qh - NL) / kSeg) {
#pragma unroll
            for (int q = g * kSeg; q < g * kSeg + kSeg && q < NR; ++q) hv = NL + q == qh ? w[q] : hv;
          }
      }
      const double tail = lane4_sum(a);
      if (k == ((s + 1) & 3)) {
        const double acc = hv * hv + tail;
        double al, rv, ta;
        reflector_of(acc, hv, tail, al, rv, ta);
        nrm[b ^ 1][mypos] = acc;
        ralpha[b ^ 1][mypos] = al;
        rv0[b ^ 1][mypos] = rv;
        rtau[b ^ 1][mypos] = ta;
        colat[b ^ 1][mypos] = c;
      }
    }
    __syncthreads();
  }
  // R[r][j] = W[r][piv[j]] above the diagonal, alpha_j on it; rows with a
  // negative diagonal flipped.  Column-major.
  if (col_ok) {
    const int jj = mypos;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int r = 4 * q + k;
      if (r < ell) {
        double v = r < jj ? wc[q * LP * 4] : (r == jj ? alph[jj] : 0.0);
        if (alph[r] < 0.0) v = -v;
        Rout[(int64_t)jj * ell + r] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = 4 * (NL + q) + k;
      if (r < ell) {
        double v = r < jj ? w[q] : (r == jj ? alph[jj] : 0.0);
        if (alph[r] < 0.0) v = -v;
        Rout[(int64_t)jj * ell + r] = v;
      }
    }
    if (k == 0) piv[jj] = c;
  }
  if (tid < ell) signg[tid] = alph[tid] < 0.0 ? -1.0 : 1.0;
}

// Qt = H_0 (H_1 (... H_{l-1} I)) with one wave per column c: Qt e_c =
// H_0 ... H_c e_c (H_s leaves e_c unchanged for s > c, v_s being zero above
// row s).  Lane i holds rows i, i + 64, i + 128, i + 192; the next
// reflector's loads are issued before the current one is applied.  The dot
// products are reduced by a butterfly (same bits on every lane).
// V column-major (V[s l + i] = v_s[i], zero above row s), tau and sign per
// step / column; l <= 256.
__global__ void __launch_bounds__(64) qrcp_formq_cols_kernel(const double* __restrict__ V,
                                                             const double* __restrict__ tau,
                                                             const double* __restrict__ sign, int ell,
                                                             double* __restrict__ Qout) {
  const int c = blockIdx.x, lane = threadIdx.x;
  double x[4], vn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = lane + 64 * r;
    x[r] = row == c ? 1.0 : 0.0;
    vn[r] = row < ell ? V[(int64_t)c * ell + row] : 0.0;
  }
  for (int s = c; s >= 0; --s) {
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = vn[r];
    if (s > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lane + 64 * r;
        vn[r] = row < ell ? V[(int64_t)(s - 1) * ell + row] : 0.0;
      }
    }
    const double ts = tau[s];
    if (ts == 0.0) continue;
    double d = (v[0] * x[0] + v[1] * x[1]) + (v[2] * x[2] + v[3] * x[3]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = d + __shfl_xor(d, off, 64);
    d = d * ts;
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = x[r] - d * v[r];
  }
  const double sg = sign[c];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = lane + 64 * r;
    if (row < ell) Qout[(int64_t)c * ell + row] = sg * x[r];
  }
}

}  // namespace

hipError_t launch_qrcp(const double* D, int64_t ldd, int trans, int ell, double* Qt, double* R,
                       int32_t* piv, double* work, hipStream_t st) {
  // work: 2 l^2 + 2 l doubles: V (l^2), scratch matrix (l^2), tau, sign
  const int64_t l2 = (int64_t)ell * ell;
  double* V = work;
  double* scratch = work + l2;
  double* tau = work + 2 * l2;
  double* sign = tau + ell;
  if (ell <= 32) {
    qrcp_reg_kernel<8><<<dim3(1), dim3(512), 0, st>>>(D, ldd, trans, ell, Qt, R, piv);
  } else if (ell <= 64) {
    qrcp_reg_kernel<16><<<dim3(1), dim3(512), 0, st>>>(D, ldd, trans, ell, Qt, R, piv);
  } else if (ell <= 96) {
    qrcp_reg_kernel<24><<<dim3(1), dim3(512), 0, st>>>(D, ldd, trans, ell, Qt, R, piv);
  } else if (ell <= 112) {
    qrcp_reg_kernel<28><<<dim3(1), dim3(512), 0, st>>>(D, ldd, trans, ell, Qt, R, piv);
  } else if (ell <= kQrcpRegMax) {
    qrcp_reg_kernel<32><<<dim3(1), dim3(512), 0, st>>>(D, ldd, trans, ell, Qt, R, piv);
  } else if (ell <= 160) {
    qrcp_big_kernel<40><<<dim3(1), dim3(640), 0, st>>>(D, ldd, trans, ell, Qt, R, piv, V);
  } else if (ell <= kBigMax) {
    qrcp_big_kernel<48><<<dim3(1), dim3(768), 0, st>>>(D, ldd, trans, ell, Qt, R, piv, V);
  } else if (ell <= kBigLMax) {
    qrcp_bigl_kernel<40, 16><<<dim3(1), dim3(896), 0, st>>>(D, ldd, trans, ell, R, piv, V, tau, sign);
    qrcp_formq_cols_kernel<<<dim3(ell), dim3(64), 0, st>>>(V, tau, sign, ell, Qt);
  } else {
    qrcp_pivot_global<<<dim3(1), dim3(1024), 0, st>>>(D, ldd, trans, ell, R, piv, V, tau, sign, scratch);
    qrcp_formq_cols_kernel<<<dim3(ell), dim3(64), 0, st>>>(V, tau, sign, ell, Qt);
  }
  return hipGetLastError();
}

}  // namespace corutv
