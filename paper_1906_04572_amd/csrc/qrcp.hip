// Column-pivoted QR of the l x l core (Sec. 3.1 eq. 8; Algorithm 1 QRCP step):
// D P = Qt R by Businger-Golub pivoting and Householder reflectors.
//
// Pivot loop: one workgroup of 1024 threads (l <= 256); four threads serve
// each logical column.  Columns are never moved: the logical -> original index map piv
// is permuted instead, and column data stays at its original position.  Two
// barriers per step: (A) every owner computes its trailing norm; (B) every
// thread redundantly finds the pivot and the reflector from shared data (no
// serial phase) and updates its own column.
//
// The arithmetic order is fixed so that the pivot sequence is a function of
// the input bits only (each product and sum rounded separately: this file is
// compiled with contraction off).  sum4 of an ordered list of terms: a_k =
// sequential sum of the terms at positions k, k+4, ... (k = 0..3), result
// (a_0 + a_1) + (a_2 + a_3) -- four independent chains instead of one.
//   tails   t_j = sum4_{i = s+1..l-1} W[i,j]*W[i,j]
//   norms   acc_j = W[s,j]*W[s,j] + t_j
//   pivot   first logical position j >= s with the largest acc_j
//   reflector  nrm = sqrt(acc_p); alpha = -nrm if x0 >= 0 else nrm;
//           v = W[s:, p] with v_0 = x0 - alpha; vtv = v0*v0 + t_p; tau = 2/vtv
//   update  d_j = sum4_{i = s..l-1} v_i*W[i,j];
//           f_j = d_j*tau; W[i,j] = W[i,j] - f_j*v_i
// Qt = H_0 H_1 ... H_{l-1} is formed afterwards by a second kernel (backward
// accumulation, one thread per column); it does not influence the pivots.
// diag(R) is made non-negative by flipping rows of R and columns of Qt.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace corutv {
namespace {

constexpr int kQrcpLdsMax = 128;  // working matrix in LDS up to this size

// W: row-major l x l (element (i, c) at W[i*l + c], c = original column).
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
    W[e] = trans ? D[(int64_t)i * ldd + c] : D[(int64_t)c * ldd + i];
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
        const double w = W[i * ell + c];
        a = a + w * w;
      }
      const double t = combine4(a);
      if (k == 0) {
        const double h = W[s * ell + c];
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
      const double x0 = W[s * ell + cp];
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
      if (k == 0) a = a + v0 * W[s * ell + c];
      for (int i = s + (k == 0 ? 4 : k); i < ell; i += 4) a = a + W[i * ell + cp] * W[i * ell + c];
      const double d = combine4(a);
      const double f = d * tau;
      if (k == 0) W[s * ell + c] = W[s * ell + c] - f * v0;
      for (int i = s + (k == 0 ? 4 : k); i < ell; i += 4)
        W[i * ell + c] = W[i * ell + c] - f * W[i * ell + cp];
    }
    // reflector of step s: v_s = (v0, W[s+1:, cp]); column cp is not touched
    // by later steps (its logical position s < every later trailing column)
    if (tid < ell) Vout[(int64_t)s * ell + tid] = tid < s ? 0.0 : (tid == s ? v0 : W[tid * ell + cp]);
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
      v = W[r * ell + pfin[jj]];
    else if (jj == r)
      v = alph[r];
    if (alph[r] < 0.0) v = -v;
    Rout[(int64_t)jj * ell + r] = v;
  }
  if (tid < ell) piv[tid] = pfin[tid];
}

__global__ void __launch_bounds__(1024) qrcp_pivot_lds(const double* D, int64_t ldd, int trans, int ell,
                                                      double* Rout, int32_t* piv, double* Vout,
                                                      double* tauout, double* signout) {
  __shared__ double W[kQrcpLdsMax * kQrcpLdsMax];
  __shared__ double nrm[256], tl[256], alph[256];
  __shared__ int pv[512];
  qrcp_pivot_body(W, nrm, tl, pv, alph, D, ldd, trans, ell, Rout, piv, Vout, tauout);
  __syncthreads();
  if ((int)threadIdx.x < ell) signout[threadIdx.x] = alph[threadIdx.x] < 0.0 ? -1.0 : 1.0;
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

// Qt = H_0 (H_1 (... H_{l-1} I)), one thread per column; Q in LDS (row-major).
// The reflector of the next step is staged into LDS (double-buffered) while
// the current one is applied, so each step has one barrier.
__device__ __forceinline__ void qrcp_formq_body(double* __restrict__ Q, double* __restrict__ vb,
                                                const double* __restrict__ V,
                                                const double* __restrict__ tau,
                                                const double* __restrict__ sign, int ell,
                                                double* __restrict__ Qout) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < ell * ell; e += nt) Q[e] = (e / ell == e % ell) ? 1.0 : 0.0;
  if (tid < ell) vb[((ell - 1) & 1) * 256 + tid] = V[(int64_t)(ell - 1) * ell + tid];
  __syncthreads();
  const int j = tid >> 2, k = tid & 3;
  for (int s = ell - 1; s >= 0; --s) {
    const double* v = vb + (s & 1) * 256;
    if (s > 0 && tid < ell) vb[((s - 1) & 1) * 256 + tid] = V[(int64_t)(s - 1) * ell + tid];
    const double ts = tau[s];
    if (ts != 0.0 && j >= s && j < ell) {
      double a = 0.0;
      for (int i = s + k; i < ell; i += 4) a += v[i] * Q[i * ell + j];
      a += __shfl_xor(a, 1, 64);
      a += __shfl_xor(a, 2, 64);
      const double d = a * ts;
      for (int i = s + k; i < ell; i += 4) Q[i * ell + j] -= d * v[i];
    }
    __syncthreads();
  }
  for (int e = tid; e < ell * ell; e += nt) {
    const int i = e % ell, c = e / ell;  // column-major output
    Qout[e] = sign[c] * Q[i * ell + c];
  }
}

__global__ void __launch_bounds__(1024) qrcp_formq_lds(const double* V, const double* tau,
                                                      const double* sign, int ell, double* Qout) {
  __shared__ double Q[kQrcpLdsMax * kQrcpLdsMax];
  __shared__ double vb[512];
  qrcp_formq_body(Q, vb, V, tau, sign, ell, Qout);
}

__global__ void __launch_bounds__(1024) qrcp_formq_global(const double* V, const double* tau,
                                                         const double* sign, int ell, double* Qout,
                                                         double* work) {
  __shared__ double vb[512];
  qrcp_formq_body(work, vb, V, tau, sign, ell, Qout);
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
  if (ell <= kQrcpLdsMax) {
    qrcp_pivot_lds<<<dim3(1), dim3(1024), 0, st>>>(D, ldd, trans, ell, R, piv, V, tau, sign);
    qrcp_formq_lds<<<dim3(1), dim3(1024), 0, st>>>(V, tau, sign, ell, Qt);
  } else {
    qrcp_pivot_global<<<dim3(1), dim3(1024), 0, st>>>(D, ldd, trans, ell, R, piv, V, tau, sign, scratch);
    qrcp_formq_global<<<dim3(1), dim3(1024), 0, st>>>(V, tau, sign, ell, Qt, scratch);
  }
  return hipGetLastError();
}

}  // namespace corutv
