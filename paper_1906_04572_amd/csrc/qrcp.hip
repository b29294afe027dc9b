// Column-pivoted QR of the l x l core (Sec. 3.1 eq. 8; Algorithm 1 QRCP step):
// D P = Qt R by Businger-Golub pivoting and Householder reflectors, in one
// workgroup (l <= 256: one thread per column for the norms, dot products and
// column updates, one thread per row for the accumulation of Qt).
//
// The arithmetic order is fixed so that the pivot sequence is a function of
// the input bits only:
//   norms   acc_j = 0; for i = s..l-1: acc_j = acc_j + W[i,j]*W[i,j]
//   pivot   first position j >= s of the largest acc_j
//   reflector  nrm = sqrt(acc_p); alpha = -nrm if x0 >= 0 else nrm;
//           v = W[s:, s] with v_0 = x0 - alpha; vtv = sequential sum of v_i*v_i;
//           tau = 2 / vtv
//   update  d_j = sequential sum of v_i*W[s+i,j]; f_j = d_j*tau;
//           W[s+i,j] = W[s+i,j] - f_j*v_i
//   Qt      dq_r = sequential sum of Qt[r,s+i]*v_i; fq_r = dq_r*tau;
//           Qt[r,s+i] = Qt[r,s+i] - fq_r*v_i
// with every product and sum rounded separately (no fused multiply-add; this
// file is compiled with contraction off), and diag(R) made non-negative at the
// end by flipping rows of R and columns of Qt.
#include "internal.hpp"

#pragma clang fp contract(off)

namespace corutv {
namespace {

constexpr int kQrcpLdsMax = 128;  // working matrix in LDS up to this size

__device__ void qrcp_body(double* W, double* Qt, double* nrm, int* pv, double* sc,
                          const double* __restrict__ D, int64_t ldd, int trans, int ell,
                          double* __restrict__ Qout, double* __restrict__ Rout,
                          int32_t* __restrict__ piv) {
  const int tid = threadIdx.x;
  const int n2 = ell * ell;
  // W row-major: W[i*ell + j] = D[i, j]; Qt row-major, identity.
  for (int e = tid; e < n2; e += blockDim.x) {
    const int i = e / ell, j = e % ell;
    W[e] = trans ? D[(int64_t)i * ldd + j] : D[(int64_t)j * ldd + i];
    Qt[e] = i == j ? 1.0 : 0.0;
  }
  if (tid < ell) pv[tid] = tid;
  __syncthreads();
  const int j = tid;  // column (for W) and row (for Qt) owned by this thread
  for (int s = 0; s < ell; ++s) {
    if (j >= s && j < ell) {
      double acc = 0.0;
      for (int i = s; i < ell; ++i) {
        const double w = W[i * ell + j];
        acc = acc + w * w;
      }
      nrm[j] = acc;
    }
    __syncthreads();
    if (tid == 0) {
      int p = s;
      double best = nrm[s];
      for (int c = s + 1; c < ell; ++c)
        if (nrm[c] > best) {
          best = nrm[c];
          p = c;
        }
      sc[4] = (double)p;
      if (p != s) {
        const int t = pv[s];
        pv[s] = pv[p];
        pv[p] = t;
      }
    }
    __syncthreads();
    const int p = (int)sc[4];
    if (p != s && tid < ell) {  // swap columns s and p, one row per thread
      const double a = W[tid * ell + s];
      W[tid * ell + s] = W[tid * ell + p];
      W[tid * ell + p] = a;
    }
    __syncthreads();
    if (tid == 0) {
      const double nr = sqrt(nrm[p]);
      if (nr == 0.0) {
        sc[0] = 0.0;  // tau = 0: H = I
      } else {
        const double x0 = W[s * ell + s];
        const double alpha = x0 >= 0.0 ? -nr : nr;
        const double v0 = x0 - alpha;
        double vtv = v0 * v0;
        for (int i = s + 1; i < ell; ++i) {
          const double vi = W[i * ell + s];
          vtv = vtv + vi * vi;
        }
        sc[0] = 2.0 / vtv;
        sc[1] = alpha;
        sc[2] = v0;
      }
    }
    __syncthreads();
    const double tau = sc[0];
    if (tau != 0.0) {
      const double v0 = sc[2];
      if (j > s && j < ell) {
        double d = v0 * W[s * ell + j];
        for (int i = s + 1; i < ell; ++i) d = d + W[i * ell + s] * W[i * ell + j];
        const double f = d * tau;
        W[s * ell + j] = W[s * ell + j] - f * v0;
        for (int i = s + 1; i < ell; ++i) W[i * ell + j] = W[i * ell + j] - f * W[i * ell + s];
      }
      if (j < ell) {  // Qt row j
        double dq = Qt[j * ell + s] * v0;
        for (int i = s + 1; i < ell; ++i) dq = dq + Qt[j * ell + i] * W[i * ell + s];
        const double fq = dq * tau;
        Qt[j * ell + s] = Qt[j * ell + s] - fq * v0;
        for (int i = s + 1; i < ell; ++i) Qt[j * ell + i] = Qt[j * ell + i] - fq * W[i * ell + s];
      }
    }
    __syncthreads();
    if (tau != 0.0) {
      if (tid == 0) W[s * ell + s] = sc[1];
      if (tid > s && tid < ell) W[tid * ell + s] = 0.0;
    }
    __syncthreads();
  }
  // outputs: R = triu(W) with rows flipped where the diagonal is negative,
  // Qt with the matching columns flipped; both column-major (ld ell).
  for (int e = tid; e < n2; e += blockDim.x) {
    const int i = e / ell, c = e % ell;
    const bool flip_r = W[i * ell + i] < 0.0;
    const double r = c >= i ? (flip_r ? -W[e] : W[e]) : 0.0;
    Rout[(int64_t)c * ell + i] = r;
    const bool flip_q = W[c * ell + c] < 0.0;
    Qout[(int64_t)c * ell + i] = flip_q ? -Qt[i * ell + c] : Qt[i * ell + c];
  }
  if (tid < ell) piv[tid] = pv[tid];
}

__global__ void __launch_bounds__(256) qrcp_lds_kernel(const double* D, int64_t ldd, int trans,
                                                       int ell, double* Qout, double* Rout,
                                                       int32_t* piv, double* work) {
  __shared__ double W[kQrcpLdsMax * kQrcpLdsMax];
  __shared__ double nrm[256];
  __shared__ int pv[256];
  __shared__ double sc[8];
  qrcp_body(W, work, nrm, pv, sc, D, ldd, trans, ell, Qout, Rout, piv);
}

__global__ void __launch_bounds__(256) qrcp_global_kernel(const double* D, int64_t ldd, int trans,
                                                          int ell, double* Qout, double* Rout,
                                                          int32_t* piv, double* work) {
  __shared__ double nrm[256];
  __shared__ int pv[256];
  __shared__ double sc[8];
  qrcp_body(work, work + (int64_t)ell * ell, nrm, pv, sc, D, ldd, trans, ell, Qout, Rout, piv);
}

}  // namespace

hipError_t launch_qrcp(const double* D, int64_t ldd, int trans, int ell, double* Qt, double* R,
                       int32_t* piv, double* work, hipStream_t st) {
  if (ell <= kQrcpLdsMax)
    qrcp_lds_kernel<<<dim3(1), dim3(256), 0, st>>>(D, ldd, trans, ell, Qt, R, piv, work);
  else
    qrcp_global_kernel<<<dim3(1), dim3(256), 0, st>>>(D, ldd, trans, ell, Qt, R, piv, work);
  return hipGetLastError();
}

}  // namespace corutv
