// ALM-CoRUTV robust PCA, elementwise part (Sec. 4, Algorithm 2; eq. 12 and
// the shrinkage operator).  One pass over the m x n data per iteration j:
//
//   r   = number of diagonal entries of T above 1/mu_j (a prefix: diag(T) is
//         non-negative and non-increasing)
//   L   = sum_{a < r} P[i, a] Q[j, a]   (P = U, Q = V T^T for an upper T;
//         P = U T, Q = V for a lower T -- the rank-r CoR-UTV thresholding)
//   x   = M - L + Y / mu_j
//   S   = sgn(x) max(|x| - lambda / mu_j, 0)
//   Z   = M - L - S,   Y <- Y + mu_j Z
//   B   = M - S + Y / mu_{j+1}   (the next iteration's CoR-UTV input)
//
// M, S and L are FP32 at the boundary; the iteration state Y and B is FP64
// and every operation is FP64.  (Late in the iteration mu reaches 1e7 mu_0,
// so the shrink threshold lambda/mu drops below the FP32 spacing of the data;
// FP32 state would leave rounding residue above the threshold on clean
// entries.)  Per-block sums of Z^2 are written for the relative residual
// zeta = ||Z||_F / ||M||_F and reduced in a fixed order.
#include "internal.hpp"

namespace corutv {
namespace {

constexpr int kRpcaBlocks = 1024;

struct RpcaArgs {
  const float* M;
  float* S;
  double* Y;
  double* B;
  float* L;
  int64_t m, n;
  int64_t ldm, lds, ldy, ldb, ldl;
  int lay_m, lay_s, lay_l;  // layouts of M, S, L; Y and B follow M
  const double* P;
  int64_t ldp;
  const double* Q;
  int64_t ldq;
  const double* T;
  int64_t ldt;
  int ell;
  double mu, mu_next, thresh;  // thresh = lambda / mu
  double inv_mu;               // 1 / mu (rank threshold)
  double* part;
};

__device__ __forceinline__ int64_t at(int lay, int64_t ld, int64_t i, int64_t j) {
  return lay == CORUTV_COL_MAJOR ? j * ld + i : i * ld + j;
}

__global__ void __launch_bounds__(256) rpca_step_kernel(RpcaArgs a) {
  __shared__ int rs;
  __shared__ double red[256];
  if (threadIdx.x == 0) {
    int r = 0;
    while (r < a.ell && a.T[(int64_t)r * a.ldt + r] > a.inv_mu) ++r;
    rs = r;
  }
  __syncthreads();
  const int r = rs;
  const bool colmaj = a.lay_m == CORUTV_COL_MAJOR;
  const int64_t total = a.m * a.n;
  double z2 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    // walk the data in its own storage order (coalesced)
    const int64_t i = colmaj ? e % a.m : e / a.n;
    const int64_t j = colmaj ? e / a.m : e % a.n;
    double l = 0.0;
    for (int c = 0; c < r; ++c) l = fma(a.P[(int64_t)c * a.ldp + i], a.Q[(int64_t)c * a.ldq + j], l);
    const int64_t om = at(a.lay_m, a.ldm, i, j);
    const double mv = (double)a.M[om];
    const double yv = a.Y ? (double)a.Y[at(a.lay_m, a.ldy, i, j)] : 0.0;
    const double x = mv - l + yv / a.mu;
    const double ax = fabs(x) - a.thresh;
    const double sv = ax > 0.0 ? copysign(ax, x) : 0.0;
    const double z = mv - l - sv;
    const double yn = yv + a.mu * z;
    a.S[at(a.lay_s, a.lds, i, j)] = (float)sv;
    a.Y[at(a.lay_m, a.ldy, i, j)] = yn;
    if (a.B) a.B[at(a.lay_m, a.ldb, i, j)] = mv - sv + yn / a.mu_next;
    if (a.L) a.L[at(a.lay_l, a.ldl, i, j)] = (float)l;
    z2 += z * z;
  }
  red[threadIdx.x] = z2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

// B = M (FP32 -> FP64, exact), same layout
__global__ void widen_kernel(const float* X, int lay, int64_t ld, int64_t m, int64_t n, double* B,
                             int64_t ldb) {
  const bool colmaj = lay == CORUTV_COL_MAJOR;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = colmaj ? e % m : e / n;
    const int64_t j = colmaj ? e / m : e % n;
    B[at(lay, ldb, i, j)] = (double)X[at(lay, ld, i, j)];
  }
}

// sum of squares of a float matrix (per-block partials, fixed order)
__global__ void __launch_bounds__(256) sumsq_kernel(const float* X, int lay, int64_t ld, int64_t m,
                                                    int64_t n, double* part) {
  __shared__ double red[256];
  const bool colmaj = lay == CORUTV_COL_MAJOR;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = colmaj ? e % m : e / n;
    const int64_t j = colmaj ? e / m : e % n;
    const double v = (double)X[at(lay, ld, i, j)];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

int rpca_partial_blocks() { return kRpcaBlocks; }

hipError_t launch_rpca_elementwise(const float* M, int lay_m, int64_t ldm, float* S, int lay_s,
                                   int64_t lds, double* Y, int64_t ldy, double* B, int64_t ldb, float* L,
                                   int lay_l, int64_t ldl, int64_t m, int64_t n, const double* P,
                                   int64_t ldp, const double* Q, int64_t ldq, const double* T,
                                   int64_t ldt, int ell, double mu, double mu_next, double lambda,
                                   double* part, hipStream_t st) {
  RpcaArgs a;
  a.M = M;
  a.S = S;
  a.Y = Y;
  a.B = B;
  a.L = L;
  a.m = m;
  a.n = n;
  a.ldm = ldm;
  a.lds = lds;
  a.ldy = ldy;
  a.ldb = ldb;
  a.ldl = ldl;
  a.lay_m = lay_m;
  a.lay_s = lay_s;
  a.lay_l = lay_l;
  a.P = P;
  a.ldp = ldp;
  a.Q = Q;
  a.ldq = ldq;
  a.T = T;
  a.ldt = ldt;
  a.ell = ell;
  a.mu = mu;
  a.mu_next = mu_next;
  a.thresh = lambda / mu;
  a.inv_mu = 1.0 / mu;
  a.part = part;
  rpca_step_kernel<<<dim3(kRpcaBlocks), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_widen(const float* X, int lay, int64_t ld, int64_t m, int64_t n, double* B, int64_t ldb,
                        hipStream_t st) {
  widen_kernel<<<dim3(kRpcaBlocks), dim3(256), 0, st>>>(X, lay, ld, m, n, B, ldb);
  return hipGetLastError();
}

hipError_t launch_sumsq(const float* X, int lay, int64_t ld, int64_t m, int64_t n, double* part,
                        hipStream_t st) {
  sumsq_kernel<<<dim3(kRpcaBlocks), dim3(256), 0, st>>>(X, lay, ld, m, n, part);
  return hipGetLastError();
}

}  // namespace corutv
