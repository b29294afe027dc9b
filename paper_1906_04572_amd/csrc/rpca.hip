// ALM-CoRUTV robust PCA, elementwise part (Sec. 4, Algorithm 2; eq. 12 and
// the shrinkage operator).  One pass over the m x n data per iteration j:
//
//   r   = number of diagonal entries of T above 1/mu_j (for the non-negative,
//         non-increasing diagonal of a QRCP these are the first r)
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
  const int* st;  // status words of the iteration's decomposition
  int nst;
  int* sticky;    // OR of every status word seen so far
  int* rank_out;  // nullable: receives r
};

__device__ __forceinline__ int64_t at(int lay, int64_t ld, int64_t i, int64_t j) {
  return lay == CORUTV_COL_MAJOR ? j * ld + i : i * ld + j;
}

// One block of the grid handles tiles of 256 consecutive elements of a storage
// line of M (a column when M is column-major, a row otherwise) times kLines
// neighbouring lines, so each thread reads its entry of the along-line factor
// (P for columns, Q for rows) once per rank-one term and reuses it for kLines
// elements.  Every element is loaded and computed at a clamped in-range index;
// only stores and the Z^2 sum are masked.
constexpr int kLines = 8;

__global__ void __launch_bounds__(256) rpca_step_kernel(RpcaArgs a) {
  __shared__ int rs;
  __shared__ double red[256];
  if (threadIdx.x == 0) rs = 0;
  __syncthreads();
  // r: how many diagonal entries of T exceed 1/mu (eq. 12)
  if ((int)threadIdx.x < a.ell && a.T[(int64_t)threadIdx.x * a.ldt + threadIdx.x] > a.inv_mu)
    atomicAdd(&rs, 1);
  __syncthreads();
  const int r = rs;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (a.sticky) {
      int acc = *a.sticky;
      for (int i = 0; i < a.nst; ++i) acc |= a.st[i];
      *a.sticky = acc;
    }
    if (a.rank_out) *a.rank_out = r;
  }
  const bool colmaj = a.lay_m == CORUTV_COL_MAJOR;
  const int64_t len = colmaj ? a.m : a.n;     // elements along a storage line
  const int64_t nlines = colmaj ? a.n : a.m;
  const double* Fa = colmaj ? a.P : a.Q;      // factor indexed along the line
  const int64_t ldfa = colmaj ? a.ldp : a.ldq;
  const double* Fb = colmaj ? a.Q : a.P;      // factor indexed by the line
  const int64_t ldfb = colmaj ? a.ldq : a.ldp;
  const int64_t ta = (len + 255) / 256, tb = (nlines + kLines - 1) / kLines;
  double z2 = 0.0;
  for (int64_t t = blockIdx.x; t < ta * tb; t += gridDim.x) {
    const int64_t p0 = (t % ta) * 256 + threadIdx.x;
    const int64_t b0 = (t / ta) * kLines;
    const bool pin = p0 < len;
    const int64_t pc = pin ? p0 : len - 1;
    int64_t bl[kLines];
    double l[kLines], mv[kLines], yv[kLines];
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      bl[u] = b0 + u < nlines ? b0 + u : nlines - 1;
      l[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      mv[u] = (double)a.M[bl[u] * a.ldm + pc];
      yv[u] = a.Y[bl[u] * a.ldy + pc];
    }
    for (int c = 0; c < r; ++c) {
      const double fa = Fa[(int64_t)c * ldfa + pc];
#pragma unroll
      for (int u = 0; u < kLines; ++u) l[u] = fma(fa, Fb[(int64_t)c * ldfb + bl[u]], l[u]);
    }
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      const double x = mv[u] - l[u] + yv[u] / a.mu;
      const double ax = fabs(x) - a.thresh;
      const double sv = ax > 0.0 ? copysign(ax, x) : 0.0;
      const double z = mv[u] - l[u] - sv;
      const double yn = yv[u] + a.mu * z;
      if (pin && b0 + u < nlines) {
        const int64_t i = colmaj ? p0 : b0 + u;
        const int64_t j = colmaj ? b0 + u : p0;
        a.S[at(a.lay_s, a.lds, i, j)] = (float)sv;
        a.Y[bl[u] * a.ldy + p0] = yn;
        if (a.B) a.B[bl[u] * a.ldb + p0] = mv[u] - sv + yn / a.mu_next;
        if (a.L) a.L[at(a.lay_l, a.ldl, i, j)] = (float)l[u];
        z2 += z * z;
      }
    }
  }
  red[threadIdx.x] = z2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

// The same step with two neighbouring elements of a storage line per thread
// (8-byte loads and stores of M, S and L, 16-byte ones of Y, B and the
// along-line factor), for lines of even length whose leading dimensions are
// even and whose bases are aligned, with S and L in M's layout.  The
// arithmetic of each element is the scalar kernel's, in the same order.
__global__ void __launch_bounds__(256) rpca_step2_kernel(RpcaArgs a) {
  __shared__ int rs;
  __shared__ double red[256];
  if (threadIdx.x == 0) rs = 0;
  __syncthreads();
  if ((int)threadIdx.x < a.ell && a.T[(int64_t)threadIdx.x * a.ldt + threadIdx.x] > a.inv_mu)
    atomicAdd(&rs, 1);
  __syncthreads();
  const int r = rs;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (a.sticky) {
      int acc = *a.sticky;
      for (int i = 0; i < a.nst; ++i) acc |= a.st[i];
      *a.sticky = acc;
    }
    if (a.rank_out) *a.rank_out = r;
  }
  const bool colmaj = a.lay_m == CORUTV_COL_MAJOR;
  const int64_t len = colmaj ? a.m : a.n;  // even
  const int64_t nlines = colmaj ? a.n : a.m;
  const double* Fa = colmaj ? a.P : a.Q;
  const int64_t ldfa = colmaj ? a.ldp : a.ldq;
  const double* Fb = colmaj ? a.Q : a.P;
  const int64_t ldfb = colmaj ? a.ldq : a.ldp;
  const int64_t ta = (len + 511) / 512, tb = (nlines + kLines - 1) / kLines;
  double z2 = 0.0;
  for (int64_t t = blockIdx.x; t < ta * tb; t += gridDim.x) {
    const int64_t p0 = (t % ta) * 512 + 2 * threadIdx.x;
    const int64_t b0 = (t / ta) * kLines;
    const bool pin = p0 < len;  // both elements (len is even)
    const int64_t pc = pin ? p0 : len - 2;
    int64_t bl[kLines];
    double l0[kLines], l1[kLines];
    float2 mv[kLines];
    double2 yv[kLines];
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      bl[u] = b0 + u < nlines ? b0 + u : nlines - 1;
      l0[u] = 0.0;
      l1[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      mv[u] = *(const float2*)(a.M + bl[u] * a.ldm + pc);
      yv[u] = *(const double2*)(a.Y + bl[u] * a.ldy + pc);
    }
    for (int c = 0; c < r; ++c) {
      const double2 fa = *(const double2*)(Fa + (int64_t)c * ldfa + pc);
#pragma unroll
      for (int u = 0; u < kLines; ++u) {
        const double fb = Fb[(int64_t)c * ldfb + bl[u]];
        l0[u] = fma(fa.x, fb, l0[u]);
        l1[u] = fma(fa.y, fb, l1[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      const double m2[2] = {(double)mv[u].x, (double)mv[u].y};
      const double y2[2] = {yv[u].x, yv[u].y};
      const double lv[2] = {l0[u], l1[u]};
      double sv[2], yn[2], bn[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double x = m2[e] - lv[e] + y2[e] / a.mu;
        const double ax = fabs(x) - a.thresh;
        sv[e] = ax > 0.0 ? copysign(ax, x) : 0.0;
        const double z = m2[e] - lv[e] - sv[e];
        yn[e] = y2[e] + a.mu * z;
        bn[e] = m2[e] - sv[e] + yn[e] / a.mu_next;
        if (pin && b0 + u < nlines) z2 += z * z;
      }
      if (pin && b0 + u < nlines) {
        const int64_t off = bl[u] * a.lds + p0;  // S, L share M's layout here
        *(float2*)(a.S + off) = make_float2((float)sv[0], (float)sv[1]);
        *(double2*)(a.Y + bl[u] * a.ldy + p0) = make_double2(yn[0], yn[1]);
        if (a.B) *(double2*)(a.B + bl[u] * a.ldb + p0) = make_double2(bn[0], bn[1]);
        if (a.L) *(float2*)(a.L + bl[u] * a.ldl + p0) = make_float2((float)lv[0], (float)lv[1]);
      }
    }
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
                                   double* part, const int* status, int nstatus, int* sticky,
                                   int* rank_out, hipStream_t st) {
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
  a.st = status;
  a.nst = nstatus;
  a.sticky = sticky;
  a.rank_out = rank_out;
  // the paired form: even lines, even leading dimensions, aligned bases, S
  // and L stored like M
  const int64_t len = lay_m == CORUTV_COL_MAJOR ? m : n;
  auto al = [](const void* p, int b) { return p == nullptr || ((uintptr_t)p % b) == 0; };
  const bool pair = len % 2 == 0 && ldm % 2 == 0 && lds % 2 == 0 && ldy % 2 == 0 && ldb % 2 == 0 &&
                    (L == nullptr || (ldl % 2 == 0 && lay_l == lay_m)) && lay_s == lay_m && al(M, 8) &&
                    al(S, 8) && al(L, 8) && al(Y, 16) && al(B, 16) && ldp % 2 == 0 && ldq % 2 == 0 &&
                    al(lay_m == CORUTV_COL_MAJOR ? (const void*)P : (const void*)Q, 16);
  if (pair)
    rpca_step2_kernel<<<dim3(kRpcaBlocks), dim3(256), 0, st>>>(a);
  else
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
