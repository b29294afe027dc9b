// Passes over the dense matrix A (Sec. 3.1 eqs. 4, 5, 7; Algorithm 1 power
// loop): Y = A W (m x n times n x l) and Z = A^T Q (n x m times m x l), the
// O(mnl) part of CoR-UTV.  The paper counts 2mnl flops per product and 2q+3
// passes over A (Sec. 3.2); each pass here streams A from HBM exactly once.
//
// Design (MI355X / gfx950):
//  * A is row-major R x C with leading dimension lda (a column-major matrix is
//    the row-major view of its transpose, so both orientations reduce to the
//    two kernels below: trans = 0 contracts over C, trans = 1 over R).
//  * MFMA 16x16x4 (FP32 or FP64).  The matrix-core A operand is the skinny
//    matrix (l rows, staged in LDS, shared by the four waves of a workgroup);
//    the B operand is A itself, loaded straight from HBM into registers with
//    16-byte vector loads (each element of A is used by exactly one lane).
//    The k index of each MFMA step is permuted so that a lane's four
//    consecutive k values come from one contiguous vector load.
//  * Output tile: all l (padded to 16) sketch columns x TW output rows, so A
//    is read once per pass.
//  * Work split: stream-K.  The reduction range is cut into 8 chunks, one per
//    XCD (workgroup w runs on XCD w mod 8), so each XCD's L2 holds only its
//    1/8 of the skinny operand; inside a chunk the (tile, k-block) units are
//    divided evenly over a persistent grid, so every CU gets the same work.
//    A skinny operand of at most 1 MB fits every L2 whole: the reduction is
//    then one chunk over the whole grid, and an output tile gathers about
//    8 g / tiles + 1 partial tiles instead of 8 (g / tiles + 1).
//    Each workgroup writes one partial tile per output tile it touches; the
//    consumer kernel sums them in a fixed order, so results are
//    deterministic (no atomics).  An FP64 pass over a short reduction (one
//    chunk) whose output has at least one tile per CU instead gives each
//    workgroup one whole tile, written straight to the output.
#include <algorithm>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace corutv {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mma;
template <>
struct Mma<float> {
  using acc = f4;
  using v16 = f4;  // 16-byte vector
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<double> {
  using acc = d4;
  using v16 = d2;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

struct SketchArgs {
  const void* A;
  int64_t lda;
  int64_t N;  // output length (rows of Y / Z)
  int64_t K;  // reduction length
  const void* S;
  const void* S2;  // bf16 forms: the lo parts of the pre-split skinny operand
  int64_t lds;
  void* P;
  int tiles, nk, nkx, gx, maxslot, nchunk;
  double* out;  // direct output (one whole tile per workgroup), or null
  int64_t ldo;
  int ell;      // columns of out that take the sums (the rest of ELLP: zero)
};

// VEC: A rows 16-byte aligned (address and leading dimension), so vector
// loads are allowed.  A template argument, not a runtime flag: a runtime
// branch between the two load paths costs the compiler its exact count of
// outstanding loads, and it then waits for more of them than needed.
// WG waves per workgroup; they share each staged block of the skinny operand,
// so a workgroup covers 16 NB WG output rows per tile.
template <typename T, int MB, bool TRANS, int NB, bool VEC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (MB <= 8 ? 3 : 2) : (MB <= 8 ? 2 : 1)))) sketch_kernel(SketchArgs a) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  using v16 = typename M::v16;
  constexpr int E16 = 16 / sizeof(T);   // elements per 16-byte vector
  constexpr int KC = 128 / sizeof(T);   // k values per LDS stage
  constexpr int KG = KC / 16;           // 16-k MFMA groups per stage
  constexpr int ELLP = MB * 16;
  constexpr int LDK = KC + E16;         // LDS row stride (one vector of pad)
  constexpr int TW = 16 * NB * WG;      // output rows per workgroup tile
  constexpr int NT = 64 * WG;           // threads
  constexpr int VPR = KC / E16;         // vectors per skinny row per stage
  constexpr int SPASS = (ELLP * VPR + NT - 1) / NT;
  // staged rows: every thread stores all SPASS of its vectors (rows past
  // ELLP are never read), so no store waits under a per-lane branch
  constexpr int ELLS = SPASS * NT / VPR;
  // two-buffer stage pipeline, except in the wide FP32 kernels
  constexpr bool kPipe2 = sizeof(T) == 8 || MB <= 8;
  // direct output (one whole tile per workgroup) in the narrow FP64 kernels
  // only: the others have no registers to spare for it
  constexpr bool kDirect = sizeof(T) == 8 && MB <= 8;
  __shared__ __attribute__((aligned(16))) T lds_s[2][ELLS * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, qd = lane & 15;
  const int x = blockIdx.x % a.nchunk;  // K chunk (chunk x on XCD x when there are 8)
  const int jw = blockIdx.x / a.nchunk;
  const T* __restrict__ A = (const T*)a.A;
  const T* __restrict__ S = (const T*)a.S;
  T* __restrict__ P = (T*)a.P;
  const int64_t U = (int64_t)a.tiles * a.nkx;
  int64_t u = (int64_t)jw * U / a.gx;
  const int64_t uend = (int64_t)(jw + 1) * U / a.gx;
  const int tfirst = (int)(u / a.nkx);
  int iter = 0;  // LDS buffer parity, continuous across tiles

  while (u < uend) {
    const int t = (int)(u / a.nkx);
    const int kb0 = (int)(u % a.nkx);
    const int kb1 = (int)min((int64_t)a.nkx, kb0 + (uend - u));
    const int gk0 = x * a.nkx + kb0;
    const int gk1 = min(x * a.nkx + kb1, a.nk);
    const int64_t nbase = (int64_t)t * TW + wave * 16 * NB;

    acc_t acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = acc_t{0, 0, 0, 0};

    if (gk0 < gk1) {
      v16 sreg[SPASS];
      // B operand registers: N-pass [nb][h][4], T-pass [h][tt][nb]

      // All loads below are unconditional, from addresses clamped into the
      // valid range, with out-of-range elements zeroed by selects afterwards:
      // loads under per-lane branches defeat the compiler's tracking of
      // outstanding loads and serialize the prefetch.
      auto load_skinny = [&](int kb) {
        // the skinny operand has at least ELLP rows and lds >= the k extent
        // of the last chunk, with zero padding (library-internal buffers)
#pragma unroll
        for (int p = 0; p < SPASS; ++p) {
          const int v = tid + NT * p;
          const int c = min(v / VPR, ELLP - 1), kv = v % VPR;
          sreg[p] = *(const v16*)(S + (int64_t)c * a.lds + (int64_t)kb * KC + kv * E16);
        }
      };
      auto store_skinny = [&](int buf) {
#pragma unroll
        for (int p = 0; p < SPASS; ++p) {
          const int v = tid + NT * p;
          const int c = v / VPR, kv = v % VPR;
          *(v16*)&lds_s[buf][c * LDK + kv * E16] = sreg[p];
        }
      };
      // raw loads from clamped addresses.  Only the last k-block of the
      // reduction reaches past K (zero_tail clears those elements); rows past
      // N give output rows that are never read.
      auto load_b = [&](int kb, T* b) {
        if constexpr (!TRANS) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int64_t n = nbase + nb * 16 + qd;
            const bool nok = n < a.N;
            const int64_t nc = nok ? n : a.N - 1;
#pragma unroll
            for (int h = 0; h < KG; ++h) {
              const int64_t k = (int64_t)kb * KC + 16 * h + 4 * g;
              T* d = b + (nb * KG + h) * 4;
              if constexpr (VEC) {
                // rows are 16-byte aligned and K (the row length) is a
                // multiple of 4, so the 4-vector at k < K stays in the row
                const T* src = A + nc * a.lda + (k < a.K ? k : 0);
                if constexpr (sizeof(T) == 4) {
                  const f4 vv = *(const f4*)src;
                  d[0] = vv[0]; d[1] = vv[1]; d[2] = vv[2]; d[3] = vv[3];
                } else {
                  const d2 v0 = *(const d2*)src;
                  const d2 v1 = *(const d2*)(src + 2);
                  d[0] = v0[0]; d[1] = v0[1]; d[2] = v1[0]; d[3] = v1[1];
                }
              } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) d[e] = A[nc * a.lda + (k + e < a.K ? k + e : 0)];
              }
            }
          }
        } else {
#pragma unroll
          for (int h = 0; h < KG; ++h)
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              const int64_t k = (int64_t)kb * KC + 16 * h + 4 * g + tt;
              const bool kok = k < a.K;
              const int64_t kc = kok ? k : a.K - 1;
              const int64_t n0 = nbase + NB * qd;
              T* d = b + (h * 4 + tt) * NB;
              if constexpr (NB == 2 && VEC) {
                // n0 is even and N (the row length) a multiple of 4: the
                // pair at n0 < N stays in the row
                const T* src = A + kc * a.lda + (n0 < a.N ? n0 : 0);
                if constexpr (sizeof(T) == 4) {
                  const f2 vv = *(const f2*)src;
                  d[0] = vv[0]; d[NB - 1] = vv[1];
                } else {
                  const d2 vv = *(const d2*)src;
                  d[0] = vv[0]; d[NB - 1] = vv[1];
                }
              } else {
#pragma unroll
                for (int e = 0; e < NB; ++e) d[e] = A[kc * a.lda + (n0 + e < a.N ? n0 + e : 0)];
              }
            }
        }
      };

      auto zero_tail = [&](int kb, T* b) {
#pragma unroll
        for (int h = 0; h < KG; ++h)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = (int64_t)kb * KC + 16 * h + 4 * g + e < a.K;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              T& v = TRANS ? b[(h * 4 + e) * NB + nb] : b[(nb * KG + h) * 4 + e];
              v = ok ? v : T(0);
            }
          }
      };

      // products of one stage of A (bc) with the staged skinny block buf
      auto products = [&](const T* bc, int buf) {
        const T* ls = &lds_s[buf][0];
#pragma unroll
        for (int h = 0; h < KG; ++h) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            // one block row of the skinny operand at a time keeps few
            // registers live (the products of different rows are independent)
            T sf[4];
            const T* src = ls + (mb * 16 + qd) * LDK + 16 * h + 4 * g;
            if constexpr (sizeof(T) == 4) {
              const f4 vv = *(const f4*)src;
              sf[0] = vv[0]; sf[1] = vv[1]; sf[2] = vv[2]; sf[3] = vv[3];
            } else {
              const d2 v0 = *(const d2*)src;
              const d2 v1 = *(const d2*)(src + 2);
              sf[0] = v0[0]; sf[1] = v0[1]; sf[2] = v1[0]; sf[3] = v1[1];
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) {
                const T bv = TRANS ? bc[(h * 4 + tt) * NB + nb] : bc[(nb * KG + h) * 4 + tt];
                acc[mb][nb] = M::op(sf[tt], bv, acc[mb][nb]);
              }
          }
        }
      };
      if constexpr (kPipe2) {
        // two A buffers alternating by stage parity (the stage is written
        // twice), so no register copy waits for a load in flight; the next
        // stage's skinny block is loaded ahead of the products
        T ba[NB * KG * 4], bb[NB * KG * 4];
        load_skinny(gk0);
        load_b(gk0, ba);
        auto stage = [&](int kb, T* bc, T* bn) {
          const int buf = iter & 1;
          store_skinny(buf);
          if (kb == a.nk - 1) zero_tail(kb, bc);
          __syncthreads();
          // prefetch the next chunk (the last chunk reloads itself: harmless)
          const int kn = kb + 1 < gk1 ? kb + 1 : kb;
          load_skinny(kn);
          load_b(kn, bn);
          __builtin_amdgcn_sched_barrier(0);
          products(bc, buf);
          // the next stage's stores wait for the loads just issued: keep
          // them behind these products
          __builtin_amdgcn_sched_barrier(0);
          ++iter;
        };
        // pairs of stages with no branch between them (a load whose only
        // use sits behind a branch is moved down to it and then waited for)
        int kb = gk0;
        for (; kb + 1 < gk1; kb += 2) {
          stage(kb, ba, bb);
          stage(kb + 1, bb, ba);
        }
        if (kb < gk1) stage(kb, ba, bb);
      } else {
        // the wide FP32 kernels (8 waves, up to 256 sketch columns): one A
        // buffer copied forward, which their registers allow
        T bcur[NB * KG * 4], bnext[NB * KG * 4];
        load_skinny(gk0);
        load_b(gk0, bcur);
        for (int kb = gk0; kb < gk1; ++kb, ++iter) {
          const int buf = iter & 1;
          store_skinny(buf);
          if (kb == a.nk - 1) zero_tail(kb, bcur);
          __syncthreads();
          const int kn = kb + 1 < gk1 ? kb + 1 : kb;
          load_skinny(kn);
          load_b(kn, bnext);
          __builtin_amdgcn_sched_barrier(0);
          products(bcur, buf);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < NB * KG * 4; ++e) bcur[e] = bnext[e];
        }
      }
    }

    if (kDirect && a.out) {
      // the whole reduction of this tile: straight to the output (lane
      // base: row n0, column g (FP64) or 4g (FP32); then uniform offsets)
      const int64_t n0 = (int64_t)t * TW + wave * 16 * NB + (TRANS ? NB * qd : qd);
      const int cg = sizeof(T) == 4 ? 4 * g : g;
      double* ob = a.out + (int64_t)cg * a.ldo + n0;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int dc = mb * 16 + (sizeof(T) == 4 ? i : 4 * i);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int dn = TRANS ? nb : nb * 16;
            if (n0 + dn < a.N) ob[(int64_t)dc * a.ldo + dn] = cg + dc < a.ell ? (double)acc[mb][nb][i] : 0.0;
          }
        }
    } else {
      // partial tile (x, jw, t - tfirst): [ELLP][TW]
      const int64_t slot = ((int64_t)x * a.gx + jw) * a.maxslot + (t - tfirst);
      T* dst = P + slot * (int64_t)ELLP * TW;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // accumulator slot i of lane (g, qd) holds row 4g + i of the 16 x 16
          // block for the FP32 instruction and row g + 4i for the FP64 one
          const int c = mb * 16 + (sizeof(T) == 4 ? 4 * g + i : g + 4 * i);
          if constexpr (!TRANS) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) dst[(int64_t)c * TW + wave * 16 * NB + nb * 16 + qd] = acc[mb][nb][i];
          } else {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) dst[(int64_t)c * TW + wave * 16 * NB + NB * qd + nb] = acc[mb][nb][i];
          }
        }
    }
    u += kb1 - kb0;
  }
}

// ---------------------------------------------------------------------------
// Reduced-precision forms (float A and operands): BF16 rounds both operands to
// nearest-even bfloat16 in the loader; BF16X3 splits x = hi + lo (hi =
// bf16(x), lo = bf16(x - hi)) and accumulates lo*hi + hi*lo + hi*hi, small
// terms first.  FP32 accumulation on v_mfma_f32_16x16x32_bf16: lane (g, qd)
// supplies k = 8g..8g+7 of a 32-k block for row qd of the skinny operand and
// for output row qd of A; accumulator slot i holds row 4g + i.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(const float* x, bf8& hi, bf8& lo, bool want_lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    if (want_lo) lo[e] = (__bf16)(x[e] - (float)h);
  }
}

// The skinny operand arrives pre-split into bf16 hi (S) and lo (S2) parts
// (split_bf16_kernel, same rounding), so it is staged into LDS as bf16 and
// fed to the matrix cores without per-wave conversion.
template <int MB, bool TRANS, int NB, bool X3, bool VEC, int WG>
__global__ void __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(MB > 8 ? 2 : 1))) sketch_bf16_kernel(SketchArgs a) {
  // k values per LDS stage: two MFMA blocks for BF16 up to 128 sketch columns
  // (more bytes of A in flight per stage); one for BF16X3 and for wider
  // sketches, whose registers allow no more
  constexpr int KC = (X3 || MB > 8) ? 32 : 64;
  constexpr int KB = KC / 32;            // MFMA blocks per stage
  constexpr int ELLP = MB * 16;
  constexpr int LDKB = KC + 8;           // LDS row stride in bf16 (16 bytes of pad)
  constexpr int TW = 16 * NB * WG;
  constexpr int NT = 64 * WG;
  constexpr int VPR = KC / 8;            // 16-byte vectors per skinny row per stage
  constexpr int SPASS = (ELLP * VPR + NT - 1) / NT;
  constexpr int ELLS = SPASS * NT / VPR;  // staged rows (past ELLP never read)
  constexpr int NPART = X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) __bf16 lds_s[NPART][2][ELLS * LDKB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, qd = lane & 15;
  const int x = blockIdx.x % a.nchunk;  // K chunk (chunk x on XCD x when there are 8)
  const int jw = blockIdx.x / a.nchunk;
  const float* __restrict__ A = (const float*)a.A;
  const __bf16* __restrict__ Sp[2] = {(const __bf16*)a.S, (const __bf16*)a.S2};
  float* __restrict__ P = (float*)a.P;
  const int64_t U = (int64_t)a.tiles * a.nkx;
  int64_t u = (int64_t)jw * U / a.gx;
  const int64_t uend = (int64_t)(jw + 1) * U / a.gx;
  const int tfirst = (int)(u / a.nkx);
  int iter = 0;

  while (u < uend) {
    const int t = (int)(u / a.nkx);
    const int kb0 = (int)(u % a.nkx);
    const int kb1 = (int)min((int64_t)a.nkx, kb0 + (uend - u));
    const int gk0 = x * a.nkx + kb0;
    const int gk1 = min(x * a.nkx + kb1, a.nk);
    const int64_t nbase = (int64_t)t * TW + wave * 16 * NB;
    f4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};

    if (gk0 < gk1) {
      f4 sreg[NPART][SPASS];  // raw 16-byte vectors of 8 bf16
      float bcur[NB * KB * 8];  // [nb][block][8 k values]
      // unconditional loads from clamped addresses; validity bits applied
      // when the prefetched chunk becomes current (see the FP32/FP64 kernel)
      auto load_skinny = [&](int kb) {
#pragma unroll
        for (int h = 0; h < NPART; ++h)
#pragma unroll
          for (int p = 0; p < SPASS; ++p) {
            const int v = tid + NT * p;
            const int c = min(v / VPR, ELLP - 1), kv = v % VPR;
            sreg[h][p] = *(const f4*)(Sp[h] + (int64_t)c * a.lds + (int64_t)kb * KC + kv * 8);
          }
      };
      auto store_skinny = [&](int buf) {
#pragma unroll
        for (int h = 0; h < NPART; ++h)
#pragma unroll
          for (int p = 0; p < SPASS; ++p) {
            const int v = tid + NT * p;
            const int c = v / VPR, kv = v % VPR;
            *(f4*)&lds_s[h][buf][c * LDKB + kv * 8] = sreg[h][p];
          }
      };
      // raw loads from clamped addresses; only the last k-block of the
      // reduction reaches past K (zero_tail), rows past N give output rows
      // that are never read
      auto load_b = [&](int kb, float* b) {
        if constexpr (!TRANS) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int64_t n = nbase + nb * 16 + qd;
            const int64_t nc = n < a.N ? n : a.N - 1;
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
              const int64_t k = (int64_t)kb * KC + 32 * kk + 8 * g;
              float* d = b + (nb * KB + kk) * 8;
              if constexpr (VEC) {
                // K is a multiple of 4: both 4-vectors at k < K stay in the row
                const float* src = A + nc * a.lda + (k < a.K ? k : 0);
                const f4 v0 = *(const f4*)src;
                const int64_t k2 = k + 4 < a.K ? k + 4 : (k < a.K ? k : 0);
                const f4 v1 = *(const f4*)(A + nc * a.lda + k2);
                d[0] = v0[0]; d[1] = v0[1]; d[2] = v0[2]; d[3] = v0[3];
                d[4] = v1[0]; d[5] = v1[1]; d[6] = v1[2]; d[7] = v1[3];
              } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) d[e] = A[nc * a.lda + (k + e < a.K ? k + e : 0)];
              }
            }
          }
        } else {
#pragma unroll
          for (int kk = 0; kk < KB; ++kk)
#pragma unroll
            for (int tt = 0; tt < 8; ++tt) {
              const int64_t k = (int64_t)kb * KC + 32 * kk + 8 * g + tt;
              const int64_t kc = k < a.K ? k : a.K - 1;
              const int64_t n0 = nbase + NB * qd;
              if constexpr (NB == 2 && VEC) {
                const f2 vv = *(const f2*)(A + kc * a.lda + (n0 < a.N ? n0 : 0));
                b[kk * 8 + tt] = vv[0];
                b[(KB + kk) * 8 + tt] = vv[1];
              } else {
#pragma unroll
                for (int e = 0; e < NB; ++e) b[(e * KB + kk) * 8 + tt] = A[kc * a.lda + (n0 + e < a.N ? n0 + e : 0)];
              }
            }
        }
      };

      auto zero_tail = [&](int kb, float* b) {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const bool ok = (int64_t)kb * KC + 32 * kk + 8 * g + e < a.K;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              float& v = b[(nb * KB + kk) * 8 + e];
              v = ok ? v : 0.f;
            }
          }
      };
      // products of one stage of A (bc) with the staged skinny block buf
      auto products = [&](const float* bc, int buf) {
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          bf8 bh[NB], bl[NB];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) split8(bc + (nb * KB + kk) * 8, bh[nb], bl[nb], X3);
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const int off = (mb * 16 + qd) * LDKB + 32 * kk + 8 * g;
            const bf8 sh = *(const bf8*)&lds_s[0][buf][off];
            bf8 sl;
            if constexpr (X3) sl = *(const bf8*)&lds_s[NPART - 1][buf][off];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              if constexpr (X3) {
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl, bh[nb], acc[mb][nb], 0, 0, 0);
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, bl[nb], acc[mb][nb], 0, 0, 0);
              }
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, bh[nb], acc[mb][nb], 0, 0, 0);
            }
          }
        }
      };
      load_skinny(gk0);
      if constexpr (MB > 8 && !X3) {
        // wide sketches in plain BF16 (one 32-k block per stage): two stages
        // of A in flight (measured slower for BF16X3, whose products fill
        // the time the second stage would cover).
        // The two prefetch buffers alternate by stage parity (the loop body
        // is written twice), so no register copy waits for a load in flight.
        float bna[NB * KB * 8], bnb[NB * KB * 8];
        load_b(gk0, bcur);
        load_b(gk0 + 1 < gk1 ? gk0 + 1 : gk1 - 1, bna);
        load_b(gk0 + 2 < gk1 ? gk0 + 2 : gk1 - 1, bnb);
        auto body = [&](int kb, float* bnx) {
          const int buf = iter & 1;
          store_skinny(buf);
          if (kb == a.nk - 1) zero_tail(kb, bcur);
          __syncthreads();
          load_skinny(kb + 1 < gk1 ? kb + 1 : kb);
          __builtin_amdgcn_sched_barrier(0);
          products(bcur, buf);
#pragma unroll
          for (int e = 0; e < NB * KB * 8; ++e) bcur[e] = bnx[e];
          load_b(kb + 3 < gk1 ? kb + 3 : gk1 - 1, bnx);
          // the next body's stores wait for the skinny loads issued above:
          // keep them behind this body's work
          __builtin_amdgcn_sched_barrier(0);
          ++iter;
        };
        // pairs of bodies with no branch between them (a load whose only use
        // sits behind a branch is moved down to it and then waited for)
        int kb = gk0;
        for (; kb + 1 < gk1; kb += 2) {
          body(kb, bna);
          body(kb + 1, bnb);
        }
        if (kb < gk1) body(kb, bna);
      } else {
        // DEPTH A buffers in rotation (the stage is written DEPTH times), so
        // no register copy waits for a load in flight; the A loads run
        // DEPTH - 1 stages ahead, issued ahead of the products, and nothing
        // waits for them before their own stage (a third buffer, loads two
        // stages ahead, measured no faster for plain BF16 at 112 columns)
        constexpr int DEPTH = 2;
        float bq[DEPTH][NB * KB * 8];
#pragma unroll
        for (int d = 0; d < DEPTH - 1; ++d) load_b(gk0 + d < gk1 ? gk0 + d : gk1 - 1, bq[d]);
        auto stage = [&](int kb, float* bc, float* bn) {
          const int buf = iter & 1;
          store_skinny(buf);
          if (kb == a.nk - 1) zero_tail(kb, bc);
          __syncthreads();
          const int kn = kb + 1 < gk1 ? kb + 1 : kb;
          load_skinny(kn);
          load_b(kb + DEPTH - 1 < gk1 ? kb + DEPTH - 1 : gk1 - 1, bn);
          __builtin_amdgcn_sched_barrier(0);
          products(bc, buf);
          __builtin_amdgcn_sched_barrier(0);
          ++iter;
        };
        int kb = gk0;
        for (; kb + DEPTH - 1 < gk1; kb += DEPTH) {
#pragma unroll
          for (int d = 0; d < DEPTH; ++d) stage(kb + d, bq[d], bq[(d + DEPTH - 1) % DEPTH]);
        }
#pragma unroll
        for (int d = 0; d < DEPTH - 1; ++d)
          if (kb + d < gk1) stage(kb + d, bq[d], bq[(d + DEPTH - 1) % DEPTH]);
      }
    }
    {
      const int64_t slot = ((int64_t)x * a.gx + jw) * a.maxslot + (t - tfirst);
      float* dst = P + slot * (int64_t)ELLP * TW;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = mb * 16 + 4 * g + i;
          if constexpr (!TRANS) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) dst[(int64_t)c * TW + wave * 16 * NB + nb * 16 + qd] = acc[mb][nb][i];
          } else {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) dst[(int64_t)c * TW + wave * 16 * NB + NB * qd + nb] = acc[mb][nb][i];
          }
        }
    }
    u += kb1 - kb0;
  }
}

// bf16 hi/lo split of the skinny operand (same rounding as split8)
__global__ void split_bf16_kernel(const float* __restrict__ S, int64_t n, __bf16* __restrict__ H,
                                  __bf16* __restrict__ L, int x3) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float v = S[e];
    const __bf16 h = (__bf16)v;
    H[e] = h;
    if (x3) L[e] = (__bf16)(v - (float)h);
  }
}

// Waves per workgroup of each pass kernel: eight (256 output rows sharing one
// staged skinny block, half the skinny operand's L2 reads per byte of A) where
// two waves per SIMD is the register limit anyway; four where the FP32 kernel
// runs three waves per SIMD or the FP64 kernel needs one SIMD's registers per
// wave.
constexpr int wg_for(int prec, int mb) {
  return prec == P_F64 ? 4 : (prec == P_F32 ? (mb > 8 ? 8 : 4) : 8);
}

template <int MB, bool TRANS, bool X3, bool VEC>
void* bf16_ptr() {
  constexpr int NB = 2;
  return (void*)&sketch_bf16_kernel<MB, TRANS, NB, X3, VEC, wg_for(P_BF16, MB)>;
}

template <bool TRANS, bool X3, bool VEC>
void* pick_bf16(int mb) {
  switch (mb) {
    case 1: return bf16_ptr<1, TRANS, X3, VEC>();
    case 2: return bf16_ptr<2, TRANS, X3, VEC>();
    case 3: return bf16_ptr<3, TRANS, X3, VEC>();
    case 4: return bf16_ptr<4, TRANS, X3, VEC>();
    case 5: return bf16_ptr<5, TRANS, X3, VEC>();
    case 6: return bf16_ptr<6, TRANS, X3, VEC>();
    case 7: return bf16_ptr<7, TRANS, X3, VEC>();
    case 8: return bf16_ptr<8, TRANS, X3, VEC>();
    case 9: return bf16_ptr<9, TRANS, X3, VEC>();
    case 10: return bf16_ptr<10, TRANS, X3, VEC>();
    case 11: return bf16_ptr<11, TRANS, X3, VEC>();
    case 12: return bf16_ptr<12, TRANS, X3, VEC>();
    case 13: return bf16_ptr<13, TRANS, X3, VEC>();
    case 14: return bf16_ptr<14, TRANS, X3, VEC>();
    case 15: return bf16_ptr<15, TRANS, X3, VEC>();
    case 16: return bf16_ptr<16, TRANS, X3, VEC>();
    default: return nullptr;
  }
}

template <typename T, int MB, bool TRANS, bool VEC>
void* kernel_ptr() {
  constexpr int NB = 2;
  return (void*)&sketch_kernel<T, MB, TRANS, NB, VEC, wg_for(sizeof(T) == 8 ? P_F64 : P_F32, MB)>;
}

template <typename T, bool TRANS, bool VEC>
void* pick(int mb) {
  switch (mb) {
    case 1: return kernel_ptr<T, 1, TRANS, VEC>();
    case 2: return kernel_ptr<T, 2, TRANS, VEC>();
    case 3: return kernel_ptr<T, 3, TRANS, VEC>();
    case 4: return kernel_ptr<T, 4, TRANS, VEC>();
    case 5: return kernel_ptr<T, 5, TRANS, VEC>();
    case 6: return kernel_ptr<T, 6, TRANS, VEC>();
    case 7: return kernel_ptr<T, 7, TRANS, VEC>();
    case 8: return kernel_ptr<T, 8, TRANS, VEC>();
    case 9: return kernel_ptr<T, 9, TRANS, VEC>();
    case 10: return kernel_ptr<T, 10, TRANS, VEC>();
    case 11: return kernel_ptr<T, 11, TRANS, VEC>();
    case 12: return kernel_ptr<T, 12, TRANS, VEC>();
    case 13: return kernel_ptr<T, 13, TRANS, VEC>();
    case 14: return kernel_ptr<T, 14, TRANS, VEC>();
    case 15: return kernel_ptr<T, 15, TRANS, VEC>();
    case 16: return kernel_ptr<T, 16, TRANS, VEC>();
    default: return nullptr;
  }
}

// Workgroups per CU to use (occupancy reported by the runtime, capped).
constexpr int kOccCap = 4;

// cached per kernel: the runtime query costs host time on every launch
std::mutex g_occ_mu;
std::map<void*, int> g_occ;

int occupancy_of(void* fn, int threads) {
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    auto it = g_occ.find(fn);
    if (it != g_occ.end()) return it->second;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)fn, threads, 0) != hipSuccess)
    occ = 1;
  if (occ < 1) occ = 1;
  occ = occ < kOccCap ? occ : kOccCap;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  g_occ[fn] = occ;
  return occ;
}

// k values per stage of each kernel family
int kc_of(int prec, int mb) { return prec == P_F64 ? 16 : (prec == P_BF16 && mb <= 8 ? 64 : 32); }

constexpr int64_t kOneChunkBytes = 1 << 20;
constexpr int kMinUnits = 16;

// gx: workgroups per XCD (the grid is 8 gx)
void geometry(int64_t N, int64_t K, int ellp, int elem, int kc, int gx, int wg, Partials* p) {
  const int nb = 2;
  const int tw = 16 * nb * wg;
  p->ellp = ellp;
  p->tw = tw;
  p->elem = elem;
  p->n = N;
  p->tiles = (int)((N + tw - 1) / tw);
  const int64_t nk = (K + kc - 1) / kc;
  // a skinny operand that fits every XCD's L2 whole needs no split by XCD
  p->nchunk = K * ellp * elem <= kOneChunkBytes ? 1 : 8;
  p->nkx = (int)((nk + p->nchunk - 1) / p->nchunk);
  if (p->nkx < 1) p->nkx = 1;
  gx = gx * 8 / p->nchunk;  // workgroups per chunk (the grid is nchunk gx)
  const int64_t U = (int64_t)p->tiles * p->nkx;
  // a small pass keeps at least kMinUnits (tile, k-block) units per
  // workgroup: fewer workgroups, and so fewer partial tiles to write and sum
  if (U < (int64_t)gx * kMinUnits) gx = (int)std::max<int64_t>(1, U / kMinUnits);
  p->gx = gx;
  int ms = 1;
  for (int j = 0; j < gx; ++j) {
    const int64_t u0 = (int64_t)j * U / gx, u1 = (int64_t)(j + 1) * U / gx;
    if (u1 <= u0) continue;
    const int s = (int)((u1 - 1) / p->nkx - u0 / p->nkx) + 1;
    if (s > ms) ms = s;
  }
  p->maxslot = ms;
}

}  // namespace

static int64_t need_elems(const Partials& p) {
  return (int64_t)p.nchunk * p.gx * p.maxslot * (int64_t)p.ellp * p.tw;
}

int64_t partials_capacity(int64_t n_out, int64_t k_len, int ellp, int prec) {
  // prec P_F32 stands for every float form (F32 and the bf16 ones)
  int64_t best = 0;
  const int elem = prec == P_F64 ? 8 : 4;
  // every stage depth and workgroup size of the float kernels (a cover)
  const int kcs[3] = {16, 32, 64}, wgs[2] = {4, 8};
  for (int v = 0; v < 3; ++v)
    for (int w = 0; w < 2; ++w) {
      if (prec == P_F64 && (kcs[v] != 16 || wgs[w] != 4)) continue;
      if (prec != P_F64 && kcs[v] == 16) continue;
      for (int occ = 1; occ <= kOccCap; ++occ) {
        Partials p;
        geometry(n_out, k_len, ellp, elem, kcs[v], 32 * occ, wgs[w], &p);
        const int64_t e = need_elems(p);
        if (e > best) best = e;
      }
    }
  return best;
}

hipError_t launch_sketch(int prec, int trans, const void* A, int64_t lda, int64_t R, int64_t C,
                         const void* S, int64_t lds, int ellp, void* part_buf, int64_t part_elems,
                         Partials* part, int num_cu, hipStream_t st, void* sbf, double* out, int64_t ldo,
                         int ell) {
  const bool f64 = prec == P_F64;
  const int mb = ellp / 16;
  const int elem = f64 ? 8 : 4;
  // Vector loads read whole 16-byte groups (4 floats, or 2 + 2 doubles) from
  // a clamped start inside the row: a row length that is a multiple of 4
  // keeps the last group of the last row inside the matrix.
  const bool vec = (((uintptr_t)A) % 16 == 0) && ((lda * elem) % 16 == 0) && (C % 4 == 0);
  void* fn = nullptr;
  if (prec == P_F64)
    fn = vec ? (trans ? pick<double, true, true>(mb) : pick<double, false, true>(mb))
             : (trans ? pick<double, true, false>(mb) : pick<double, false, false>(mb));
  else if (prec == P_F32)
    fn = vec ? (trans ? pick<float, true, true>(mb) : pick<float, false, true>(mb))
             : (trans ? pick<float, true, false>(mb) : pick<float, false, false>(mb));
  else if (prec == P_BF16)
    fn = vec ? (trans ? pick_bf16<true, false, true>(mb) : pick_bf16<false, false, true>(mb))
             : (trans ? pick_bf16<true, false, false>(mb) : pick_bf16<false, false, false>(mb));
  else if (prec == P_BF16X3)
    fn = vec ? (trans ? pick_bf16<true, true, true>(mb) : pick_bf16<false, true, true>(mb))
             : (trans ? pick_bf16<true, true, false>(mb) : pick_bf16<false, true, false>(mb));
  if (!fn) return hipErrorInvalidValue;
  const int64_t N = trans ? C : R;
  const int64_t K = trans ? R : C;
  const int wg = wg_for(prec == P_F64 ? P_F64 : (prec == P_F32 ? P_F32 : P_BF16), mb);
  int gx = (num_cu / 8) * occupancy_of(fn, 64 * wg);
  if (gx < 1) gx = 1;
  const int kc = kc_of(prec, mb);
  geometry(N, K, ellp, elem, kc, gx, wg, part);
  // a short reduction over an output of many tiles: one whole tile per
  // workgroup, written straight to the output (no partial tiles to sum)
  const bool direct = out && f64 && mb <= 8 && part->nchunk == 1 && part->tiles >= num_cu;
  if (direct) {
    part->gx = part->tiles;
    part->maxslot = 1;
  } else {
    while (need_elems(*part) > part_elems && gx > 1) {
      gx = gx > 8 ? gx - 8 : gx - 1;
      geometry(N, K, ellp, elem, kc, gx, wg, part);
    }
    if (need_elems(*part) > part_elems) return hipErrorInvalidValue;
  }
  part->direct = direct;
  part->ptr = part_buf;
  SketchArgs a;
  a.A = A;
  a.lda = lda;
  a.N = N;
  a.K = K;
  a.S = S;
  a.S2 = nullptr;
  a.lds = lds;
  if (prec == P_BF16 || prec == P_BF16X3) {
    // split the float skinny operand (ellp rows of stride lds) into bf16
    if (!sbf) return hipErrorInvalidValue;
    const int64_t ne = (int64_t)ellp * lds;
    __bf16* H = (__bf16*)sbf;
    __bf16* L = H + ne;
    split_bf16_kernel<<<dim3(1024), dim3(256), 0, st>>>((const float*)S, ne, H, L, prec == P_BF16X3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.S = H;
    a.S2 = L;
  }
  a.P = part_buf;
  a.tiles = part->tiles;
  a.nk = (int)((K + kc - 1) / kc);
  a.nkx = part->nkx;
  a.nchunk = part->nchunk;
  a.gx = part->gx;
  a.maxslot = part->maxslot;
  a.out = direct ? out : nullptr;
  a.ldo = ldo;
  a.ell = ell;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)fn, dim3(part->nchunk * part->gx), dim3(64 * wg), args, 0, st);
}

}  // namespace corutv
