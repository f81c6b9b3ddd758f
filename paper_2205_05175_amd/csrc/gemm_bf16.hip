// Split-BF16 three-term MFMA GEMM on FP32 planar-complex / real operands (gfx950).
//
// Every FP32 operand element x is split while it is staged into LDS as hi = bf16(x) and
// lo = bf16(x - hi), and each real product is formed as hi*hi' + hi*lo' + lo*hi' with
// v_mfma_f32_16x16x32_bf16, accumulated in FP32 (the dropped lo*lo' term is ~2^-16 of the
// product). Operand tiles live in LDS as [row][k] with k contiguous so that each lane reads its
// eight consecutive k values of a fragment with one 16-byte load. Same operand descriptors and
// epilogue as the FP32 kernel; no split over K (used for the large products only).
#include <cstdint>

#include "engine.h"

namespace rtcc {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int kThr = 256;
constexpr int kBK = 32;           // one MFMA k-step
constexpr int kLDK = kBK + 8;     // padded LDS row (80 bytes)

struct Params {
  const float* Are;
  const float* Aim;
  int64_t lda;
  const float* Bre;
  const float* Bim;
  int64_t ldb;
  float* Cre;
  float* Cim;
  int64_t ldc;
  int M, N, K;
  float alpha, beta;
};

__device__ inline bf8 neg(bf8 x) {
  us8 u = __builtin_bit_cast(us8, x);
  u ^= (unsigned short)0x8000;
  return __builtin_bit_cast(bf8, u);
}

__device__ inline f4 mma(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// Register-staged FP32 tile: ROWS x COLS with COLS contiguous in memory.
template <int ROWS, int COLS, int NPL>
struct Regs {
  static constexpr int NV = ROWS * COLS / 4 / kThr;
  static_assert(NV >= 1 && NV * 4 * kThr == ROWS * COLS, "tile not divisible among threads");
  float r[NPL][NV][4];
  __device__ inline void load(const float* const* base, int64_t ld, bool vec, int row0, int col0, int rowLim,
                              int colLim, int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = v * kThr + tid;
      const int row = idx / (COLS / 4), col = (idx % (COLS / 4)) * 4;
      const int gr = row0 + row, gc = col0 + col;
      const int64_t off = (int64_t)gr * ld + gc;
      if (vec && gr < rowLim && gc + 4 <= colLim) {
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
          f4 x = *reinterpret_cast<const f4*>(base[pl] + off);
          r[pl][v][0] = x[0];
          r[pl][v][1] = x[1];
          r[pl][v][2] = x[2];
          r[pl][v][3] = x[3];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = gr < rowLim && gc + e < colLim;
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) r[pl][v][e] = ok ? base[pl][off + e] : 0.f;
        }
      }
    }
  }
  // S[pl][h][x][k]; ROWS_ARE_K: memory rows are k (else memory rows are x)
  template <bool ROWS_ARE_K, int XDIM>
  __device__ inline void store(__bf16* S, int tid) const {
    typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = v * kThr + tid;
      const int row = idx / (COLS / 4), col = (idx % (COLS / 4)) * 4;
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        bf4 hi, lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x = r[pl][v][e];
          hi[e] = (__bf16)x;
          lo[e] = (__bf16)(x - (float)hi[e]);
        }
        __bf16* base = S + (size_t)pl * 2 * XDIM * kLDK;
        if (!ROWS_ARE_K) {
          // four consecutive k of one row: one 8-byte store per half
          *reinterpret_cast<bf4*>(&base[row * kLDK + col]) = hi;
          *reinterpret_cast<bf4*>(&base[XDIM * kLDK + row * kLDK + col]) = lo;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            base[(col + e) * kLDK + row] = hi[e];
            base[XDIM * kLDK + (col + e) * kLDK + row] = lo[e];
          }
        }
      }
    }
  }
};

template <int BM, int BN, int AC, int BC, int TA, int TB>
__global__ __launch_bounds__(kThr) void gemm_bf16x3_kernel(Params p, int vec) {
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  __shared__ __attribute__((aligned(16))) __bf16 As[NA * 2 * BM * kLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NB * 2 * BN * kLDK];
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  f4 accr[FM][FN], acci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accr[i][j] = f4{0, 0, 0, 0};
      acci[i][j] = f4{0, 0, 0, 0};
    }
  const float* Ap[2] = {p.Are, p.Aim};
  const float* Bp[2] = {p.Bre, p.Bim};
  Regs<TA ? kBK : BM, TA ? BM : kBK, NA> ra;
  Regs<TB ? BN : kBK, TB ? kBK : BN, NB> rb;
  auto fetch = [&](int k0) {
    if (TA) ra.load(Ap, p.lda, vec, k0, m0, p.K, p.M, tid);
    else ra.load(Ap, p.lda, vec, m0, k0, p.M, p.K, tid);
    if (TB) rb.load(Bp, p.ldb, vec, n0, k0, p.N, p.K, tid);
    else rb.load(Bp, p.ldb, vec, k0, n0, p.K, p.N, tid);
  };
  fetch(0);
  const int g = lane >> 4, c16 = lane & 15;
  for (int k0 = 0; k0 < p.K; k0 += kBK) {
    ra.template store<TA != 0, BM>(As, tid);
    rb.template store<TB == 0, BN>(Bs, tid);
    __syncthreads();
    if (k0 + kBK < p.K) fetch(k0 + kBK);
    // all fragments of this wave (hi, lo for each plane), then term-major MFMA issue so that
    // consecutive MFMAs update different accumulators
    bf8 bfr[FN][NB][2], afr[FM][NA][2];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int pl = 0; pl < NB; ++pl)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          bfr[j][pl][h] = *reinterpret_cast<const bf8*>(
              &Bs[((pl * 2 + h) * BN + wn * WN + j * 16 + c16) * kLDK + 8 * g]);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int pl = 0; pl < NA; ++pl)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          afr[i][pl][h] = *reinterpret_cast<const bf8*>(
              &As[((pl * 2 + h) * BM + wm * WM + i * 16 + c16) * kLDK + 8 * g]);
    // (ha, hb): the three split products hi*hi, hi*lo, lo*hi
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int ha = t == 2 ? 1 : 0, hb = t == 1 ? 1 : 0;
      // Re(C) += Re(A) Re(B)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) accr[i][j] = mma(afr[i][0][ha], bfr[j][0][hb], accr[i][j]);
      // Im(C) += Re(A) Im(B)
      if (BC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acci[i][j] = mma(afr[i][0][ha], bfr[j][NB - 1][hb], acci[i][j]);
      }
      // Im(C) += Im(A) Re(B)
      if (AC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acci[i][j] = mma(afr[i][NA - 1][ha], bfr[j][0][hb], acci[i][j]);
      }
      // Re(C) -= Im(A) Im(B)
      if (AC && BC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accr[i][j] = mma(neg(afr[i][NA - 1][ha]), bfr[j][NB - 1][hb], accr[i][j]);
      }
    }
    __syncthreads();
  }

  constexpr bool CC = AC || BC;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + 4 * g + r;
        const int col = n0 + wn * WN + j * 16 + c16;
        if (row >= p.M || col >= p.N) continue;
        const int64_t off = (int64_t)row * p.ldc + col;
        float outr = p.alpha * accr[i][j][r], outi = p.alpha * acci[i][j][r];
        if (p.beta != 0.f) {
          outr += p.beta * p.Cre[off];
          if (CC) outi += p.beta * p.Cim[off];
        }
        p.Cre[off] = outr;
        if (CC) p.Cim[off] = outi;
      }
}

template <int BM, int BN, int AC, int BC>
void launch(hipStream_t st, const Params& p, int ta, int tb, int vec) {
  dim3 grid((unsigned)cdiv(p.N, BN), (unsigned)cdiv(p.M, BM));
  const int sel = ta * 2 + tb;
  switch (sel) {
    case 0: hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, BN, AC, BC, 0, 0>), grid, dim3(kThr), 0, st, p, vec); break;
    case 1: hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, BN, AC, BC, 0, 1>), grid, dim3(kThr), 0, st, p, vec); break;
    case 2: hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, BN, AC, BC, 1, 0>), grid, dim3(kThr), 0, st, p, vec); break;
    default: hipLaunchKernelGGL((gemm_bf16x3_kernel<BM, BN, AC, BC, 1, 1>), grid, dim3(kThr), 0, st, p, vec); break;
  }
  RTCC_HIP(hipGetLastError());
}

template <int BM, int BN>
void launch_typed(hipStream_t st, const Params& p, int ta, int tb, int vec) {
  const int sel = (p.Aim ? 2 : 0) + (p.Bim ? 1 : 0);
  switch (sel) {
    case 1: launch<BM, BN, 0, 1>(st, p, ta, tb, vec); break;
    case 2: launch<BM, BN, 1, 0>(st, p, ta, tb, vec); break;
    case 3: launch<BM, BN, 1, 1>(st, p, ta, tb, vec); break;
    default: launch<BM, BN, 0, 0>(st, p, ta, tb, vec); break;
  }
}

}  // namespace

// Returns false (nothing launched) for real x real products or a real output.
bool gemm_bf16x3(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<float> A, GemmOp<float> B,
                 float* Cre, float* Cim, int64_t ldc, double beta) {
  if (M <= 0 || N <= 0 || K <= 0) return false;
  const bool AC = A.im != nullptr, BC = B.im != nullptr;
  if (!Cim && (AC || BC)) return false;
  if (!AC && !BC) return false;
  Params p{A.re, A.im, A.ld, B.re, B.im, B.ld, Cre, Cim, ldc, (int)M, (int)N, (int)K, (float)alpha, (float)beta};
  auto al = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  const int vec = al(A.re) && (!AC || al(A.im)) && al(B.re) && (!BC || al(B.im)) && A.ld % 4 == 0 && B.ld % 4 == 0;
  // grids that cannot fill the chip go to the FP32 kernel, which can split over K (unless the
  // split is forced onto every product by a zero threshold)
  if (E.bf16_min_flops > 0 && cdiv(M, 64) * cdiv(N, 64) < 256) return false;
  // complex x complex products hold more fragments: narrower tiles
  const bool cc = AC && BC;
  const int64_t t128 = cdiv(M, 128) * cdiv(N, cc ? 64 : 128);
  if (t128 >= 384) {
    if (cc) launch_typed<128, 64>(E.stream, p, A.trans, B.trans, vec);
    else launch_typed<128, 128>(E.stream, p, A.trans, B.trans, vec);
  } else {
    launch_typed<64, 64>(E.stream, p, A.trans, B.trans, vec);
  }
  E.gemm_flops += 2 * M * N * K * (cc ? 4 : 2);
  if (E.trace)
    fprintf(stderr, "[rtcc] gemm-bf16x3 M=%lld N=%lld K=%lld %s%s ta=%d tb=%d vec=%d\n", (long long)M, (long long)N,
            (long long)K, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans, vec);
  return true;
}

}  // namespace rtcc
