// LDS-tiled MFMA GEMM for gfx950 on planar complex / real operands, FP64 and FP32.
//
// C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n). Each operand is real or planar
// complex (separate Re/Im planes with identical strides). Real x complex products issue two
// MFMAs per fragment pair, complex x complex four (the Im(A) fragment is negated once in
// registers for the Re(C) update). The 256-thread workgroup holds a BM x BN tile split
// into 2 x 2 wave tiles; each wave covers its tile with 16x16 MFMA blocks
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32). Skinny products with long K are split
// over K into per-split partial planes and reduced by a second kernel in a fixed order, so
// results are bitwise repeatable.
#include "engine.h"

namespace rtcc {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element r of a lane lies in row lane/16 + 4r, column lane%16
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element r of a lane lies in row 4*(lane/16) + r, column lane%16
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
struct GemmParams {
  const T* Are;
  const T* Aim;
  int64_t lda;
  int ta;
  const T* Bre;
  const T* Bim;
  int64_t ldb;
  int tb;
  T* Cre;
  T* Cim;
  int64_t ldc;
  int M, N, K;
  int kchunk;            // K range handled by one blockIdx.z
  int64_t split_stride;  // elements between partial planes (split-K); 0 = write C directly
  T alpha, beta;
};

constexpr int kBK = 16;
constexpr int kThreads = 256;

template <typename T, int BM, int BN, int AC, int BC>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmParams<T> p) {
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  constexpr int PADA = 1, PADB = 1;
  __shared__ T As[NA][kBK][BM + PADA];
  __shared__ T Bs[NB][kBK][BN + PADB];
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  using V4 = typename Mfma<T>::v4;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);

  V4 accr[FM][FN], acci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accr[i][j] = V4{0, 0, 0, 0};
      acci[i][j] = V4{0, 0, 0, 0};
    }

  const T* Ap[2] = {p.Are, p.Aim};
  const T* Bp[2] = {p.Bre, p.Bim};

  for (int k0 = kbeg; k0 < kend; k0 += kBK) {
    // ---- stage A(m0:m0+BM, k0:k0+BK) into As[pl][k][m]
    if (!p.ta) {
#pragma unroll
      for (int it = 0; it < BM * kBK / kThreads; ++it) {
        int idx = it * kThreads + tid;
        int k = idx % kBK, m = idx / kBK;
        int gm = m0 + m, gk = k0 + k;
        bool ok = gm < p.M && gk < kend;
        int64_t off = (int64_t)gm * p.lda + gk;
#pragma unroll
        for (int pl = 0; pl < NA; ++pl) As[pl][k][m] = ok ? Ap[pl][off] : T(0);
      }
    } else {
#pragma unroll
      for (int it = 0; it < BM * kBK / kThreads; ++it) {
        int idx = it * kThreads + tid;
        int m = idx % BM, k = idx / BM;
        int gm = m0 + m, gk = k0 + k;
        bool ok = gm < p.M && gk < kend;
        int64_t off = (int64_t)gk * p.lda + gm;
#pragma unroll
        for (int pl = 0; pl < NA; ++pl) As[pl][k][m] = ok ? Ap[pl][off] : T(0);
      }
    }
    // ---- stage B(k0:k0+BK, n0:n0+BN) into Bs[pl][k][n]
    if (!p.tb) {
#pragma unroll
      for (int it = 0; it < BN * kBK / kThreads; ++it) {
        int idx = it * kThreads + tid;
        int n = idx % BN, k = idx / BN;
        int gn = n0 + n, gk = k0 + k;
        bool ok = gn < p.N && gk < kend;
        int64_t off = (int64_t)gk * p.ldb + gn;
#pragma unroll
        for (int pl = 0; pl < NB; ++pl) Bs[pl][k][n] = ok ? Bp[pl][off] : T(0);
      }
    } else {
#pragma unroll
      for (int it = 0; it < BN * kBK / kThreads; ++it) {
        int idx = it * kThreads + tid;
        int k = idx % kBK, n = idx / kBK;
        int gn = n0 + n, gk = k0 + k;
        bool ok = gn < p.N && gk < kend;
        int64_t off = (int64_t)gn * p.ldb + gk;
#pragma unroll
        for (int pl = 0; pl < NB; ++pl) Bs[pl][k][n] = ok ? Bp[pl][off] : T(0);
      }
    }
    __syncthreads();

#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const int kr = kk + (lane >> 4), col = lane & 15;
      T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kr][wm * WM + i * 16 + col];
        if (AC) ai[i] = As[NA - 1][kr][wm * WM + i * 16 + col];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kr][wn * WN + j * 16 + col];
        if (BC) bi[j] = Bs[NB - 1][kr][wn * WN + j * 16 + col];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (AC && BC) {
            accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
            accr[i][j] = Mfma<T>::mma(-ai[i], bi[j], accr[i][j]);
            acci[i][j] = Mfma<T>::mma(ar[i], bi[j], acci[i][j]);
            acci[i][j] = Mfma<T>::mma(ai[i], br[j], acci[i][j]);
          } else if (AC) {
            accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
            acci[i][j] = Mfma<T>::mma(ai[i], br[j], acci[i][j]);
          } else if (BC) {
            accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
            acci[i][j] = Mfma<T>::mma(ar[i], bi[j], acci[i][j]);
          } else {
            accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
          }
        }
    }
    __syncthreads();
  }

  // ---- epilogue: each lane holds four rows of one column of every 16x16 block
  constexpr bool CC = AC || BC;
  const int cc = lane & 15;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm * WM + i * 16 + Mfma<T>::row(lane, r);
        int col = n0 + wn * WN + j * 16 + cc;
        if (row >= p.M || col >= p.N) continue;
        T vr = accr[i][j][r], vi = acci[i][j][r];
        if (p.split_stride) {
          int64_t off = (int64_t)blockIdx.z * p.split_stride + (int64_t)row * p.N + col;
          p.Cre[off] = vr;
          if (CC) p.Cim[off] = vi;
        } else {
          int64_t off = (int64_t)row * p.ldc + col;
          T outr = p.alpha * vr, outi = p.alpha * vi;
          if (p.beta != T(0)) {
            outr += p.beta * p.Cre[off];
            if (CC) outi += p.beta * p.Cim[off];
          }
          p.Cre[off] = outr;
          if (CC) p.Cim[off] = outi;
        }
      }
}

// Sum the split-K partial planes in a fixed order and apply alpha/beta.
template <typename T>
__global__ void splitk_reduce(const T* Pre, const T* Pim, int splits, int64_t stride, int M, int N, T* Cre,
                              T* Cim, int64_t ldc, T alpha, T beta) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  int row = (int)(idx / N), col = (int)(idx % N);
  T sr = 0, si = 0;
  for (int s = 0; s < splits; ++s) {
    sr += Pre[s * stride + idx];
    if (Pim) si += Pim[s * stride + idx];
  }
  int64_t off = (int64_t)row * ldc + col;
  T outr = alpha * sr, outi = alpha * si;
  if (beta != T(0)) {
    outr += beta * Cre[off];
    if (Cim) outi += beta * Cim[off];
  }
  Cre[off] = outr;
  if (Cim && Pim) Cim[off] = outi;
}

template <typename T, int BM, int BN, int AC, int BC>
static void launch_gemm(hipStream_t st, const GemmParams<T>& p, int splits) {
  dim3 grid((unsigned)cdiv(p.N, BN), (unsigned)cdiv(p.M, BM), (unsigned)splits);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, AC, BC>), grid, dim3(kThreads), 0, st, p);
  RTCC_HIP(hipGetLastError());
}

template <typename T>
void gemm(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<T> A, GemmOp<T> B, T* Cre, T* Cim,
          int64_t ldc, double beta) {
  if (M <= 0 || N <= 0) return;
  RTCC_CHECK(M < (1LL << 31) && N < (1LL << 31) && K < (1LL << 31), kEInval, "gemm: dimension too large");
  const bool AC = A.im != nullptr, BC = B.im != nullptr, CC = Cim != nullptr;
  RTCC_CHECK(CC || (!AC && !BC), kEInval, "gemm: complex product into a real output");
  if (K <= 0) {
    int64_t d[2] = {M, N}, s[2] = {ldc, 1};
    permute_axpby<T>(E.stream, 2, d, Cre, Cim, s, Cre, Cim, s, 0.0, beta);
    return;
  }
  if (!AC && !BC && CC) {
    // real product into a complex output: the imaginary plane is only scaled
    int64_t d[2] = {M, N}, s[2] = {ldc, 1};
    permute_axpby<T>(E.stream, 2, d, Cim, (T*)nullptr, s, Cim, (T*)nullptr, s, 0.0, beta);
    Cim = nullptr;
  }
  GemmParams<T> p;
  p.Are = A.re;
  p.Aim = A.im;
  p.lda = A.ld;
  p.ta = A.trans;
  p.Bre = B.re;
  p.Bim = B.im;
  p.ldb = B.ld;
  p.tb = B.trans;
  p.M = (int)M;
  p.N = (int)N;
  p.K = (int)K;
  p.alpha = (T)alpha;
  p.beta = (T)beta;
  constexpr int BM = 64, BN = 64;
  const int64_t tiles = cdiv(M, BM) * cdiv(N, BN);
  int splits = 1;
  if (tiles < 512 && K >= 8 * kBK) {
    int64_t want = std::max<int64_t>(1, 1024 / tiles);
    splits = (int)std::min<int64_t>(want, cdiv(K, 4 * kBK));
  }
  int64_t kchunk = cdiv(cdiv(K, splits), kBK) * kBK;
  splits = (int)cdiv(K, kchunk);
  p.kchunk = (int)kchunk;
  size_t mark = E.scratch.used;
  T* Pre = nullptr;
  T* Pim = nullptr;
  if (splits > 1) {
    p.split_stride = M * N;
    Pre = E.scratch.get<T>(splits * M * N);
    if (AC || BC) Pim = E.scratch.get<T>(splits * M * N);
    p.Cre = Pre;
    p.Cim = Pim;
    p.ldc = N;
  } else {
    p.split_stride = 0;
    p.Cre = Cre;
    p.Cim = Cim;
    p.ldc = ldc;
  }
  const int sel = (AC ? 2 : 0) + (BC ? 1 : 0);
  switch (sel) {
    case 0: launch_gemm<T, BM, BN, 0, 0>(E.stream, p, splits); break;
    case 1: launch_gemm<T, BM, BN, 0, 1>(E.stream, p, splits); break;
    case 2: launch_gemm<T, BM, BN, 1, 0>(E.stream, p, splits); break;
    default: launch_gemm<T, BM, BN, 1, 1>(E.stream, p, splits); break;
  }
  if (splits > 1) {
    int64_t n = M * N;
    hipLaunchKernelGGL(splitk_reduce<T>, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, E.stream, Pre, Pim, splits,
                       M * N, (int)M, (int)N, Cre, Cim, ldc, (T)alpha, (T)beta);
    RTCC_HIP(hipGetLastError());
  }
  E.scratch.reset(mark);
  E.gemm_flops += 2 * M * N * K * ((AC && BC) ? 4 : (AC || BC) ? 2 : 1);
}

template void gemm<double>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<double>, GemmOp<double>, double*,
                           double*, int64_t, double);
template void gemm<float>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<float>, GemmOp<float>, float*, float*,
                          int64_t, double);

}  // namespace rtcc
