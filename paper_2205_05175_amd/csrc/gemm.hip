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
#include <cstdint>

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
  int kchunk;            // K range handled by one split
  int splits;            // blockIdx.z = member * splits + split
  int64_t split_stride;  // elements between partial planes (split-K); 0 = write C directly
  int64_t sa, sb, sc;    // batch strides of A, B and C (elements; 0 = shared)
  T alpha, beta;
};

constexpr int kBK = 16;
constexpr int kThreads = 256;

// Register-staged load of one operand tile of ROWS x COLS elements whose COLS index is contiguous
// in memory (row stride ld). VEC consecutive elements are fetched per load when the whole vector
// is in range and the operand is VEC-aligned; out-of-range elements read as zero.
template <typename T, int ROWS, int COLS, int VEC, int NPL>
struct TileRegs {
  static constexpr int NV = ROWS * COLS / VEC / kThreads;
  static_assert(NV >= 1 && NV * VEC * kThreads == ROWS * COLS, "tile not divisible among threads");
  T r[NPL][NV][VEC];

  __device__ inline void load(const T* const* base, int64_t ld, int row0, int col0, int rowLim, int colLim,
                              int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = v * kThreads + tid;
      const int row = idx / (COLS / VEC), colv = (idx % (COLS / VEC)) * VEC;
      const int gr = row0 + row, gc = col0 + colv;
      const int64_t off = (int64_t)gr * ld + gc;
      if (VEC > 1 && gr < rowLim && gc + VEC <= colLim) {
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
          if constexpr (VEC == 4) {
            typedef T v4t __attribute__((ext_vector_type(4)));
            v4t x = *reinterpret_cast<const v4t*>(base[pl] + off);
            r[pl][v][0] = x[0]; r[pl][v][1] = x[1]; r[pl][v][2] = x[2]; r[pl][v][3] = x[3];
          } else if constexpr (VEC == 2) {
            typedef T v2t __attribute__((ext_vector_type(2)));
            v2t x = *reinterpret_cast<const v2t*>(base[pl] + off);
            r[pl][v][0] = x[0]; r[pl][v][1] = x[1];
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const bool ok = gr < rowLim && gc + e < colLim;
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) r[pl][v][e] = ok ? base[pl][off + e] : T(0);
        }
      }
    }
  }
  // store into an LDS tile S[k][x]; KMAJOR: the memory rows are k (contiguous x), else rows are x
  template <bool ROWS_ARE_K, int LD>
  __device__ inline void store(T* S, int plane_stride, int tid) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int idx = v * kThreads + tid;
      const int row = idx / (COLS / VEC), colv = (idx % (COLS / VEC)) * VEC;
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
          if (ROWS_ARE_K) S[pl * plane_stride + row * LD + colv + e] = r[pl][v][e];
          else S[pl * plane_stride + (colv + e) * LD + row] = r[pl][v][e];
        }
    }
  }
};

// TA: A stored as [k][m] (else [m][k]); TB: B stored as [n][k] (else [k][n]).
template <typename T, int BM, int BN, int AC, int BC, int TA, int TB, int VEC>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmParams<T> p) {
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  constexpr int LDA = BM + 1, LDB = BN + 1;  // padded LDS rows
  __shared__ T As[NA * kBK * LDA];
  __shared__ T Bs[NB * kBK * LDB];
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  using V4 = typename Mfma<T>::v4;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int zb = blockIdx.z / p.splits, zs = blockIdx.z - zb * p.splits;
  const int kbeg = zs * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);

  V4 accr[FM][FN], acci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accr[i][j] = V4{0, 0, 0, 0};
      acci[i][j] = V4{0, 0, 0, 0};
    }
  const int64_t oa = (int64_t)zb * p.sa, ob = (int64_t)zb * p.sb;
  const T* Ap[2] = {p.Are + oa, AC ? p.Aim + oa : nullptr};
  const T* Bp[2] = {p.Bre + ob, BC ? p.Bim + ob : nullptr};

  // A tile: TA ? (rows k, cols m) : (rows m, cols k);  B tile: TB ? (rows n, cols k) : (rows k, cols n).
  // A narrow tile (32 rows or columns) has fewer elements than VEC per thread: use shorter vectors.
  constexpr int VA = VEC < (kBK * BM) / kThreads ? VEC : (kBK * BM) / kThreads;
  constexpr int VB = VEC < (kBK * BN) / kThreads ? VEC : (kBK * BN) / kThreads;
  TileRegs<T, TA ? kBK : BM, TA ? BM : kBK, VA, NA> ra;
  TileRegs<T, TB ? BN : kBK, TB ? kBK : BN, VB, NB> rb;
  auto fetch = [&](int k0) {
    if (TA) ra.load(Ap, p.lda, k0, m0, kend, p.M, tid);
    else ra.load(Ap, p.lda, m0, k0, p.M, kend, tid);
    if (TB) rb.load(Bp, p.ldb, n0, k0, p.N, kend, tid);
    else rb.load(Bp, p.ldb, k0, n0, kend, p.N, tid);
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kBK) {
    ra.template store<TA != 0, LDA>(As, kBK * LDA, tid);
    rb.template store<TB == 0, LDB>(Bs, kBK * LDB, tid);
    __syncthreads();
    if (k0 + kBK < kend) fetch(k0 + kBK);  // next tile in flight while this one is multiplied
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const int kr = kk + (lane >> 4), col = lane & 15;
      T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[kr * LDA + wm * WM + i * 16 + col];
        if (AC) ai[i] = As[kBK * LDA + kr * LDA + wm * WM + i * 16 + col];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[kr * LDB + wn * WN + j * 16 + col];
        if (BC) bi[j] = Bs[kBK * LDB + kr * LDB + wn * WN + j * 16 + col];
      }
      T nai[FM];
      if (AC && BC) {
#pragma unroll
        for (int i = 0; i < FM; ++i) nai[i] = -ai[i];
      }
      // term-major issue: consecutive MFMAs update different accumulators
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
      if (BC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acci[i][j] = Mfma<T>::mma(ar[i], bi[j], acci[i][j]);
      }
      if (AC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acci[i][j] = Mfma<T>::mma(ai[i], br[j], acci[i][j]);
      }
      if (AC && BC) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) accr[i][j] = Mfma<T>::mma(nai[i], bi[j], accr[i][j]);
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
          int64_t off = (int64_t)zb * p.sc + (int64_t)row * p.ldc + col;
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

// Sum the split-K partial planes and apply alpha/beta. A block handles 16 outputs with 16
// lanes each; lane l sums the splits l, l+16, ... and the 16 lane sums are added in lane order,
// so the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce(const T* Pre, const T* Pim, int splits, int64_t stride, int M,
                                                     int N, T* Cre, T* Cim, int64_t ldc, int64_t sc, T alpha,
                                                     T beta) {
  __shared__ T shr[16][17], shi[16][17];
  const int ol = threadIdx.x & 15, sl = threadIdx.x >> 4;
  // member blockIdx.y: partial planes y * splits ... y * splits + splits - 1
  Pre += (int64_t)blockIdx.y * splits * stride;
  if (Pim) Pim += (int64_t)blockIdx.y * splits * stride;
  Cre += (int64_t)blockIdx.y * sc;
  if (Cim) Cim += (int64_t)blockIdx.y * sc;
  const int64_t idx = (int64_t)blockIdx.x * 16 + ol;
  const bool ok = idx < (int64_t)M * N;
  T sr = 0, si = 0;
  if (ok)
    for (int s = sl; s < splits; s += 16) {
      sr += Pre[s * stride + idx];
      if (Pim) si += Pim[s * stride + idx];
    }
  shr[sl][ol] = sr;
  shi[sl][ol] = si;
  __syncthreads();
  if (sl == 0 && ok) {
    T ar = 0, ai = 0;
    for (int k = 0; k < 16; ++k) {
      ar += shr[k][ol];
      ai += shi[k][ol];
    }
    int row = (int)(idx / N), col = (int)(idx % N);
    int64_t off = (int64_t)row * ldc + col;
    T outr = alpha * ar, outi = alpha * ai;
    if (beta != T(0)) {
      outr += beta * Cre[off];
      if (Cim) outi += beta * Cim[off];
    }
    Cre[off] = outr;
    if (Cim && Pim) Cim[off] = outi;
  }
}

// Few splits: one thread per output sums the partial planes in split order.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_few(const T* Pre, const T* Pim, int splits, int64_t stride,
                                                         int M, int N, T* Cre, T* Cim, int64_t ldc, int64_t sc,
                                                         T alpha, T beta) {
  Pre += (int64_t)blockIdx.y * splits * stride;
  if (Pim) Pim += (int64_t)blockIdx.y * splits * stride;
  Cre += (int64_t)blockIdx.y * sc;
  if (Cim) Cim += (int64_t)blockIdx.y * sc;
  const int64_t n = (int64_t)M * N;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * 256) {
    T ar = 0, ai = 0;
    for (int s = 0; s < splits; ++s) {
      ar += Pre[s * stride + idx];
      if (Pim) ai += Pim[s * stride + idx];
    }
    const int row = (int)(idx / N), col = (int)(idx - (int64_t)row * N);
    const int64_t off = (int64_t)row * ldc + col;
    T outr = alpha * ar, outi = alpha * ai;
    if (beta != T(0)) {
      outr += beta * Cre[off];
      if (Cim) outi += beta * Cim[off];
    }
    Cre[off] = outr;
    if (Cim && Pim) Cim[off] = outi;
  }
}

template <typename T>
void splitk_reduce_launch(hipStream_t st, const T* Pre, const T* Pim, int splits, int64_t M, int64_t N, T* Cre,
                          T* Cim, int64_t ldc, int64_t sc, int nbatch, double alpha, double beta) {
  const int64_t n = M * N;
  if (splits <= 24) {
    hipLaunchKernelGGL(splitk_reduce_few<T>, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 8192), (unsigned)nbatch),
                       dim3(256), 0, st, Pre, Pim, splits, n, (int)M, (int)N, Cre, Cim, ldc, sc, (T)alpha, (T)beta);
  } else {
    hipLaunchKernelGGL(splitk_reduce<T>, dim3((unsigned)cdiv(n, 16), (unsigned)nbatch), dim3(256), 0, st, Pre, Pim,
                       splits, n, (int)M, (int)N, Cre, Cim, ldc, sc, (T)alpha, (T)beta);
  }
  RTCC_HIP(hipGetLastError());
}
template void splitk_reduce_launch<float>(hipStream_t, const float*, const float*, int, int64_t, int64_t, float*,
                                          float*, int64_t, int64_t, int, double, double);
template void splitk_reduce_launch<double>(hipStream_t, const double*, const double*, int, int64_t, int64_t, double*,
                                           double*, int64_t, int64_t, int, double, double);

template <typename T, int BM, int BN, int AC, int BC, int TA, int TB, int VEC>
static void launch_one(hipStream_t st, const GemmParams<T>& p, int zdim) {
  dim3 grid((unsigned)cdiv(p.N, BN), (unsigned)cdiv(p.M, BM), (unsigned)zdim);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, AC, BC, TA, TB, VEC>), grid, dim3(kThreads), 0, st, p);
  RTCC_HIP(hipGetLastError());
}

template <typename T, int BM, int BN, int AC, int BC>
static void launch_gemm(hipStream_t st, const GemmParams<T>& p, int splits, bool vec) {
  constexpr int V = 16 / sizeof(T);
  const int sel = (p.ta ? 2 : 0) + (p.tb ? 1 : 0);
  if (vec) {
    switch (sel) {
      case 0: launch_one<T, BM, BN, AC, BC, 0, 0, V>(st, p, splits); break;
      case 1: launch_one<T, BM, BN, AC, BC, 0, 1, V>(st, p, splits); break;
      case 2: launch_one<T, BM, BN, AC, BC, 1, 0, V>(st, p, splits); break;
      default: launch_one<T, BM, BN, AC, BC, 1, 1, V>(st, p, splits); break;
    }
  } else {
    switch (sel) {
      case 0: launch_one<T, BM, BN, AC, BC, 0, 0, 1>(st, p, splits); break;
      case 1: launch_one<T, BM, BN, AC, BC, 0, 1, 1>(st, p, splits); break;
      case 2: launch_one<T, BM, BN, AC, BC, 1, 0, 1>(st, p, splits); break;
      default: launch_one<T, BM, BN, AC, BC, 1, 1, 1>(st, p, splits); break;
    }
  }
}

template <typename T, int BM, int BN>
static void launch_typed(hipStream_t st, const GemmParams<T>& p, int splits, bool vec) {
  const int sel = (p.Aim ? 2 : 0) + (p.Bim ? 1 : 0);
  switch (sel) {
    case 0: launch_gemm<T, BM, BN, 0, 0>(st, p, splits, vec); break;
    case 1: launch_gemm<T, BM, BN, 0, 1>(st, p, splits, vec); break;
    case 2: launch_gemm<T, BM, BN, 1, 0>(st, p, splits, vec); break;
    default: launch_gemm<T, BM, BN, 1, 1>(st, p, splits, vec); break;
  }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <typename T>
void gemm(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<T> A, GemmOp<T> B, T* Cre, T* Cim,
          int64_t ldc, double beta, GemmBatch bt) {
  if (M <= 0 || N <= 0 || bt.n <= 0) return;
  RTCC_CHECK(M < (1LL << 31) && N < (1LL << 31) && K < (1LL << 31), kEInval, "gemm: dimension too large");
  RTCC_CHECK(bt.n <= 65535, kEInval, "gemm: batch too large");
  const bool AC = A.im != nullptr, BC = B.im != nullptr, CC = Cim != nullptr;
  RTCC_CHECK(CC || (!AC && !BC), kEInval, "gemm: complex product into a real output");
  const int nbt = bt.n;
  if (K <= 0) {
    int64_t d[3] = {nbt, M, N}, s[3] = {bt.c, ldc, 1};
    permute_axpby<T>(E.stream, 3, d, Cre, Cim, s, Cre, Cim, s, 0.0, beta);
    return;
  }
  if (!AC && !BC && CC) {
    // real product into a complex output: the imaginary plane is only scaled
    int64_t d[3] = {nbt, M, N}, s[3] = {bt.c, ldc, 1};
    permute_axpby<T>(E.stream, 3, d, Cim, (T*)nullptr, s, Cim, (T*)nullptr, s, 0.0, beta);
    Cim = nullptr;
  }
  if constexpr (sizeof(T) == 4) {
    if (nbt == 1 && E.bf16x3 && 2.0 * (double)M * (double)N * (double)K >= E.bf16_min_flops &&
        gemm_bf16x3(E, M, N, K, alpha, A, B, Cre, Cim, ldc, beta))
      return;
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
  p.sa = bt.a;
  p.sb = bt.b;
  p.sc = bt.c;
  p.alpha = (T)alpha;
  p.beta = (T)beta;
  // 16-byte vector loads need every plane pointer, leading dimension and batch stride VEC-aligned
  constexpr int V = 16 / sizeof(T);
  const bool vec = aligned16(A.re) && (!AC || aligned16(A.im)) && aligned16(B.re) && (!BC || aligned16(B.im)) &&
                   A.ld % V == 0 && B.ld % V == 0 && bt.a % V == 0 && bt.b % V == 0;
  // FP32: 128 x 128 tiles when the grid still holds >= 2 tiles per CU; FP64 (longer MFMA,
  // more registers per tile): always 64 x 64 for occupancy. Small grids split over K.
  constexpr int LBM = 128, LBN = 128;
  // short K, one side of at most 32 against a long other side: a 32 x 256 (or 256 x 32) tile wastes
  // little (long K goes to split-K instead)
  const int narrow = K > 256                                            ? 0
                     : (M <= 32 && N >= 256) || (M <= 96 && N >= 8192)   ? 1
                     : (N <= 32 && M >= 256) || (N <= 96 && M >= 8192)   ? 2
                                                                         : 0;
  const bool large = !narrow && sizeof(T) == 4 && cdiv(M, LBM) * cdiv(N, LBN) * nbt >= 512;
  const int BM = narrow == 1 ? 32 : narrow == 2 ? 256 : large ? LBM : 64;
  const int BN = narrow == 1 ? 256 : narrow == 2 ? 32 : large ? LBN : 64;
  const int64_t tiles = cdiv(M, BM) * cdiv(N, BN) * nbt;
  // fewer than ~2 workgroups per CU: split K (chunks of >= 256) toward ~1024 workgroups
  int splits = 1;
  if (!large && !narrow && tiles < 512 && K >= 512) {
    int64_t want = std::max<int64_t>(1, 1024 / tiles);
    splits = (int)std::min<int64_t>({want, cdiv(K, 256), 1024, 65535 / nbt});
  }
  int64_t kchunk = cdiv(cdiv(K, splits), kBK) * kBK;
  splits = (int)cdiv(K, kchunk);
  p.kchunk = (int)kchunk;
  p.splits = splits;
  size_t mark = E.scratch.used;
  T* Pre = nullptr;
  T* Pim = nullptr;
  if (splits > 1) {
    p.split_stride = M * N;
    Pre = E.scratch.get<T>((int64_t)nbt * splits * M * N);
    if (AC || BC) Pim = E.scratch.get<T>((int64_t)nbt * splits * M * N);
    p.Cre = Pre;
    p.Cim = Pim;
    p.ldc = N;
  } else {
    p.split_stride = 0;
    p.Cre = Cre;
    p.Cim = Cim;
    p.ldc = ldc;
  }
  if (narrow == 1) launch_typed<T, 32, 256>(E.stream, p, nbt * splits, vec);
  else if (narrow == 2) launch_typed<T, 256, 32>(E.stream, p, nbt * splits, vec);
  else if (large) launch_typed<T, LBM, LBN>(E.stream, p, nbt * splits, vec);
  else launch_typed<T, 64, 64>(E.stream, p, nbt * splits, vec);
  if (splits > 1) splitk_reduce_launch<T>(E.stream, Pre, Pim, splits, M, N, Cre, Cim, ldc, bt.c, nbt, alpha, beta);
  E.scratch.reset(mark);
  E.gemm_flops += 2 * M * N * K * nbt * ((AC && BC) ? 4 : (AC || BC) ? 2 : 1);
  if (E.trace)
    fprintf(stderr, "[rtcc] gemm M=%lld N=%lld K=%lld batch=%d %s%s ta=%d tb=%d tile=%dx%d splits=%d vec=%d\n",
            (long long)M, (long long)N, (long long)K, nbt, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans, BM,
            BN, splits, (int)vec);
}

template void gemm<double>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<double>, GemmOp<double>, double*,
                           double*, int64_t, double, GemmBatch);
template void gemm<float>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<float>, GemmOp<float>, float*, float*,
                          int64_t, double, GemmBatch);

}  // namespace rtcc
