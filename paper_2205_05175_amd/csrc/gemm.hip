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
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

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
template <typename T, int BM, int BN, int AC, int BC, int TA, int TB, int VEC, int BK = kBK>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmParams<T> p) {
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  constexpr int LDA = BM + 1, LDB = BN + 1;  // padded LDS rows
  __shared__ T As[NA * BK * LDA];
  __shared__ T Bs[NB * BK * LDB];
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
  constexpr int VA = VEC < (BK * BM) / kThreads ? VEC : (BK * BM) / kThreads;
  constexpr int VB = VEC < (BK * BN) / kThreads ? VEC : (BK * BN) / kThreads;
  TileRegs<T, TA ? BK : BM, TA ? BM : BK, VA, NA> ra;
  TileRegs<T, TB ? BN : BK, TB ? BK : BN, VB, NB> rb;
  auto fetch = [&](int k0) {
    if (TA) ra.load(Ap, p.lda, k0, m0, kend, p.M, tid);
    else ra.load(Ap, p.lda, m0, k0, p.M, kend, tid);
    if (TB) rb.load(Bp, p.ldb, n0, k0, p.N, kend, tid);
    else rb.load(Bp, p.ldb, k0, n0, kend, p.N, tid);
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    ra.template store<TA != 0, LDA>(As, BK * LDA, tid);
    rb.template store<TB == 0, LDB>(Bs, BK * LDB, tid);
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);  // next tile in flight while this one is multiplied
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), col = lane & 15;
      T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[kr * LDA + wm * WM + i * 16 + col];
        if (AC) ai[i] = As[BK * LDA + kr * LDA + wm * WM + i * 16 + col];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[kr * LDB + wn * WN + j * 16 + col];
        if (BC) bi[j] = Bs[BK * LDB + kr * LDB + wn * WN + j * 16 + col];
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

  // ---- epilogue: each lane holds four rows of one column of every 16x16 block. With beta != 0 the
  // old C values of a row block are all loaded before any of its stores (a store may alias a later
  // load, so loads interleaved with stores would each wait a full memory latency).
  constexpr bool CC = AC || BC;
  const int cc = lane & 15;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    T oldr[FN][4], oldi[FN][4];
    const bool acc = !p.split_stride && p.beta != T(0);
    if (acc) {
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + Mfma<T>::row(lane, r);
          const int col = n0 + wn * WN + j * 16 + cc;
          const bool ok = row < p.M && col < p.N;
          const int64_t off = (int64_t)zb * p.sc + (int64_t)row * p.ldc + col;
          oldr[j][r] = ok ? p.Cre[off] : T(0);
          oldi[j][r] = (CC && ok) ? p.Cim[off] : T(0);
        }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + Mfma<T>::row(lane, r);
        const int col = n0 + wn * WN + j * 16 + cc;
        if (row >= p.M || col >= p.N) continue;
        const T vr = accr[i][j][r], vi = acci[i][j][r];
        if (p.split_stride) {
          const int64_t off = (int64_t)blockIdx.z * p.split_stride + (int64_t)row * p.N + col;
          p.Cre[off] = vr;
          if (CC) p.Cim[off] = vi;
        } else {
          const int64_t off = (int64_t)zb * p.sc + (int64_t)row * p.ldc + col;
          T outr = p.alpha * vr, outi = p.alpha * vi;
          if (acc) {
            outr += p.beta * oldr[j][r];
            outi += p.beta * oldi[j][r];
          }
          p.Cre[off] = outr;
          if (CC) p.Cim[off] = outi;
        }
      }
  }
}

// Sum the split-K partial planes and apply alpha/beta. A block of 1024 threads handles 16 outputs
// with 64 lanes each (a wave reads four partial planes, 64 contiguous bytes from each): lane l sums
// the splits l, l + 64, ... in order with eight loads in flight, and the 64 lane sums of an output
// are added by a fixed pairwise tree, so the result does not depend on scheduling. The many-split
// products (a small output with K split hundreds of ways) have few outputs: the wide blocks keep
// every partial load of a block in flight at once.
template <typename T>
__global__ __launch_bounds__(1024) void splitk_reduce(const T* Pre, const T* Pim, int splits, int64_t stride, int M,
                                                      int N, T* Cre, T* Cim, int64_t ldc, int64_t sc, T alpha,
                                                      T beta) {
  constexpr int kLanes = 64;
  __shared__ T shr[kLanes][17], shi[kLanes][17];
  const int ol = threadIdx.x & 15, sl = threadIdx.x >> 4;
  // member blockIdx.y: partial planes y * splits ... y * splits + splits - 1
  Pre += (int64_t)blockIdx.y * splits * stride;
  if (Pim) Pim += (int64_t)blockIdx.y * splits * stride;
  Cre += (int64_t)blockIdx.y * sc;
  if (Cim) Cim += (int64_t)blockIdx.y * sc;
  const int64_t idx = (int64_t)blockIdx.x * 16 + ol;
  const bool ok = idx < (int64_t)M * N;
  T sr = 0, si = 0;
  if (ok) {
    int s = sl;
    for (; s + 7 * kLanes < splits; s += 8 * kLanes) {
      T vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        vr[u] = Pre[(int64_t)(s + kLanes * u) * stride + idx];
        vi[u] = Pim ? Pim[(int64_t)(s + kLanes * u) * stride + idx] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sr += vr[u];
        si += vi[u];
      }
    }
    for (; s < splits; s += kLanes) {
      sr += Pre[(int64_t)s * stride + idx];
      if (Pim) si += Pim[(int64_t)s * stride + idx];
    }
  }
  shr[sl][ol] = sr;
  shi[sl][ol] = si;
  __syncthreads();
  // lane sums: (0 + 32), (1 + 33), ... then (0 + 16), ... down to lane 0
#pragma unroll
  for (int h = kLanes / 2; h >= 1; h >>= 1) {
    if (sl < h) {
      shr[sl][ol] += shr[sl + h][ol];
      shi[sl][ol] += shi[sl + h][ol];
    }
    __syncthreads();
  }
  if (sl == 0 && ok) {
    const T ar = shr[0][ol], ai = shi[0][ol];
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
    int s = 0;
    for (; s + 4 <= splits; s += 4) {
      T vr[4], vi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        vr[u] = Pre[(int64_t)(s + u) * stride + idx];
        vi[u] = Pim ? Pim[(int64_t)(s + u) * stride + idx] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ar += vr[u];
        ai += vi[u];
      }
    }
    for (; s < splits; ++s) {
      ar += Pre[(int64_t)s * stride + idx];
      if (Pim) ai += Pim[(int64_t)s * stride + idx];
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

// Few splits, FP32 rows of a multiple of 4 with 16-byte aligned planes: the same sums (split order, then
// alpha and beta) for four consecutive outputs per thread with 16-byte loads and stores.
__global__ __launch_bounds__(256) void splitk_reduce_few4(const float* Pre, const float* Pim, int splits,
                                                          int64_t stride, int M, int N, float* Cre, float* Cim,
                                                          int64_t ldc, int64_t sc, float alpha, float beta) {
  Pre += (int64_t)blockIdx.y * splits * stride;
  if (Pim) Pim += (int64_t)blockIdx.y * splits * stride;
  Cre += (int64_t)blockIdx.y * sc;
  if (Cim) Cim += (int64_t)blockIdx.y * sc;
  const int64_t n4 = (int64_t)M * N / 4;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += (int64_t)gridDim.x * 256) {
    const int64_t idx = 4 * q;
    float4 ar = make_float4(0.f, 0.f, 0.f, 0.f), ai = ar;
    int s = 0;
    for (; s + 4 <= splits; s += 4) {
      float4 vr[4], vi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        vr[u] = *reinterpret_cast<const float4*>(Pre + (int64_t)(s + u) * stride + idx);
        vi[u] = Pim ? *reinterpret_cast<const float4*>(Pim + (int64_t)(s + u) * stride + idx)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ar.x += vr[u].x; ar.y += vr[u].y; ar.z += vr[u].z; ar.w += vr[u].w;
        ai.x += vi[u].x; ai.y += vi[u].y; ai.z += vi[u].z; ai.w += vi[u].w;
      }
    }
    for (; s < splits; ++s) {
      const float4 v = *reinterpret_cast<const float4*>(Pre + (int64_t)s * stride + idx);
      ar.x += v.x; ar.y += v.y; ar.z += v.z; ar.w += v.w;
      if (Pim) {
        const float4 w = *reinterpret_cast<const float4*>(Pim + (int64_t)s * stride + idx);
        ai.x += w.x; ai.y += w.y; ai.z += w.z; ai.w += w.w;
      }
    }
    const int row = (int)(idx / N), col = (int)(idx - (int64_t)row * N);
    const int64_t off = (int64_t)row * ldc + col;
    float4 outr = make_float4(alpha * ar.x, alpha * ar.y, alpha * ar.z, alpha * ar.w);
    float4 outi = make_float4(alpha * ai.x, alpha * ai.y, alpha * ai.z, alpha * ai.w);
    if (beta != 0.f) {
      const float4 cr = *reinterpret_cast<const float4*>(Cre + off);
      outr.x += beta * cr.x; outr.y += beta * cr.y; outr.z += beta * cr.z; outr.w += beta * cr.w;
      if (Cim) {
        const float4 ci = *reinterpret_cast<const float4*>(Cim + off);
        outi.x += beta * ci.x; outi.y += beta * ci.y; outi.z += beta * ci.z; outi.w += beta * ci.w;
      }
    }
    *reinterpret_cast<float4*>(Cre + off) = outr;
    if (Cim && Pim) *reinterpret_cast<float4*>(Cim + off) = outi;
  }
}

template <typename T>
void splitk_reduce_launch(hipStream_t st, const T* Pre, const T* Pim, int splits, int64_t M, int64_t N, T* Cre,
                          T* Cim, int64_t ldc, int64_t sc, int nbatch, double alpha, double beta) {
  const int64_t n = M * N;
  if constexpr (sizeof(T) == 4) {
    const auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    if (splits <= 24 && N % 4 == 0 && ldc % 4 == 0 && sc % 4 == 0 && al16(Pre) && (!Pim || al16(Pim)) && al16(Cre) &&
        (!Cim || al16(Cim))) {
      hipLaunchKernelGGL(splitk_reduce_few4, dim3((unsigned)std::min<int64_t>(cdiv(n / 4, 256), 8192), (unsigned)nbatch),
                         dim3(256), 0, st, Pre, Pim, splits, n, (int)M, (int)N, Cre, Cim, ldc, sc, (float)alpha,
                         (float)beta);
      RTCC_HIP(hipGetLastError());
      return;
    }
  }
  if (splits <= 24) {
    hipLaunchKernelGGL(splitk_reduce_few<T>, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 8192), (unsigned)nbatch),
                       dim3(256), 0, st, Pre, Pim, splits, n, (int)M, (int)N, Cre, Cim, ldc, sc, (T)alpha, (T)beta);
  } else {
    hipLaunchKernelGGL(splitk_reduce<T>, dim3((unsigned)cdiv(n, 16), (unsigned)nbatch), dim3(1024), 0, st, Pre, Pim,
                       splits, n, (int)M, (int)N, Cre, Cim, ldc, sc, (T)alpha, (T)beta);
  }
  RTCC_HIP(hipGetLastError());
}
template void splitk_reduce_launch<float>(hipStream_t, const float*, const float*, int, int64_t, int64_t, float*,
                                          float*, int64_t, int64_t, int, double, double);
template void splitk_reduce_launch<double>(hipStream_t, const double*, const double*, int, int64_t, int64_t, double*,
                                           double*, int64_t, int64_t, int, double, double);

// ---- tiny products ------------------------------------------------------------------------------
// M * N and K small: too few tiles to hide a tile kernel's stage latency. A workgroup takes 16
// consecutive outputs of member blockIdx.y; 16 threads share the k range of each output (thread
// slice s takes k = s, s + 16, ...) and the 16 slice sums are added in slice order.
template <typename T, int AC, int BC>
__global__ __launch_bounds__(256) void gemm_dot_kernel(GemmParams<T> p) {
  __shared__ T shr[16][17], shi[16][17];
  const int ol = threadIdx.x & 15, ks = threadIdx.x >> 4;
  const int64_t o = (int64_t)blockIdx.x * 16 + ol;
  const bool ok = o < (int64_t)p.M * p.N;
  const int m = ok ? (int)(o / p.N) : 0, n = ok ? (int)(o - (int64_t)m * p.N) : 0;
  const int64_t zb = blockIdx.y;
  const T* Ar = p.Are + zb * p.sa;
  const T* Ai = AC ? p.Aim + zb * p.sa : nullptr;
  const T* Br = p.Bre + zb * p.sb;
  const T* Bi = BC ? p.Bim + zb * p.sb : nullptr;
  // element (m, k) of A at am + k * ak; element (k, n) of B at bn + k * bk
  const int64_t am = p.ta ? m : (int64_t)m * p.lda, ak = p.ta ? p.lda : 1;
  const int64_t bn = p.tb ? (int64_t)n * p.ldb : n, bk = p.tb ? 1 : p.ldb;
  T ar = 0, ai = 0;
  auto madd = [&](T xr, T xi, T yr, T yi) {
    ar = fma(xr, yr, ar);
    if (AC && BC) ar = fma(-xi, yi, ar);
    if (BC) ai = fma(xr, yi, ai);
    if (AC) ai = fma(xi, yr, ai);
  };
  if (ok) {
    int k = ks;
    for (; k + 3 * 16 < p.K; k += 4 * 16) {
      T xr[4], xi[4], yr[4], yi[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t kk = k + 16 * u;
        xr[u] = Ar[am + kk * ak];
        xi[u] = AC ? Ai[am + kk * ak] : T(0);
        yr[u] = Br[bn + kk * bk];
        yi[u] = BC ? Bi[bn + kk * bk] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) madd(xr[u], xi[u], yr[u], yi[u]);
    }
    for (; k < p.K; k += 16)
      madd(Ar[am + (int64_t)k * ak], AC ? Ai[am + (int64_t)k * ak] : T(0), Br[bn + (int64_t)k * bk],
           BC ? Bi[bn + (int64_t)k * bk] : T(0));
  }
  shr[ks][ol] = ar;
  shi[ks][ol] = ai;
  __syncthreads();
  if (ks != 0 || !ok) return;
  T sr = 0, si = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    sr += shr[s][ol];
    si += shi[s][ol];
  }
  constexpr bool CC = AC || BC;
  const int64_t off = zb * p.sc + (int64_t)m * p.ldc + n;
  T outr = p.alpha * sr, outi = p.alpha * si;
  if (p.beta != T(0)) {
    outr += p.beta * p.Cre[off];
    if (CC) outi += p.beta * p.Cim[off];
  }
  p.Cre[off] = outr;
  if (CC) p.Cim[off] = outi;
}

// ---- matrix-vector products (one of M, N is 1) -------------------------------------------------
// y(n) = alpha * sum_k x(k) W(k, n) + beta * y(n), x with element stride incx, y with stride incy.
// With split_stride != 0 the k-range of split s goes to the partial plane y + s * split_stride
// (unit stride) and splitk_reduce_launch finishes the sum.
template <typename T>
struct GemvParams {
  const T* xre;
  const T* xim;
  int64_t incx;
  const T* wre;
  const T* wim;
  int64_t ldw;
  T* yre;
  T* yim;
  int64_t incy;
  int N, K, kchunk;
  int64_t split_stride;
  T alpha, beta;
  // two-level indices (GEN kernels): W(k, n) = W[(k / K2) sk1 + (k % K2) sk2 + (n / N2) sn1 + (n % N2) sn2];
  // q64, r64 = 64 / K2, 64 % K2
  int N2, K2, q64, r64;
  int64_t sn1, sn2, sk1, sk2;
};

// Row layout W(k, n) = W[k * ldw + n] (GEN: the two-level form, lanes along n): consecutive lanes take
// consecutive n (coalesced rows of W); each thread walks its k-range with eight rows of loads in
// flight and sums in k order.
template <typename T, int XC, int WC, int GEN>
__global__ __launch_bounds__(256) void gemv_row_kernel(GemvParams<T> p) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= p.N) return;  // no barriers below
  const int s = blockIdx.y;
  const int kb = s * p.kchunk, ke = min(p.K, kb + p.kchunk);
  const int64_t nn = GEN ? (int64_t)(n / p.N2) * p.sn1 + (int64_t)(n % p.N2) * p.sn2 : n;
  int k1 = GEN ? kb / p.K2 : 0, k2 = GEN ? kb % p.K2 : 0;
  // offset of row k of W; called once per k, in increasing k
  auto kofs = [&](int k) -> int64_t {
    if (!GEN) return (int64_t)k * p.ldw + nn;
    const int64_t o = (int64_t)k1 * p.sk1 + (int64_t)k2 * p.sk2 + nn;
    if (++k2 == p.K2) {
      k2 = 0;
      ++k1;
    }
    return o;
  };
  T ar = 0, ai = 0;
  auto madd = [&](T xr, T xi, T wr, T wi) {
    ar = fma(xr, wr, ar);
    if (XC && WC) ar = fma(-xi, wi, ar);
    if (WC) ai = fma(xr, wi, ai);
    if (XC) ai = fma(xi, wr, ai);
  };
  int k = kb;
  for (; k + 8 <= ke; k += 8) {
    T wr[8], wi[8], xr[8], xi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t o = kofs(k + u);
      wr[u] = p.wre[o];
      wi[u] = WC ? p.wim[o] : T(0);
      xr[u] = p.xre[(int64_t)(k + u) * p.incx];
      xi[u] = XC ? p.xim[(int64_t)(k + u) * p.incx] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) madd(xr[u], xi[u], wr[u], wi[u]);
  }
  for (; k < ke; ++k) {
    const int64_t o = kofs(k);
    madd(p.xre[(int64_t)k * p.incx], XC ? p.xim[(int64_t)k * p.incx] : T(0), p.wre[o], WC ? p.wim[o] : T(0));
  }
  constexpr bool CC = XC || WC;
  if (p.split_stride) {
    const int64_t o = (int64_t)s * p.split_stride + n;
    p.yre[o] = ar;
    if (CC) p.yim[o] = ai;
  } else {
    const int64_t o = (int64_t)n * p.incy;
    T outr = p.alpha * ar, outi = p.alpha * ai;
    if (p.beta != T(0)) {
      outr += p.beta * p.yre[o];
      if (CC) outi += p.beta * p.yim[o];
    }
    p.yre[o] = outr;
    if (CC) p.yim[o] = outi;
  }
}

// Column layout W(k, n) = W[n * ldw + k] (GEN: the two-level form, lanes along k): one wave per n,
// lanes stride over k (coalesced), four loads in flight per lane; the 64 lane sums are combined in a
// fixed butterfly order.
template <typename T, int XC, int WC, int GEN>
__global__ __launch_bounds__(256) void gemv_col_kernel(GemvParams<T> p) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= p.N) return;  // whole waves leave together; no barriers below
  const int s = blockIdx.y;
  const int kb = s * p.kchunk, ke = min(p.K, kb + p.kchunk);
  const int64_t nn = GEN ? (int64_t)(n / p.N2) * p.sn1 + (int64_t)(n % p.N2) * p.sn2 : (int64_t)n * p.ldw;
  const T* wr = p.wre + nn;
  const T* wi = WC ? p.wim + nn : nullptr;
  int k1 = GEN ? (kb + lane) / p.K2 : 0, k2 = GEN ? (kb + lane) % p.K2 : 0;
  // offset of element k (this lane's k, k + 64, ...) in the row of n; called once per k, in order
  auto kofs = [&](int k) -> int64_t {
    if (!GEN) return k;
    const int64_t o = (int64_t)k1 * p.sk1 + (int64_t)k2 * p.sk2;
    k2 += p.r64;
    k1 += p.q64;
    if (k2 >= p.K2) {
      k2 -= p.K2;
      ++k1;
    }
    return o;
  };
  T ar = 0, ai = 0;
  auto madd = [&](T xr, T xi, T vr, T vi) {
    ar = fma(xr, vr, ar);
    if (XC && WC) ar = fma(-xi, vi, ar);
    if (WC) ai = fma(xr, vi, ai);
    if (XC) ai = fma(xi, vr, ai);
  };
  int k = kb + lane;
  for (; k + 3 * 64 < ke; k += 4 * 64) {
    T vr[4], vi[4], xr[4], xi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + 64 * u;
      const int64_t o = kofs(kk);
      vr[u] = wr[o];
      vi[u] = WC ? wi[o] : T(0);
      xr[u] = p.xre[(int64_t)kk * p.incx];
      xi[u] = XC ? p.xim[(int64_t)kk * p.incx] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) madd(xr[u], xi[u], vr[u], vi[u]);
  }
  for (; k < ke; k += 64) {
    const int64_t o = kofs(k);
    madd(p.xre[(int64_t)k * p.incx], XC ? p.xim[(int64_t)k * p.incx] : T(0), wr[o], WC ? wi[o] : T(0));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ar += __shfl_xor(ar, off);
    ai += __shfl_xor(ai, off);
  }
  if (lane != 0) return;
  constexpr bool CC = XC || WC;
  if (p.split_stride) {
    const int64_t o = (int64_t)s * p.split_stride + n;
    p.yre[o] = ar;
    if (CC) p.yim[o] = ai;
  } else {
    const int64_t o = (int64_t)n * p.incy;
    T outr = p.alpha * ar, outi = p.alpha * ai;
    if (p.beta != T(0)) {
      outr += p.beta * p.yre[o];
      if (CC) outi += p.beta * p.yim[o];
    }
    p.yre[o] = outr;
    if (CC) p.yim[o] = outi;
  }
}

// Two-level index form of W for the GEN kernels (see GemvParams).
struct GemvLayout {
  int64_t N2, sn1, sn2, K2, sk1, sk2;
};

// x(k), W(k, n) as described above (or in the two-level form L when non-null); y complex when x or W
// is. Returns the number of splits used.
template <typename T>
static int gemv(Engine& E, bool col, int64_t N, int64_t K, double alpha, const T* xre, const T* xim, int64_t incx,
                const T* wre, const T* wim, int64_t ldw, T* yre, T* yim, int64_t incy, double beta,
                const GemvLayout* L = nullptr) {
  GemvParams<T> p;
  p.N2 = L ? (int)L->N2 : 1;
  p.K2 = L ? (int)L->K2 : 1;
  p.sn1 = L ? L->sn1 : 0;
  p.sn2 = L ? L->sn2 : 0;
  p.sk1 = L ? L->sk1 : 0;
  p.sk2 = L ? L->sk2 : 0;
  p.q64 = 64 / p.K2;
  p.r64 = 64 % p.K2;
  p.xre = xre;
  p.xim = xim;
  p.incx = incx;
  p.wre = wre;
  p.wim = wim;
  p.ldw = ldw;
  p.N = (int)N;
  p.K = (int)K;
  p.alpha = (T)alpha;
  p.beta = (T)beta;
  // enough independent k-ranges for ~2048 workgroups of row threads / ~8192 column waves
  int64_t kchunk;
  unsigned gx;
  if (col) {
    gx = (unsigned)cdiv(N, 4);
    const int64_t want = std::max<int64_t>(1, 8192 / N);
    kchunk = cdiv(cdiv(K, std::min<int64_t>(want, cdiv(K, 256))), 64) * 64;
  } else {
    gx = (unsigned)cdiv(N, 256);
    kchunk = cdiv(std::max<int64_t>({16, cdiv(K * gx, 2048), cdiv(K, 65535)}), 8) * 8;
  }
  const int splits = (int)cdiv(K, kchunk);
  p.kchunk = (int)kchunk;
  size_t mark = E.scratch.used;
  T* Pre = nullptr;
  T* Pim = nullptr;
  const bool CC = xim || wim;
  if (splits > 1) {
    Pre = E.scratch.get<T>((int64_t)splits * N);
    if (CC) Pim = E.scratch.get<T>((int64_t)splits * N);
    p.yre = Pre;
    p.yim = Pim;
    p.incy = 1;
    p.split_stride = N;
  } else {
    p.yre = yre;
    p.yim = yim;
    p.incy = incy;
    p.split_stride = 0;
  }
  const dim3 grid(gx, (unsigned)splits);
  const int sel = (xim ? 2 : 0) + (wim ? 1 : 0);
#define RTCC_GEMV(XC, WC)                                                                              \
  if (L && col) hipLaunchKernelGGL((gemv_col_kernel<T, XC, WC, 1>), grid, dim3(256), 0, E.stream, p);   \
  else if (L) hipLaunchKernelGGL((gemv_row_kernel<T, XC, WC, 1>), grid, dim3(256), 0, E.stream, p);     \
  else if (col) hipLaunchKernelGGL((gemv_col_kernel<T, XC, WC, 0>), grid, dim3(256), 0, E.stream, p);   \
  else hipLaunchKernelGGL((gemv_row_kernel<T, XC, WC, 0>), grid, dim3(256), 0, E.stream, p);
  switch (sel) {
    case 0: RTCC_GEMV(0, 0) break;
    case 1: RTCC_GEMV(0, 1) break;
    case 2: RTCC_GEMV(1, 0) break;
    default: RTCC_GEMV(1, 1) break;
  }
#undef RTCC_GEMV
  RTCC_HIP(hipGetLastError());
  // partial planes [split][n] -> y(n) at stride incy (an N x 1 "matrix" with row stride incy)
  if (splits > 1) splitk_reduce_launch<T>(E.stream, Pre, Pim, splits, N, 1, yre, yim, incy, 0, 1, alpha, beta);
  E.scratch.reset(mark);
  return splits;
}

template <typename T, int BM, int BN, int AC, int BC, int TA, int TB, int VEC, int BK = kBK>
static void launch_one(hipStream_t st, const GemmParams<T>& p, int zdim) {
  dim3 grid((unsigned)cdiv(p.N, BN), (unsigned)cdiv(p.M, BM), (unsigned)zdim);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, AC, BC, TA, TB, VEC, BK>), grid, dim3(kThreads), 0, st, p);
  RTCC_HIP(hipGetLastError());
}

template <typename T, int BM, int BN, int AC, int BC, int BK, bool VECONLY>
static void launch_gemm(hipStream_t st, const GemmParams<T>& p, int splits, bool vec) {
  constexpr int V = 16 / sizeof(T);
  const int sel = (p.ta ? 2 : 0) + (p.tb ? 1 : 0);
  if (vec || VECONLY) {
    switch (sel) {
      case 0: launch_one<T, BM, BN, AC, BC, 0, 0, V, BK>(st, p, splits); break;
      case 1: launch_one<T, BM, BN, AC, BC, 0, 1, V, BK>(st, p, splits); break;
      case 2: launch_one<T, BM, BN, AC, BC, 1, 0, V, BK>(st, p, splits); break;
      default: launch_one<T, BM, BN, AC, BC, 1, 1, V, BK>(st, p, splits); break;
    }
  } else {
    switch (sel) {
      case 0: launch_one<T, BM, BN, AC, BC, 0, 0, 1, BK>(st, p, splits); break;
      case 1: launch_one<T, BM, BN, AC, BC, 0, 1, 1, BK>(st, p, splits); break;
      case 2: launch_one<T, BM, BN, AC, BC, 1, 0, 1, BK>(st, p, splits); break;
      default: launch_one<T, BM, BN, AC, BC, 1, 1, 1, BK>(st, p, splits); break;
    }
  }
}

// VECONLY: instantiated for 16-byte-aligned operands only (the caller falls back to 64 x 64 tiles)
template <typename T, int BM, int BN, int BK = kBK, bool VECONLY = false>
static void launch_typed(hipStream_t st, const GemmParams<T>& p, int splits, bool vec) {
  const int sel = (p.Aim ? 2 : 0) + (p.Bim ? 1 : 0);
  switch (sel) {
    case 0: launch_gemm<T, BM, BN, 0, 0, BK, VECONLY>(st, p, splits, vec); break;
    case 1: launch_gemm<T, BM, BN, 0, 1, BK, VECONLY>(st, p, splits, vec); break;
    case 2: launch_gemm<T, BM, BN, 1, 0, BK, VECONLY>(st, p, splits, vec); break;
    default: launch_gemm<T, BM, BN, 1, 1, BK, VECONLY>(st, p, splits, vec); break;
  }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// ---- tuning table -------------------------------------------------------------------------------
namespace {
struct TuneKey {
  int prec, ac, bc, ta, tb;
  int64_t M, N, K;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, M, N, K, ac, bc, ta, tb) < std::tie(o.prec, o.M, o.N, o.K, o.ac, o.bc, o.ta, o.tb);
  }
};
std::map<TuneKey, GemmChoice> g_tune;
std::mutex g_tune_mu;

// the tile configurations the dispatcher below instantiates: {bm * 1000 + bn, bk, aligned operands only}
struct TileCfg {
  int mn, bk;
  bool veconly;
};
constexpr TileCfg kTileCfgs[] = {{64064, kBK, false}, {128128, kBK, false}, {32064, 32, true}, {32128, 16, true},
                                 {64032, 32, true},   {64096, 32, true},    {32032, 64, true}, {32096, 32, true},
                                 {96032, 32, true},   {32096, 64, true},    {64032, 64, true}, {32064, 64, true}};
}  // namespace

GemmChoice tuned_choice(int prec, int64_t M, int64_t N, int64_t K, bool ac, bool bc, int ta, int tb) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.empty()) return GemmChoice();
  auto it = g_tune.find(TuneKey{prec, ac, bc, ta != 0, tb != 0, M, N, K});
  return it == g_tune.end() ? GemmChoice() : it->second;
}

int load_tuning(const char* path) {
  std::map<TuneKey, GemmChoice> tab;
  if (path) {
    FILE* f = fopen(path, "r");
    RTCC_CHECK(f != nullptr, kEInval, std::string("cannot open tuning table ") + path);
    char line[512];
    int ln = 0;
    while (fgets(line, sizeof line, f)) {
      ++ln;
      char* hash = strchr(line, '#');
      if (hash) *hash = 0;
      long long M, N, K;
      int prec, ac, bc, ta, tb;
      GemmChoice c;
      const int got = sscanf(line, "%d %lld %lld %lld %d %d %d %d %d %d %d %d", &prec, &M, &N, &K, &ac, &bc, &ta, &tb,
                             &c.kind, &c.p1, &c.p2, &c.splits);
      if (got <= 0) continue;  // blank or comment line
      const bool ok = got == 12 && prec >= 0 && prec <= 2 && M > 0 && N > 0 && K > 0 && c.kind >= 0 && c.kind <= 2 &&
                      c.splits >= 0;
      if (!ok) {
        fclose(f);
        throw Error(kEInval, std::string("malformed tuning table line ") + std::to_string(ln) + " in " + path);
      }
      tab[TuneKey{prec, ac != 0, bc != 0, ta != 0, tb != 0, M, N, K}] = c;
    }
    fclose(f);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(tab);
  return (int)g_tune.size();
}

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
  // kernel choice: forced (kernel tests, the autotuner), else the tuning table, else the rules below
  GemmChoice ch;
  if (E.force) ch = *E.force;
  else if (E.use_tuning && nbt == 1 && M > 1 && N > 1)
    ch = tuned_choice(sizeof(T) == 8 ? 0 : E.bf16x3 ? 2 : 1, M, N, K, AC, BC, A.trans, B.trans);
  if constexpr (sizeof(T) == 4) {
    if (ch.kind == 2) {
      const bool done = nbt == 1 && E.bf16x3 && gemm_bf16x3(E, M, N, K, alpha, A, B, Cre, Cim, ldc, beta, ch.p1,
                                                           ch.splits, ch.p2);
      RTCC_CHECK(done || !E.force, kEInval, "gemm: the split-BF16 kernel cannot take this product");
      if (done) return;
      ch = GemmChoice();
    } else if (ch.kind == 0 && nbt == 1 && E.bf16x3 && 2.0 * (double)M * (double)N * (double)K >= E.bf16_min_flops &&
               gemm_bf16x3(E, M, N, K, alpha, A, B, Cre, Cim, ldc, beta)) {
      return;
    }
  }
  RTCC_CHECK(ch.kind != 2, kEInval, "gemm: the split-BF16 kernel needs FP32 operands");
  if (ch.kind == 0 && nbt == 1 && (M == 1 || N == 1)) {
    int splits;
    if (M == 1)  // x(k) = A(0, k), W(k, n) = B(k, n), y(n) = C(0, n)
      splits = gemv<T>(E, B.trans != 0, N, K, alpha, A.re, A.im, A.trans ? A.ld : 1, B.re, B.im, B.ld, Cre, Cim, 1,
                       beta);
    else  // x(k) = B(k, 0), W(k, m) = A(m, k), y(m) = C(m, 0)
      splits = gemv<T>(E, A.trans == 0, M, K, alpha, B.re, B.im, B.trans ? 1 : B.ld, A.re, A.im, A.ld, Cre, Cim, ldc,
                       beta);
    E.gemm_flops += 2 * M * N * K * ((AC && BC) ? 4 : (AC || BC) ? 2 : 1);
    if (E.trace)
      fprintf(stderr, "[rtcc] gemv M=%lld N=%lld K=%lld %s%s ta=%d tb=%d splits=%d\n", (long long)M, (long long)N,
              (long long)K, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans, splits);
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
  // Tile choice (measured on skinny shapes, which are latency- and bandwidth-bound):
  //  - short K (<= 256) with one side of at most 32 (96 against a very long other side): a thin tile
  //    along the long side; the whole K of a tile is a few stages;
  //  - an output of at most 128 x 128 with long K: a tile fitted to the output and K split into
  //    ~512-2048 fixed-order partial sums;
  //  - FP32 with >= 512 tiles of 128 x 128: those; otherwise 64 x 64, K split when the grid is small.
  if (ch.kind == 0 && M * N <= 8192 && K <= 256) {
    p.kchunk = (int)K;
    p.splits = 1;
    p.split_stride = 0;
    p.Cre = Cre;
    p.Cim = Cim;
    p.ldc = ldc;
    const dim3 grid((unsigned)cdiv(M * N, 16), (unsigned)nbt);
    const int sel = (AC ? 2 : 0) + (BC ? 1 : 0);
    switch (sel) {
      case 0: hipLaunchKernelGGL((gemm_dot_kernel<T, 0, 0>), grid, dim3(256), 0, E.stream, p); break;
      case 1: hipLaunchKernelGGL((gemm_dot_kernel<T, 0, 1>), grid, dim3(256), 0, E.stream, p); break;
      case 2: hipLaunchKernelGGL((gemm_dot_kernel<T, 1, 0>), grid, dim3(256), 0, E.stream, p); break;
      default: hipLaunchKernelGGL((gemm_dot_kernel<T, 1, 1>), grid, dim3(256), 0, E.stream, p); break;
    }
    RTCC_HIP(hipGetLastError());
    E.gemm_flops += 2 * M * N * K * nbt * ((AC && BC) ? 4 : (AC || BC) ? 2 : 1);
    if (E.trace)
      fprintf(stderr, "[rtcc] gemm M=%lld N=%lld K=%lld batch=%d %s%s ta=%d tb=%d dot\n", (long long)M, (long long)N,
              (long long)K, nbt, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans);
    return;
  }
  const int narrow = K > 256                                            ? 0
                     : (M <= 32 && N >= 256) || (M <= 96 && N >= 8192)   ? 1
                     : (N <= 32 && M >= 256) || (N <= 96 && M >= 8192)   ? 2
                                                                         : 0;
  const bool skinny = !narrow && M <= 128 && N <= 128 && K >= 512 && vec;
  const bool large = !narrow && !skinny && sizeof(T) == 4 && cdiv(M, 128) * cdiv(N, 128) * nbt >= 512;
  int BM = 64, BN = 64, BK = kBK, target = 1024;
  if (narrow == 1) {
    BM = 32;
    BN = K <= 32 ? 64 : 128;
    BK = K <= 32 ? 32 : 16;
  } else if (narrow == 2) {
    BM = 64;
    BN = N <= 32 ? 32 : 96;
    BK = 32;
  } else if (skinny) {
    if (M <= N || M <= 32) {
      BM = 32;
      BN = N <= 32 ? 32 : N <= 64 ? 64 : N <= 96 ? 96 : 128;
    } else {
      BN = 32;
      BM = M <= 64 ? 64 : 96;
    }
    BK = BM == 32 && BN == 32 ? 64 : BN == 128 ? 16 : 32;
    target = BM * BN <= 1024 ? 2048 : BM * BN <= 2048 ? 1024 : 512;
  } else if (large) {
    BM = BN = 128;
  }
  const bool fixed = narrow || large;
  if (narrow && !vec) BM = BN = 64, BK = kBK;  // thin tiles are built for aligned operands only
  const int64_t tiles = cdiv(M, BM) * cdiv(N, BN) * nbt;
  int splits = 1;
  if (skinny) {
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({target / tiles, cdiv(K, 64), 65535 / nbt}));
  } else if (!fixed && tiles < 512 && K >= 512) {
    // fewer than ~2 workgroups per CU: split K (chunks of >= 256) toward ~1024 workgroups
    int64_t want = std::max<int64_t>(1, 1024 / tiles);
    splits = (int)std::min<int64_t>({want, cdiv(K, 256), 1024, 65535 / nbt});
  }
  if (ch.kind == 1) {
    const TileCfg* cfg = nullptr;
    for (const TileCfg& c : kTileCfgs)
      if (c.mn == ch.p1 && c.bk == ch.p2 && (sizeof(T) == 4 || c.mn != 128128)) cfg = &c;
    const bool ok = cfg && (vec || !cfg->veconly) && ch.splits >= 1;
    RTCC_CHECK(ok || !E.force, kEInval, "gemm: the chosen tile kernel is not available for this product");
    if (ok) {
      BM = ch.p1 / 1000;
      BN = ch.p1 % 1000;
      BK = ch.p2;
      splits = (int)std::min<int64_t>({(int64_t)ch.splits, cdiv(K, BK), 65535 / nbt});
    }
  }
  int64_t kchunk = cdiv(cdiv(K, splits), BK) * BK;
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
  const int z = nbt * splits;
  const int cfg = BM * 1000 + BN;
  // timing of the large complex x complex products, those the split-BF16 context gives the split kernel
  // (2 M N K >= bf16_min_flops): the tile kernel alone (see Engine::mark_mode)
  const double cc_flops = 8.0 * M * N * K * nbt;
  const bool ccm = E.mark && E.mark_mode == 2 && AC && BC && 2.0 * M * N * K * nbt >= E.bf16_min_flops &&
                   !(sizeof(T) == 4 && E.bf16x3);
  const double cc_bytes =
      2.0 * sizeof(T) * nbt * (M * K + K * N + M * N * (beta != 0.0 ? 2 : 1));
  if (ccm) E.mark(E.mark_user, 0, cc_flops, cc_bytes, E.stream);
  const bool lm = E.ladder && E.mark && E.mark_mode == 1;  // a ladder GEMM (its kernel alone)
  if (lm) E.mark(E.mark_user, 0, E.ladder_flops, 0.0, E.stream);
  if (BK == kBK && BM == 64 && BN == 64) launch_typed<T, 64, 64>(E.stream, p, z, vec);
  else if (cfg == 128128) {
    if constexpr (sizeof(T) == 4) launch_typed<T, 128, 128>(E.stream, p, z, vec);
  } else if (cfg == 32064 && BK == 32) launch_typed<T, 32, 64, 32, true>(E.stream, p, z, vec);
  else if (cfg == 32064 && BK == 64) launch_typed<T, 32, 64, 64, true>(E.stream, p, z, vec);
  else if (cfg == 32128) launch_typed<T, 32, 128, 16, true>(E.stream, p, z, vec);
  else if (cfg == 64032 && BK == 32) launch_typed<T, 64, 32, 32, true>(E.stream, p, z, vec);
  else if (cfg == 64032 && BK == 64) launch_typed<T, 64, 32, 64, true>(E.stream, p, z, vec);
  else if (cfg == 64096) launch_typed<T, 64, 96, 32, true>(E.stream, p, z, vec);
  else if (cfg == 32032) launch_typed<T, 32, 32, 64, true>(E.stream, p, z, vec);
  else if (cfg == 32096 && BK == 32) launch_typed<T, 32, 96, 32, true>(E.stream, p, z, vec);
  else if (cfg == 32096 && BK == 64) launch_typed<T, 32, 96, 64, true>(E.stream, p, z, vec);
  else if (cfg == 96032) launch_typed<T, 96, 32, 32, true>(E.stream, p, z, vec);
  else RTCC_CHECK(false, kEInval, "gemm: no kernel for the chosen tile");
  if (ccm) E.mark(E.mark_user, 1, cc_flops, cc_bytes, E.stream);
  if (lm) E.mark(E.mark_user, 1, E.ladder_flops, 0.0, E.stream);
  if (splits > 1) splitk_reduce_launch<T>(E.stream, Pre, Pim, splits, M, N, Cre, Cim, ldc, bt.c, nbt, alpha, beta);
  E.scratch.reset(mark);
  E.gemm_flops += 2 * M * N * K * nbt * ((AC && BC) ? 4 : (AC || BC) ? 2 : 1);
  if (E.trace)
    fprintf(stderr, "[rtcc] gemm M=%lld N=%lld K=%lld batch=%d %s%s ta=%d tb=%d tile=%dx%dx%d splits=%d vec=%d\n",
            (long long)M, (long long)N, (long long)K, nbt, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans, BM,
            BN, BK, splits, (int)vec);
}

template <typename T>
void gemv_strided(Engine& E, int64_t N, int64_t K, double alpha, const T* xre, const T* xim, int64_t incx,
                  const T* wre, const T* wim, int64_t N2, int64_t sn1, int64_t sn2, int64_t K2, int64_t sk1,
                  int64_t sk2, T* yre, T* yim, int64_t incy, double beta) {
  if (N <= 0) return;
  RTCC_CHECK(N < (1LL << 31) && K < (1LL << 31) && N2 >= 1 && K2 >= 1 && N % N2 == 0 && (K == 0 || K % K2 == 0),
             kEInval, "gemv_strided: bad extents");
  const bool XC = xim != nullptr, WC = wim != nullptr;
  RTCC_CHECK(yim || (!XC && !WC), kEInval, "gemv_strided: complex product into a real output");
  if (K <= 0) {
    int64_t d[1] = {N}, st[1] = {incy};
    permute_axpby<T>(E.stream, 1, d, yre, yim, st, yre, yim, st, 0.0, beta);
    return;
  }
  if (!XC && !WC && yim) {  // real product into a complex output: the imaginary plane is only scaled
    int64_t d[1] = {N}, st[1] = {incy};
    permute_axpby<T>(E.stream, 1, d, yim, (T*)nullptr, st, yim, (T*)nullptr, st, 0.0, beta);
    yim = nullptr;
  }
  // lanes along the index with unit (or the smaller) innermost stride
  const bool col = !(sn2 == 1 || (sk2 != 1 && sn2 < sk2));
  const GemvLayout L{N2, sn1, sn2, K2, sk1, sk2};
  const int splits = gemv<T>(E, col, N, K, alpha, xre, xim, incx, wre, wim, 0, yre, yim, incy, beta, &L);
  E.gemm_flops += 2 * N * K * ((XC && WC) ? 4 : (XC || WC) ? 2 : 1);
  if (E.trace)
    fprintf(stderr,
            "[rtcc] gemv-strided N=%lld (%lld x %lld: %lld %lld) K=%lld (%lld x %lld: %lld %lld) %s%s %s splits=%d\n",
            (long long)N, (long long)(N / N2), (long long)N2, (long long)sn1, (long long)sn2, (long long)K,
            (long long)(K / K2), (long long)K2, (long long)sk1, (long long)sk2, XC ? "c" : "r", WC ? "c" : "r",
            col ? "col" : "row", splits);
}

template void gemv_strided<double>(Engine&, int64_t, int64_t, double, const double*, const double*, int64_t,
                                   const double*, const double*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                   double*, double*, int64_t, double);
template void gemv_strided<float>(Engine&, int64_t, int64_t, double, const float*, const float*, int64_t,
                                  const float*, const float*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                  float*, float*, int64_t, double);

template void gemm<double>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<double>, GemmOp<double>, double*,
                           double*, int64_t, double, GemmBatch);
template void gemm<float>(Engine&, int64_t, int64_t, int64_t, double, GemmOp<float>, GemmOp<float>, float*, float*,
                          int64_t, double, GemmBatch);

}  // namespace rtcc
