// Split-BF16 three-term MFMA GEMM on FP32 planar-complex / real operands (gfx950).
//
// Each FP32 operand element x is split as hi = bf16(x), lo = bf16(x - hi), and every real product
// is formed as hi*hi' + hi*lo' + lo*hi' with v_mfma_f32_32x32x16_bf16, accumulated in FP32 (the
// dropped lo*lo' term is ~2^-16 of the product). The split is a separate pass that also brings both
// operands into one layout, "packed": per plane (Re hi, Re lo[, Im hi, Im lo]) a bf16 matrix of
// [rows][K] stored k-blocked and half-major as [K / 16][2][rows][8] (the 8 k of one half of a 16-wide
// k block of a row are 16 contiguous bytes, and the rows of one half follow each other), rows padded
// to a multiple of the tile's rows (128 for A, 256 for B) and K to a multiple of 32 with zeros, so
// the GEMM copies whole contiguous stage tiles without bounds checks, and a stage tile copied as is
// into LDS serves the MFMA fragments without bank conflicts (lanes 0-31 read rows r..r+31 of half 0,
// lanes 32-63 the same rows of half 1: two contiguous 512-byte runs). Packed layouts of constant
// operands (the integrals) are made once and cached.
//
// GEMM: 512 threads, a 128 x 256 output tile per workgroup, 2 x 4 waves of 64 x 64 (2 x 2 MFMA
// blocks of 32 x 32 each), two waves per SIMD so that one wave's MFMAs cover the other's LDS and
// barrier waits; the wide N side halves the B-plane traffic per flop (outputs too small for 16 such
// tiles take 2 x 2 waves of 256 threads and 128 x 128 tiles instead). Two ways to feed LDS, one per
// kernel: (register-staged) per 16-wide k stage the packed tiles pass through registers into one of
// two padded LDS buffers: stage s + 1 is written and stage s + 2 fetched while stage s is multiplied;
// (DMA ring) the stage tiles go from memory straight into a ring of three or four LDS buffers with
// 16-byte direct-to-LDS loads, issued two or three stages ahead, so no registers or LDS write
// instructions carry them. Both take one barrier per stage. Lane l of a
// 32x32x16 MFMA holds A[l%32][8(l/32)+j] and B[8(l/32)+j][l%32] and its output r lies at row
// 8(r/4) + 4(l/32) + r%4, column l%32. Small grids split K into fixed-order partial sums.
// Workgroups are numbered so that each of the eight XCDs (which take workgroups round-robin) works
// on a contiguous band of tiles.
#include <cstdint>
#include <cstdio>
#include <string>

#include "engine.h"

namespace rtcc {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16 __attribute__((ext_vector_type(16)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 128;             // output tile rows; columns 64 * WN (WN waves along N)
constexpr int kBK = 32;              // k stage
constexpr int kRowPad = 128;         // packed rows are a multiple of this (of 256 for wide B tiles)
constexpr int kKPad = 32;            // packed K is a multiple of this

// ---- packing ------------------------------------------------------------------------------------
// dst plane (2 c + h) = h ? lo : hi of plane c of the source, k-blocked as [Kp / 16][2][Rp][8]: one
// 16-wide k stage of 128 rows is two contiguous 2 KB runs. Element (r, k) of the source is
// src[r * ld + k] (trans = 0) or src[k * ld + r] (trans = 1). A thread makes one row's 16-wide k
// block: consecutive lanes take consecutive rows, so the 16-byte chunks they store are contiguous;
// the loads are four 16-byte vectors (trans = 0, aligned; the two halves of a wave read the two
// halves of each row's 128-byte run) or 16 loads coalesced across rows (trans = 1).
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ sre, const float* __restrict__ sim,
                                                   int64_t ld, int trans, int R, int K, int Rp, int Kp, int vec,
                                                   __bf16* __restrict__ dst) {
  // a wave takes 32 rows and two neighbouring k blocks: lanes 0-31 block 2 y, lanes 32-63 block 2 y + 1,
  // so with trans = 0 each row's 128-byte run is read by one load instruction
  const int t = threadIdx.x, r = blockIdx.x * 128 + (t >> 6) * 32 + (t & 31);
  const int kb = 2 * blockIdx.y + ((t >> 5) & 1), k0 = kb * 16;
  if (r >= Rp || kb * 16 >= Kp) return;
  const int64_t plane = (int64_t)Rp * Kp;
  const int64_t o0 = ((int64_t)(2 * kb) * Rp + r) * 8, o1 = o0 + (int64_t)Rp * 8;  // halves k0..7, k8..15
  const int np = sim ? 2 : 1;
  for (int c = 0; c < np; ++c) {
    const float* src = c ? sim : sre;
    float x[16];
    if (r < R && vec && k0 + 16 <= K) {
      const float4* p4 = reinterpret_cast<const float4*>(src + (int64_t)r * ld + k0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 f = p4[q];
        x[4 * q] = f.x;
        x[4 * q + 1] = f.y;
        x[4 * q + 2] = f.z;
        x[4 * q + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = k0 + kk;
        x[kk] = (r < R && k < K) ? src[trans ? (int64_t)k * ld + r : (int64_t)r * ld + k] : 0.f;
      }
    }
    bf8 hi[2], lo[2];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const __bf16 h = (__bf16)x[kk];
      hi[kk >> 3][kk & 7] = h;
      lo[kk >> 3][kk & 7] = (__bf16)(x[kk] - (float)h);
    }
    __bf16* dh = dst + (2 * c) * plane;
    __bf16* dl = dst + (2 * c + 1) * plane;
    *reinterpret_cast<bf8*>(dh + o0) = hi[0];
    *reinterpret_cast<bf8*>(dh + o1) = hi[1];
    *reinterpret_cast<bf8*>(dl + o0) = lo[0];
    *reinterpret_cast<bf8*>(dl + o1) = lo[1];
  }
}

struct Packed {
  const __bf16* p = nullptr;
  int64_t plane = 0;  // elements per plane
  int Rp = 0, Kp = 0, np = 1;
};

Packed pack_operand(Engine& E, const float* re, const float* im, int64_t ld, int trans, int64_t R, int64_t K,
                    bool konst, int rowpad) {
  Packed P;
  P.Rp = (int)(cdiv(R, rowpad) * rowpad);
  P.Kp = (int)(cdiv(K, kKPad) * kKPad);
  P.np = im ? 2 : 1;
  P.plane = (int64_t)P.Rp * P.Kp;
  const size_t bytes = (size_t)P.plane * 2 * P.np * sizeof(__bf16);
  RTCC_CHECK(P.Kp / 32 <= 65535, kEInval, "gemm_bf16x3: K too large");
  const bool vec = !trans && ld % 4 == 0 && ((uintptr_t)re % 16) == 0 && (!im || ((uintptr_t)im % 16) == 0);
  const dim3 grid((unsigned)cdiv(P.Rp, 128), (unsigned)(P.Kp / 32));
  auto fill = [&](void* dst, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, st, re, im, ld, trans, (int)R, (int)K, P.Rp, P.Kp, (int)vec,
                       (__bf16*)dst);
    RTCC_HIP(hipGetLastError());
  };
  char key[160];
  snprintf(key, sizeof key, "bf16x3:%p/%p/%lld/%d/%lld/%lld/%d", (const void*)re, (const void*)im, (long long)ld,
           trans, (long long)R, (long long)K, P.Rp);
  if (konst && E.cache) {
    P.p = (const __bf16*)const_cache_get(E.cache, key, bytes, fill);
    return P;
  }
  if (memo_fixed(E, re)) {
    // an operand fixed for the current call: packed once, reused by later products of this call
    bool hit = false;
    void* dst = memo_get(E, key, bytes, &hit);
    if (dst) {
      if (!hit) fill(dst, E.stream);
      if (E.trace) fprintf(stderr, "[rtcc] memo-pack %s src=%p\n", hit ? "hit" : "new", (const void*)re);
      P.p = (const __bf16*)dst;
      return P;
    }
  }
  {
    if (E.trace)
      fprintf(stderr, "[rtcc] pack-operand src=%p ld=%lld trans=%d R=%lld K=%lld\n", (const void*)re, (long long)ld, trans,
              (long long)R, (long long)K);
    void* dst = E.scratch.get<char>((int64_t)bytes);
    fill(dst, E.stream);
    P.p = (const __bf16*)dst;
  }
  return P;
}

// ---- GEMM ---------------------------------------------------------------------------------------
struct Params {
  const __bf16* A;  // packed [NA * 2][Mp][Kp]
  const __bf16* B;  // packed [NB * 2][Np][Kp]
  int64_t pa, pb;   // plane strides
  int Kp, Mp, Np;   // padded K and rows
  int M, N;
  int tiles_m, tiles_n, ntiles;
  int band;  // output-tile rows per band of the workgroup -> tile map
  int kchunk, splits;
  float* Cre;
  float* Cim;
  int64_t ldc;
  int64_t split_stride;  // > 0: write partial planes [split][M][N]
  float alpha, beta;
};

__device__ inline bf8 neg(bf8 x) {
  us8 u = __builtin_bit_cast(us8, x);
  u ^= (unsigned short)0x8000;
  return __builtin_bit_cast(bf8, u);
}

__device__ inline f16 mma(bf8 a, bf8 b, f16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }

// Split and tile (tm, tn) of workgroup b: the eight XCDs take workgroups round-robin; renumber so
// XCD x owns a contiguous range of (split, tile) pairs, split slowest, and walk the tiles of one
// split in bands of p.band tile rows (tiles of a band share B columns, all share the split's k range).
__device__ inline void tile_of(int b, const Params& p, int* split, int* tm, int* tn) {
  const int n = p.ntiles * p.splits, q = n / 8, r = n % 8, x = b % 8, j = b / 8;
  const int lin = x * q + min(x, r) + j;
  *split = lin / p.ntiles;
  const int id = lin - *split * p.ntiles;
  const int G = p.band;
  const int band = id / (G * p.tiles_n);
  const int first = band * G;
  const int rows = min(G, p.tiles_m - first);
  const int in = id - band * G * p.tiles_n;
  *tm = first + in % rows;
  *tn = in / rows;
}

// Epilogue of one wave's 64 x 64 output block at (r0, c0): alpha * acc + beta * C, or the raw partial
// sums into split plane `split`. With beta != 0 the old C values of each 32 x 32 block are all loaded
// before its stores (a store may alias a later load, so loads interleaved with stores would each wait
// a full memory latency).
template <int AC, int BC, int NJ>
__device__ inline void store_tile(const Params& p, const f16 (&accr)[2][NJ], const f16 (&acci)[2][NJ], int split,
                                  int r0, int c0, int lane) {
  constexpr bool CC = AC || BC;
  const int l32 = lane & 31;
  const bool acc = !p.split_stride && p.beta != 0.f;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      float oldr[16], oldi[16];
      if (acc) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = r0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int col = c0 + j * 32 + l32;
          const bool ok = row < p.M && col < p.N;
          const int64_t off = (int64_t)row * p.ldc + col;
          oldr[r] = ok ? p.Cre[off] : 0.f;
          oldi[r] = (CC && ok) ? p.Cim[off] : 0.f;
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = r0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = c0 + j * 32 + l32;
        if (row >= p.M || col >= p.N) continue;
        const float vr = accr[i][j][r], vi = acci[i][j][r];
        if (p.split_stride) {
          const int64_t off = (int64_t)split * p.split_stride + (int64_t)row * p.N + col;
          p.Cre[off] = vr;
          if (CC) p.Cim[off] = vi;
        } else {
          const int64_t off = (int64_t)row * p.ldc + col;
          float outr = p.alpha * vr, outi = p.alpha * vi;
          if (acc) {
            outr += p.beta * oldr[r];
            outi += p.beta * oldi[r];
          }
          p.Cre[off] = outr;
          if (CC) p.Cim[off] = outi;
        }
      }
      // one 32 x 32 block at a time: keeps the scheduler from holding every block's values in registers
      __builtin_amdgcn_sched_barrier(0);
    }
}

// The three split products of one 16-wide k step for one wave: (hi, hi), (hi, lo), (lo, hi) for every
// pair of its 2 x 2 blocks; packed plane index 2 c + h.
template <int AC, int BC>
__device__ inline void mma_step(const bf8 (&af)[2][2 * (AC ? 2 : 1)], const bf8 (&bfr)[2][2 * (BC ? 2 : 1)],
                                f16 (&accr)[2][2], f16 (&acci)[2][2]) {
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int ha = t == 2 ? 1 : 0, hb = t == 1 ? 1 : 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) accr[i][j] = mma(af[i][ha], bfr[j][hb], accr[i][j]);
    if (BC) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acci[i][j] = mma(af[i][ha], bfr[j][2 + hb], acci[i][j]);
    }
    if (AC) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acci[i][j] = mma(af[i][2 + ha], bfr[j][hb], acci[i][j]);
    }
    if (AC && BC) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accr[i][j] = mma(neg(af[i][2 + ha]), bfr[j][2 + hb], accr[i][j]);
    }
  }
}

template <int N>
__device__ inline void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

typedef __attribute__((address_space(3))) void* lds_ptr;

// Fragments (16 bytes per lane) from LDS: NA at byte addresses ba + OA[i] and NB at bb + OB[i], read
// in one asm block that waits for them before it ends. The compiler does not see these reads, so it
// puts none of its own waits for the direct-to-LDS loads in front of them (it cannot tell the ring
// buffers apart and would drain every load in flight); the kernel orders them with its explicit waits
// and barriers. The offsets are template arguments (ds_read_b128 immediates).
#define RTCC_DSR(o, a, n) "ds_read_b128 %" #o ", %" #a " offset:%" #n "\n"
template <int A0, int A1, int A2, int A3, int A4, int A5, int A6, int A7, int B0, int B1, int B2, int B3>
__device__ inline void lds_read_8_4(unsigned ba, unsigned bb, u4 (&a)[8], u4 (&b)[4]) {
  asm volatile(RTCC_DSR(0, 12, 14) RTCC_DSR(1, 12, 15) RTCC_DSR(2, 12, 16) RTCC_DSR(3, 12, 17) RTCC_DSR(4, 12, 18)
                   RTCC_DSR(5, 12, 19) RTCC_DSR(6, 12, 20) RTCC_DSR(7, 12, 21) RTCC_DSR(8, 13, 22) RTCC_DSR(9, 13, 23)
                       RTCC_DSR(10, 13, 24) RTCC_DSR(11, 13, 25) "s_waitcnt lgkmcnt(0)"
               : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3]), "=&v"(a[4]), "=&v"(a[5]), "=&v"(a[6]),
                 "=&v"(a[7]), "=&v"(b[0]), "=&v"(b[1]), "=&v"(b[2]), "=&v"(b[3])
               : "v"(ba), "v"(bb), "n"(A0), "n"(A1), "n"(A2), "n"(A3), "n"(A4), "n"(A5), "n"(A6), "n"(A7), "n"(B0),
                 "n"(B1), "n"(B2), "n"(B3));
}
template <int O0, int O1, int O2, int O3, int O4, int O5, int O6, int O7>
__device__ inline void lds_read_8(unsigned base, u4 (&a)[8]) {
  asm volatile(RTCC_DSR(0, 8, 9) RTCC_DSR(1, 8, 10) RTCC_DSR(2, 8, 11) RTCC_DSR(3, 8, 12) RTCC_DSR(4, 8, 13)
                   RTCC_DSR(5, 8, 14) RTCC_DSR(6, 8, 15) RTCC_DSR(7, 8, 16) "s_waitcnt lgkmcnt(0)"
               : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3]), "=&v"(a[4]), "=&v"(a[5]), "=&v"(a[6]),
                 "=&v"(a[7])
               : "v"(base), "n"(O0), "n"(O1), "n"(O2), "n"(O3), "n"(O4), "n"(O5), "n"(O6), "n"(O7));
}
#undef RTCC_DSR


// DMA-ring kernel. LDS holds NBUF stage images, each the plain copy of the stage's packed tiles: A
// planes [PA][2][128][8] then B planes [PB][2][BN][8] (bf16). Each wave copies D 1 KB pieces of a stage
// with 16-byte direct-to-LDS loads (lane l: bytes 16 l .. 16 l + 15 of the piece). Stage s + NBUF - 1
// is requested right after the barrier of stage s, into the buffer stage s - 1 used; before that
// barrier each wave waits until at most the loads of the later stages it has requested are still in
// flight (s_waitcnt counts one wave's memory instructions in order), so after the barrier every
// wave's share of stage s is in LDS. The main loop is unrolled by NBUF so every buffer index is a
// constant.
// TWO = 1: at most half the LDS and 256 registers per lane, so that two workgroups share a CU (their
// barriers are independent, so one's MFMAs run while the other waits at a stage boundary).
template <int AC, int BC, int LADDER, int WN, int TWO>
__global__ __launch_bounds__(128 * WN, 2) void gemm_bf16x3_dma(Params p) {
  constexpr int kThr = 128 * WN, kBN = 64 * WN, NW = kThr / 64;
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  constexpr int PA = 2 * NA, PB = 2 * NB;
  constexpr int SK = 16;
  constexpr int ACH = PA * 2 * kBM, BCH = PB * 2 * kBN;  // 16-byte pieces per stage
  constexpr int SB = (ACH + BCH) * 16;                   // stage bytes
  constexpr int LDSB = TWO ? 80 * 1024 : 160 * 1024;
  constexpr int NBUF = LDSB / SB >= 4 ? 4 : LDSB / SB >= 3 ? 3 : 2;
  static_assert(SB * NBUF <= LDSB, "LDS ring too large");
  constexpr int NI = (ACH + BCH) / 64;  // 1 KB loads per stage
  static_assert(NI % NW == 0 && (ACH / 64) * 64 == ACH, "stage does not divide among the waves");
  constexpr int D = NI / NW;            // loads per wave and stage
  __shared__ __attribute__((aligned(1024))) char ring[NBUF][SB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int split, tm, tn;
  tile_of(blockIdx.x, p, &split, &tm, &tn);
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int kbeg = split * p.kchunk, kend = min(p.Kp, kbeg + p.kchunk);
  const int nst = (kend - kbeg) / SK;

  // source of this wave's load d (piece j = wave * D + d): plane, half and first row of a 64-row run
  const __bf16* src[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int j = wave * D + d, q = j * 64;  // first piece of the load
    if (q < ACH) {
      const int pl = q / (2 * kBM), h = (q / kBM) & 1, r = q % kBM;
      src[d] = p.A + pl * p.pa + ((int64_t)h * p.Mp + m0 + r + lane) * 8;
    } else {
      const int qb = q - ACH;
      const int pl = qb / (2 * kBN), h = (qb / kBN) & 1, r = qb % kBN;
      src[d] = p.B + pl * p.pb + ((int64_t)h * p.Np + n0 + r + lane) * 8;
    }
  }
  // k block kb of a plane starts 2 kb rows-of-halves later
  const int64_t stepA = (int64_t)2 * p.Mp * 8, stepB = (int64_t)2 * p.Np * 8;
  auto request = [&](int st, char* buf) {
    const int64_t kb = kbeg / SK + st;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int j = wave * D + d;
      const __bf16* g = src[d] + kb * (j * 64 < ACH ? stepA : stepB);
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_ptr)(buf + j * 1024), 16, 0, 0);
    }
  };

  f16 accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        accr[i][j][e] = 0.f;
        acci[i][j][e] = 0.f;
      }

  const int l32 = lane & 31, hh = lane >> 5;
#pragma unroll
  for (int u = 0; u < NBUF - 1; ++u)
    if (u < nst) request(u, ring[u]);
  for (int base = 0; base < nst; base += NBUF) {
#pragma unroll
    for (int u = 0; u < NBUF; ++u) {
      const int s = base + u;
      if (s < nst) {
        // loads of later stages this wave may leave in flight: min(NBUF - 2, nst - 1 - s) stages
        const int later = min(NBUF - 2, nst - 1 - s);
        if (later >= 2) wait_vmcnt<2 * D>();
        else if (later == 1) wait_vmcnt<D>();
        else wait_vmcnt<0>();
        asm volatile("s_barrier" ::: "memory");
        if (s + NBUF - 1 < nst) request(s + NBUF - 1, ring[(u + NBUF - 1) % NBUF]);
        // fragment (i, pl) of A at byte ((pl * 2 + hh) * 128 + wm * 64 + i * 32 + l32) * 16 of the buffer,
        // (j, pl) of B at ACH * 16 + ((pl * 2 + hh) * BN + wn * 64 + j * 32 + l32) * 16
        const unsigned ba = (unsigned)(uintptr_t)(lds_ptr)ring[u] + (unsigned)((hh * kBM + wm * 64 + l32) * 16);
        const unsigned bb =
            (unsigned)(uintptr_t)(lds_ptr)ring[u] + (unsigned)(ACH * 16 + (hh * kBN + wn * 64 + l32) * 16);
        constexpr int PLA = 2 * kBM * 16, PLB = 2 * kBN * 16;  // bytes per packed plane in a stage
        // fragment arrays ordered [block][plane]: A (i, pl) at i * PA + pl, B (j, pl) at j * PB + pl
        u4 fa[2 * PA], fb[2 * PB];
        if constexpr (PA == 4 && PB == 2) {
          lds_read_8_4<0, PLA, 2 * PLA, 3 * PLA, 512, PLA + 512, 2 * PLA + 512, 3 * PLA + 512, 0, PLB, 512,
                       PLB + 512>(ba, bb, fa, fb);
        } else if constexpr (PA == 2 && PB == 4) {
          lds_read_8_4<0, PLB, 2 * PLB, 3 * PLB, 512, PLB + 512, 2 * PLB + 512, 3 * PLB + 512, 0, PLA, 512,
                       PLA + 512>(bb, ba, fb, fa);
        } else {
          lds_read_8<0, PLA, 2 * PLA, 3 * PLA, 512, PLA + 512, 2 * PLA + 512, 3 * PLA + 512>(ba, fa);
          lds_read_8<0, PLB, 2 * PLB, 3 * PLB, 512, PLB + 512, 2 * PLB + 512, 3 * PLB + 512>(bb, fb);
        }
        bf8 af[2][PA], bfr[2][PB];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pl = 0; pl < PA; ++pl) af[i][pl] = __builtin_bit_cast(bf8, fa[i * PA + pl]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int pl = 0; pl < PB; ++pl) bfr[j][pl] = __builtin_bit_cast(bf8, fb[j * PB + pl]);
        mma_step<AC, BC>(af, bfr, accr, acci);
      }
    }
  }
  store_tile<AC, BC, 2>(p, accr, acci, split, m0 + wm * 64, n0 + wn * 64, lane);
}

// WN waves along N (2 or 4): a 128 x 64 WN tile, 128 WN threads; workgroup `bid` of the product p.
template <int AC, int BC, int WN>
__device__ __forceinline__ void nt_body(const Params& p, int bid) {
  constexpr int kThr = 128 * WN, kBN = 64 * WN;
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;  // complex planes
  constexpr int PA = 2 * NA, PB = 2 * NB;            // packed planes (hi, lo per complex plane)
  constexpr int SK = 16;                             // k per LDS stage (one MFMA step)
  constexpr int LDK = 24;                            // LDS row: 48 bytes, 16-byte aligned rows
  // two LDS buffers: stage s + 1 is written while stage s is multiplied
  __shared__ __attribute__((aligned(16))) __bf16 As[2][PA * kBM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][PB * kBN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int split, tm, tn;
  tile_of(bid, p, &split, &tm, &tn);
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int kbeg = split * p.kchunk, kend = min(p.Kp, kbeg + p.kchunk);

  f16 accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        accr[i][j][e] = 0.f;
        acci[i][j][e] = 0.f;
      }

  // a plane tile of one stage: rows x 16 k = 2 chunks of 16 bytes per row. B: one chunk per plane
  // and thread (row t % kBN, half t / kBN); A (128 rows): planes (t / 256) + kThr / 256 * q, row
  // t % 128, half (t / 128) % 2. Consecutive lanes write consecutive LDS rows (conflict-free).
  constexpr int AST = kThr / 256, NRA = PA / AST;  // A planes per thread
  const int brow = tid % kBN, bq = tid / kBN;
  const int arow = tid & 127, aq = (tid >> 7) & 1, apl = tid >> 8;
  u4 ra[NRA], rb[PB];
  // half-major k blocks: half h of row r in k block kb at ((2 kb + h) * R + r) * 8
  auto fetch = [&](int k0) {
    const int64_t kb = k0 / SK;
#pragma unroll
    for (int q = 0; q < NRA; ++q)
      ra[q] = *reinterpret_cast<const u4*>(p.A + (apl + AST * q) * p.pa + ((2 * kb + aq) * p.Mp + m0 + arow) * 8);
#pragma unroll
    for (int pl = 0; pl < PB; ++pl)
      rb[pl] = *reinterpret_cast<const u4*>(p.B + pl * p.pb + ((2 * kb + bq) * p.Np + n0 + brow) * 8);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NRA; ++q)
      *reinterpret_cast<u4*>(&As[buf][((apl + AST * q) * kBM + arow) * LDK + 8 * aq]) = ra[q];
#pragma unroll
    for (int pl = 0; pl < PB; ++pl) *reinterpret_cast<u4*>(&Bs[buf][(pl * kBN + brow) * LDK + 8 * bq]) = rb[pl];
  };

  const int l32 = lane & 31, hk = 8 * (lane >> 5);
  const int nst = (kend - kbeg) / SK;
  if (nst > 0) {
    fetch(kbeg);
    stash(0);
    if (nst > 1) fetch(kbeg + SK);
    __syncthreads();
  }
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    bf8 af[2][PA], bfr[2][PB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int pl = 0; pl < PA; ++pl)
        af[i][pl] = *reinterpret_cast<const bf8*>(&As[buf][(pl * kBM + wm * 64 + i * 32 + l32) * LDK + hk]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int pl = 0; pl < PB; ++pl)
        bfr[j][pl] = *reinterpret_cast<const bf8*>(&Bs[buf][(pl * kBN + wn * 64 + j * 32 + l32) * LDK + hk]);
    mma_step<AC, BC>(af, bfr, accr, acci);
    // next stage into the other buffer (last read before the previous barrier), then prefetch
    if (s + 1 < nst) {
      stash(buf ^ 1);
      if (s + 2 < nst) fetch(kbeg + (s + 2) * SK);
    }
    __syncthreads();
  }

  store_tile<AC, BC, 2>(p, accr, acci, split, m0 + wm * 64, n0 + wn * 64, lane);
}

// Up to three independent products of the same kind in one launch: workgroups [0, wg1) take p0,
// [wg1, wg2) p1, the rest p2 (a single product passes wg1 = wg2 = its grid). LADDER = 1: the same
// kernel under a name of its own for the particle-particle ladder.
template <int AC, int BC, int LADDER, int WN>
__global__ __launch_bounds__(128 * WN) void gemm_bf16x3_nt(Params p0, Params p1, Params p2, int wg1, int wg2) {
  const int b = blockIdx.x;
  if (b < wg1) nt_body<AC, BC, WN>(p0, b);
  else if (b < wg2) nt_body<AC, BC, WN>(p1, b - wg1);
  else nt_body<AC, BC, WN>(p2, b - wg2);
}

// Two products of the same kind in one launch: workgroups [0, wg0) take p0, the rest p1 (the two GEMMs
// of the symmetric / antisymmetric ladder, which alone would each fill only part of the chip).
template <int AC, int BC, int LADDER, int WN>
__global__ __launch_bounds__(128 * WN) void gemm_bf16x3_nt2(Params p0, Params p1, int wg0) {
  if ((int)blockIdx.x < wg0) nt_body<AC, BC, WN>(p0, blockIdx.x);
  else nt_body<AC, BC, WN>(p1, blockIdx.x - wg0);
}

// Wide-wave kernel: 256 threads, a 128 x 256 output tile, 2 x 2 waves of 64 x 128 (2 x 4 MFMA blocks of
// 32 x 32), one wave per SIMD. Per 16-wide k stage a wave reads 2 PA A fragments and 4 PB B fragments for
// 12 PA PB / 2 MFMAs (c x r: 16 fragments for 48 MFMAs, a third fewer LDS reads per MFMA than 64 x 64 wave
// tiles); the B fragments are used block by block, so the MFMAs of block j run while the reads of block
// j + 1 are still in flight. Register-staged double-buffered LDS as in gemm_bf16x3_nt.
template <int AC, int BC, int LADDER>
__global__ __launch_bounds__(256) void gemm_bf16x3_w4(Params p) {
  constexpr int kBN = 256;
  constexpr int NA = AC ? 2 : 1, NB = BC ? 2 : 1;
  constexpr int PA = 2 * NA, PB = 2 * NB;
  constexpr int SK = 16, LDK = 24;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][PA * kBM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][PB * kBN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int split, tm, tn;
  tile_of(blockIdx.x, p, &split, &tm, &tn);
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int kbeg = split * p.kchunk, kend = min(p.Kp, kbeg + p.kchunk);

  f16 accr[2][4], acci[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        accr[i][j][e] = 0.f;
        acci[i][j][e] = 0.f;
      }

  // stage tiles: A [PA][128 rows][2 halves], thread t: row t % 128, half t / 128, every plane;
  // B [PB][256 rows][2 halves], thread t: row t, both halves, every plane
  const int arow = tid & 127, aq = tid >> 7;
  u4 ra[PA], rb[PB][2];
  auto fetch = [&](int k0) {
    const int64_t kb = k0 / SK;
#pragma unroll
    for (int pl = 0; pl < PA; ++pl)
      ra[pl] = *reinterpret_cast<const u4*>(p.A + pl * p.pa + ((2 * kb + aq) * p.Mp + m0 + arow) * 8);
#pragma unroll
    for (int pl = 0; pl < PB; ++pl)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        rb[pl][h] = *reinterpret_cast<const u4*>(p.B + pl * p.pb + ((2 * kb + h) * p.Np + n0 + tid) * 8);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int pl = 0; pl < PA; ++pl) *reinterpret_cast<u4*>(&As[buf][(pl * kBM + arow) * LDK + 8 * aq]) = ra[pl];
#pragma unroll
    for (int pl = 0; pl < PB; ++pl)
#pragma unroll
      for (int h = 0; h < 2; ++h) *reinterpret_cast<u4*>(&Bs[buf][(pl * kBN + tid) * LDK + 8 * h]) = rb[pl][h];
  };

  const int l32 = lane & 31, hk = 8 * (lane >> 5);
  const int nst = (kend - kbeg) / SK;
  if (nst > 0) {
    fetch(kbeg);
    stash(0);
    if (nst > 1) fetch(kbeg + SK);
    __syncthreads();
  }
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    bf8 af[2][PA], an[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int pl = 0; pl < PA; ++pl)
        af[i][pl] = *reinterpret_cast<const bf8*>(&As[buf][(pl * kBM + wm * 64 + i * 32 + l32) * LDK + hk]);
    if (AC && BC) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) an[i][h] = neg(af[i][2 + h]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 bfr[PB];
#pragma unroll
      for (int pl = 0; pl < PB; ++pl)
        bfr[pl] = *reinterpret_cast<const bf8*>(&Bs[buf][(pl * kBN + wn * 128 + j * 32 + l32) * LDK + hk]);
      // three split products; within each, the two row blocks' updates alternate so that an
      // accumulator's consecutive MFMAs are several instructions apart
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int ha = t == 2 ? 1 : 0, hb = t == 1 ? 1 : 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) accr[i][j] = mma(af[i][ha], bfr[hb], accr[i][j]);
        if (BC) {
#pragma unroll
          for (int i = 0; i < 2; ++i) acci[i][j] = mma(af[i][ha], bfr[2 + hb], acci[i][j]);
        }
        if (AC) {
#pragma unroll
          for (int i = 0; i < 2; ++i) acci[i][j] = mma(af[i][2 + ha], bfr[hb], acci[i][j]);
        }
        if (AC && BC) {
#pragma unroll
          for (int i = 0; i < 2; ++i) accr[i][j] = mma(an[i][ha], bfr[2 + hb], accr[i][j]);
        }
      }
    }
    if (s + 1 < nst) {
      stash(buf ^ 1);
      if (s + 2 < nst) fetch(kbeg + (s + 2) * SK);
    }
    __syncthreads();
  }
  store_tile<AC, BC, 4>(p, accr, acci, split, m0 + wm * 64, n0 + wn * 128, lane);
}

}  // namespace

// Returns false (nothing launched) for real x real products or a real output.
bool gemm_bf16x3(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<float> A, GemmOp<float> B,
                 float* Cre, float* Cim, int64_t ldc, double beta, int force_wn, int force_splits, int force_kernel) {
  if (M <= 0 || N <= 0 || K <= 0) return false;
  const bool AC = A.im != nullptr, BC = B.im != nullptr;
  if (!Cim && (AC || BC)) return false;
  if (!AC && !BC) return false;
  RTCC_CHECK(M < (1LL << 30) && N < (1LL << 30) && K < (1LL << 30), kEInval, "gemm_bf16x3: dimension too large");
  size_t mark = E.scratch.used;
  // 2 x 4 waves (128 x 256 tiles); outputs too small for 16 such tiles (e.g. 400 x 400) use 2 x 2 waves
  // (128 x 128), which doubles their tile count (measured: 41-55 -> 28-41 us at 400 x 400 x 5776)
  RTCC_CHECK(force_wn == 0 || force_wn == 2 || force_wn == 4, kEInval, "gemm_bf16x3: waves along N must be 2 or 4");
  const int kern = force_kernel ? force_kernel : E.bf16_kernel;
  RTCC_CHECK(kern >= 1 && kern <= 4, kEInval, "gemm_bf16x3: unknown kernel variant");
  const int WN = force_wn ? force_wn : kern == 3 ? 2 : kern == 4 ? 4 : cdiv(M, kBM) * cdiv(N, 256) < 16 ? 2 : 4,
            kBN = 64 * WN;
  // A as [M][K] rows; B as [N][K] rows (B(k, n) = trans ? b[n * ld + k] : b[k * ld + n])
  const Packed pa = pack_operand(E, A.re, A.im, A.ld, A.trans, M, K, A.konst, kRowPad);
  const Packed pb = pack_operand(E, B.re, B.im, B.ld, B.trans ? 0 : 1, N, K, B.konst, kBN);
  Params p;
  p.A = pa.p;
  p.B = pb.p;
  p.pa = pa.plane;
  p.pb = pb.plane;
  p.Kp = pa.Kp;
  p.Mp = pa.Rp;
  p.Np = pb.Rp;
  p.M = (int)M;
  p.N = (int)N;
  p.tiles_m = (int)cdiv(M, kBM);
  p.tiles_n = (int)cdiv(N, kBN);
  p.ntiles = p.tiles_m * p.tiles_n;
  p.band = E.tile_band;
  p.alpha = (float)alpha;
  p.beta = (float)beta;
  // Split K when it shortens the estimated time: workgroups run in rounds of one per CU (256), a
  // tile takes ~tile_flops / (35% of the per-CU split-BF16 rate, as measured), and s > 1 splits add
  // a reduction that streams s partial planes and C (cache-resident: ~12 TB/s measured). A split
  // grid stays within kSplitWG workgroups: the right-hand side issues its large products from
  // three concurrent streams, and a split product that claims every CU holds the others back
  // longer than its split gains (measured for the o=20, v=76 step: 144-176 of 256 best, 192 0.5% and
  // 256 3% slower; below 144 the 1520 x 1520 products lose their split and the step is 4% slower).
  const int stages = p.Kp / kBK;
  const double tile_time = 2.0 * kBM * kBN * (double)p.Kp * ((AC && BC) ? 4 : 2) / (0.35 * 2516.6e12 / 3 / 256);
  const double plane_bytes = (double)M * N * 4.0 * 2.0;
  int splits = 1;
  double best = 1e300;
  const int kSplitWG = E.split_wg;
  for (int sp = 1; sp <= 16 && (sp == 1 || stages / sp >= 4); ++sp) {
    if (sp > 1 && p.ntiles * sp > kSplitWG) break;
    const double rounds = (double)cdiv((int64_t)p.ntiles * sp, 256);
    const double t = rounds * tile_time / sp + (sp > 1 ? (2.0 * sp + 2.0) * plane_bytes / 12e12 : 0.0);
    if (t < best * 0.97) {
      best = t;
      splits = sp;
    }
  }
  if (force_splits > 0) splits = (int)std::min<int64_t>(force_splits, std::max(stages, 1));
  const int per = (int)cdiv(stages, splits);
  p.kchunk = per * kBK;
  splits = (int)cdiv(stages, per);
  p.splits = splits;
  float *Pre = nullptr, *Pim = nullptr;
  if (splits > 1) {
    p.split_stride = M * N;
    Pre = E.scratch.get<float>(splits * M * N);
    Pim = E.scratch.get<float>(splits * M * N);
    p.Cre = Pre;
    p.Cim = Pim;
    p.ldc = N;
  } else {
    p.split_stride = 0;
    p.Cre = Cre;
    p.Cim = Cim;
    p.ldc = ldc;
  }
  const int nwg = p.ntiles * splits;
  const dim3 grid((unsigned)nwg);
  const bool lad = E.ladder != 0;
  if (lad && E.mark && E.mark_mode == 1) E.mark(E.mark_user, 0, E.ladder_flops, 0.0, E.stream);
  // timing of the complex x complex register-staged 128 x 256 kernel: algorithmic flops and bytes
  // (operands read once, the output written once and read once when accumulated into)
  const bool ccm = E.mark && E.mark_mode == 2 && AC && BC && !lad && kern == 1 && WN == 4;
  const double cc_flops = 8.0 * M * N * K, cc_bytes = 8.0 * (M * K + N * K + M * N * (beta != 0.0 ? 2 : 1));
  if (ccm) E.mark(E.mark_user, 0, cc_flops, cc_bytes, E.stream);
  const dim3 block(kern == 4 ? 256 : 128 * WN);
  RTCC_CHECK(kern != 3 || WN == 2, kEInval, "gemm_bf16x3: the two-per-CU kernel takes 128 x 128 tiles");
  RTCC_CHECK(kern != 4 || WN == 4, kEInval, "gemm_bf16x3: the wide-wave kernel takes 128 x 256 tiles");
  if (kern == 4) {  // 128 x 256 tiles, four waves of 64 x 128
    if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_w4<1, 0, 1>), grid, block, 0, E.stream, p);
    else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_w4<1, 1, 0>), grid, block, 0, E.stream, p);
    else if (AC) hipLaunchKernelGGL((gemm_bf16x3_w4<1, 0, 0>), grid, block, 0, E.stream, p);
    else hipLaunchKernelGGL((gemm_bf16x3_w4<0, 1, 0>), grid, block, 0, E.stream, p);
  } else if (kern == 3) {  // 128 x 128 tiles, two workgroups per CU
    if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 1, 2, 1>), grid, block, 0, E.stream, p);
    else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 1, 0, 2, 1>), grid, block, 0, E.stream, p);
    else if (AC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 0, 2, 1>), grid, block, 0, E.stream, p);
    else hipLaunchKernelGGL((gemm_bf16x3_dma<0, 1, 0, 2, 1>), grid, block, 0, E.stream, p);
  } else if (kern == 2) {
    if (WN == 4) {
      if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 1, 4, 0>), grid, block, 0, E.stream, p);
      else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 1, 0, 4, 0>), grid, block, 0, E.stream, p);
      else if (AC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 0, 4, 0>), grid, block, 0, E.stream, p);
      else hipLaunchKernelGGL((gemm_bf16x3_dma<0, 1, 0, 4, 0>), grid, block, 0, E.stream, p);
    } else {
      if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 1, 2, 0>), grid, block, 0, E.stream, p);
      else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 1, 0, 2, 0>), grid, block, 0, E.stream, p);
      else if (AC) hipLaunchKernelGGL((gemm_bf16x3_dma<1, 0, 0, 2, 0>), grid, block, 0, E.stream, p);
      else hipLaunchKernelGGL((gemm_bf16x3_dma<0, 1, 0, 2, 0>), grid, block, 0, E.stream, p);
    }
  } else if (WN == 4) {
    if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 0, 1, 4>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 1, 0, 4>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else if (AC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 0, 0, 4>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else hipLaunchKernelGGL((gemm_bf16x3_nt<0, 1, 0, 4>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
  } else {
    if (lad && AC && !BC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 0, 1, 2>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 1, 0, 2>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else if (AC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 0, 0, 2>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
    else hipLaunchKernelGGL((gemm_bf16x3_nt<0, 1, 0, 2>), grid, block, 0, E.stream, p, p, p, nwg, nwg);
  }
  RTCC_HIP(hipGetLastError());
  if (lad && E.mark && E.mark_mode == 1) E.mark(E.mark_user, 1, E.ladder_flops, 0.0, E.stream);
  if (ccm) E.mark(E.mark_user, 1, cc_flops, cc_bytes, E.stream);
  if (splits > 1) splitk_reduce_launch<float>(E.stream, Pre, Pim, splits, M, N, Cre, Cim, ldc, 0, 1, alpha, beta);
  E.scratch.reset(mark);
  E.gemm_flops += 2 * M * N * K * ((AC && BC) ? 4 : 2);
  if (E.trace)
    fprintf(stderr, "[rtcc] gemm-bf16x3 M=%lld N=%lld K=%lld %s%s ta=%d tb=%d wn=%d splits=%d kernel=%d konst=%d%d\n",
            (long long)M, (long long)N, (long long)K, AC ? "c" : "r", BC ? "c" : "r", A.trans, B.trans, WN, splits, kern,
            (int)A.konst, (int)B.konst);
  return true;
}

bool gemm_bf16x3_pair(Engine& E, const Bf16Job (&jobs)[2]) {
  for (const Bf16Job& j : jobs) {
    if (j.M <= 0 || j.N <= 0 || j.K <= 0 || !j.A.im || j.B.im || !j.Cim) return false;
    RTCC_CHECK(j.M < (1LL << 30) && j.N < (1LL << 30) && j.K < (1LL << 30), kEInval,
               "gemm_bf16x3_pair: dimension too large");
  }
  if (E.bf16_kernel != 1) return false;
  constexpr int WN = 4, kBN = 64 * WN;
  size_t mark = E.scratch.used;
  Params p[2];
  int64_t tiles = 0;
  int stages = 0;
  for (int h = 0; h < 2; ++h) {
    const Bf16Job& j = jobs[h];
    const Packed pa = pack_operand(E, j.A.re, j.A.im, j.A.ld, j.A.trans, j.M, j.K, j.A.konst, kRowPad);
    const Packed pb = pack_operand(E, j.B.re, j.B.im, j.B.ld, j.B.trans ? 0 : 1, j.N, j.K, j.B.konst, kBN);
    Params& q = p[h];
    q.A = pa.p;
    q.B = pb.p;
    q.pa = pa.plane;
    q.pb = pb.plane;
    q.Kp = pa.Kp;
    q.Mp = pa.Rp;
    q.Np = pb.Rp;
    q.M = (int)j.M;
    q.N = (int)j.N;
    q.tiles_m = (int)cdiv(j.M, kBM);
    q.tiles_n = (int)cdiv(j.N, kBN);
    q.ntiles = q.tiles_m * q.tiles_n;
    q.band = E.tile_band;
    q.alpha = (float)j.alpha;
    q.beta = (float)j.beta;
    tiles += q.ntiles;
    stages = std::max(stages, q.Kp / kBK);
  }
  // one K split for both, from the single-product cost model over the summed tiles (the longer K sets
  // the per-tile time) within the same workgroup cap
  const double tile_time = 2.0 * kBM * kBN * (double)stages * kBK * 2 / (0.35 * 2516.6e12 / 3 / 256);
  double plane_bytes = 0.0;
  for (const Bf16Job& j : jobs) plane_bytes += (double)j.M * j.N * 8.0;
  int splits = 1;
  double best = 1e300;
  // the pair replaces two launches of up to 160 workgroups that ran one after the other: up to one
  // workgroup per CU (measured in the (20,76) step: 3 splits, 252 workgroups, 114 us for both GEMMs
  // against 2 x 79 us apart; 2 splits 133 us; 4 splits 146 us)
  constexpr int kSplitWG = 256;
  for (int sp = 1; sp <= 16 && (sp == 1 || stages / sp >= 4); ++sp) {
    if (sp > 1 && tiles * sp > kSplitWG) break;
    const double rounds = (double)cdiv(tiles * sp, 256);
    const double t = rounds * tile_time / sp + (sp > 1 ? (2.0 * sp + 2.0) * plane_bytes / 12e12 : 0.0);
    if (t < best * 0.97) {
      best = t;
      splits = sp;
    }
  }
  if (E.pair_splits > 0) splits = std::min(E.pair_splits, std::max(stages, 1));
  float* P[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  for (int h = 0; h < 2; ++h) {
    const Bf16Job& j = jobs[h];
    Params& q = p[h];
    const int st = q.Kp / kBK, per = (int)cdiv(st, splits);
    q.kchunk = per * kBK;
    q.splits = (int)cdiv(st, per);
    if (q.splits > 1) {
      q.split_stride = j.M * j.N;
      P[h][0] = E.scratch.get<float>(q.splits * j.M * j.N);
      P[h][1] = E.scratch.get<float>(q.splits * j.M * j.N);
      q.Cre = P[h][0];
      q.Cim = P[h][1];
      q.ldc = j.N;
    } else {
      q.split_stride = 0;
      q.Cre = j.Cre;
      q.Cim = j.Cim;
      q.ldc = j.ldc;
    }
  }
  const int wg0 = p[0].ntiles * p[0].splits, wg = wg0 + p[1].ntiles * p[1].splits;
  const bool lad = E.ladder != 0;
  if (lad && E.mark && E.mark_mode == 1) E.mark(E.mark_user, 0, E.ladder_flops, 0.0, E.stream);
  if (lad) hipLaunchKernelGGL((gemm_bf16x3_nt2<1, 0, 1, WN>), dim3((unsigned)wg), dim3(128 * WN), 0, E.stream, p[0], p[1], wg0);
  else hipLaunchKernelGGL((gemm_bf16x3_nt2<1, 0, 0, WN>), dim3((unsigned)wg), dim3(128 * WN), 0, E.stream, p[0], p[1], wg0);
  RTCC_HIP(hipGetLastError());
  if (lad && E.mark && E.mark_mode == 1) E.mark(E.mark_user, 1, E.ladder_flops, 0.0, E.stream);
  for (int h = 0; h < 2; ++h) {
    const Bf16Job& j = jobs[h];
    if (p[h].splits > 1)
      splitk_reduce_launch<float>(E.stream, P[h][0], P[h][1], p[h].splits, j.M, j.N, j.Cre, j.Cim, j.ldc, 0, 1,
                                  j.alpha, j.beta);
    E.gemm_flops += 2 * j.M * j.N * j.K * 2;
    if (E.trace)
      fprintf(stderr, "[rtcc] gemm-bf16x3 pair %d/2 M=%lld N=%lld K=%lld cr ta=%d tb=%d wn=%d splits=%d\n", h + 1,
              (long long)j.M, (long long)j.N, (long long)j.K, j.A.trans, j.B.trans, WN, p[h].splits);
  }
  E.scratch.reset(mark);
  return true;
}

bool gemm_bf16x3_multi(Engine& E, const Bf16Job* jobs, int n) {
  if (n < 2 || n > 3 || E.bf16_kernel != 1) return false;
  const bool AC = jobs[0].A.im != nullptr, BC = jobs[0].B.im != nullptr;
  if (!AC && !BC) return false;
  for (int h = 0; h < n; ++h) {
    const Bf16Job& j = jobs[h];
    if (j.M <= 0 || j.N <= 0 || j.K <= 0 || (j.A.im != nullptr) != AC || (j.B.im != nullptr) != BC || !j.Cim)
      return false;
    RTCC_CHECK(j.M < (1LL << 30) && j.N < (1LL << 30) && j.K < (1LL << 30), kEInval,
               "gemm_bf16x3_multi: dimension too large");
  }
  constexpr int WN = 4, kBN = 64 * WN;
  size_t mark = E.scratch.used;
  Params p[3];
  int64_t tiles = 0;
  int stages = 0;
  double flops = 0.0, bytes = 0.0, plane_bytes = 0.0;
  for (int h = 0; h < n; ++h) {
    const Bf16Job& j = jobs[h];
    const Packed pa = pack_operand(E, j.A.re, j.A.im, j.A.ld, j.A.trans, j.M, j.K, j.A.konst, kRowPad);
    const Packed pb = pack_operand(E, j.B.re, j.B.im, j.B.ld, j.B.trans ? 0 : 1, j.N, j.K, j.B.konst, kBN);
    Params& q = p[h];
    q.A = pa.p;
    q.B = pb.p;
    q.pa = pa.plane;
    q.pb = pb.plane;
    q.Kp = pa.Kp;
    q.Mp = pa.Rp;
    q.Np = pb.Rp;
    q.M = (int)j.M;
    q.N = (int)j.N;
    q.tiles_m = (int)cdiv(j.M, kBM);
    q.tiles_n = (int)cdiv(j.N, kBN);
    q.ntiles = q.tiles_m * q.tiles_n;
    q.band = E.tile_band;
    q.alpha = (float)j.alpha;
    q.beta = (float)j.beta;
    tiles += q.ntiles;
    stages = std::max(stages, q.Kp / kBK);
    flops += 2.0 * j.M * j.N * j.K * ((AC && BC) ? 4 : 2);
    bytes += 8.0 * (j.M * j.K + j.N * j.K + j.M * j.N * (j.beta != 0.0 ? 2 : 1));
    plane_bytes += (double)j.M * j.N * 8.0;
  }
  // one K split for all, from the single-product cost model over the summed tiles (the longest K sets the
  // per-tile time), within one workgroup per CU: the launch replaces products that ran one after another
  const double tile_time = 2.0 * kBM * kBN * (double)stages * kBK * ((AC && BC) ? 4 : 2) / (0.35 * 2516.6e12 / 3 / 256);
  int splits = 1;
  double best = 1e300;
  const int kSplitWG = E.group_wg;
  for (int sp = 1; sp <= 16 && (sp == 1 || stages / sp >= 4); ++sp) {
    if (sp > 1 && tiles * sp > kSplitWG) break;
    const double rounds = (double)cdiv(tiles * sp, 256);
    const double t = rounds * tile_time / sp + (sp > 1 ? (2.0 * sp + 2.0) * plane_bytes / 12e12 : 0.0);
    if (t < best * 0.97) {
      best = t;
      splits = sp;
    }
  }
  float* P[3][2] = {};
  int wg[3] = {0, 0, 0};
  for (int h = 0; h < n; ++h) {
    const Bf16Job& j = jobs[h];
    Params& q = p[h];
    const int st = q.Kp / kBK, per = (int)cdiv(st, splits);
    q.kchunk = per * kBK;
    q.splits = (int)cdiv(st, per);
    if (q.splits > 1) {
      q.split_stride = j.M * j.N;
      P[h][0] = E.scratch.get<float>(q.splits * j.M * j.N);
      P[h][1] = E.scratch.get<float>(q.splits * j.M * j.N);
      q.Cre = P[h][0];
      q.Cim = P[h][1];
      q.ldc = j.N;
    } else {
      q.split_stride = 0;
      q.Cre = j.Cre;
      q.Cim = j.Cim;
      q.ldc = j.ldc;
    }
    wg[h] = q.ntiles * q.splits;
  }
  if (n == 2) p[2] = p[1];
  const int wg1 = wg[0], wg2 = wg[0] + wg[1], total = wg2 + (n == 3 ? wg[2] : 0);
  // timed as one launch of the complex x complex kernel (see Engine::mark_mode)
  const bool ccm = E.mark && E.mark_mode == 2 && AC && BC;
  if (ccm) E.mark(E.mark_user, 0, flops, bytes, E.stream);
  const dim3 grid((unsigned)total), block(128 * WN);
  if (AC && BC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 1, 0, 4>), grid, block, 0, E.stream, p[0], p[1], p[2], wg1, wg2);
  else if (AC) hipLaunchKernelGGL((gemm_bf16x3_nt<1, 0, 0, 4>), grid, block, 0, E.stream, p[0], p[1], p[2], wg1, wg2);
  else hipLaunchKernelGGL((gemm_bf16x3_nt<0, 1, 0, 4>), grid, block, 0, E.stream, p[0], p[1], p[2], wg1, wg2);
  RTCC_HIP(hipGetLastError());
  if (ccm) E.mark(E.mark_user, 1, flops, bytes, E.stream);
  for (int h = 0; h < n; ++h) {
    const Bf16Job& j = jobs[h];
    if (p[h].splits > 1)
      splitk_reduce_launch<float>(E.stream, P[h][0], P[h][1], p[h].splits, j.M, j.N, j.Cre, j.Cim, j.ldc, 0, 1,
                                  j.alpha, j.beta);
    E.gemm_flops += 2 * j.M * j.N * j.K * ((AC && BC) ? 4 : 2);
    if (E.trace)
      fprintf(stderr, "[rtcc] gemm-bf16x3 multi %d/%d M=%lld N=%lld K=%lld %s%s ta=%d tb=%d wn=%d splits=%d\n", h + 1,
              n, (long long)j.M, (long long)j.N, (long long)j.K, AC ? "c" : "r", BC ? "c" : "r", j.A.trans,
              j.B.trans, WN, p[h].splits);
  }
  E.scratch.reset(mark);
  return true;
}

}  // namespace rtcc
