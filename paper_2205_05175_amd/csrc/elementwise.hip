// Memory-bound kernels: strided permute-axpby, state (un)packing, RK stage updates, field,
// and fixed-order wavefront reductions.
#include <cstdio>
#include <cstdlib>

#include "elementwise.h"

namespace rtcc {

// ---- strided permute-axpby: out = alpha * permute(in) + beta * out -------------------------------
// Dimensions that are contiguous on both sides are merged first. If the output's fastest dimension x
// is also the input's fastest, every thread handles V consecutive elements along x (16-byte vectors
// when aligned). Otherwise (a transpose) 32 x 32 tiles over x and p, the input's fastest dimension,
// go through LDS: read with p across lanes, written with x across lanes. Indices are decoded with
// 32-bit multiply-shift division (exact for numerators below 2^31).
struct FDiv {
  uint32_t m, s, d;
};
static FDiv make_fdiv(int64_t d) {
  // Granlund-Montgomery: l = ceil(log2 d), m = floor(2^(31+l) / d) + 1, n / d = (n * m) >> (31 + l)
  int l = 0;
  while ((1LL << l) < d) ++l;
  FDiv f;
  f.m = (uint32_t)(((uint64_t)1 << (31 + l)) / (uint64_t)d + 1);
  f.s = 31 + l;
  f.d = (uint32_t)d;
  return f;
}
__device__ inline uint32_t fdiv(uint32_t n, const FDiv& f) { return (uint32_t)(((uint64_t)n * f.m) >> f.s); }

constexpr int kPT = 32;
struct PermGeom {
  int nout;  // outer dimensions (<= kMaxDim - 1), outermost first
  FDiv od[kMaxDim];
  int64_t ois[kMaxDim], oos[kMaxDim];
  FDiv dx, dp;  // tile dims (transpose) or x and x / V (element kernel: dp = groups per row)
  int64_t isp, isx, osp, osx;
  FDiv tx;      // tiles along x (transpose kernel)
  FDiv tp;      // tiles along p
  uint32_t nwork;  // tiles or element groups
  int load_x_fast;
};

__device__ inline void decode_outer(const PermGeom& g, uint32_t rem, int64_t* ib, int64_t* ob) {
  int64_t a = 0, b = 0;
  for (int k = g.nout - 1; k >= 0; --k) {
    const uint32_t q = fdiv(rem, g.od[k]);
    const uint32_t c = rem - q * g.od[k].d;
    rem = q;
    a += (int64_t)c * g.ois[k];
    b += (int64_t)c * g.oos[k];
  }
  *ib = a;
  *ob = b;
}

template <typename T, int V>
__global__ __launch_bounds__(256) void permute_elem_kernel(PermGeom g, const T* __restrict__ inre,
                                                           const T* __restrict__ inim, T* outre, T* outim, T alpha,
                                                           T beta) {
  typedef T vt __attribute__((ext_vector_type(V)));
  for (uint32_t w = blockIdx.x * 256 + threadIdx.x; w < g.nwork; w += gridDim.x * 256) {
    const uint32_t row = fdiv(w, g.dp);            // dp = groups of V per row
    const uint32_t x = (w - row * g.dp.d) * V;
    int64_t ib, ob;
    decode_outer(g, row, &ib, &ob);
    ib += (int64_t)x * g.isx;
    ob += (int64_t)x * g.osx;
    // every load (input and, for beta != 0, output planes) is issued before the first store
    if constexpr (V > 1) {
      const vt r = inre ? *reinterpret_cast<const vt*>(inre + ib) : vt{};
      const vt ri = (outim && inre && inim) ? *reinterpret_cast<const vt*>(inim + ib) : vt{};
      const vt cr = beta != T(0) ? *reinterpret_cast<const vt*>(outre + ob) : vt{};
      const vt ci = (outim && beta != T(0)) ? *reinterpret_cast<const vt*>(outim + ob) : vt{};
      *reinterpret_cast<vt*>(outre + ob) = r * alpha + beta * cr;
      if (outim) *reinterpret_cast<vt*>(outim + ob) = ri * alpha + beta * ci;
    } else {
      const T r = inre ? inre[ib] : T(0);
      const T ri = (outim && inre && inim) ? inim[ib] : T(0);
      const T cr = beta != T(0) ? outre[ob] : T(0);
      const T ci = (outim && beta != T(0)) ? outim[ob] : T(0);
      outre[ob] = alpha * r + beta * cr;
      if (outim) outim[ob] = alpha * ri + beta * ci;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void permute_tile_kernel(PermGeom g, const T* __restrict__ inre,
                                                           const T* __restrict__ inim, T* outre, T* outim, T alpha,
                                                           T beta) {
  __shared__ T sre[kPT][kPT + 1];
  __shared__ T sim[kPT][kPT + 1];
  const int t = threadIdx.x;
  for (uint32_t tile = blockIdx.x; tile < g.nwork; tile += gridDim.x) {
    uint32_t rem = fdiv(tile, g.tx);
    const int bx = (int)(tile - rem * g.tx.d);
    const uint32_t r2 = fdiv(rem, g.tp);
    const int bp = (int)(rem - r2 * g.tp.d);
    int64_t ib, ob;
    decode_outer(g, r2, &ib, &ob);
    const int p0 = bp * kPT, x0 = bx * kPT;
    const int dpn = (int)g.dp.d, dxn = (int)g.dx.d;
#pragma unroll
    for (int r = 0; r < kPT * kPT / 256; ++r) {
      const int f = t & (kPT - 1), sidx = (t >> 5) + r * (256 / kPT);
      const int ip = g.load_x_fast ? sidx : f, ix = g.load_x_fast ? f : sidx;
      if (p0 + ip < dpn && x0 + ix < dxn) {
        const int64_t off = ib + (int64_t)(p0 + ip) * g.isp + (int64_t)(x0 + ix) * g.isx;
        sre[ix][ip] = inre[off];
        if (outim) sim[ix][ip] = inim ? inim[off] : T(0);
      }
    }
    __syncthreads();
    constexpr int R = kPT * kPT / 256;
    T cr[R], ci[R];  // old output values (beta != 0), all loaded before the stores
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ix = t & (kPT - 1), ip = (t >> 5) + r * (256 / kPT);
      cr[r] = T(0);
      ci[r] = T(0);
      if (beta != T(0) && p0 + ip < dpn && x0 + ix < dxn) {
        const int64_t off = ob + (int64_t)(p0 + ip) * g.osp + (int64_t)(x0 + ix) * g.osx;
        cr[r] = outre[off];
        if (outim) ci[r] = outim[off];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ix = t & (kPT - 1), ip = (t >> 5) + r * (256 / kPT);
      if (p0 + ip < dpn && x0 + ix < dxn) {
        const int64_t off = ob + (int64_t)(p0 + ip) * g.osp + (int64_t)(x0 + ix) * g.osx;
        outre[off] = alpha * sre[ix][ip] + beta * cr[r];
        if (outim) outim[off] = alpha * sim[ix][ip] + beta * ci[r];
      }
    }
    __syncthreads();
  }
}

// Transposes of small matrices (both transposed extents <= 128, e.g. 76 x 76): 32 x 32 tiles would
// leave up to 40% of their slots empty, so a workgroup moves one whole dx x dp matrix through LDS
// (dynamic size; rows padded to an odd length), reading with p (the input's fastest dimension)
// across lanes and writing with x (the output's) across lanes, eight elements in flight per thread.
template <typename T>
__global__ __launch_bounds__(256) void permute_mat_kernel(PermGeom g, int ld, const T* __restrict__ inre,
                                                          const T* __restrict__ inim, T* outre, T* outim, T alpha,
                                                          T beta) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sre = reinterpret_cast<T*>(lds_raw);
  const int dxn = (int)g.dx.d, dpn = (int)g.dp.d, n = dxn * dpn;
  T* sim = sre + dxn * ld;
  const int t = threadIdx.x;
  constexpr int U = 8;
  for (uint32_t w = blockIdx.x; w < g.nwork; w += gridDim.x) {
    int64_t ib, ob;
    decode_outer(g, w, &ib, &ob);
    for (int e0 = 0; e0 < n; e0 += 256 * U) {
      T vr[U], vi[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + t + 256 * u;
        vr[u] = T(0);
        vi[u] = T(0);
        if (e < n) {
          const int x = (int)fdiv((uint32_t)e, g.dp), p = e - x * dpn;
          const int64_t off = ib + (int64_t)p * g.isp + (int64_t)x * g.isx;
          vr[u] = inre[off];
          if (inim) vi[u] = inim[off];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + t + 256 * u;
        if (e < n) {
          const int x = (int)fdiv((uint32_t)e, g.dp), p = e - x * dpn;
          sre[x * ld + p] = vr[u];
          if (outim) sim[x * ld + p] = vi[u];
        }
      }
    }
    __syncthreads();
    for (int e0 = 0; e0 < n; e0 += 256 * U) {
      // the outputs' old values (beta != 0) are all loaded before any of the U stores
      T cr[U], ci[U];
      int64_t offs[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + t + 256 * u;
        const int p = (int)fdiv((uint32_t)e, g.dx), x = e - p * dxn;
        offs[u] = ob + (int64_t)p * g.osp + (int64_t)x * g.osx;
        cr[u] = T(0);
        ci[u] = T(0);
        if (e < n && beta != T(0)) {
          cr[u] = outre[offs[u]];
          if (outim) ci[u] = outim[offs[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + t + 256 * u;
        if (e < n) {
          const int p = (int)fdiv((uint32_t)e, g.dx), x = e - p * dxn;
          outre[offs[u]] = alpha * sre[x * ld + p] + beta * cr[u];
          if (outim) outim[offs[u]] = alpha * sim[x * ld + p] + beta * ci[u];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
void permute_axpby(hipStream_t st, int nd, const int64_t* dims, const T* inre, const T* inim, const int64_t* instr,
                   T* outre, T* outim, const int64_t* outstr, double alpha, double beta) {
  RTCC_CHECK(nd >= 0 && nd <= kMaxDim, kEInval, "permute: too many dimensions");
  if (alpha == 0.0) {
    inre = nullptr;
    inim = nullptr;
  }
  auto absl = [](int64_t x) { return x < 0 ? -x : x; };
  // drop unit dimensions; an empty tensor is a no-op
  int64_t d[kMaxDim], is[kMaxDim], os[kMaxDim];
  int n = 0;
  int64_t total = 1;
  for (int i = 0; i < nd; ++i) {
    if (dims[i] == 0) return;
    if (dims[i] == 1) continue;
    d[n] = dims[i];
    is[n] = inre ? instr[i] : 0;
    os[n] = outstr[i];
    total *= dims[i];
    ++n;
  }
  RTCC_CHECK(total < (1LL << 31), kEInval, "permute: tensor too large");
  // order by output stride, outermost first, then merge dimensions contiguous on both sides
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      if (absl(os[b]) > absl(os[a])) {
        std::swap(d[a], d[b]);
        std::swap(is[a], is[b]);
        std::swap(os[a], os[b]);
      }
  {
    int m = 0;
    for (int i = 0; i < n; ++i) {
      if (m > 0 && os[m - 1] == os[i] * d[i] && is[m - 1] == is[i] * d[i]) {
        d[m - 1] *= d[i];
        is[m - 1] = is[i];
        os[m - 1] = os[i];
      } else {
        d[m] = d[i];
        is[m] = is[i];
        os[m] = os[i];
        ++m;
      }
    }
    n = m;
  }
  PermGeom g;
  const int ix = n - 1;  // output-fastest (ix = -1: a scalar)
  int ip = -1;
  if (inre && ix >= 0)
    for (int i = 0; i < ix; ++i)
      if (is[i] != 0 && absl(is[i]) < absl(is[ix]) && (ip < 0 || absl(is[i]) < absl(is[ip]))) ip = i;
  static const bool trace = [] {
    const char* t = std::getenv("RTCC_TRACE");
    return t && t[0] == '1';
  }();
  const int64_t dxv = ix >= 0 ? d[ix] : 1;
  g.isx = ix >= 0 ? is[ix] : 0;
  g.osx = ix >= 0 ? os[ix] : 0;
  if (ip < 0) {
    // element kernel over (outer..., x)
    constexpr int VW = 16 / sizeof(T);
    bool vec = dxv % VW == 0 && g.osx == 1 && (g.isx == 1 || !inre) && ((uintptr_t)outre % 16) == 0 &&
               (!outim || (uintptr_t)outim % 16 == 0) && (!inre || (uintptr_t)inre % 16 == 0) &&
               (!inim || (uintptr_t)inim % 16 == 0);
    for (int i = 0; i < ix; ++i) vec = vec && is[i] % VW == 0 && os[i] % VW == 0;
    const int V = vec ? VW : 1;
    g.nout = ix > 0 ? ix : 0;
    for (int k = 0; k < g.nout; ++k) {
      g.od[k] = make_fdiv(d[k]);
      g.ois[k] = is[k];
      g.oos[k] = os[k];
    }
    g.dp = make_fdiv(dxv / V);
    g.nwork = (uint32_t)(total / V);
    if (trace)
      fprintf(stderr, "[rtcc] permute %s elem x=%lld(is %lld os %lld) V=%d outer=%d groups=%u cplx=%d beta=%g\n",
              sizeof(T) == 8 ? "f64" : "f32", (long long)dxv, (long long)g.isx, (long long)g.osx, V, g.nout, g.nwork,
              outim ? 1 : 0, beta);
    const unsigned blocks = (unsigned)std::min<int64_t>(cdiv((int64_t)g.nwork, 256), 16384);
    if (V > 1)
      hipLaunchKernelGGL((permute_elem_kernel<T, VW>), dim3(blocks), dim3(256), 0, st, g, inre, inim, outre, outim,
                         (T)alpha, (T)beta);
    else
      hipLaunchKernelGGL((permute_elem_kernel<T, 1>), dim3(blocks), dim3(256), 0, st, g, inre, inim, outre, outim,
                         (T)alpha, (T)beta);
    RTCC_HIP(hipGetLastError());
    return;
  }
  // transpose: tiles over (p, x), outer = the rest
  g.dx = make_fdiv(dxv);
  g.dp = make_fdiv(d[ip]);
  g.isp = is[ip];
  g.osp = os[ip];
  g.load_x_fast = 0;
  g.nout = 0;
  int64_t outer = 1;
  for (int i = 0; i < ix; ++i) {
    if (i == ip) continue;
    g.od[g.nout] = make_fdiv(d[i]);
    g.ois[g.nout] = is[i];
    g.oos[g.nout] = os[i];
    outer *= d[i];
    ++g.nout;
  }
  // whole small matrices when 32 x 32 tiles would be partly empty and the matrix fits in LDS
  const int64_t dpv = d[ip];
  const int ldm = (int)(dpv % 2 == 0 ? dpv + 1 : dpv + 2);  // odd row length: conflict-free column reads
  const int64_t mat_bytes = dxv * ldm * (int64_t)sizeof(T) * (outim ? 2 : 1);
  if (dxv <= 128 && dpv <= 128 && (dxv % kPT != 0 || dpv % kPT != 0) && mat_bytes <= 65536 && outer >= 256) {
    g.nwork = (uint32_t)outer;
    if (trace)
      fprintf(stderr, "[rtcc] permute %s mat x=%lld(is %lld os %lld) p=%lld(is %lld os %lld) outer=%lld cplx=%d beta=%g\n",
              sizeof(T) == 8 ? "f64" : "f32", (long long)dxv, (long long)g.isx, (long long)g.osx, (long long)dpv,
              (long long)g.isp, (long long)g.osp, (long long)outer, outim ? 1 : 0, beta);
    const unsigned blocks = (unsigned)std::min<int64_t>(outer, 16384);
    hipLaunchKernelGGL(permute_mat_kernel<T>, dim3(blocks), dim3(256), (size_t)mat_bytes, st, g, ldm, inre, inim, outre,
                       outim, (T)alpha, (T)beta);
    RTCC_HIP(hipGetLastError());
    return;
  }
  const int64_t tx = cdiv(dxv, kPT), tp = cdiv(d[ip], kPT);
  g.tx = make_fdiv(tx);
  g.tp = make_fdiv(tp);
  const int64_t ntiles = outer * tx * tp;
  RTCC_CHECK(ntiles < (1LL << 31), kEInval, "permute: too many tiles");
  g.nwork = (uint32_t)ntiles;
  if (trace)
    fprintf(stderr, "[rtcc] permute %s tile x=%lld(is %lld os %lld) p=%lld(is %lld os %lld) outer=%lld tiles=%lld cplx=%d beta=%g\n",
            sizeof(T) == 8 ? "f64" : "f32", (long long)dxv, (long long)g.isx, (long long)g.osx, (long long)d[ip],
            (long long)g.isp, (long long)g.osp, (long long)outer, (long long)ntiles, outim ? 1 : 0, beta);
  const unsigned blocks = (unsigned)std::min<int64_t>(ntiles, 16384);
  hipLaunchKernelGGL(permute_tile_kernel<T>, dim3(blocks), dim3(256), 0, st, g, inre, inim, outre, outim, (T)alpha,
                     (T)beta);
  RTCC_HIP(hipGetLastError());
}
template void permute_axpby<double>(hipStream_t, int, const int64_t*, const double*, const double*, const int64_t*,
                                    double*, double*, const int64_t*, double, double);
template void permute_axpby<float>(hipStream_t, int, const int64_t*, const float*, const float*, const int64_t*,
                                   float*, float*, const int64_t*, double, double);

// ---- state vector <-> planar amplitudes ------------------------------------------------
// y layout (complex128 interleaved): [T1 o*v | T2 o*o*v*v | L1 o*v | L2 o*o*v*v]
template <typename T>
__device__ inline void state_segment(int64_t i, int64_t n1, int64_t n2, int64_t ntot, int* seg, int64_t* j,
                                     int64_t* b) {
  *b = i / ntot;
  int64_t r = i - *b * ntot;
  if (r < n1) { *seg = 0; *j = r; }
  else if (r < n1 + n2) { *seg = 1; *j = r - n1; }
  else if (r < 2 * n1 + n2) { *seg = 2; *j = r - n1 - n2; }
  else { *seg = 3; *j = r - 2 * n1 - n2; }
}

template <typename T>
__global__ void unpack_kernel(const double2* __restrict__ y, int64_t n1, int64_t n2, int64_t total, Planes4<T> P) {
  const int64_t ntot = 2 * (n1 + n2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    double2 z = y[i];
    int seg;
    int64_t j, b;
    state_segment<T>(i, n1, n2, ntot, &seg, &j, &b);
    j += b * P.bs[seg];
    P.re[seg][j] = (T)z.x;
    P.im[seg][j] = (T)z.y;
  }
}

template <typename T>
void unpack_state(hipStream_t st, const void* y, int o, int v, Planes4<T> P, int nb) {
  int64_t n1 = (int64_t)o * v, n2 = n1 * n1, total = 2 * (n1 + n2) * nb;
  int64_t blocks = std::min<int64_t>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(unpack_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, (const double2*)y, n1, n2, total, P);
  RTCC_HIP(hipGetLastError());
}

// out = scale * (-i R_T, +i R_L)
template <typename T>
__global__ void pack_kernel(int64_t n1, int64_t n2, int64_t total, Planes4<T> P, double2* out, double scale) {
  const int64_t ntot = 2 * (n1 + n2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int seg;
    int64_t j, b;
    state_segment<T>(i, n1, n2, ntot, &seg, &j, &b);
    j += b * P.bs[seg];
    double sgn = seg < 2 ? -1.0 : 1.0;
    double re = (double)P.re[seg][j], im = (double)P.im[seg][j];
    // (sgn i)(re + i im) = -sgn im + i sgn re
    out[i] = make_double2(-sgn * im * scale, sgn * re * scale);
  }
}

template <typename T>
void pack_rhs(hipStream_t st, int o, int v, Planes4<T> P, void* out, double scale, int nb) {
  int64_t n1 = (int64_t)o * v, n2 = n1 * n1, total = 2 * (n1 + n2) * nb;
  int64_t blocks = std::min<int64_t>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(pack_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, n1, n2, total, P, (double2*)out,
                     scale);
  RTCC_HIP(hipGetLastError());
}

// planes P = y + sum_j c_j k_j (the combination in FP64, then rounded to T): an RK stage input formed
// and converted in one pass, in place of a state_combo into an FP64 state and an unpack_state of it.
// Same arithmetic in the same order as those two passes.
struct ComboArgs {
  const double2* k[8];
  double c[8];
  int nk;
};

template <typename T>
__global__ void combo_unpack_kernel(const double2* __restrict__ y, ComboArgs cb, int64_t n1, int64_t n2,
                                    int64_t total, Planes4<T> P) {
  const int64_t ntot = 2 * (n1 + n2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = y[i];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= cb.nk) break;
      const double2 kk = cb.k[j][i];
      a.x += cb.c[j] * kk.x;
      a.y += cb.c[j] * kk.y;
    }
    int seg;
    int64_t jj, b;
    state_segment<T>(i, n1, n2, ntot, &seg, &jj, &b);
    jj += b * P.bs[seg];
    P.re[seg][jj] = (T)a.x;
    P.im[seg][jj] = (T)a.y;
  }
}

template <typename T>
void combo_unpack(hipStream_t st, int o, int v, int nb, const void* y, int nk, const void* const* ks, const double* cs,
                  Planes4<T> P) {
  RTCC_CHECK(nk <= 8, kEInval, "combo_unpack: too many terms");
  ComboArgs cb;
  cb.nk = 0;
  for (int j = 0; j < nk; ++j) {
    if (cs[j] == 0.0) continue;
    cb.k[cb.nk] = (const double2*)ks[j];
    cb.c[cb.nk] = cs[j];
    cb.nk++;
  }
  const int64_t n1 = (int64_t)o * v, n2 = n1 * n1, total = 2 * (n1 + n2) * nb;
  const int64_t blocks = std::min<int64_t>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(combo_unpack_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, (const double2*)y, cb, n1, n2,
                     total, P);
  RTCC_HIP(hipGetLastError());
}
template void combo_unpack<double>(hipStream_t, int, int, int, const void*, int, const void* const*, const double*,
                                   Planes4<double>);
template void combo_unpack<float>(hipStream_t, int, int, int, const void*, int, const void* const*, const double*,
                                  Planes4<float>);

template void unpack_state<double>(hipStream_t, const void*, int, int, Planes4<double>, int);
template void unpack_state<float>(hipStream_t, const void*, int, int, Planes4<float>, int);
template void pack_rhs<double>(hipStream_t, int, int, Planes4<double>, void*, double, int);
template void pack_rhs<float>(hipStream_t, int, int, Planes4<float>, void*, double, int);

// ---- field-dressed Fock matrix f(t) = f0 - sum_a E_a mu_a -------------------------------------
template <typename T>
__global__ void fock_kernel(int64_t nn, const double* f0, const double* mu, double ex, double ey, double ez, double s0,
                            T* f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  f[i] = (T)(s0 * f0[i] - ex * mu[i] - ey * mu[nn + i] - ez * mu[2 * nn + i]);
}

template <typename T>
void field_fock(hipStream_t st, int n, const double* f0, const double* mu, const double E[3], double s0, T* f) {
  int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(fock_kernel<T>, dim3((unsigned)cdiv(nn, 256)), dim3(256), 0, st, nn, f0, mu, E[0], E[1], E[2],
                     s0, f);
  RTCC_HIP(hipGetLastError());
}
template void field_fock<double>(hipStream_t, int, const double*, const double*, const double*, double, double*);
template void field_fock<float>(hipStream_t, int, const double*, const double*, const double*, double, float*);

// Field evaluated on the device at t = *tdev + toff (Eq. field; kinds other than the Gaussian
// pulse give zero), so a captured step can be replayed at successive times.
template <typename T>
__global__ void fock_time_kernel(int64_t nn, const double* f0, const double* mu, FieldDev fd, const double* tdev,
                                 double toff, T* f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  double a = 0.0;
  if (fd.kind == 1) {
    double x = tdev[0] + toff - fd.t0;
    a = -fd.E0 * exp(-0.5 * x * x / (fd.sigma * fd.sigma)) * cos(fd.omega * x);
  }
  f[i] = (T)(f0[i] - a * (fd.n[0] * mu[i] + fd.n[1] * mu[nn + i] + fd.n[2] * mu[2 * nn + i]));
}

template <typename T>
void field_fock_t(hipStream_t st, int n, const double* f0, const double* mu, const FieldDev& fd, const double* tdev,
                  double toff, T* f) {
  int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(fock_time_kernel<T>, dim3((unsigned)cdiv(nn, 256)), dim3(256), 0, st, nn, f0, mu, fd, tdev,
                     toff, f);
  RTCC_HIP(hipGetLastError());
}
template void field_fock_t<double>(hipStream_t, int, const double*, const double*, const FieldDev&, const double*,
                                   double, double*);
template void field_fock_t<float>(hipStream_t, int, const double*, const double*, const FieldDev&, const double*,
                                  double, float*);

template <typename T>
__global__ void fock_time_batch_kernel(int64_t nn, const double* f0, const double* mu, const FieldDev* fds,
                                       const double* tdev, double toff, T* f, int64_t fbs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const FieldDev& fd = fds[blockIdx.y];
  double a = 0.0;
  if (fd.kind == 1) {
    double x = tdev[0] + toff - fd.t0;
    a = -fd.E0 * exp(-0.5 * x * x / (fd.sigma * fd.sigma)) * cos(fd.omega * x);
  } else if (fd.kind == kFieldConstant) {
    a = 1.0;
  }
  f[blockIdx.y * fbs + i] = (T)(f0[i] - a * (fd.n[0] * mu[i] + fd.n[1] * mu[nn + i] + fd.n[2] * mu[2 * nn + i]));
}

template <typename T>
void field_fock_tb(hipStream_t st, int n, const double* f0, const double* mu, const FieldDev* fds, int nb,
                   const double* tdev, double toff, T* f, int64_t fbs) {
  int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(fock_time_batch_kernel<T>, dim3((unsigned)cdiv(nn, 256), (unsigned)nb), dim3(256), 0, st, nn,
                     f0, mu, fds, tdev, toff, f, fbs);
  RTCC_HIP(hipGetLastError());
}
template void field_fock_tb<double>(hipStream_t, int, const double*, const double*, const FieldDev*, int,
                                    const double*, double, double*, int64_t);
template void field_fock_tb<float>(hipStream_t, int, const double*, const double*, const FieldDev*, int,
                                   const double*, double, float*, int64_t);

// Fields reach the device as kernel arguments (copied at launch), never through a host staging buffer.
struct FieldChunk {
  FieldDev f[8];
  int n;
};
__global__ void store_fields_kernel(FieldChunk ch, FieldDev* out) {
  if ((int)threadIdx.x < ch.n) out[threadIdx.x] = ch.f[threadIdx.x];
}
void upload_fields(hipStream_t st, const FieldDev* host, int n, FieldDev* dev) {
  for (int b = 0; b < n; b += 8) {
    FieldChunk ch;
    ch.n = std::min(8, n - b);
    for (int i = 0; i < ch.n; ++i) ch.f[i] = host[b + i];
    hipLaunchKernelGGL(store_fields_kernel, dim3(1), dim3(64), 0, st, ch, dev + b);
    RTCC_HIP(hipGetLastError());
  }
}

// One block per (component a, member b): strided per-thread sums, then the 256 thread sums
// are combined in a fixed tree order through LDS.
__global__ __launch_bounds__(256) void dipole_batch_kernel(int64_t nn, const double* rre, const double* rim,
                                                           int64_t rbs, const double* mu, const double* mu_ref,
                                                           double* out) {
  __shared__ double sr[256], si[256];
  const int a = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const double* pr = rre + b * rbs;
  const double* pi = rim + b * rbs;
  const double* m = mu + a * nn;
  double xr = 0.0, xi = 0.0;
  for (int64_t i = tid; i < nn; i += 256) {
    xr += pr[i] * m[i];
    xi += pi[i] * m[i];
  }
  sr[tid] = xr;
  si[tid] = xi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      sr[tid] += sr[tid + w];
      si[tid] += si[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[6 * b + 2 * a] = mu_ref[a] + sr[0];
    out[6 * b + 2 * a + 1] = si[0];
  }
}

void dipole_batch(hipStream_t st, int nb, int64_t nn, const double* rho_re, const double* rho_im, int64_t rbs,
                  const double* mu, const double* mu_ref, double* out) {
  hipLaunchKernelGGL(dipole_batch_kernel, dim3(3, (unsigned)nb), dim3(256), 0, st, nn, rho_re, rho_im, rbs, mu,
                     mu_ref, out);
  RTCC_HIP(hipGetLastError());
}

__global__ void scalar_kernel(double* p, double v, int add) { p[0] = add ? p[0] + v : v; }
void scalar_update(hipStream_t st, double* p, double v, bool add) {
  hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(1), 0, st, p, v, add ? 1 : 0);
  RTCC_HIP(hipGetLastError());
}

// ---- RK combinations on the FP64 state ----------------------------------------------------------
struct Combo {
  const double2* k[8];
  double c[8];
  int nk;
};

__global__ void combo_kernel(int64_t n, const double2* __restrict__ y, Combo cb, double2* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = y ? y[i] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= cb.nk) break;
      double2 kk = cb.k[j][i];
      a.x += cb.c[j] * kk.x;
      a.y += cb.c[j] * kk.y;
    }
    out[i] = a;
  }
}

void state_combo(hipStream_t st, int64_t n, const void* y, int nk, const void* const* ks, const double* cs, void* out) {
  RTCC_CHECK(nk <= 8, kEInval, "state_combo: too many terms");
  Combo cb;
  cb.nk = 0;
  for (int j = 0; j < nk; ++j) {
    if (cs[j] == 0.0) continue;
    cb.k[cb.nk] = (const double2*)ks[j];
    cb.c[cb.nk] = cs[j];
    cb.nk++;
  }
  int64_t blocks = std::min<int64_t>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(combo_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, (const double2*)y, cb, (double2*)out);
  RTCC_HIP(hipGetLastError());
}

// ---- fixed-order reductions -------------------------------------------------------------------
// Stage 1: each block reduces a contiguous chunk (wavefront shuffles, then LDS across waves);
// stage 2: one block reduces the per-block partials in index order.
constexpr int kRedBlocks = 512;

__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
__device__ inline double wave_max(double x) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  return x;
}

// mode 0: sum of Re(a*conj?)...  we use explicit modes:
//   MODE_DOT_RC  : sum_i (ar_i + i ai_i) * b_i        (complex a planar, real b)  -> 2 doubles
//   MODE_MAXDIFF : max_i |y5_i - y4_i| (interleaved complex)                        -> 1 double
//   MODE_VDOT    : sum_i conj(a_i) b_i (interleaved complex)                          -> 2 doubles
//   MODE_NONFIN  : count of non-finite entries (interleaved complex)                 -> 1 double
template <typename T, int MODE>
__global__ void reduce_stage1(int64_t n, const void* a, const void* b, const void* c, double* partial) {
  __shared__ double sh0[4], sh1[4];
  int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  int64_t beg = (int64_t)blockIdx.x * chunk, end = min(n, beg + chunk);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    if (MODE == 0) {
      const T* ar = (const T*)a;
      const T* ai = (const T*)c;
      double bv = ((const double*)b)[i];
      s0 += (double)ar[i] * bv;
      s1 += (double)ai[i] * bv;
    } else if (MODE == 1) {
      double2 p = ((const double2*)a)[i], q = b ? ((const double2*)b)[i] : make_double2(0.0, 0.0);
      double dx = p.x - q.x, dy = p.y - q.y;
      s0 = fmax(s0, sqrt(dx * dx + dy * dy));
    } else if (MODE == 2) {
      double2 p = ((const double2*)a)[i], q = ((const double2*)b)[i];
      s0 += p.x * q.x + p.y * q.y;
      s1 += p.x * q.y - p.y * q.x;
    } else {
      double2 p = ((const double2*)a)[i];
      if (!isfinite(p.x) || !isfinite(p.y)) s0 += 1.0;
    }
  }
  if (MODE == 1) s0 = wave_max(s0);
  else {
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
  }
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh0[w] = s0;
    sh1[w] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r0 = sh0[0], r1 = sh1[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      if (MODE == 1) r0 = fmax(r0, sh0[k]);
      else {
        r0 += sh0[k];
        r1 += sh1[k];
      }
    }
    partial[2 * blockIdx.x] = r0;
    partial[2 * blockIdx.x + 1] = r1;
  }
}

template <int MODE>
__global__ void reduce_stage2(int nb, const double* partial, double* out) {
  if (threadIdx.x != 0) return;
  double r0 = partial[0], r1 = partial[1];
  for (int k = 1; k < nb; ++k) {
    if (MODE == 1) r0 = fmax(r0, partial[2 * k]);
    else {
      r0 += partial[2 * k];
      r1 += partial[2 * k + 1];
    }
  }
  out[0] = r0;
  out[1] = r1;
}

template <typename T, int MODE>
static void reduce(hipStream_t st, int64_t n, const void* a, const void* b, const void* c, double* partial,
                   double* out) {
  int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, cdiv(n, 256)));
  hipLaunchKernelGGL((reduce_stage1<T, MODE>), dim3(nb), dim3(256), 0, st, n, a, b, c, partial);
  RTCC_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_stage2<MODE>, dim3(1), dim3(64), 0, st, nb, partial, out);
  RTCC_HIP(hipGetLastError());
}

template <typename T>
void dot_planar_real(hipStream_t st, int64_t n, const T* are, const T* aim, const double* b, double* partial,
                     double* out2) {
  reduce<T, 0>(st, n, are, b, aim, partial, out2);
}
template void dot_planar_real<double>(hipStream_t, int64_t, const double*, const double*, const double*, double*,
                                      double*);
template void dot_planar_real<float>(hipStream_t, int64_t, const float*, const float*, const double*, double*,
                                     double*);

void max_abs_diff(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2) {
  reduce<double, 1>(st, n, a, b, nullptr, partial, out2);
}
void vdot(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2) {
  reduce<double, 2>(st, n, a, b, nullptr, partial, out2);
}
void count_nonfinite(hipStream_t st, int64_t n, const void* a, double* partial, double* out2) {
  reduce<double, 3>(st, n, a, nullptr, nullptr, partial, out2);
}

// ---- adjoint helpers on the interleaved state ---------------------------------------------------
// out (= or +=) scale * post( M( pre(a + cb * b) ) ) with M = Shat or Shat^-1:
//   Shat   (x_T, x_L) = (-i Ginv x_L, +i Ginv x_T),   Ginv: singles x/2, doubles (2 x_ijab + x_ijba)/3
//   Shat^-1(x_T, x_L) = (-i G x_L,    +i G x_T),      G:    singles 2 x, doubles 2 x_ijab - x_ijba
// pre / post: complex conjugation when requested. a, b and out must not overlap.
__global__ void hamil_kernel(int o, int v, const double2* __restrict__ a, const double2* __restrict__ b, double2 cb,
                             int inverse, int conj_in, int conj_out, double scale, int accumulate,
                             double2* __restrict__ out) {
  const int64_t n1 = (int64_t)o * v, n2 = n1 * n1, nst = 2 * (n1 + n2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nst; i += (int64_t)gridDim.x * blockDim.x) {
    const bool tpart = i < n1 + n2;
    const int64_t r = tpart ? i : i - (n1 + n2);  // offset inside the T or L half
    const int64_t src = tpart ? i + (n1 + n2) : i - (n1 + n2);  // same offset in the other half
    auto load = [&](int64_t k) {
      double2 x = a[k];
      if (b) {
        double2 y = b[k];
        x.x += cb.x * y.x - cb.y * y.y;
        x.y += cb.x * y.y + cb.y * y.x;
      }
      if (conj_in) x.y = -x.y;
      return x;
    };
    double2 x;
    if (r < n1) {
      double2 z = load(src);
      double f = inverse ? 2.0 : 0.5;
      x = make_double2(f * z.x, f * z.y);
    } else {
      const int64_t d = r - n1, bb = d % v, aa = (d / v) % v, pre = d / (v * (int64_t)v);
      const int64_t sw = src - d + (pre * v + bb) * v + aa;  // (i j b a) in the other half
      double2 z = load(src), zs = load(sw);
      if (inverse) x = make_double2(2.0 * z.x - zs.x, 2.0 * z.y - zs.y);
      else x = make_double2((2.0 * z.x + zs.x) / 3.0, (2.0 * z.y + zs.y) / 3.0);
    }
    // multiply by -i (T half of the output) or +i (L half): (-i)(x + iy) = y - ix
    double2 res = tpart ? make_double2(x.y, -x.x) : make_double2(-x.y, x.x);
    if (conj_out) res.y = -res.y;
    res.x *= scale;
    res.y *= scale;
    if (accumulate) {
      res.x += out[i].x;
      res.y += out[i].y;
    }
    out[i] = res;
  }
}

void hamil_apply(hipStream_t st, int o, int v, const void* a, const void* b, const double cb[2], bool inverse,
                 bool conj_in, bool conj_out, double scale, bool accumulate, void* out) {
  const int64_t n1 = (int64_t)o * v, nst = 2 * (n1 + n1 * n1);
  int64_t blocks = std::min<int64_t>(cdiv(nst, 256), 8192);
  hipLaunchKernelGGL(hamil_kernel, dim3((unsigned)blocks), dim3(256), 0, st, o, v, (const double2*)a,
                     (const double2*)b, make_double2(cb ? cb[0] : 0.0, cb ? cb[1] : 0.0), inverse ? 1 : 0,
                     conj_in ? 1 : 0, conj_out ? 1 : 0, scale, accumulate ? 1 : 0, (double2*)out);
  RTCC_HIP(hipGetLastError());
}

// Radius of the evaluation circle: rho / max|u| (rho when u = 0).
__device__ inline double circle_radius(const double* maxu, double rho) {
  return maxu[0] > 0.0 ? rho / maxu[0] : rho;
}

// out[j] = y + r w^j u for the m points w^j = exp(2 pi i j / m)
__global__ void circle_points_kernel(int64_t nst, const double2* __restrict__ y, const double2* __restrict__ u,
                                     const double* maxu, double rho, int m, double2* __restrict__ out) {
  const double r = circle_radius(maxu, rho);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nst * m; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i / nst);
    const int64_t k = i - (int64_t)j * nst;
    double sn, cs;
    sincospi(2.0 * j / m, &sn, &cs);
    const double2 uu = u[k], yy = y[k];
    out[i] = make_double2(yy.x + r * (cs * uu.x - sn * uu.y), yy.y + r * (cs * uu.y + sn * uu.x));
  }
}

void circle_points(hipStream_t st, int64_t nst, const void* y, const void* u, const double* maxu, double rho, int m,
                   void* out) {
  int64_t blocks = std::min<int64_t>(cdiv(nst * m, 256), 8192);
  hipLaunchKernelGGL(circle_points_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nst, (const double2*)y,
                     (const double2*)u, maxu, rho, m, (double2*)out);
  RTCC_HIP(hipGetLastError());
}

// out = (1 / (m r)) sum_j conj(w^j) F_j: the first-order Taylor coefficient of a polynomial of degree < m + 1
// sampled on the circle (exact, no truncation error)
__global__ void circle_coef1_kernel(int64_t nst, const double2* __restrict__ F, const double* maxu, double rho, int m,
                                    double2* __restrict__ out) {
  const double r = circle_radius(maxu, rho);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nst; k += (int64_t)gridDim.x * blockDim.x) {
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < m; ++j) {
      double sn, cs;
      sincospi(2.0 * j / m, &sn, &cs);
      const double2 f = F[(int64_t)j * nst + k];
      sx += cs * f.x + sn * f.y;  // conj(w) f = (cs - i sn)(fx + i fy)
      sy += cs * f.y - sn * f.x;
    }
    out[k] = make_double2(sx / (m * r), sy / (m * r));
  }
}

void circle_coef1(hipStream_t st, int64_t nst, const void* F, const double* maxu, double rho, int m, void* out) {
  int64_t blocks = std::min<int64_t>(cdiv(nst, 256), 8192);
  hipLaunchKernelGGL(circle_coef1_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nst, (const double2*)F, maxu, rho,
                     m, (double2*)out);
  RTCC_HIP(hipGetLastError());
}

void max_abs(hipStream_t st, int64_t n, const void* a, double* partial, double* out2) {
  reduce<double, 1>(st, n, a, nullptr, nullptr, partial, out2);
}

// ---- divergence guard: |T2| and the non-finite entries of an interleaved state ----------------
// Stage 1: each block sums |y_i|^2 over its part of [t2b, t2e) and counts the non-finite entries of
// its part of [0, nst); stage 2 adds the block partials in index order and writes
// out[0] = sqrt(sum) (NaN if any entry is non-finite) and out[1] = the count.
__global__ void guard_stage1(int64_t nst, int64_t t2b, int64_t t2e, const double2* __restrict__ y,
                             double* partial) {
  __shared__ double sh0[4], sh1[4];
  const int64_t chunk = (nst + gridDim.x - 1) / gridDim.x;
  const int64_t beg = (int64_t)blockIdx.x * chunk, end = min(nst, beg + chunk);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const double2 p = y[i];
    if (!isfinite(p.x) || !isfinite(p.y)) s1 += 1.0;
    else if (i >= t2b && i < t2e) s0 += p.x * p.x + p.y * p.y;
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh0[w] = s0;
    sh1[w] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r0 = sh0[0], r1 = sh1[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      r0 += sh0[k];
      r1 += sh1[k];
    }
    partial[2 * blockIdx.x] = r0;
    partial[2 * blockIdx.x + 1] = r1;
  }
}

__global__ void guard_stage2(int nb, const double* partial, double* out) {
  if (threadIdx.x != 0) return;
  double r0 = 0.0, r1 = 0.0;
  for (int k = 0; k < nb; ++k) {
    r0 += partial[2 * k];
    r1 += partial[2 * k + 1];
  }
  out[0] = r1 > 0.0 ? __builtin_nan("") : sqrt(r0);
  out[1] = r1;
}

void state_guard(hipStream_t st, int64_t nst, int64_t t2b, int64_t t2e, const void* y, double* partial,
                 double* out2) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kGuardBlocks, cdiv(nst, 256)));
  hipLaunchKernelGGL(guard_stage1, dim3(nb), dim3(256), 0, st, nst, t2b, t2e, (const double2*)y, partial);
  RTCC_HIP(hipGetLastError());
  hipLaunchKernelGGL(guard_stage2, dim3(1), dim3(64), 0, st, nb, partial, out2);
  RTCC_HIP(hipGetLastError());
}

// ---- ground-state Jacobi update on the interleaved state: x += R / D ---------------------------
// R given as planar residuals (r1 = o*v, r2 = o*o*v*v), D from the diagonal of the spatial Fock matrix
template <typename T>
__global__ void jacobi_kernel(int o, int v, const double* fdiag, const T* r1, const T* r2, double2* x1, double2* x2,
                              double2* e1, double2* e2) {
  int64_t n1 = (int64_t)o * v, n2 = n1 * n1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += (int64_t)gridDim.x * blockDim.x) {
    double d, rr, ri;
    if (i < n1) {
      int a = (int)(i % v), ii = (int)(i / v);
      d = fdiag[ii] - fdiag[o + a];
      rr = r1[i];
      ri = r1[i + n1];
      double2 q = make_double2(rr / d, ri / d);
      e1[i] = q;
      x1[i] = make_double2(x1[i].x + q.x, x1[i].y + q.y);
    } else {
      int64_t j = i - n1;
      int b = (int)(j % v), a = (int)((j / v) % v), jj = (int)((j / v / v) % o), ii = (int)(j / v / v / o);
      d = fdiag[ii] + fdiag[jj] - fdiag[o + a] - fdiag[o + b];
      rr = r2[j];
      ri = r2[j + n2];
      double2 q = make_double2(rr / d, ri / d);
      e2[j] = q;
      x2[j] = make_double2(x2[j].x + q.x, x2[j].y + q.y);
    }
  }
}

template <typename T>
void jacobi_update(hipStream_t st, int o, int v, const double* fdiag, const T* r1, const T* r2, void* x1, void* x2,
                   void* e1, void* e2) {
  int64_t n = (int64_t)o * v + (int64_t)o * o * v * v;
  int64_t blocks = std::min<int64_t>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(jacobi_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, o, v, fdiag, r1, r2, (double2*)x1,
                     (double2*)x2, (double2*)e1, (double2*)e2);
  RTCC_HIP(hipGetLastError());
}
template void jacobi_update<double>(hipStream_t, int, int, const double*, const double*, const double*, void*, void*,
                                    void*, void*);

// max |R| over planar residual arrays (convergence test)
template <typename T>
__global__ void maxabs_planar_kernel(int64_t n, const T* re, const T* im, double* partial) {
  __shared__ double sh[4];
  int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  int64_t beg = (int64_t)blockIdx.x * chunk, end = min(n, beg + chunk);
  double m = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    double a = re[i], b = im[i];
    double x = sqrt(a * a + b * b);
    m = (x != x) ? INFINITY : fmax(m, x);
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, sh[k]);
    partial[2 * blockIdx.x] = r;
    partial[2 * blockIdx.x + 1] = 0.0;
  }
}

template <typename T>
void maxabs_planar(hipStream_t st, int64_t n, const T* re, const T* im, double* partial, double* out2) {
  int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, cdiv(n, 256)));
  hipLaunchKernelGGL(maxabs_planar_kernel<T>, dim3(nb), dim3(256), 0, st, n, re, im, partial);
  RTCC_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_stage2<1>, dim3(1), dim3(64), 0, st, nb, partial, out2);
  RTCC_HIP(hipGetLastError());
}
template void maxabs_planar<double>(hipStream_t, int64_t, const double*, const double*, double*, double*);

// ---- ring-intermediate combinations --------------------------------------------------------------
// With p = (m,e), q = (j,b) and X(p,q) = X[p * Q + q] for X in {Bd, Pd, Bx, Px} (planar complex):
//   W[q * 2P + p] = Bd + Pd / 2,   W[q * 2P + P + p] = Bx + Px / 2      (transposed, via LDS)
//   H[p * 2Q + 2q] = Bd + Pd,      H[p * 2Q + 2q + 1] = Bx + Px          (optional)
// 32 x 32 tiles of (p, q); member blockIdx.z of a batch at the given batch strides.
template <typename T>
struct RingArgs {
  const T* x[8];  // Bd, Pd, Bx, Px: re, im
  T* w[2];        // W re, im
  T* h[2];        // H re, im (nullptr: not formed)
  int64_t P, Q, tiles_q;
  int64_t xbs, wbs, hbs;
};

template <typename T>
__global__ __launch_bounds__(256) void ring_combo_kernel(RingArgs<T> a) {
  __shared__ T sw[4][32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t p0 = (blockIdx.x / a.tiles_q) * 32, q0 = (blockIdx.x % a.tiles_q) * 32;
  const int64_t z = blockIdx.z;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t p = p0 + ty + 8 * k, q = q0 + tx;
    if (p < a.P && q < a.Q) {
      const int64_t i = z * a.xbs + p * a.Q + q;
      T v[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = a.x[c][i];
      // v: Bd re, Bd im, Pd re, Pd im, Bx re, Bx im, Px re, Px im
      sw[0][ty + 8 * k][tx] = v[0] + T(0.5) * v[2];
      sw[1][ty + 8 * k][tx] = v[1] + T(0.5) * v[3];
      sw[2][ty + 8 * k][tx] = v[4] + T(0.5) * v[6];
      sw[3][ty + 8 * k][tx] = v[5] + T(0.5) * v[7];
      if (a.h[0]) {
        const int64_t o = z * a.hbs + p * 2 * a.Q + 2 * q;
        a.h[0][o] = v[0] + v[2];
        a.h[0][o + 1] = v[4] + v[6];
        a.h[1][o] = v[1] + v[3];
        a.h[1][o + 1] = v[5] + v[7];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t q = q0 + ty + 8 * k, p = p0 + tx;
    if (p < a.P && q < a.Q) {
      const int64_t o = z * a.wbs + q * 2 * a.P + p;
      a.w[0][o] = sw[0][tx][ty + 8 * k];
      a.w[1][o] = sw[1][tx][ty + 8 * k];
      a.w[0][o + a.P] = sw[2][tx][ty + 8 * k];
      a.w[1][o + a.P] = sw[3][tx][ty + 8 * k];
    }
  }
}

template <typename T>
void ring_combo(hipStream_t st, int64_t P, int64_t Q, int nb, const T* const x[8], int64_t xbs, T* wre, T* wim,
                int64_t wbs, T* hre, T* him, int64_t hbs) {
  RTCC_CHECK(P > 0 && Q > 0 && nb >= 1 && nb <= 65535, kEInval, "ring_combo: bad extents");
  RingArgs<T> a;
  for (int c = 0; c < 8; ++c) a.x[c] = x[c];
  a.w[0] = wre;
  a.w[1] = wim;
  a.h[0] = hre;
  a.h[1] = him;
  a.P = P;
  a.Q = Q;
  a.tiles_q = cdiv(Q, 32);
  a.xbs = xbs;
  a.wbs = wbs;
  a.hbs = hbs;
  const int64_t tiles = cdiv(P, 32) * a.tiles_q;
  RTCC_CHECK(tiles < (1LL << 31), kEInval, "ring_combo: too many tiles");
  hipLaunchKernelGGL(ring_combo_kernel<T>, dim3((unsigned)tiles, 1, (unsigned)nb), dim3(256), 0, st, a);
  RTCC_HIP(hipGetLastError());
}
template void ring_combo<double>(hipStream_t, int64_t, int64_t, int, const double* const[8], int64_t, double*,
                                 double*, int64_t, double*, double*, int64_t);
template void ring_combo<float>(hipStream_t, int64_t, int64_t, int, const float* const[8], int64_t, float*, float*,
                                int64_t, float*, float*, int64_t);

// ---- amplitude combinations ------------------------------------------------------------------------
// For every (i,j): tau = t2 + t1_ia t1_jb, taut = t2 + t1_ia t1_jb / 2, t2s = 2 t2 - t2[b,a] and (if l2)
// l2s = 2 l2 - l2[b,a], planar complex, [i][j][a][b] row-major. A workgroup takes one (i,j) and one
// pair of mirrored 32 x 32 (a,b) tiles (ta <= tb), so the transposed partner of every element is in
// LDS and each element of t2 and l2 is read once; t2 and l2 go to separate workgroups (blockIdx.z =
// 2 member + which). Member at batch stride bs1 for t1 and bs[k] for the doubles (t2, l2, tau, taut,
// t2s, l2s).
template <typename T>
struct AmpArgs {
  const T* t1[2];
  const T* t2[2];
  const T* l2[2];
  T* tau[2];
  T* taut[2];
  T* t2s[2];
  T* l2s[2];
  T* stk[2][2];  // stacked (X-s, X) copies: [t2 / l2][re / im], or null
  int o, v, nt;
  int64_t bs1, bs[6], sbs[2];
};

template <typename T>
__global__ __launch_bounds__(256) void amp_combo_kernel(AmpArgs<T> g) {
  __shared__ T s[2][2][32][33];  // [tile A / mirror tile B][re / im]
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // pair index -> (ta, tb), ta <= tb: row ta holds nt - ta pairs
  int q = blockIdx.x, ta = 0;
  while (q >= g.nt - ta) {
    q -= g.nt - ta;
    ++ta;
  }
  const int tb = ta + q;
  const int ij = blockIdx.y, i = ij / g.o, j = ij - i * g.o;
  const int64_t z = blockIdx.z >> 1, vv = (int64_t)g.v * g.v;
  const int which = blockIdx.z & 1;
  const int64_t base = (int64_t)ij * vv;  // (i,j) block; member offsets per tensor below
  const int a0 = ta * 32, b0 = tb * 32;
  const bool mirror = ta != tb;
  const T* t1r = g.t1[0] + z * g.bs1 + (int64_t)i * g.v;
  const T* t1i = g.t1[1] + z * g.bs1 + (int64_t)i * g.v;
  const T* u1r = g.t1[0] + z * g.bs1 + (int64_t)j * g.v;
  const T* u1i = g.t1[1] + z * g.bs1 + (int64_t)j * g.v;
  {
    const T* const* X = which == 0 ? g.t2 : g.l2;
    if (which == 1 && !X[0]) return;  // uniform over the workgroup
    T* const* XS = which == 0 ? g.t2s : g.l2s;
    const int64_t xo = z * g.bs[which], so = z * g.bs[which == 0 ? 4 : 5];
    const int64_t to = z * g.bs[2], uo = z * g.bs[3];
    // tile A = X[a0 + r][b0 + c], tile B = X[b0 + r][a0 + c]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = ty + 8 * k;
      for (int c = 0; c < 2; ++c) {
        s[0][c][r][tx] = (a0 + r < g.v && b0 + tx < g.v) ? X[c][xo + base + (int64_t)(a0 + r) * g.v + b0 + tx] : T(0);
        if (mirror)
          s[1][c][r][tx] =
              (b0 + r < g.v && a0 + tx < g.v) ? X[c][xo + base + (int64_t)(b0 + r) * g.v + a0 + tx] : T(0);
      }
    }
    __syncthreads();
    for (int h = 0; h < (mirror ? 2 : 1); ++h) {
      const int ra = h == 0 ? a0 : b0, cb = h == 0 ? b0 : a0;  // this tile's row (a) and column (b) origins
      const int ht = mirror ? 1 - h : 0;                        // the tile holding the transposed partners
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = ty + 8 * k, a = ra + r, b = cb + tx;
        if (a >= g.v || b >= g.v) continue;
        const int64_t off = base + (int64_t)a * g.v + b;
        const T xr = s[h][0][r][tx], xi = s[h][1][r][tx];
        const T yr = s[ht][0][tx][r], yi = s[ht][1][tx][r];  // X[b][a]
        const T sr = T(2) * xr - yr, si = T(2) * xi - yi;
        XS[0][so + off] = sr;
        XS[1][so + off] = si;
        if (g.stk[which][0]) {
          T* const* K = g.stk[which];
          const int64_t ov = (int64_t)g.o * g.v, ia = (int64_t)i * g.v + a, ko = z * g.sbs[which];
          if (which == 0) {  // [i][a][s][j][b]: s = 0 t2s, s = 1 t2
            const int64_t q = ko + ia * 2 * ov + (int64_t)j * g.v + b;
            K[0][q] = sr;
            K[1][q] = si;
            K[0][q + ov] = xr;
            K[1][q + ov] = xi;
          } else {  // [i][a][j][b][s]: s = 0 l2s, s = 1 l2, as one two-element store per plane
            typedef T T2 __attribute__((ext_vector_type(2)));
            const int64_t q = ko + ((ia * g.o + j) * g.v + b) * 2;
            *reinterpret_cast<T2*>(K[0] + q) = T2{sr, xr};
            *reinterpret_cast<T2*>(K[1] + q) = T2{si, xi};
          }
        }
        if (which == 0) {
          const T pr = t1r[a] * u1r[b] - t1i[a] * u1i[b];
          const T pi = t1r[a] * u1i[b] + t1i[a] * u1r[b];
          g.tau[0][to + off] = xr + pr;
          g.tau[1][to + off] = xi + pi;
          g.taut[0][uo + off] = xr + T(0.5) * pr;
          g.taut[1][uo + off] = xi + T(0.5) * pi;
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
void amp_combo(hipStream_t st, int o, int v, int nb, const T* const t1[2], int64_t bs1, const T* const t2[2],
               const T* const l2[2], const int64_t bs[6], T* const tau[2], T* const taut[2], T* const t2s[2],
               T* const l2s[2], T* const stk_t[2], int64_t sbs_t, T* const stk_l[2], int64_t sbs_l) {
  RTCC_CHECK(o > 0 && v > 0 && nb >= 1 && nb <= 32767 && (int64_t)o * o <= 65535, kEInval, "amp_combo: bad extents");
  RTCC_CHECK(!stk_l || ((uintptr_t)stk_l[0] % (2 * sizeof(T)) == 0 && (uintptr_t)stk_l[1] % (2 * sizeof(T)) == 0 &&
                        sbs_l % 2 == 0),
             kEInval, "amp_combo: misaligned stacked lambda copy");
  AmpArgs<T> g;
  for (int c = 0; c < 2; ++c) {
    g.stk[0][c] = stk_t ? stk_t[c] : nullptr;
    g.stk[1][c] = (stk_l && l2) ? stk_l[c] : nullptr;
  }
  g.sbs[0] = sbs_t;
  g.sbs[1] = sbs_l;
  for (int c = 0; c < 2; ++c) {
    g.t1[c] = t1[c];
    g.t2[c] = t2[c];
    g.l2[c] = l2 ? l2[c] : nullptr;
    g.tau[c] = tau[c];
    g.taut[c] = taut[c];
    g.t2s[c] = t2s[c];
    g.l2s[c] = l2 ? l2s[c] : nullptr;
  }
  g.o = o;
  g.v = v;
  g.nt = (int)cdiv(v, 32);
  g.bs1 = bs1;
  for (int k = 0; k < 6; ++k) g.bs[k] = bs[k];
  const unsigned pairs = (unsigned)(g.nt * (g.nt + 1) / 2);
  hipLaunchKernelGGL(amp_combo_kernel<T>, dim3(pairs, (unsigned)(o * o), (unsigned)(2 * nb)), dim3(256), 0, st, g);
  RTCC_HIP(hipGetLastError());
}
template void amp_combo<double>(hipStream_t, int, int, int, const double* const[2], int64_t, const double* const[2],
                                const double* const[2], const int64_t[6], double* const[2], double* const[2],
                                double* const[2], double* const[2], double* const[2], int64_t,
                                double* const[2], int64_t);
template void amp_combo<float>(hipStream_t, int, int, int, const float* const[2], int64_t, const float* const[2],
                               const float* const[2], const int64_t[6], float* const[2], float* const[2],
                               float* const[2], float* const[2], float* const[2], int64_t, float* const[2],
                               int64_t);

// ---- doubles residual assembly ------------------------------------------------------------------
// out[ijab] += base[ijab] + lad[ijab] + z[ijab] + zt[iajb] + z[jiba] + zt[jbia]. A workgroup takes a
// 32 x 32 (a, b) tile of one (i, j) block; the partners z[jiba] + zt[jbia] are read along a (the
// contiguous index of both) into LDS and taken transposed.
template <typename T>
struct PairArgs {
  T* out[2];
  const T* base[2];
  const T* lad[2];
  const T* z[2];
  const T* zt[2];
  int o, v, nt;
  int64_t obs, lbs, zbs, tbs;
};

template <typename T>
__global__ __launch_bounds__(256) void pair_combo_kernel(PairArgs<T> g) {
  __shared__ T s[2][32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int ta = blockIdx.x / g.nt, tb = blockIdx.x - ta * g.nt;
  const int ij = blockIdx.y, i = ij / g.o, j = ij - i * g.o;
  const int64_t m = blockIdx.z, v = g.v, vv = v * v, ov = (int64_t)g.o * v;
  const int a0 = ta * 32, b0 = tb * 32;
  // partners: row r <-> b = b0 + r, column tx <-> a = a0 + tx
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ty + 8 * k, a = a0 + tx, b = b0 + r;
    if (a >= g.v || b >= g.v) continue;
    const int64_t zo = m * g.zbs + ((int64_t)j * g.o + i) * vv + (int64_t)b * v + a;
    const int64_t to = m * g.tbs + (int64_t)j * v * ov + (int64_t)b * ov + (int64_t)i * v + a;
#pragma unroll
    for (int c = 0; c < 2; ++c) s[c][r][tx] = g.z[c][zo] + g.zt[c][to];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ty + 8 * k, a = a0 + r, b = b0 + tx;
    if (a >= g.v || b >= g.v) continue;
    const int64_t off = (int64_t)ij * vv + (int64_t)a * v + b;
    const int64_t to = m * g.tbs + (int64_t)i * v * ov + (int64_t)a * ov + (int64_t)j * v + b;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T x = g.out[c][m * g.obs + off];
      if (g.base[c]) x += g.base[c][off];
      x += g.lad[c][m * g.lbs + off];
      x += g.z[c][m * g.zbs + off];
      x += g.zt[c][to];
      x += s[c][tx][r];
      g.out[c][m * g.obs + off] = x;
    }
  }
}

template <typename T>
void pair_combo(hipStream_t st, int o, int v, int nb, T* const out[2], int64_t obs, const T* const base[2],
                const T* const lad[2], int64_t lbs, const T* const z[2], int64_t zbs, const T* const zt[2],
                int64_t tbs) {
  RTCC_CHECK(o > 0 && v > 0 && nb >= 1 && nb <= 65535 && (int64_t)o * o <= 65535, kEInval, "pair_combo: bad extents");
  PairArgs<T> g;
  for (int c = 0; c < 2; ++c) {
    g.out[c] = out[c];
    g.base[c] = base[c];
    g.lad[c] = lad[c];
    g.z[c] = z[c];
    g.zt[c] = zt[c];
  }
  g.o = o;
  g.v = v;
  g.nt = (int)cdiv(v, 32);
  g.obs = obs;
  g.lbs = lbs;
  g.zbs = zbs;
  g.tbs = tbs;
  hipLaunchKernelGGL(pair_combo_kernel<T>, dim3((unsigned)(g.nt * g.nt), (unsigned)(o * o), (unsigned)nb), dim3(256),
                     0, st, g);
  RTCC_HIP(hipGetLastError());
}
template void pair_combo<double>(hipStream_t, int, int, int, double* const[2], int64_t, const double* const[2],
                                 const double* const[2], int64_t, const double* const[2], int64_t,
                                 const double* const[2], int64_t);
template void pair_combo<float>(hipStream_t, int, int, int, float* const[2], int64_t, const float* const[2],
                                const float* const[2], int64_t, const float* const[2], int64_t, const float* const[2],
                                int64_t);

}  // namespace rtcc
