// Symmetric / antisymmetric form of the particle-particle ladder.
//
// The closed-shell ladder Z_ij^ab = sum_ef <ab|ef> X_ij^ef (X = tau or lambda2) has the pair symmetry
// X_ji^fe = X_ij^ef, and <ab|ef> = <ba|fe>. Splitting X by the exchange e <-> f,
//   X+_ij^(ef) = X_ij^ef + X_ij^fe (e < f),  X_ij^ee (e = f),     X-_ij^(ef) = X_ij^ef - X_ij^fe (e < f),
// and the integrals the same way, V+-_(ef),(ab) = (<ab|ef> +- <ab|fe>) / 2, gives
//   Z_ij^ab = S_ij^ab + A_ij^ab,  S = sum_{e<=f} X+ V+,  A = sum_{e<f} X- V-,
// where S is symmetric and A antisymmetric under i <-> j and under a <-> b. So S is needed only for
// i <= j, a <= b and A only for i < j, a < b: two GEMMs over the triangles, o(o+1)/2 x v(v+1)/2 x
// v(v+1)/2 and o(o-1)/2 x v(v-1)/2 x v(v-1)/2, a quarter of the flops of the full o^2 x v^2 x v^2
// product. The paper notes that the ground-state coupled-cluster machinery carries over to the
// time-dependent equations (Theory, propagation of the RT-CC equations); this is one such device.
//
// Pair (p, q) with p <= q (diag = 1) or p < q (diag = 0) of n is stored at the row-major position of
// the upper triangle: rows p = 0, 1, ... in order, q ascending within a row.
#include "elementwise.h"

namespace rtcc {

namespace {

__device__ __host__ inline int64_t tri_index(int p, int q, int n, int diag) {
  return (int64_t)p * (n - 1 + diag) - (int64_t)p * (p - 1) / 2 + (q - p - (1 - diag));
}

// (i, j) with i <= j from its pair index
__device__ inline void tri_decode(int idx, int n, int& i, int& j) {
  i = 0;
  while (idx >= n - i) {
    idx -= n - i;
    ++i;
  }
  j = i + idx;
}

// grid: x over the v*v (e, f) grid, y over (block, i <= j)
template <typename T>
__global__ __launch_bounds__(256) void fold_kernel(int o, int v, const T* __restrict__ xre, const T* __restrict__ xim,
                                                   T* __restrict__ pre, T* __restrict__ pim, T* __restrict__ mre,
                                                   T* __restrict__ mim) {
  const int po = o * (o + 1) / 2, pm = o * (o - 1) / 2;
  const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
  const int blk = blockIdx.y / po, pidx = blockIdx.y - blk * po;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= v * v) return;
  const int e = idx / v, f = idx - e * v;
  if (f < e) return;
  int i, j;
  tri_decode(pidx, o, i, j);
  const int64_t base = ((int64_t)blk * o * o + (int64_t)i * o + j) * v * v;
  const T ar = xre[base + (int64_t)e * v + f], ai = xim[base + (int64_t)e * v + f];
  const T br = xre[base + (int64_t)f * v + e], bi = xim[base + (int64_t)f * v + e];
  const int64_t op = ((int64_t)blk * po + pidx) * pv + tri_index(e, f, v, 1);
  pre[op] = e == f ? ar : ar + br;
  pim[op] = e == f ? ai : ai + bi;
  if (i < j && e < f) {
    const int64_t om = ((int64_t)blk * pm + tri_index(i, j, o, 0)) * mv + tri_index(e, f, v, 0);
    mre[om] = ar - br;
    mim[om] = ai - bi;
  }
}

// grid: x over the v*v (a, b) grid, y over (block, i, j)
template <typename T>
__global__ __launch_bounds__(256) void unfold_kernel(int o, int v, const T* __restrict__ sre, const T* __restrict__ sim,
                                                     const T* __restrict__ are, const T* __restrict__ aim,
                                                     T* __restrict__ zre, T* __restrict__ zim) {
  const int po = o * (o + 1) / 2, pm = o * (o - 1) / 2;
  const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
  const int blk = blockIdx.y / (o * o), ij = blockIdx.y - blk * o * o;
  const int i = ij / o, j = ij - i * o;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= v * v) return;
  const int a = idx / v, b = idx - a * v;
  const int p = min(i, j), q = max(i, j), c = min(a, b), d = max(a, b);
  const int64_t os = ((int64_t)blk * po + tri_index(p, q, o, 1)) * pv + tri_index(c, d, v, 1);
  T zr = sre[os], zi = sim[os];
  if (i != j && a != b) {
    const int64_t oa = ((int64_t)blk * pm + tri_index(p, q, o, 0)) * mv + tri_index(c, d, v, 0);
    const T s = (i < j) == (a < b) ? T(1) : T(-1);
    zr += s * are[oa];
    zi += s * aim[oa];
  }
  const int64_t oz = ((int64_t)blk * o * o + ij) * v * v + idx;
  zre[oz] = zr;
  zim[oz] = zi;
}

// 32-bit pair index (every triangle of the LDS-staged kernels has fewer than 2^31 entries)
__device__ inline int tri32(int p, int q, int n, int diag) {
  return p * (n - 1 + diag) - p * (p - 1) / 2 + (q - p - (1 - diag));
}

constexpr int kLdsV = 96;  // largest v of the LDS-staged fold / unfold (one v x v plane per workgroup)

// One workgroup per (block, i <= j, plane): the v x v plane X[blk][i][j] is read once, coalesced, into LDS;
// then each (e, f) with e <= f writes its X+ entry (and for i < j, e < f its X- entry): within a row e the
// outputs are consecutive.
template <typename T>
__global__ __launch_bounds__(256) void fold_lds_kernel(int o, int v, const T* __restrict__ xre,
                                                       const T* __restrict__ xim, T* __restrict__ pre,
                                                       T* __restrict__ pim, T* __restrict__ mre, T* __restrict__ mim) {
  __shared__ T sx[kLdsV * kLdsV];
  const int po = o * (o + 1) / 2, pm = o * (o - 1) / 2;
  const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
  const int blk = blockIdx.y / po, pidx = blockIdx.y - blk * po;
  int i, j;
  tri_decode(pidx, o, i, j);
  const int vv = v * v;
  const int64_t base = ((int64_t)blk * o * o + (int64_t)i * o + j) * vv;
  const T* x = blockIdx.x ? xim : xre;
  T* outp = (blockIdx.x ? pim : pre) + ((int64_t)blk * po + pidx) * pv;
  T* outm = (blockIdx.x ? mim : mre) + (i < j ? ((int64_t)blk * pm + tri_index(i, j, o, 0)) * mv : 0);
  for (int k = threadIdx.x; k < vv; k += blockDim.x) sx[k] = x[base + k];
  __syncthreads();
  for (int k = threadIdx.x; k < vv; k += blockDim.x) {
    const int e = k / v, f = k - e * v;
    if (f < e) continue;
    const T a = sx[k], b = sx[f * v + e];
    outp[tri32(e, f, v, 1)] = e == f ? a : a + b;
    if (i < j && e < f) outm[tri32(e, f, v, 0)] = a - b;
  }
}

// One workgroup per (block, i <= j, plane): the S+ row (and for i < j the S- row) is read once into LDS and
// both output planes Z[blk][i][j] and Z[blk][j][i] are written, coalesced.
template <typename T>
__global__ __launch_bounds__(256) void unfold_lds_kernel(int o, int v, const T* __restrict__ sre,
                                                         const T* __restrict__ sim, const T* __restrict__ are,
                                                         const T* __restrict__ aim, T* __restrict__ zre,
                                                         T* __restrict__ zim) {
  __shared__ T sp[kLdsV * (kLdsV + 1) / 2];
  __shared__ T sm[kLdsV * (kLdsV - 1) / 2];
  const int po = o * (o + 1) / 2, pm = o * (o - 1) / 2;
  const int pv = v * (v + 1) / 2, mv = v * (v - 1) / 2;
  const int blk = blockIdx.y / po, pidx = blockIdx.y - blk * po;
  int i, j;
  tri_decode(pidx, o, i, j);
  const int vv = v * v;
  const T* s = (blockIdx.x ? sim : sre) + ((int64_t)blk * po + pidx) * pv;
  const T* a = (blockIdx.x ? aim : are) + (i < j ? ((int64_t)blk * pm + tri_index(i, j, o, 0)) * mv : 0);
  T* z = blockIdx.x ? zim : zre;
  const int64_t oij = ((int64_t)blk * o * o + (int64_t)i * o + j) * vv;
  const int64_t oji = ((int64_t)blk * o * o + (int64_t)j * o + i) * vv;
  for (int k = threadIdx.x; k < pv; k += blockDim.x) sp[k] = s[k];
  if (i < j)
    for (int k = threadIdx.x; k < mv; k += blockDim.x) sm[k] = a[k];
  __syncthreads();
  for (int k = threadIdx.x; k < vv; k += blockDim.x) {
    const int aa = k / v, bb = k - aa * v;
    const int c = min(aa, bb), d = max(aa, bb);
    const T sv = sp[tri32(c, d, v, 1)];
    if (i == j) {
      z[oij + k] = sv;
    } else {
      const T av = aa == bb ? T(0) : (aa < bb ? sm[tri32(c, d, v, 0)] : -sm[tri32(c, d, v, 0)]);
      z[oij + k] = sv + av;
      z[oji + k] = sv - av;
    }
  }
}

// V+ [(e <= f)][(a <= b)] and V- [(e < f)][(a < b)] from the v^2 x v^2 matrix V[(ab)][(ef)] = <ab|ef>
__global__ __launch_bounds__(256) void sym_build_kernel(int v, const double* __restrict__ V, double* __restrict__ vp,
                                                        double* __restrict__ vm) {
  const int64_t vv = (int64_t)v * v, pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
  const int64_t ef = (int64_t)blockIdx.y, ab = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ab >= vv) return;
  const int e = (int)(ef / v), f = (int)(ef - (int64_t)e * v), a = (int)(ab / v), b = (int)(ab - (int64_t)a * v);
  if (f < e || b < a) return;
  const double x = V[ab * vv + ef], y = V[ab * vv + (int64_t)f * v + e];
  vp[tri_index(e, f, v, 1) * pv + tri_index(a, b, v, 1)] = 0.5 * (x + y);
  if (e < f && a < b) vm[tri_index(e, f, v, 0) * mv + tri_index(a, b, v, 0)] = 0.5 * (x - y);
}

}  // namespace

template <typename T>
void ladder_fold(hipStream_t st, int nblk, int o, int v, const T* xre, const T* xim, T* pre, T* pim, T* mre, T* mim,
                 bool lds) {
  const int po = o * (o + 1) / 2;
  RTCC_CHECK((int64_t)nblk * po < 65536, kEInval, "ladder_fold: too many pair rows");
  if (lds && v <= kLdsV) {
    hipLaunchKernelGGL(fold_lds_kernel<T>, dim3(2, (unsigned)(nblk * po)), dim3(256), 0, st, o, v, xre, xim, pre, pim,
                       mre, mim);
    RTCC_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(fold_kernel<T>, dim3((unsigned)cdiv((int64_t)v * v, 256), (unsigned)(nblk * po)), dim3(256), 0, st,
                     o, v, xre, xim, pre, pim, mre, mim);
  RTCC_HIP(hipGetLastError());
}

template <typename T>
void ladder_unfold(hipStream_t st, int nblk, int o, int v, const T* sre, const T* sim, const T* are, const T* aim,
                   T* zre, T* zim, bool lds) {
  RTCC_CHECK((int64_t)nblk * o * o < 65536, kEInval, "ladder_unfold: too many pair rows");
  if (lds && v <= kLdsV) {
    hipLaunchKernelGGL(unfold_lds_kernel<T>, dim3(2, (unsigned)(nblk * (o * (o + 1) / 2))), dim3(256), 0, st, o, v,
                       sre, sim, are, aim, zre, zim);
    RTCC_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(unfold_kernel<T>, dim3((unsigned)cdiv((int64_t)v * v, 256), (unsigned)(nblk * o * o)), dim3(256),
                     0, st, o, v, sre, sim, are, aim, zre, zim);
  RTCC_HIP(hipGetLastError());
}

void ladder_sym_build(hipStream_t st, int v, const double* vvvv, double* vp, double* vm) {
  const int64_t vv = (int64_t)v * v;
  RTCC_CHECK(vv < 65536, kEInval, "ladder_sym_build: v too large");
  hipLaunchKernelGGL(sym_build_kernel, dim3((unsigned)cdiv(vv, 256), (unsigned)vv), dim3(256), 0, st, v, vvvv, vp, vm);
  RTCC_HIP(hipGetLastError());
}

template void ladder_fold<double>(hipStream_t, int, int, int, const double*, const double*, double*, double*, double*,
                                  double*, bool);
template void ladder_fold<float>(hipStream_t, int, int, int, const float*, const float*, float*, float*, float*,
                                 float*, bool);
template void ladder_unfold<double>(hipStream_t, int, int, int, const double*, const double*, const double*,
                                    const double*, double*, double*, bool);
template void ladder_unfold<float>(hipStream_t, int, int, int, const float*, const float*, const float*, const float*,
                                   float*, float*, bool);

}  // namespace rtcc
