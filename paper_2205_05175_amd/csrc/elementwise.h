// Declarations of the memory-bound kernels (state layout, RK combinations, reductions).
#pragma once
#include "engine.h"

namespace rtcc {

// Planar T1, T2, L1, L2 (or their residuals); member b of a batch at re[i] + b * bs[i] (same for im).
template <typename T>
struct Planes4 {
  T* re[4];
  T* im[4];
  int64_t bs[4];
};
// y holds nb consecutive states (nb = 1 for a single state).
template <typename T>
void unpack_state(hipStream_t st, const void* y, int o, int v, Planes4<T> P, int nb = 1);
template <typename T>
void pack_rhs(hipStream_t st, int o, int v, Planes4<T> P, void* out, double scale, int nb = 1);
// P = y + sum_j cs[j] ks[j] (nk <= 8 FP64 states of nb members; terms with cs[j] == 0 skipped), one pass.
template <typename T>
void combo_unpack(hipStream_t st, int o, int v, int nb, const void* y, int nk, const void* const* ks, const double* cs,
                  Planes4<T> P);
template <typename T>
void field_fock(hipStream_t st, int n, const double* f0, const double* mu, const double E[3], double s0, T* f);
// Field on the device: the rtcc_field kinds (0 none, 1 Gaussian pulse, 2 kick = none while
// stepping) and kFieldConstant, the constant field vector n (E0 and the pulse shape unused).
constexpr int kFieldConstant = 3;
struct FieldDev {
  int kind;
  double E0, omega, sigma, t0, n[3];
};
template <typename T>
void field_fock_t(hipStream_t st, int n, const double* f0, const double* mu, const FieldDev& fd, const double* tdev,
                  double toff, T* f);
// Batched: member b uses fds[b] (DEVICE) and writes f + b * fbs.
template <typename T>
void field_fock_tb(hipStream_t st, int n, const double* f0, const double* mu, const FieldDev* fds, int nb,
                   const double* tdev, double toff, T* f, int64_t fbs);
// dev[0..n) = host[0..n), enqueued as kernel arguments (the host array may change right after the call).
void upload_fields(hipStream_t st, const FieldDev* host, int n, FieldDev* dev);
// out[6 b + 2 a + (0, 1)] = (Re, Im) of mu_ref[a] + sum_pq rho_b[pq] mu_a[pq] for every member b;
// rho_b at rho_re / rho_im + b * rbs (n*n entries). Fixed summation order.
void dipole_batch(hipStream_t st, int nb, int64_t nn, const double* rho_re, const double* rho_im, int64_t rbs,
                  const double* mu, const double* mu_ref, double* out);
void scalar_update(hipStream_t st, double* p, double v, bool add);
void state_combo(hipStream_t st, int64_t n, const void* y, int nk, const void* const* ks, const double* cs, void* out);
template <typename T>
void dot_planar_real(hipStream_t st, int64_t n, const T* are, const T* aim, const double* b, double* partial,
                     double* out2);
void max_abs_diff(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2);
void vdot(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2);
void count_nonfinite(hipStream_t st, int64_t n, const void* a, double* partial, double* out2);
// Symmetric / antisymmetric ladder (ladder.hip). nblk blocks of o*o*v*v consecutive entries X[blk][i][j][e][f]
// (pair-symmetric: X_ji^fe = X_ij^ef) -> X+ rows (blk, i <= j) x (e <= f) and X- rows (blk, i < j) x (e < f);
// back: Z[blk][i][j][a][b] = S+(pairs) +- S-(pairs) over the full square. Row-major upper-triangle pair order.
// lds: stage one (i, j) plane per workgroup through LDS (v <= 96; otherwise, or with lds = false, element
// kernels that read the transposed entries from global memory).
template <typename T>
void ladder_fold(hipStream_t st, int nblk, int o, int v, const T* xre, const T* xim, T* pre, T* pim, T* mre, T* mim,
                 bool lds = true);
template <typename T>
void ladder_unfold(hipStream_t st, int nblk, int o, int v, const T* sre, const T* sim, const T* are, const T* aim,
                   T* zre, T* zim, bool lds = true);
// V+ (v(v+1)/2 square) and V- (v(v-1)/2 square) from <ab|ef> as the v^2 x v^2 matrix [(ab)][(ef)].
void ladder_sym_build(hipStream_t st, int v, const double* vvvv, double* vp, double* vm);

// Largest number of reduction blocks of state_guard (it needs 2 * kGuardBlocks partial doubles).
constexpr int kGuardBlocks = 512;
// out2[0] = Frobenius norm of the entries [t2b, t2e) of the interleaved complex vector y (NaN if any of
// its nst entries is non-finite), out2[1] = number of non-finite entries. Fixed summation order.
void state_guard(hipStream_t st, int64_t nst, int64_t t2b, int64_t t2e, const void* y, double* partial,
                 double* out2);
// Adjoint helpers (interleaved complex states of o, v): see elementwise.hip.
void hamil_apply(hipStream_t st, int o, int v, const void* a, const void* b, const double cb[2], bool inverse,
                 bool conj_in, bool conj_out, double scale, bool accumulate, void* out);
void circle_points(hipStream_t st, int64_t nst, const void* y, const void* u, const double* maxu, double rho, int m,
                   void* out);
void circle_coef1(hipStream_t st, int64_t nst, const void* F, const double* maxu, double rho, int m, void* out);
void max_abs(hipStream_t st, int64_t n, const void* a, double* partial, double* out2);
template <typename T>
void jacobi_update(hipStream_t st, int o, int v, const double* fdiag, const T* r1, const T* r2, void* x1, void* x2,
                   void* e1, void* e2);
template <typename T>
void maxabs_planar(hipStream_t st, int64_t n, const T* re, const T* im, double* partial, double* out2);

// W = (Bd + Pd / 2 | Bx + Px / 2) transposed into [q][2][p], H = (Bd + Pd, Bx + Px) interleaved into [p][q][2]
// (H skipped when hre is null); x = {Bd, Pd, Bx, Px} as (re, im) pairs, each [p][q] contiguous.
template <typename T>
void ring_combo(hipStream_t st, int64_t P, int64_t Q, int nb, const T* const x[8], int64_t xbs, T* wre, T* wim,
                int64_t wbs, T* hre, T* him, int64_t hbs);
// tau = t2 + t1 t1, taut = t2 + t1 t1 / 2, t2s = 2 t2 - t2[ijba], l2s = 2 l2 - l2[ijba] (l2 may be null),
// planar (re, im) pointer pairs; t1 at batch stride bs1, the doubles (t2, l2, tau, taut, t2s, l2s) at bs[k].
// Optionally (non-null) also the stacked copies stk_t[i][a][s][j][b] = (t2s, t2)[s] and
// stk_l[i][a][j][b][s] = (l2s, l2)[s] at batch strides sbs_t, sbs_l.
template <typename T>
void amp_combo(hipStream_t st, int o, int v, int nb, const T* const t1[2], int64_t bs1, const T* const t2[2],
               const T* const l2[2], const int64_t bs[6], T* const tau[2], T* const taut[2], T* const t2s[2],
               T* const l2s[2], T* const stk_t[2], int64_t sbs_t, T* const stk_l[2], int64_t sbs_l);
// out[ijab] += base[ijab] + lad[ijab] + z[ijab] + zt[iajb] + z[jiba] + zt[jbia]: planar (re, im) pointer
// pairs, base (shared by all members; either plane may be null) [o][o][v][v], lad and z [o][o][v][v], zt
// [o][v][o][v], each at its own batch stride.
template <typename T>
void pair_combo(hipStream_t st, int o, int v, int nb, T* const out[2], int64_t obs, const T* const base[2],
                const T* const lad[2], int64_t lbs, const T* const z[2], int64_t zbs, const T* const zt[2],
                int64_t tbs);
}  // namespace rtcc
