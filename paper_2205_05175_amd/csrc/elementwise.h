// Declarations of the memory-bound kernels (state layout, RK combinations, reductions).
#pragma once
#include "engine.h"

namespace rtcc {

template <typename T>
struct Planes4 {
  T* re[4];
  T* im[4];
};
template <typename T>
void unpack_state(hipStream_t st, const void* y, int o, int v, Planes4<T> P);
template <typename T>
void pack_rhs(hipStream_t st, int o, int v, Planes4<T> P, void* out, double scale);
template <typename T>
void field_fock(hipStream_t st, int n, const double* f0, const double* mu, const double E[3], double s0, T* f);
struct FieldDev {
  int kind;
  double E0, omega, sigma, t0, n[3];
};
template <typename T>
void field_fock_t(hipStream_t st, int n, const double* f0, const double* mu, const FieldDev& fd, const double* tdev,
                  double toff, T* f);
void scalar_update(hipStream_t st, double* p, double v, bool add);
void state_combo(hipStream_t st, int64_t n, const void* y, int nk, const void* const* ks, const double* cs, void* out);
template <typename T>
void dot_planar_real(hipStream_t st, int64_t n, const T* are, const T* aim, const double* b, double* partial,
                     double* out2);
void max_abs_diff(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2);
void vdot(hipStream_t st, int64_t n, const void* a, const void* b, double* partial, double* out2);
void count_nonfinite(hipStream_t st, int64_t n, const void* a, double* partial, double* out2);
template <typename T>
void jacobi_update(hipStream_t st, int o, int v, const double* fdiag, const T* r1, const T* r2, void* x1, void* x2,
                   void* e1, void* e2);
template <typename T>
void maxabs_planar(hipStream_t st, int64_t n, const T* re, const T* im, double* partial, double* out2);

}  // namespace rtcc
