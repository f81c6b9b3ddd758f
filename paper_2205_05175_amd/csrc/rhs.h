// Closed-shell RT-CCSD right-hand side: integral blocks, workspace and the contraction list.
#pragma once
#include <vector>

#include "elementwise.h"
#include "engine.h"

namespace rtcc {

// Device arena for long-lived tensors of one context.
struct Arena {
  std::vector<void*> blocks;
  int nb = 1;  // members per tensor allocated by real() / cplx() (batch stride = one member)
  ~Arena() { release(); }
  void release() {
    for (void* p : blocks) (void)hipFree(p);
    blocks.clear();
  }
  template <typename T>
  T* alloc(int64_t n) {
    void* p = nullptr;
    size_t bytes = std::max<int64_t>(n, 1) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) throw Error(kENoMem, "device allocation failed");
    blocks.push_back(p);
    return (T*)p;
  }
  template <typename T>
  Ten<T> real(std::initializer_list<int64_t> dims) {
    int64_t n = 1;
    for (auto d : dims) n *= d;
    Ten<T> t = make_ten<T>(alloc<T>(nb * n), nullptr, dims);
    t.bs = nb > 1 ? n : 0;
    return t;
  }
  // planar complex: all real planes of the batch, then all imaginary planes
  template <typename T>
  Ten<T> cplx(std::initializer_list<int64_t> dims) {
    int64_t n = 1;
    for (auto d : dims) n *= d;
    T* p = alloc<T>(2 * nb * n);
    Ten<T> t = make_ten<T>(p, p + nb * n, dims);
    t.bs = nb > 1 ? n : 0;
    return t;
  }
};

// Physicists' integral blocks <pq|rs> = (pr|qs) and the combinations L_pqrs = 2<pq|rs> - <pq|sr>.
template <typename T>
struct Ints {
  Ten<T> oooo, ooov, oovv, ovov, ovvo, ovvv, vvvv, Loovv, Looov, Lovvv, Lovvo;
  Ten<T> vvp, vvm;  // symmetric / antisymmetric ladder integrals over the (e <= f) and (e < f) pairs
};

template <typename T>
struct Work {
  int o = 0, v = 0, n = 0;
  Ten<T> f, fov, foo, fvv;                         // field-dressed Fock matrix (real) and blocks
  Ten<T> t1, l1, t2, X, tau, l2, taut, t2s, l2s;    // amplitudes; X = [tau; l2] (ladder operand)
  Ten<T> Fae, Fmi, Fme, Hvv, Hoo, Gvv, Goo, Q, Gx;  // one-body
  Ten<T> W, M, Mp, Hooov, Z1, Y, U, U2, Y3, Y3B, Y3C, Y6, B4, B5, B7, D, Nn, Xin, Qnf;
  Ten<T> Lad, LadT, LadL;
  Ten<T> Xp, Xm, Sp, Sm;                           // symmetric / antisymmetric ladder operands and products
  Ten<T> Pd, Px, Bd, Bx, WW, Wd, Wx, HH, HHd, HHx, HH5, T2R, L2R, Zt, ZLt, B2, B3, Wr, WrB, WrC;
  Ten<T> Z, ZL, S1t;                               // (1+P) brackets; t1-t1 ring piece
  Ten<T> R1, R2, S1, S2;                           // residuals: R_T (T1,T2), R_L (L1,L2)
  Ten<T> S1b, S1c, Wr2, Wr2B, Wr2C;                // partial Lambda1 sums of the concurrent groups
  Ten<T> rho, Dvv, Doo, P1;                        // one-particle density
};

template <typename T>
void build_ints(Engine& E, Arena& A, int o, int v, const double* eri_dev, Ints<T>& I);
// Workspace for nb members (nb > 1: every tensor batched, see Engine::nb).
template <typename T>
void build_work(Arena& A, int o, int v, Work<T>& w, int nb = 1);
// Residuals at the amplitudes held in w (t1, t2, l1, l2) and the Fock matrix w.f.
// twobody=false evaluates the residuals of the one-body operator w.f alone.
template <typename T>
void residuals(Engine& E, const Ints<T>& I, Work<T>& w, bool twobody, bool lambda);
// rho such that mu_a = mu_ref_a + sum_pq rho_pq mu_a,pq
template <typename T>
void density(Engine& E, Work<T>& w);

}  // namespace rtcc
