// Closed-shell (spin-adapted) RT-CCSD right-hand side.
//
// Residuals of the paper's equations of motion (Theory: Eq. derivT for the cluster
// amplitudes, Eq. derivL for Lambda, Hbar of Eq. simtranH) in closed-shell variables
// t_i^a = t_{ia,aa}, t_ij^ab = t_{i alpha j beta}^{a alpha b beta} (Lambda mapped the same
// way), for a general (field-dressed, non-canonical) Fock matrix and a non-stationary state.
// The factorisation keeps every contraction at o^3 v^3 or below except the particle-particle
// ladder sum_ef <ab|ef> X_ij^ef, which is one real-by-complex GEMM over the stacked operand
// X = [tau; lambda2] shared by the T2 and Lambda2 equations. Hbar_abef and Hbar_abei are
// never formed: their t1 and tau dressings are contracted with tau or lambda first.
#include "rhs.h"

namespace rtcc {

namespace {

template <typename T>
Ten<T> view(const Ten<T>& base, int64_t off, std::initializer_list<int64_t> dims, std::initializer_list<int64_t> strides) {
  Ten<T> t;
  t.re = base.re + off;
  t.im = base.im ? base.im + off : nullptr;
  t.nd = (int)dims.size();
  int i = 0;
  for (auto d : dims) t.d[i++] = d;
  i = 0;
  for (auto s : strides) t.s[i++] = s;
  t.bs = base.bs;
  return t;
}

// block[p,q,r,s] = <pq|rs> = (pr|qs) from the chemists'-order n^4 array
template <typename T>
void extract(Engine& E, const double* eri, int n, int p0, int q0, int r0, int s0, const Ten<double>& out) {
  int64_t nn = n;
  const double* base = eri + (int64_t)p0 * nn * nn * nn + (int64_t)r0 * nn * nn + (int64_t)q0 * nn + s0;
  int64_t is[4] = {nn * nn * nn, nn, nn * nn, 1};
  permute_axpby<double>(E.stream, 4, out.d, base, nullptr, is, out.re, nullptr, out.s, 1.0, 0.0);
}

template <typename T>
void mark_constant(Ints<T>& I) {
  for (Ten<T>* t : {&I.oooo, &I.ooov, &I.oovv, &I.ovov, &I.ovvo, &I.ovvv, &I.vvvv, &I.Loovv, &I.Looov, &I.Lovvv,
                    &I.Lovvo, &I.vvp, &I.vvm})
    t->konst = true;
}

__global__ void convert_kernel(int64_t n, const double* in, float* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

}  // namespace

template <typename T>
void build_ints(Engine& E, Arena& A, int o, int v, const double* eri, Ints<T>& I);

template <>
void build_ints<double>(Engine& E, Arena& A, int o, int v, const double* eri, Ints<double>& I) {
  const int n = o + v;
  I.oooo = A.real<double>({o, o, o, o});
  I.ooov = A.real<double>({o, o, o, v});
  I.oovv = A.real<double>({o, o, v, v});
  I.ovov = A.real<double>({o, v, o, v});
  I.ovvo = A.real<double>({o, v, v, o});
  I.ovvv = A.real<double>({o, v, v, v});
  I.vvvv = A.real<double>({v, v, v, v});
  extract<double>(E, eri, n, 0, 0, 0, 0, I.oooo);
  extract<double>(E, eri, n, 0, 0, 0, o, I.ooov);
  extract<double>(E, eri, n, 0, 0, o, o, I.oovv);
  extract<double>(E, eri, n, 0, o, 0, o, I.ovov);
  extract<double>(E, eri, n, 0, o, o, 0, I.ovvo);
  extract<double>(E, eri, n, 0, o, o, o, I.ovvv);
  extract<double>(E, eri, n, o, o, o, o, I.vvvv);
  const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
  I.vvp = A.real<double>({pv, pv});
  I.vvm = A.real<double>({mv, mv});
  ladder_sym_build(E.stream, v, I.vvvv.re, I.vvp.re, I.vvm.re);
  I.Loovv = A.real<double>({o, o, v, v});
  I.Looov = A.real<double>({o, o, o, v});
  I.Lovvv = A.real<double>({o, v, v, v});
  I.Lovvo = A.real<double>({o, v, v, o});
  padd<double>(E, 2.0, "mnef->mnef", I.oovv, I.Loovv, 0.0);
  padd<double>(E, -1.0, "mnfe->mnef", I.oovv, I.Loovv, 1.0);
  padd<double>(E, 2.0, "mnie->mnie", I.ooov, I.Looov, 0.0);
  padd<double>(E, -1.0, "nmie->mnie", I.ooov, I.Looov, 1.0);
  padd<double>(E, 2.0, "maef->maef", I.ovvv, I.Lovvv, 0.0);
  padd<double>(E, -1.0, "mafe->maef", I.ovvv, I.Lovvv, 1.0);
  padd<double>(E, 2.0, "nafi->nafi", I.ovvo, I.Lovvo, 0.0);
  padd<double>(E, -1.0, "naif->nafi", I.ovov, I.Lovvo, 1.0);
  mark_constant(I);
}

template <>
void build_ints<float>(Engine& E, Arena& A, int o, int v, const double* eri, Ints<float>& I) {
  Arena tmp;
  Ints<double> D;
  build_ints<double>(E, tmp, o, v, eri, D);
  auto cvt = [&](const Ten<double>& src) {
    Ten<float> t = make_ten<float>(A.alloc<float>(src.size()), nullptr, {});
    t.nd = src.nd;
    for (int i = 0; i < src.nd; ++i) {
      t.d[i] = src.d[i];
      t.s[i] = src.s[i];
    }
    int64_t nel = src.size();
    if (nel == 0) return t;  // e.g. the antisymmetric ladder block at v = 1
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)std::min<int64_t>(cdiv(nel, 256), 65536)), dim3(256), 0,
                       E.stream, nel, src.re, t.re);
    RTCC_HIP(hipGetLastError());
    return t;
  };
  I.oooo = cvt(D.oooo);
  I.ooov = cvt(D.ooov);
  I.oovv = cvt(D.oovv);
  I.ovov = cvt(D.ovov);
  I.ovvo = cvt(D.ovvo);
  I.ovvv = cvt(D.ovvv);
  I.vvvv = cvt(D.vvvv);
  I.vvp = cvt(D.vvp);
  I.vvm = cvt(D.vvm);
  I.Loovv = cvt(D.Loovv);
  I.Looov = cvt(D.Looov);
  I.Lovvv = cvt(D.Lovvv);
  I.Lovvo = cvt(D.Lovvo);
  mark_constant(I);
  RTCC_HIP(hipStreamSynchronize(E.stream));  // tmp is freed on return
}

template <typename T>
void build_work(Arena& A, int o, int v, Work<T>& w, int nb) {
  const int64_t n = o + v, ov = (int64_t)o * v, oovv = ov * ov;
  struct Restore {
    Arena& a;
    ~Restore() { a.nb = 1; }
  } restore{A};
  A.nb = nb;
  w.o = o;
  w.v = v;
  w.n = (int)n;
  w.f = A.real<T>({n, n});
  w.fov = view(w.f, o, {o, v}, {n, 1});
  w.foo = view(w.f, 0, {o, o}, {n, 1});
  w.fvv = view(w.f, o * n + o, {v, v}, {n, 1});
  w.t1 = A.cplx<T>({o, v});
  w.l1 = A.cplx<T>({o, v});
  w.t2 = A.cplx<T>({o, o, v, v});
  w.X = A.cplx<T>({2, o, o, v, v});
  w.tau = view(w.X, 0, {o, o, v, v}, {o * v * v, v * v, v, 1});
  w.l2 = view(w.X, oovv, {o, o, v, v}, {o * v * v, v * v, v, 1});
  w.taut = A.cplx<T>({o, o, v, v});
  w.t2s = A.cplx<T>({o, o, v, v});
  w.l2s = A.cplx<T>({o, o, v, v});
  w.Fae = A.cplx<T>({v, v});
  w.Fmi = A.cplx<T>({o, o});
  w.Fme = A.cplx<T>({o, v});
  w.Hvv = A.cplx<T>({v, v});
  w.Hoo = A.cplx<T>({o, o});
  w.Gvv = A.cplx<T>({v, v});
  w.Goo = A.cplx<T>({o, o});
  w.Q = A.cplx<T>({o, o});
  w.Gx = A.cplx<T>({v, v});
  w.W = A.cplx<T>({o, o, o, o});
  w.M = A.cplx<T>({o, o, o, o});
  w.Mp = A.cplx<T>({o, o, o, o});
  w.Hooov = A.cplx<T>({o, o, o, v});
  w.Xin = A.cplx<T>({o, o});
  w.Qnf = A.cplx<T>({o, v});
  w.Z1 = A.cplx<T>({o, o, v, o});
  w.Y = A.cplx<T>({o, o, v, o});
  w.U = A.cplx<T>({o, o, v, o});
  w.U2 = A.cplx<T>({o, o, o, v});
  w.Y3 = A.cplx<T>({o, o, o, v});
  w.Y3B = A.cplx<T>({o, o, o, v});
  w.Y3C = A.cplx<T>({o, o, o, v});
  w.Y6 = A.cplx<T>({o, o, v, o});
  w.B4 = A.cplx<T>({o, o, v, o});
  w.B5 = A.cplx<T>({o, o, o, v});
  w.B7 = A.cplx<T>({o, o, v, o});
  w.D = A.cplx<T>({o, o, v, o});
  w.Nn = A.cplx<T>({o, o, o, v});
  w.Lad = A.cplx<T>({2, o, o, v, v});
  w.LadT = view(w.Lad, 0, {o, o, v, v}, {o * v * v, v * v, v, 1});
  w.LadL = view(w.Lad, oovv, {o, o, v, v}, {o * v * v, v * v, v, 1});
  {
    const int64_t po = (int64_t)o * (o + 1) / 2, pm = (int64_t)o * (o - 1) / 2;
    const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
    w.Xp = A.cplx<T>({2, po, pv});
    w.Sp = A.cplx<T>({2, po, pv});
    w.Xm = A.cplx<T>({2, std::max<int64_t>(pm, 1), std::max<int64_t>(mv, 1)});
    w.Sm = A.cplx<T>({2, std::max<int64_t>(pm, 1), std::max<int64_t>(mv, 1)});
  }
  // ring intermediates, element X_mbej stored at (m,e,j,b)
  w.Pd = A.cplx<T>({o, v, o, v});
  w.Px = A.cplx<T>({o, v, o, v});
  w.Bd = A.cplx<T>({o, v, o, v});
  w.Bx = A.cplx<T>({o, v, o, v});
  // W_mbej (s=0 direct, s=1 exchange) stored at (j,b,s,m,e): the T ring GEMM reads it as [n][k]
  w.WW = A.cplx<T>({o, v, 2, o, v});
  w.Wd = view(w.WW, 0, {o, v, o, v}, {v, 1, 2 * ov * v, 2 * ov});
  w.Wx = view(w.WW, ov, {o, v, o, v}, {v, 1, 2 * ov * v, 2 * ov});
  // Hbar_mbej (s=0 direct, s=1 exchange) stored at (m,e,j,b,s): the Lambda ring GEMM reads it as [n][k]
  w.HH = A.cplx<T>({o, v, o, v, 2});
  w.HH5 = w.HH;
  w.HHd = view(w.HH, 0, {o, v, o, v}, {2 * ov * v, 2 * ov, 2 * v, 2});
  w.HHx = view(w.HH, 1, {o, v, o, v}, {2 * ov * v, 2 * ov, 2 * v, 2});
  // stacked left operands of the ring GEMMs: (i,a,s,m,e) for T and (i,a,m,e,s) for Lambda
  w.T2R = A.cplx<T>({o, v, 2, o, v});
  w.L2R = A.cplx<T>({o, v, o, v, 2});
  w.Zt = A.cplx<T>({o, v, o, v});
  w.ZLt = A.cplx<T>({o, v, o, v});
  w.B2 = A.cplx<T>({o, v, o, v});
  w.B3 = A.cplx<T>({o, v, o, v});
  // the three l2s x t2 intermediates of each of the two Lambda1 groups, formed together
  w.Wr = A.cplx<T>({o, v, o, v});
  w.WrB = A.cplx<T>({o, v, o, v});
  w.WrC = A.cplx<T>({o, v, o, v});
  w.Z = A.cplx<T>({o, o, v, v});
  w.S1t = A.cplx<T>({o, v, o, o});
  w.ZL = A.cplx<T>({o, o, v, v});
  w.R1 = A.cplx<T>({o, v});
  w.R2 = A.cplx<T>({o, o, v, v});
  w.S1 = A.cplx<T>({o, v});
  w.S1b = A.cplx<T>({o, v});
  w.S1c = A.cplx<T>({o, v});
  w.Wr2 = A.cplx<T>({v, o, o, v});
  w.Wr2B = A.cplx<T>({v, o, o, v});
  w.Wr2C = A.cplx<T>({v, o, o, v});
  w.S2 = A.cplx<T>({o, o, v, v});
  w.rho = A.cplx<T>({n, n});
  w.Dvv = A.cplx<T>({v, v});
  w.Doo = A.cplx<T>({o, o});
  w.P1 = A.cplx<T>({o, o});
}

// out += base + lad + z + zt[iajb] + (z + zt[iajb])[jiba] over [o][o][v][v] (zt stored [o][v][o][v])
template <typename T>
void pair_add(Engine& E, const Ten<T>& base, const Ten<T>& lad, const Ten<T>& z, const Ten<T>& zt, const Ten<T>& out) {
  const int o = (int)out.d[0], v = (int)out.d[2];
  auto dense = [&](const Ten<T>& x, int64_t d0, int64_t d1, int64_t d2, int64_t d3) {
    return x.nd == 4 && x.d[0] == d0 && x.d[1] == d1 && x.d[2] == d2 && x.d[3] == d3 && x.s[3] == 1 &&
           x.s[2] == d3 && x.s[1] == d2 * d3 && x.s[0] == d1 * d2 * d3;
  };
  RTCC_CHECK(dense(out, o, o, v, v) && dense(base, o, o, v, v) && dense(lad, o, o, v, v) && dense(z, o, o, v, v) &&
                 dense(zt, o, v, o, v) && out.im && lad.im && z.im && zt.im && base.bs == 0 && (E.nb == 1 || out.bs != 0),
             kEInval, "pair_add: unexpected layout");
  if (E.trace) fprintf(stderr, "[rtcc] pair_add\n");
  T* const op[2] = {out.re, out.im};
  const T* const bp[2] = {base.re, base.im};
  const T* const lp[2] = {lad.re, lad.im};
  const T* const zp[2] = {z.re, z.im};
  const T* const tp[2] = {zt.re, zt.im};
  pair_combo<T>(E.stream, o, v, E.nb, op, out.bs, bp, lp, lad.bs, zp, z.bs, tp, zt.bs);
}

template <typename T>
void residuals(Engine& E, const Ints<T>& I, Work<T>& w, bool tb, bool lambda) {
  // Contractions go to engine `cur`. With branch engines, independent parts (which share only
  // intermediates finished before their fork, and each write their own outputs and temporaries)
  // run concurrently on three streams, in two fork/join sections.
  Engine* cur = &E;
  auto C = [&](double a, const char* s, const Ten<T>& x, const Ten<T>& y, const Ten<T>& z, double b) {
    ein<T>(*cur, a, s, x, y, z, b);
  };
  auto P = [&](double a, const char* s, const Ten<T>& x, const Ten<T>& z, double b) {
    padd<T>(*cur, a, s, x, z, b);
  };
  const bool par = tb && lambda && E.br[0] && E.br[1];
  if (E.trace)
    fprintf(stderr, "[rtcc] tensors t1=%p t2=%p l1=%p l2=%p tau=%p taut=%p t2s=%p l2s=%p W=%p Hooov=%p\n",
            (void*)w.t1.re, (void*)w.t2.re, (void*)w.l1.re, (void*)w.l2.re, (void*)w.tau.re, (void*)w.taut.re,
            (void*)w.t2s.re, (void*)w.l2s.re, (void*)w.W.re, (void*)w.Hooov.re);
  const int o = w.o, v = w.v;
  const Ten<T>&t1 = w.t1, &t2 = w.t2, &l1 = w.l1, &l2 = w.l2, &tau = w.tau;

  // ---- amplitude combinations: tau = t2 + t1 t1, taut = t2 + t1 t1 / 2, t2s = 2 t2 - t2[ijba] and
  // l2s = 2 l2 - l2[ijba], one pass over t2 and l2
  {
    const T* a1[2] = {t1.re, t1.im};
    const T* a2[2] = {t2.re, t2.im};
    const T* b2[2] = {l2.re, l2.im};
    T* o_tau[2] = {tau.re, tau.im};
    T* o_taut[2] = {w.taut.re, w.taut.im};
    T* o_t2s[2] = {w.t2s.re, w.t2s.im};
    T* o_l2s[2] = {w.l2s.re, w.l2s.im};
    const int64_t bs[6] = {t2.bs, l2.bs, tau.bs, w.taut.bs, w.t2s.bs, w.l2s.bs};
    // with the t1 terms, also the stacked left operands of the ring products
    T* o_tr[2] = {w.T2R.re, w.T2R.im};
    T* o_lr[2] = {w.L2R.re, w.L2R.im};
    amp_combo<T>(E.stream, o, v, E.nb, a1, t1.bs, a2, lambda ? b2 : nullptr, bs, o_tau, o_taut, o_t2s, o_l2s,
                 tb ? o_tr : nullptr, w.T2R.bs, (tb && lambda) ? o_lr : nullptr, w.L2R.bs);
  }
  // the amplitudes and their combinations are fixed from here on: derived layouts of them are kept
  // (per engine) for the rest of this call
  struct MemoScope {
    Engine* e[3];
    ~MemoScope() {
      for (Engine* x : e)
        if (x) memo_end(*x);
    }
  } memo_scope{{&E, par ? E.br[0] : nullptr, par ? E.br[1] : nullptr}};
  for (Engine* x : memo_scope.e)
    if (x) memo_begin(*x, {t1.re, t2.re, l1.re, l2.re, tau.re, w.taut.re, w.t2s.re, w.l2s.re});

  // Concurrent part 1 (with branch engines): the main engine builds the one-body intermediates,
  // the T1 residual, W, Hbar_mnie and the Hbar_mnie-free parts of the ring intermediates; branch 0
  // the ladder and Z1; branch 1 the t2-integral ring pieces and the Lambda intermediates G, U. Then
  // the main engine completes the ring intermediates (the Hbar_mnie terms and the combinations) and
  // part 2 forks the residuals. Hbar_amef is never formed: its uses take <ma|fe> and the t1 term
  // separately.
  if (par) fork_branches(E);

  // ---- one-body intermediates
  P(1, "ae->ae", w.fvv, w.Fae, 0);
  C(-0.5, "me,ma->ae", w.fov, t1, w.Fae, 1);
  P(1, "mi->mi", w.foo, w.Fmi, 0);
  C(0.5, "ie,me->mi", t1, w.fov, w.Fmi, 1);
  P(1, "me->me", w.fov, w.Fme, 0);
  if (tb) {
    C(1, "mf,mafe->ae", t1, I.Lovvv, w.Fae, 1);
    C(-1, "mnaf,mnef->ae", w.taut, I.Loovv, w.Fae, 1);
    C(1, "ne,mnie->mi", t1, I.Looov, w.Fmi, 1);
    C(1, "inef,mnef->mi", w.taut, I.Loovv, w.Fmi, 1);
    C(1, "nf,mnef->me", t1, I.Loovv, w.Fme, 1);
  }
  P(1, "ae->ae", w.Fae, w.Hvv, 0);
  C(-0.5, "ma,me->ae", t1, w.Fme, w.Hvv, 1);
  P(1, "mi->mi", w.Fmi, w.Hoo, 0);
  C(0.5, "ie,me->mi", t1, w.Fme, w.Hoo, 1);

  // ---- T1 residual
  P(1, "ia->ia", w.fov, w.R1, 0);
  C(1, "ie,ae->ia", t1, w.Fae, w.R1, 1);
  C(-1, "ma,mi->ia", t1, w.Fmi, w.R1, 1);
  C(1, "imae,me->ia", w.t2s, w.Fme, w.R1, 1);
  if (tb) {
    C(1, "nf,nafi->ia", t1, I.Lovvo, w.R1, 1);
    C(1, "imef,mafe->ia", t2, I.Lovvv, w.R1, 1);
    C(-1, "mnae,mnie->ia", t2, I.Looov, w.R1, 1);
  }

  // ---- two-electron intermediates
  if (tb) {
    P(1, "mnij->mnij", I.oooo, w.W, 0);
    C(1, "je,mnie->mnij", t1, I.ooov, w.W, 1);
    C(1, "ie,nmje->mnij", t1, I.ooov, w.W, 1);
    C(1, "ijef,mnef->mnij", tau, I.oovv, w.W, 1);
    P(1, "mnie->mnie", I.ooov, w.Hooov, 0);
    C(1, "if,mnfe->mnie", t1, I.oovv, w.Hooov, 1);
    // the parts of the ring intermediates that do not need Hbar_mnie
    P(1, "mbej->mejb", I.ovvo, w.Bd, 0);
    C(1, "jf,mbef->mejb", t1, I.ovvv, w.Bd, 1);
    P(-1, "mbje->mejb", I.ovov, w.Bx, 0);
    C(-1, "jf,mbfe->mejb", t1, I.ovvv, w.Bx, 1);

    if (par) cur = E.br[0];
    // particle-particle ladder: one GEMM over the stacked [tau; lambda2] rows, or the two GEMMs of its
    // symmetric / antisymmetric form over the pair triangles (a quarter of the flops)
    const int nblk = E.nb * (lambda || E.nb > 1 ? 2 : 1);
    if (E.sym_ladder) {
      const int64_t vv = (int64_t)v * v;
      RTCC_CHECK(E.nb == 1 || (w.X.bs == 2 * (int64_t)o * o * vv && w.Lad.bs == w.X.bs &&
                               w.Xp.bs == 2 * w.Xp.d[1] * w.Xp.d[2] && w.Xm.bs == 2 * w.Xm.d[1] * w.Xm.d[2] &&
                               w.Sp.bs == w.Xp.bs && w.Sm.bs == w.Xm.bs),
                 kEInval, "ladder operands are not member-contiguous");
      const int64_t po = (int64_t)o * (o + 1) / 2, pm = (int64_t)o * (o - 1) / 2;
      const int64_t pv = (int64_t)v * (v + 1) / 2, mv = (int64_t)v * (v - 1) / 2;
      ladder_fold<T>(cur->stream, nblk, o, v, w.X.re, w.X.im, w.Xp.re, w.Xp.im, w.Xm.re, w.Xm.im, E.ladder_lds);
      const bool split16 = sizeof(T) == 4 && cur->bf16x3;
      const int64_t rows_[2] = {nblk * po, nblk * pm}, kn[2] = {pv, mv};
      const Ten<T>* ops[2][3] = {{&w.Xp, &I.vvp, &w.Sp}, {&w.Xm, &I.vvm, &w.Sm}};
      bool paired = false;
      if constexpr (sizeof(T) == 4) {
        // split-BF16: both GEMMs in one launch when both qualify for the split kernel and the tuning
        // table holds no choice of its own for either
        bool ok = split16 && cur->pair_splits >= 0 && rows_[1] > 0 && kn[1] > 0;
        for (int h = 0; h < 2 && ok; ++h)
          ok = 2.0 * (double)rows_[h] * (double)kn[h] * (double)kn[h] >= cur->bf16_min_flops &&
               (!cur->use_tuning || tuned_choice(2, rows_[h], kn[h], kn[h], true, false, 0, 1).kind == 0);
        if (ok) {
          Bf16Job jobs[2];
          for (int h = 0; h < 2; ++h)
            jobs[h] = Bf16Job{rows_[h], kn[h], kn[h], 1.0, GemmOp<float>{ops[h][0]->re, ops[h][0]->im, kn[h], 0},
                              GemmOp<float>{ops[h][1]->re, nullptr, kn[h], 1, true}, ops[h][2]->re, ops[h][2]->im,
                              kn[h], 0.0};
          E.ladder_flops = 4.0 * (double)(rows_[0] * kn[0] * kn[0] + rows_[1] * kn[1] * kn[1]);
          cur->ladder_flops = E.ladder_flops;
          cur->ladder = 1;
          if (E.trace) fprintf(stderr, "[rtcc] ladder X+V+ and X-V- paired\n");
          paired = gemm_bf16x3_pair(*cur, jobs);
          cur->ladder = 0;
        }
      }
      for (int h = 0; h < 2 && !paired; ++h) {
        if (rows_[h] == 0 || kn[h] == 0) continue;
        GemmOp<T> a{ops[h][0]->re, ops[h][0]->im, kn[h], 0};
        GemmOp<T> b{ops[h][1]->re, nullptr, kn[h], 1, true};  // V+- are symmetric matrices
        E.ladder_flops = 4.0 * (double)rows_[h] * (double)kn[h] * (double)kn[h];
        cur->ladder_flops = E.ladder_flops;
        if (E.trace) fprintf(stderr, "[rtcc] ladder %s M=%lld N=K=%lld\n", h ? "X-V-" : "X+V+", (long long)rows_[h],
                             (long long)kn[h]);
        cur->ladder = 1;
        gemm<T>(*cur, rows_[h], kn[h], kn[h], 1.0, a, b, ops[h][2]->re, ops[h][2]->im, kn[h], 0.0);
        cur->ladder = 0;
      }
      ladder_unfold<T>(cur->stream, nblk, o, v, w.Sp.re, w.Sp.im, w.Sm.re, w.Sm.im, w.Lad.re, w.Lad.im,
                       E.ladder_lds);
    } else {
      // batched: the members' [tau; lambda2] blocks are consecutive rows of one operand
      const int64_t rows = nblk * (int64_t)o * o, vv = (int64_t)v * v;
      RTCC_CHECK(E.nb == 1 || w.X.bs == 2 * (int64_t)o * o * vv, kEInval, "ladder operand is not member-contiguous");
      GemmOp<T> a{w.X.re, w.X.im, vv, 0};
      GemmOp<T> b{I.vvvv.re, nullptr, vv, 1, true};  // B(ef, ab) = <ab|ef> = <ef|ab>: V is symmetric
      E.ladder_flops = 4.0 * (double)rows * (double)vv * (double)vv;  // real x complex: 2 MACs per entry
      cur->ladder_flops = E.ladder_flops;
      if (E.trace) fprintf(stderr, "[rtcc] ladder full M=%lld N=K=%lld\n", (long long)rows, (long long)vv);
      cur->ladder = 1;
      gemm<T>(*cur, rows, vv, vv, 1.0, a, b, w.Lad.re, w.Lad.im, vv, 0.0);
      cur->ladder = 0;
    }
    C(1, "ijef,mafe->ijam", tau, I.ovvv, w.Z1, 0);

    // ring intermediates (element X_mbej at (m,e,j,b))
    if (par) cur = E.br[1];
    {
      const EinTerm<T> ring[2] = {{1, "njfb,mnef->mejb", &t2, &I.Loovv, &w.Pd, 0},
                                  {1, "jnfb,mnfe->mejb", &t2, &I.oovv, &w.Px, 0}};
      if (!ein_multi<T>(*cur, ring, 2))
        for (const EinTerm<T>& x : ring) C(x.alpha, x.spec, *x.A, *x.B, *x.C, x.beta);
    }
    C(-1, "jnfb,mnef->mejb", t2, I.oovv, w.Pd, 1);
  }
  // Lambda intermediates used by more than one of the concurrent parts
  if (lambda && tb) {
    C(-1, "mnef,mnaf->ae", w.t2s, w.l2, w.Gvv, 0);
    C(1, "mnef,inef->mi", w.t2s, w.l2, w.Goo, 0);
    C(1, "imef,kf->imek", w.l2s, t1, w.U, 0);
    C(1, "imef,ke->imkf", w.l2s, t1, w.U2, 0);
  }
  if (par) join_branches(E);
  cur = &E;
  if (tb) {
    C(-1, "nb,nmje->mejb", t1, w.Hooov, w.Bd, 1);
    C(1, "nb,mnje->mejb", t1, w.Hooov, w.Bx, 1);
    // Wd = Bd + Pd/2, Wx = Bx + Px/2 (the T side) and Hd = Bd + Pd, Hx = Bx + Px (the Lambda side)
    // in one pass, written straight into the stacked layouts the ring GEMMs read
    const T* x[8] = {w.Bd.re, w.Bd.im, w.Pd.re, w.Pd.im, w.Bx.re, w.Bx.im, w.Px.re, w.Px.im};
    const int64_t ov = (int64_t)o * v;
    ring_combo<T>(E.stream, ov, ov, E.nb, x, w.Bd.bs, w.WW.re, w.WW.im, w.WW.bs, lambda ? w.HH.re : nullptr,
                  lambda ? w.HH.im : nullptr, w.HH.bs);
  }
  if (par) fork_branches(E);

  // ---- T2 residual: R2 = <ij|ab> + tau.W + ladder + (1 + P(ia,jb)) Z
  C(1, "ijae,be->ijab", t2, w.Hvv, w.Z, 0);
  C(-1, "imab,mj->ijab", t2, w.Hoo, w.Z, 1);
  if (tb) {
    C(1, "iasme,jbsme->iajb", w.T2R, w.WW, w.Zt, 0);
    C(1, "mjae,meib->iajb", t2, w.Wx, w.Zt, 1);
    C(-1, "mb,ijam->ijab", t1, w.Z1, w.Z, 1);
    // t1 t1 ring pieces: S[m,b,i,j] = sum_e t_ie <mb|ej> + t_je <mb|ie>
    {
      const Ten<T>& S = w.S1t;
      C(1, "ie,mbej->mbij", t1, I.ovvo, S, 0);
      C(1, "je,mbie->mbij", t1, I.ovov, S, 1);
      C(-1, "ma,mbij->ijab", t1, S, w.Z, 1);
    }
    C(1, "ie,jeba->ijab", t1, I.ovvv, w.Z, 1);
    C(-1, "ma,ijmb->ijab", t1, I.ooov, w.Z, 1);
    C(1, "mnab,mnij->ijab", tau, w.W, w.R2, 0);
    // R2 += <ij|ab> + ladder + Z + Zt[iajb] + (the same two)[jiba], one pass
    pair_add(*cur, I.oovv, w.LadT, w.Z, w.Zt, w.R2);
  } else {
    P(1, "ijab->ijab", w.Z, w.R2, 0);
    P(1, "ijab->jiba", w.Z, w.R2, 1);
  }
  if (!lambda) return;

  // ---- Lambda2 residual
  if (par) cur = E.br[0];
  C(1, "ijae,eb->ijab", l2, w.Hvv, w.ZL, 0);
  C(-1, "imab,jm->ijab", l2, w.Hoo, w.ZL, 1);
  C(1, "ia,jb->ijab", l1, w.Fme, w.ZL, 1);
  if (tb) {
    C(1, "ijef,mf->ijem", l2, t1, w.Y, 0);
    C(1, "ijef,mnef->ijmn", l2, tau, w.M, 0);
    // l1 . Hbar_ejab with Hbar_amef = <ma|fe> - t_na <nm|ef>: the integral part, then the t1 part
    // through X_in = sum_e l_ie t_ne
    C(1, "ie,jeba->ijab", l1, I.ovvv, w.ZL, 1);
    C(1, "ie,ne->in", l1, t1, w.Xin, 0);
    C(-1, "in,njab->ijab", w.Xin, I.oovv, w.ZL, 1);
    C(-1, "ma,ijmb->ijab", l1, w.Hooov, w.ZL, 1);
    C(1, "iames,jbmes->iajb", w.L2R, w.HH5, w.ZLt, 0);
    C(1, "mjae,ibme->iajb", l2, w.HHx, w.ZLt, 1);
    C(1, "ijae,be->ijab", I.oovv, w.Gvv, w.ZL, 1);
    C(-1, "imab,mj->ijab", I.oovv, w.Goo, w.ZL, 1);
    C(-1, "ijem,meba->ijab", w.Y, I.ovvv, w.ZL, 1);
    C(1, "mnab,ijmn->ijab", l2, w.W, w.S2, 0);
    C(1, "ijmn,mnab->ijab", w.M, I.oovv, w.S2, 1);
    pair_add(*cur, I.oovv, w.LadL, w.ZL, w.ZLt, w.S2);
  } else {
    P(1, "ijab->ijab", w.ZL, w.S2, 0);
    P(1, "ijab->jiba", w.ZL, w.S2, 1);
  }

  // ---- Lambda1 residual: S1 = Fme + l1.Hvv - l1.Hoo + ... + A1 - A2, in three groups with their
  // own partial sums (S1, S1b, S1c), balanced over the three streams: group B (the Wr part of A1)
  // on the first branch after the Lambda2 residual, group A after the T2 residual on the main
  // engine, group C (the Y3 part of A1 and A2) on the second branch; summed after the join.
  if (tb) {
    // group B (the Wr part of A1)
    // Wr in the product's own row-major layout (i f | n g), which the next contraction reads as
    // rows i over one contiguous run of its summed letters; the three l2s x t2 products are independent
    // and go out as one launch where the split-BF16 kernel takes them
    const EinTerm<T> wr[3] = {{1, "imef,nmeg->ifng", &w.l2s, &t2, &w.Wr, 0},
                              {1, "imef,nmgf->ieng", &w.l2s, &t2, &w.WrB, 0},
                              {1, "imef,nmfg->ieng", &w.l2s, &t2, &w.WrC, 0}};
    if (!ein_multi<T>(*cur, wr, 3))
      for (const EinTerm<T>& x : wr) C(x.alpha, x.spec, *x.A, *x.B, *x.C, x.beta);
    C(-1, "ifng,nfag->ia", w.Wr, I.ovvv, w.S1b, 0);
    C(1, "ieng,nega->ia", w.WrB, I.Lovvv, w.S1b, 1);
    C(-1, "ieng,nega->ia", w.WrC, I.ovvv, w.S1b, 1);
  }
  if (par) cur = &E;
  P(1, "ia->ia", w.Fme, w.S1, 0);
  C(1, "ie,ea->ia", l1, w.Hvv, w.S1, 1);
  C(-1, "ma,im->ia", l1, w.Hoo, w.S1, 1);
  // Fock parts of A1 and A2 (present without two-electron integrals too)
  C(1, "imef,nmef->in", w.l2s, t2, w.Q, 0);
  C(-1, "in,na->ia", w.Q, w.Fme, w.S1, 1);
  C(1, "mnae,mnfe->af", w.l2s, t2, w.Gx, 0);
  C(-1, "if,af->ia", w.Fme, w.Gx, w.S1, 1);
  if (!tb) return;
  // group A
  C(2, "me,iame->ia", l1, w.HHd, w.S1, 1);
  C(1, "me,iame->ia", l1, w.HHx, w.S1, 1);
  // G_ef (-2 Hbar_eifa + Hbar_eiaf) = -G_ef L_ieaf + Q_nf L_nifa with Q_nf = sum_e t_ne G_ef
  C(-1, "ef,ieaf->ia", w.Gvv, I.Lovvv, w.S1, 1);
  C(1, "ne,ef->nf", t1, w.Gvv, w.Qnf, 0);
  C(1, "nf,nifa->ia", w.Qnf, I.Loovv, w.S1, 1);
  C(-2, "mn,mina->ia", w.Goo, w.Hooov, w.S1, 1);
  C(1, "mn,imna->ia", w.Goo, w.Hooov, w.S1, 1);
  // A1 = sum_mef l2s_im^ef Hbar_efam
  C(1, "imef,mafe->ia", w.l2s, I.ovvv, w.S1, 1);
  C(2, "mg,imag->ia", t1, w.LadL, w.S1, 1);
  C(-1, "mg,imga->ia", t1, w.LadL, w.S1, 1);
  C(1, "mg,kega->meka", t1, I.ovvv, w.B2, 0);
  C(-1, "imek,meka->ia", w.U, w.B2, w.S1, 1);
  C(1, "mg,kfag->mfka", t1, I.ovvv, w.B3, 0);
  C(-1, "imkf,mfka->ia", w.U2, w.B3, w.S1, 1);
  C(1, "imef,klef->imkl", w.l2s, tau, w.Mp, 0);
  C(1, "mg,klag->klma", t1, I.oovv, w.Nn, 0);
  C(1, "imkl,klma->ia", w.Mp, w.Nn, w.S1, 1);
  C(1, "imnk,knma->ia", w.Mp, I.ooov, w.S1, 1);
  C(-1, "imnf,nfam->ia", w.U2, I.ovvo, w.S1, 1);
  C(-1, "imen,nema->ia", w.U, I.ovov, w.S1, 1);
  // group C: the Y3 part of A1, then -A2 = -sum_mne l2s_mn^ae Hbar_iemn
  if (par) cur = E.br[1];
  {
    const EinTerm<T> y3[3] = {{1, "imnf,kmfg->inkg", &w.U2, &t2, &w.Y3, 0},
                              {1, "imnf,kmgf->inkg", &w.U2, &t2, &w.Y3B, 0},
                              {1, "imen,kmeg->inkg", &w.U, &t2, &w.Y3C, 0}};
    if (!ein_multi<T>(*cur, y3, 3))
      for (const EinTerm<T>& x : y3) C(x.alpha, x.spec, *x.A, *x.B, *x.C, x.beta);
  }
  C(1, "inkg,nkag->ia", w.Y3, I.oovv, w.S1c, 0);
  C(-1, "inkg,nkag->ia", w.Y3B, I.Loovv, w.S1c, 1);
  C(1, "inkg,nkga->ia", w.Y3C, I.oovv, w.S1c, 1);
  C(-1, "mnae,mnie->ia", w.l2s, I.ooov, w.S1c, 1);
  C(1, "mnae,ke->mnak", w.l2s, t1, w.Y6, 0);
  C(1, "mnak,ikmn->ia", w.Y6, w.W, w.S1c, 1);
  C(-1, "mnae,nmei->ia", w.l2s, w.Z1, w.S1c, 1);
  // Wr2 as (a m | k f): the product's output rows (a m) and columns (k f), and for the next
  // contraction rows a over the contiguous run of its summed letters
  {
    const EinTerm<T> wr2[3] = {{1, "mnae,nkef->amkf", &w.l2s, &t2, &w.Wr2, 0},
                               {1, "mnae,nkfe->amkf", &w.l2s, &t2, &w.Wr2B, 0},
                               {1, "mnae,mkfe->ankf", &w.l2s, &t2, &w.Wr2C, 0}};
    if (!ein_multi<T>(*cur, wr2, 3))
      for (const EinTerm<T>& x : wr2) C(x.alpha, x.spec, *x.A, *x.B, *x.C, x.beta);
  }
  C(-1, "amkf,ikmf->ia", w.Wr2, I.Looov, w.S1c, 1);
  C(1, "amkf,ikmf->ia", w.Wr2B, I.ooov, w.S1c, 1);
  C(1, "ankf,kinf->ia", w.Wr2C, I.ooov, w.S1c, 1);
  C(1, "mf,iefn->mien", t1, I.ovvo, w.B4, 0);
  C(-1, "mnae,mien->ia", w.l2s, w.B4, w.S1c, 1);
  C(1, "mf,ikfg->mikg", t1, I.oovv, w.B5, 0);
  C(-1, "kneg,mikg->mnei", t2, w.B5, w.D, 0);
  C(1, "mf,ikfg->mikg", t1, I.Loovv, w.B5, 0);
  C(1, "knge,mikg->mnei", t2, w.B5, w.D, 1);
  C(1, "nf,ikgf->nikg", t1, I.oovv, w.B5, 0);
  C(-1, "mkge,nikg->mnei", t2, w.B5, w.D, 1);
  C(-1, "mnae,mnei->ia", w.l2s, w.D, w.S1c, 1);
  C(1, "nf,iemf->niem", t1, I.ovov, w.B7, 0);
  C(-1, "mnae,niem->ia", w.l2s, w.B7, w.S1c, 1);
  if (par) join_branches(E);
  cur = &E;
  P(1, "ia->ia", w.S1b, w.S1, 1);
  P(1, "ia->ia", w.S1c, w.S1, 1);
}

template <typename T>
void density(Engine& E, Work<T>& w) {
  auto C = [&](double a, const char* s, const Ten<T>& x, const Ten<T>& y, const Ten<T>& z, double b) {
    ein<T>(E, a, s, x, y, z, b);
  };
  auto P = [&](double a, const char* s, const Ten<T>& x, const Ten<T>& z, double b) { padd<T>(E, a, s, x, z, b); };
  const int64_t o = w.o, v = w.v, n = w.n;
  const Ten<T>&t1 = w.t1, &t2 = w.t2, &l1 = w.l1, &l2 = w.l2;
  Ten<T> roo = view(w.rho, 0, {o, o}, {n, 1});
  Ten<T> rov = view(w.rho, o, {o, v}, {n, 1});
  Ten<T> rvo = view(w.rho, o * n, {v, o}, {n, 1});
  Ten<T> rvv = view(w.rho, o * n + o, {v, v}, {n, 1});
  P(2, "ijab->ijab", l2, w.l2s, 0);
  P(-1, "ijab->ijba", l2, w.l2s, 1);
  P(2, "ijab->ijab", t2, w.t2s, 0);
  P(-1, "ijab->ijba", t2, w.t2s, 1);
  C(1, "ijab,ijae->be", w.l2s, t2, w.Dvv, 0);
  C(1, "ijab,imab->jm", w.l2s, t2, w.Doo, 0);
  C(1, "ma,ia->mi", t1, l1, w.P1, 0);
  P(0, "ai->ai", rvo, rvo, 0);
  P(-2, "mi->mi", w.P1, roo, 0);
  P(-2, "jm->mj", w.Doo, roo, 1);
  P(2, "me->me", t1, rov, 0);
  P(2, "me->me", l1, rov, 1);
  C(-2, "mi,ie->me", w.P1, t1, rov, 1);
  C(2, "ia,imae->me", l1, w.t2s, rov, 1);
  C(-2, "mb,be->me", t1, w.Dvv, rov, 1);
  C(-2, "jm,je->me", w.Doo, t1, rov, 1);
  C(2, "ia,ie->ae", l1, t1, rvv, 0);
  P(2, "be->be", w.Dvv, rvv, 1);
}

template void build_work<double>(Arena&, int, int, Work<double>&, int);
template void build_work<float>(Arena&, int, int, Work<float>&, int);
template void residuals<double>(Engine&, const Ints<double>&, Work<double>&, bool, bool);
template void residuals<float>(Engine&, const Ints<float>&, Work<float>&, bool, bool);
template void density<double>(Engine&, Work<double>&);
template void density<float>(Engine&, Work<float>&);

}  // namespace rtcc
