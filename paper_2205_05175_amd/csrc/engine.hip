// Two-operand contraction engine: einsum specs mapped onto the MFMA GEMM.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "engine.h"

namespace rtcc {

namespace {

struct Spec {
  std::string a, b, c;
};

Spec parse3(const char* spec) {
  std::string s(spec);
  size_t comma = s.find(','), arrow = s.find("->");
  RTCC_CHECK(comma != std::string::npos && arrow != std::string::npos && comma < arrow, kEInval,
             std::string("bad contraction spec: ") + spec);
  return {s.substr(0, comma), s.substr(comma + 1, arrow - comma - 1), s.substr(arrow + 2)};
}

template <typename T>
int64_t dim_of(const Ten<T>& X, const std::string& sx, char c) {
  return X.d[sx.find(c)];
}
template <typename T>
int64_t str_of(const Ten<T>& X, const std::string& sx, char c) {
  return X.s[sx.find(c)];
}

// Can the letters of `g` (outer to inner) be merged into one index of X? Returns the stride of
// the merged index in *inner (0 when every letter has extent 1) and the extent in *ext.
template <typename T>
bool mergeable(const Ten<T>& X, const std::string& sx, const std::string& g, int64_t* inner, int64_t* ext) {
  int64_t expect = -1, e = 1;
  *inner = 0;
  for (int i = (int)g.size() - 1; i >= 0; --i) {
    int64_t d = dim_of(X, sx, g[i]);
    int64_t s = str_of(X, sx, g[i]);
    e *= d;
    if (d == 1) continue;
    if (expect < 0) {
      *inner = s;
      expect = s * d;
    } else {
      if (s != expect) return false;
      expect = s * d;
    }
  }
  *ext = e;
  return true;
}

// View X as the logical matrix X(rows = g1, cols = g2). Returns false if a permute is needed.
template <typename T>
bool view2d(const Ten<T>& X, const std::string& sx, const std::string& g1, const std::string& g2, GemmOp<T>* op) {
  int64_t i1, e1, i2, e2;
  if (!mergeable(X, sx, g1, &i1, &e1) || !mergeable(X, sx, g2, &i2, &e2)) return false;
  op->re = X.re;
  op->im = X.im;
  if (e2 == 1 || i2 == 1) {  // row-major: X(r, c) = X[r*ld + c]
    op->trans = 0;
    op->ld = (e1 == 1) ? std::max<int64_t>(e2, 1) : i1;
    return true;
  }
  if (e1 == 1 || i1 == 1) {  // column-major: X(r, c) = X[c*ld + r]
    op->trans = 1;
    op->ld = i2;
    return true;
  }
  return false;
}

template <typename T>
void strides_for(const Ten<T>& X, const std::string& sx, const std::string& order, int64_t* d, int64_t* s) {
  for (size_t i = 0; i < order.size(); ++i) {
    d[i] = dim_of(X, sx, order[i]);
    s[i] = str_of(X, sx, order[i]);
  }
}

// Copy X into a fresh row-major buffer with letter order `order`.
template <typename T>
Ten<T> permuted_copy(Engine& E, const Ten<T>& X, const std::string& sx, const std::string& order) {
  Ten<T> Y;
  Y.nd = (int)order.size();
  int64_t n = 1;
  for (int i = 0; i < Y.nd; ++i) {
    Y.d[i] = dim_of(X, sx, order[i]);
    n *= Y.d[i];
  }
  int64_t st = 1;
  for (int i = Y.nd - 1; i >= 0; --i) {
    Y.s[i] = st;
    st *= Y.d[i];
  }
  Y.re = E.scratch.get<T>(std::max<int64_t>(n, 1));
  Y.im = X.im ? E.scratch.get<T>(std::max<int64_t>(n, 1)) : nullptr;
  int64_t d[kMaxDim], is[kMaxDim];
  strides_for(X, sx, order, d, is);
  permute_axpby<T>(E.stream, Y.nd, d, X.re, X.im, is, Y.re, Y.im, Y.s, 1.0, 0.0);
  return Y;
}

std::string ordered(const std::string& from, const std::string& keep) {
  std::string r;
  for (char c : from)
    if (keep.find(c) != std::string::npos) r += c;
  return r;
}

}  // namespace

template <typename T>
void ein(Engine& E, double alpha, const char* specstr, const Ten<T>& A, const Ten<T>& B, const Ten<T>& C,
         double beta) {
  Spec sp = parse3(specstr);
  RTCC_CHECK((int)sp.a.size() == A.nd && (int)sp.b.size() == B.nd && (int)sp.c.size() == C.nd, kEInval,
             std::string("rank mismatch in ") + specstr);
  // letter classes
  std::string Ml, Nl, Kl;
  for (char c : sp.c) {
    bool ina = sp.a.find(c) != std::string::npos, inb = sp.b.find(c) != std::string::npos;
    RTCC_CHECK(ina != inb, kEInval, std::string("batch/unknown index in ") + specstr);
    RTCC_CHECK(dim_of(C, sp.c, c) == (ina ? dim_of(A, sp.a, c) : dim_of(B, sp.b, c)), kEInval,
               std::string("extent mismatch in ") + specstr);
  }
  for (char c : sp.a) {
    bool inb = sp.b.find(c) != std::string::npos, inc = sp.c.find(c) != std::string::npos;
    RTCC_CHECK(inb || inc, kEInval, std::string("summed-only index in ") + specstr);
    if (inb && !inc) {
      RTCC_CHECK(dim_of(A, sp.a, c) == dim_of(B, sp.b, c), kEInval, std::string("extent mismatch in ") + specstr);
    }
  }
  for (char c : sp.b) {
    bool ina = sp.a.find(c) != std::string::npos, inc = sp.c.find(c) != std::string::npos;
    RTCC_CHECK(ina || inc, kEInval, std::string("summed-only index in ") + specstr);
  }
  RTCC_CHECK(C.cplx() || (!A.cplx() && !B.cplx()), kEInval, std::string("complex into real in ") + specstr);

  std::string Kfrom[2] = {ordered(sp.a, sp.b + ""), ordered(sp.b, sp.a)};
  for (auto& k : Kfrom) {
    std::string kk;
    for (char c : k)
      if (sp.c.find(c) == std::string::npos) kk += c;
    k = kk;
  }
  std::string Mfrom[2] = {ordered(sp.c, sp.a), ordered(sp.a, sp.c)};
  std::string Nfrom[2] = {ordered(sp.c, sp.b), ordered(sp.b, sp.c)};

  // choose letter orders that minimise permuted bytes
  int64_t best = -1;
  std::string bm, bn, bk;
  for (int im = 0; im < 2; ++im)
    for (int in = 0; in < 2; ++in)
      for (int ik = 0; ik < 2; ++ik) {
        GemmOp<T> oa, ob, oc;
        int64_t cost = 0;
        if (!view2d(A, sp.a, Mfrom[im], Kfrom[ik], &oa)) cost += A.size() * (A.cplx() ? 2 : 1);
        if (!view2d(B, sp.b, Kfrom[ik], Nfrom[in], &ob)) cost += B.size() * (B.cplx() ? 2 : 1);
        if (!view2d(C, sp.c, Mfrom[im], Nfrom[in], &oc)) cost += 3 * C.size() * (C.cplx() ? 2 : 1);
        if (best < 0 || cost < best) {
          best = cost;
          bm = Mfrom[im];
          bn = Nfrom[in];
          bk = Kfrom[ik];
        }
      }
  int64_t M = 1, N = 1, K = 1;
  for (char c : bm) M *= dim_of(C, sp.c, c);
  for (char c : bn) N *= dim_of(C, sp.c, c);
  for (char c : bk) K *= dim_of(A, sp.a, c);

  if (E.trace) {
    GemmOp<T> xa, xb, xc;
    bool pa = !view2d(A, sp.a, bm, bk, &xa), pb = !view2d(B, sp.b, bk, bn, &xb), pc = !view2d(C, sp.c, bm, bn, &xc);
    fprintf(stderr, "[rtcc] ein %-22s M=%lld N=%lld K=%lld permute:%s%s%s (A %lld, B %lld, C %lld elems)\n", specstr,
            (long long)M, (long long)N, (long long)K, pa ? " A" : "", pb ? " B" : "", pc ? " C" : "",
            (long long)A.size(), (long long)B.size(), (long long)C.size());
  }
  size_t mark = E.scratch.used;
  GemmOp<T> oa, ob, oc;
  Ten<T> Ap = A, Bp = B;
  std::string sa = sp.a, sb = sp.b;
  if (!view2d(A, sp.a, bm, bk, &oa)) {
    Ap = permuted_copy(E, A, sp.a, bm + bk);
    sa = bm + bk;
    view2d(Ap, sa, bm, bk, &oa);
  }
  if (!view2d(B, sp.b, bk, bn, &ob)) {
    Bp = permuted_copy(E, B, sp.b, bk + bn);
    sb = bk + bn;
    view2d(Bp, sb, bk, bn, &ob);
  }
  if (view2d(C, sp.c, bm, bn, &oc)) {
    if (oc.trans == 0) {
      gemm<T>(E, M, N, K, alpha, oa, ob, C.re, C.im, oc.ld, beta);
    } else {
      // C^T(n,m) = B^T(n,k) A^T(k,m)
      GemmOp<T> bt = ob, at = oa;
      bt.trans ^= 1;
      at.trans ^= 1;
      gemm<T>(E, N, M, K, alpha, bt, at, C.re, C.im, oc.ld, beta);
    }
  } else {
    T* tre = E.scratch.get<T>(std::max<int64_t>(M * N, 1));
    T* tim = C.im ? E.scratch.get<T>(std::max<int64_t>(M * N, 1)) : nullptr;
    gemm<T>(E, M, N, K, 1.0, oa, ob, tre, tim, N, 0.0);
    // temp is row-major over letters bm+bn; add into C
    std::string tl = bm + bn;
    int64_t d[kMaxDim], is[kMaxDim], os[kMaxDim];
    int64_t st = 1;
    for (int i = (int)tl.size() - 1; i >= 0; --i) {
      d[i] = dim_of(C, sp.c, tl[i]);
      is[i] = st;
      st *= d[i];
      os[i] = str_of(C, sp.c, tl[i]);
    }
    permute_axpby<T>(E.stream, (int)tl.size(), d, tre, tim, is, C.re, C.im, os, alpha, beta);
  }
  E.scratch.reset(mark);
}

template <typename T>
void padd(Engine& E, double alpha, const char* specstr, const Ten<T>& A, const Ten<T>& C, double beta) {
  std::string s(specstr);
  size_t arrow = s.find("->");
  RTCC_CHECK(arrow != std::string::npos, kEInval, std::string("bad permute spec: ") + specstr);
  std::string sa = s.substr(0, arrow), sc = s.substr(arrow + 2);
  RTCC_CHECK((int)sa.size() == A.nd && (int)sc.size() == C.nd && sa.size() == sc.size(), kEInval,
             std::string("rank mismatch in ") + specstr);
  RTCC_CHECK(C.cplx() || !A.cplx(), kEInval, std::string("complex into real in ") + specstr);
  int64_t d[kMaxDim], is[kMaxDim], os[kMaxDim];
  for (size_t i = 0; i < sc.size(); ++i) {
    size_t j = sa.find(sc[i]);
    RTCC_CHECK(j != std::string::npos && A.d[j] == C.d[i], kEInval, std::string("bad permute spec: ") + specstr);
    d[i] = C.d[i];
    is[i] = A.s[j];
    os[i] = C.s[i];
  }
  if (A.cplx() || !C.cplx()) {
    permute_axpby<T>(E.stream, C.nd, d, A.re, A.im, is, C.re, C.im, os, alpha, beta);
  } else {
    // real input into complex output: imaginary plane is scaled by beta only
    permute_axpby<T>(E.stream, C.nd, d, A.re, (const T*)nullptr, is, C.re, C.im, os, alpha, beta);
  }
}

template void ein<double>(Engine&, double, const char*, const Ten<double>&, const Ten<double>&, const Ten<double>&,
                          double);
template void ein<float>(Engine&, double, const char*, const Ten<float>&, const Ten<float>&, const Ten<float>&,
                         double);
template void padd<double>(Engine&, double, const char*, const Ten<double>&, const Ten<double>&, double);
template void padd<float>(Engine&, double, const char*, const Ten<float>&, const Ten<float>&, double);

}  // namespace rtcc
