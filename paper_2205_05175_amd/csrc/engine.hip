// Two-operand contraction engine: einsum specs mapped onto the MFMA GEMM.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

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
  op->konst = X.konst;
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
  if (E.trace) fprintf(stderr, "[rtcc] permute-operand src=%p %s->%s n=%lld\n", (const void*)X.re, sx.c_str(), order.c_str(), (long long)n);
  permute_axpby<T>(E.stream, Y.nd, d, X.re, X.im, is, Y.re, Y.im, Y.s, 1.0, 0.0);
  return Y;
}

}  // namespace

struct ConstCache {
  struct Entry {
    void* re = nullptr;
    void* im = nullptr;
    int nd = 0;
    int64_t d[kMaxDim] = {0}, s[kMaxDim] = {0};
  };
  std::map<std::string, Entry> entries;
  std::vector<void*> allocs;
  size_t bytes = 0;
  hipStream_t side = nullptr;
};

ConstCache* const_cache_create() { return new ConstCache(); }
void const_cache_destroy(ConstCache* c) {
  if (!c) return;
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}
size_t const_cache_bytes(const ConstCache* c) { return c ? c->bytes : 0; }

void* const_cache_get(ConstCache* c, const std::string& key, size_t bytes,
                      const std::function<void(void*, hipStream_t)>& fill) {
  auto it = c->entries.find(key);
  if (it != c->entries.end()) return it->second.re;
  void* p = nullptr;
  RTCC_HIP(hipMalloc(&p, std::max<size_t>(bytes, 1)));
  c->allocs.push_back(p);
  c->bytes += bytes;
  if (!c->side) RTCC_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  fill(p, c->side);
  RTCC_HIP(hipStreamSynchronize(c->side));
  ConstCache::Entry e;
  e.re = p;
  c->entries[key] = e;
  return p;
}

namespace {

// A constant operand permuted into letter order `order`, made on first use and kept. The copy is
// made on the cache's own stream and waited for, so it is complete before any later work (also when
// the first use happens while the engine's stream is being captured into a graph).
// A permuted copy of a tensor that is fixed for the current call, kept in the engine's memo so that
// later contractions asking for the same layout reuse it; the copy counts as fixed itself.
template <typename T>
Ten<T> memo_permute(Engine& E, const Ten<T>& X, const std::string& sx, const std::string& order) {
  char key[64 + 24 * 3 * kMaxDim];
  int len = snprintf(key, 64, "p/%p/%p/%d", (const void*)X.re, (const void*)X.im, X.nd);
  for (int i = 0; i < X.nd; ++i) len += snprintf(key + len, 40, "/%lld:%lld", (long long)X.d[i], (long long)X.s[i]);
  for (char c : order) len += snprintf(key + len, 8, "/%d", (int)sx.find(c));
  int64_t n = 1;
  for (char c : order) n *= dim_of(X, sx, c);
  bool hit = false;
  void* buf = memo_get(E, key, (size_t)std::max<int64_t>(n, 1) * sizeof(T) * (X.im ? 2 : 1), &hit);
  if (!buf) return permuted_copy(E, X, sx, order);
  Ten<T> Y;
  Y.nd = (int)order.size();
  for (int i = 0; i < Y.nd; ++i) Y.d[i] = dim_of(X, sx, order[i]);
  int64_t st = 1;
  for (int i = Y.nd - 1; i >= 0; --i) {
    Y.s[i] = st;
    st *= Y.d[i];
  }
  Y.re = reinterpret_cast<T*>(buf);
  Y.im = X.im ? Y.re + std::max<int64_t>(n, 1) : nullptr;
  if (!hit) {
    int64_t d[kMaxDim], is[kMaxDim];
    strides_for(X, sx, order, d, is);
    permute_axpby<T>(E.stream, Y.nd, d, X.re, X.im, is, Y.re, Y.im, Y.s, 1.0, 0.0);
  }
  if (E.trace) fprintf(stderr, "[rtcc] memo-permute %s src=%p %s->%s\n", hit ? "hit" : "new", (const void*)X.re, sx.c_str(), order.c_str());
  E.memo->fixed.push_back(Y.re);
  return Y;
}

template <typename T>
Ten<T> cached_permute(Engine& E, const Ten<T>& X, const std::string& sx, const std::string& order) {
  ConstCache& cc = *E.cache;
  char head[64];
  snprintf(head, sizeof head, "%p/%p/%d:", (const void*)X.re, (const void*)X.im, (int)sizeof(T));
  std::string key(head);
  for (char c : order) key += std::to_string(dim_of(X, sx, c)) + "," + std::to_string(str_of(X, sx, c)) + ";";
  auto it = cc.entries.find(key);
  Ten<T> Y;
  Y.nd = (int)order.size();
  Y.konst = true;
  if (it != cc.entries.end()) {
    const auto& e = it->second;
    Y.re = (T*)e.re;
    Y.im = (T*)e.im;
    for (int i = 0; i < Y.nd; ++i) {
      Y.d[i] = e.d[i];
      Y.s[i] = e.s[i];
    }
    return Y;
  }
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
  const int planes = X.im ? 2 : 1;
  void* p = nullptr;
  RTCC_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * planes * sizeof(T)));
  cc.allocs.push_back(p);
  cc.bytes += (size_t)std::max<int64_t>(n, 1) * planes * sizeof(T);
  Y.re = (T*)p;
  Y.im = X.im ? Y.re + std::max<int64_t>(n, 1) : nullptr;
  if (!cc.side) RTCC_HIP(hipStreamCreateWithFlags(&cc.side, hipStreamNonBlocking));
  int64_t d[kMaxDim], is[kMaxDim];
  strides_for(X, sx, order, d, is);
  permute_axpby<T>(cc.side, Y.nd, d, X.re, X.im, is, Y.re, Y.im, Y.s, 1.0, 0.0);
  RTCC_HIP(hipStreamSynchronize(cc.side));
  ConstCache::Entry e;
  e.re = Y.re;
  e.im = Y.im;
  e.nd = Y.nd;
  for (int i = 0; i < Y.nd; ++i) {
    e.d[i] = Y.d[i];
    e.s[i] = Y.s[i];
  }
  cc.entries[key] = e;
  return Y;
}

std::string ordered(const std::string& from, const std::string& keep) {
  std::string r;
  for (char c : from)
    if (keep.find(c) != std::string::npos) r += c;
  return r;
}

// The operand with the batch axis (letter 'Z', outermost) prepended when it is batched.
template <typename T>
Ten<T> batch_ext(const Ten<T>& X, int nb, std::string* spec) {
  RTCC_CHECK(X.nd < kMaxDim, kEInval, "batched tensor of too many dimensions");
  Ten<T> Y = X;
  Y.nd = X.nd + 1;
  Y.d[0] = nb;
  Y.s[0] = X.bs;
  for (int i = 0; i < X.nd; ++i) {
    Y.d[i + 1] = X.d[i];
    Y.s[i + 1] = X.s[i];
  }
  *spec = "Z" + *spec;
  return Y;
}

struct Plan {
  std::string m, n, k;  // letter groups of the GEMM (outer to inner)
  std::string h;        // batch letter ("Z") or empty
  int64_t cost = -1;    // elements that must be permuted
};

// Best letter orders for one choice of batch letters H (letters of H are neither M, N nor K).
template <typename T>
Plan plan_for(const Ten<T>& A, const std::string& sa, const Ten<T>& B, const std::string& sb, const Ten<T>& C,
              const std::string& sc, const std::string& H) {
  auto drop = [&](const std::string& x) {
    std::string r;
    for (char c : x)
      if (H.find(c) == std::string::npos) r += c;
    return r;
  };
  const std::string a = drop(sa), b = drop(sb), c = drop(sc);
  std::string Kfrom[2] = {ordered(a, b), ordered(b, a)};
  for (auto& k : Kfrom) {
    std::string kk;
    for (char x : k)
      if (c.find(x) == std::string::npos) kk += x;
    k = kk;
  }
  std::string Mfrom[2] = {ordered(c, a), ordered(a, c)};
  std::string Nfrom[2] = {ordered(c, b), ordered(b, c)};
  Plan best;
  best.h = H;
  for (int im = 0; im < 2; ++im)
    for (int in = 0; in < 2; ++in)
      for (int ik = 0; ik < 2; ++ik) {
        GemmOp<T> oa, ob, oc;
        int64_t cost = 0;
        // a constant operand's permuted layouts are cached: free after the first use
        if (!view2d(A, sa, Mfrom[im], Kfrom[ik], &oa) && !A.konst) cost += A.size() * (A.cplx() ? 2 : 1);
        if (!view2d(B, sb, Kfrom[ik], Nfrom[in], &ob) && !B.konst) cost += B.size() * (B.cplx() ? 2 : 1);
        if (!view2d(C, sc, Mfrom[im], Nfrom[in], &oc)) cost += 3 * C.size() * (C.cplx() ? 2 : 1);
        if (best.cost < 0 || cost < best.cost) {
          best.cost = cost;
          best.m = Mfrom[im];
          best.n = Nfrom[in];
          best.k = Kfrom[ik];
        }
      }
  return best;
}

// y(n) = alpha sum_k x(k) W(k, n) + beta y(n) with W read in place through two-level indices (see
// gemv_strided): x and y must each be one strided index (letters kl and nl), each letter group of W at
// most two strided runs, and the lanes' direction (W's unit- or smallest-stride group) dense. Not taken
// when W's permuted layout is kept anyway (a cached constant, an operand fixed for this call). Returns
// false (nothing launched) when the form does not apply.
template <typename T>
bool gemv_two_level(Engine& E, double alpha, const Ten<T>& X, const std::string& sx, const Ten<T>& W,
                    const std::string& sw, const Ten<T>& C, const std::string& sc, const std::string& nl,
                    const std::string& kl, double beta, const char* specstr) {
  if ((W.konst && E.cache) || memo_fixed(E, W.re)) return false;
  auto by_stride = [&](std::string g) {
    std::stable_sort(g.begin(), g.end(), [&](char a, char b) { return str_of(W, sw, a) > str_of(W, sw, b); });
    return g;
  };
  // the letters g (outer to inner) as an outer and an inner run of W: extent of the inner run, strides
  auto split2 = [&](const std::string& g, int64_t* n2, int64_t* s1, int64_t* s2) {
    for (size_t q = 0; q < g.size(); ++q) {  // q = 0: one run
      int64_t i1 = 0, e1 = 1, i2 = 0, e2 = 1;
      if (!mergeable(W, sw, g.substr(q), &i2, &e2)) continue;
      if (q > 0 && !mergeable(W, sw, g.substr(0, q), &i1, &e1)) continue;
      *n2 = e2;
      *s1 = i1;
      *s2 = i2;
      return true;
    }
    return false;
  };
  const std::string kord[2] = {kl, by_stride(kl)}, nord[2] = {nl, by_stride(nl)};
  for (const std::string& ko : kord)
    for (const std::string& no : nord) {
      int64_t incx, ex, incy, ey, N2, sn1, sn2, K2, sk1, sk2;
      if (!mergeable(X, sx, ko, &incx, &ex) || !mergeable(C, sc, no, &incy, &ey)) continue;
      if (!split2(no, &N2, &sn1, &sn2) || !split2(ko, &K2, &sk1, &sk2)) continue;
      const bool row = sn2 == 1 || (sk2 != 1 && sn2 < sk2);
      if (row ? !(sn2 >= 1 && sn2 <= 2 && N2 >= 16) : !(sk2 >= 1 && sk2 <= 2 && K2 >= 16)) continue;
      if (E.trace) fprintf(stderr, "[rtcc] ein %-22s two-level gemv (no permute)\n", specstr);
      gemv_strided<T>(E, ey, ex, alpha, X.re, X.im, incx, W.re, W.im, N2, sn1, sn2, K2, sk1, sk2, C.re, C.im, incy,
                      beta);
      return true;
    }
  return false;
}

}  // namespace

void memo_begin(Engine& E, std::initializer_list<const void*> fixed) {
  if (!E.memo) return;
  E.memo->entries.clear();
  E.memo->used = 0;
  E.memo->fixed.assign(fixed.begin(), fixed.end());
  E.memo->on = true;
}

void memo_end(Engine& E) {
  if (!E.memo) return;
  E.memo->on = false;
  E.memo->entries.clear();
  E.memo->fixed.clear();
  E.memo->used = 0;
}

bool memo_fixed(const Engine& E, const void* p) {
  if (!E.memo || !E.memo->on || !p) return false;
  for (const void* q : E.memo->fixed)
    if (q == p) return true;
  return false;
}

void* memo_get(Engine& E, const std::string& key, size_t bytes, bool* hit) {
  Memo& m = *E.memo;
  auto it = m.entries.find(key);
  if (it != m.entries.end()) {
    *hit = true;
    return it->second;
  }
  *hit = false;
  const size_t b = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
  if (m.used + b > m.cap) return nullptr;
  void* p = m.base + m.used;
  m.used += b;
  m.entries[key] = p;
  return p;
}

void fork_branches(Engine& E) {
  RTCC_CHECK(E.br[0] && E.br[1] && E.ev_fork, kEInval, "fork_branches: engine has no branch engines");
  RTCC_HIP(hipEventRecord(E.ev_fork, E.stream));
  for (Engine* b : E.br) {
    b->cache = E.cache;
    b->mark = E.mark;
    b->mark_user = E.mark_user;
    b->mark_mode = E.mark_mode;
    b->trace = E.trace;
    b->bf16x3 = E.bf16x3;
    b->bf16_min_flops = E.bf16_min_flops;
    b->bf16_kernel = E.bf16_kernel;
    b->pair_splits = E.pair_splits;
    b->group_products = E.group_products;
    b->split_wg = E.split_wg;
    b->group_wg = E.group_wg;
    b->tile_band = E.tile_band;
    b->use_tuning = E.use_tuning;
    b->nb = E.nb;
    b->gemm_flops = 0;
    RTCC_HIP(hipStreamWaitEvent(b->stream, E.ev_fork, 0));
  }
}

void join_branches(Engine& E) {
  RTCC_CHECK(E.br[0] && E.br[1], kEInval, "join_branches: engine has no branch engines");
  for (int k = 0; k < 2; ++k) {
    RTCC_HIP(hipEventRecord(E.ev_join[k], E.br[k]->stream));
    RTCC_HIP(hipStreamWaitEvent(E.stream, E.ev_join[k], 0));
    E.gemm_flops += E.br[k]->gemm_flops;
  }
}

// The index classes of a contraction: every output letter in exactly one input with the output's
// extent, every input letter in the output or in the other input with matching extents; a complex
// output unless both inputs are real. Throws kEInval otherwise.
template <typename T>
void check_spec(const Spec& sp, const char* specstr, const Ten<T>& A0, const Ten<T>& B0, const Ten<T>& C0) {
  RTCC_CHECK((int)sp.a.size() == A0.nd && (int)sp.b.size() == B0.nd && (int)sp.c.size() == C0.nd, kEInval,
             std::string("rank mismatch in ") + specstr);
  for (const std::string* x : {&sp.a, &sp.b, &sp.c})
    RTCC_CHECK(x->find('Z') == std::string::npos, kEInval, std::string("reserved index Z in ") + specstr);
  // letter classes
  for (char c : sp.c) {
    bool ina = sp.a.find(c) != std::string::npos, inb = sp.b.find(c) != std::string::npos;
    RTCC_CHECK(ina != inb, kEInval, std::string("batch/unknown index in ") + specstr);
    RTCC_CHECK(dim_of(C0, sp.c, c) == (ina ? dim_of(A0, sp.a, c) : dim_of(B0, sp.b, c)), kEInval,
               std::string("extent mismatch in ") + specstr);
  }
  for (char c : sp.a) {
    bool inb = sp.b.find(c) != std::string::npos, inc = sp.c.find(c) != std::string::npos;
    RTCC_CHECK(inb || inc, kEInval, std::string("summed-only index in ") + specstr);
    if (inb && !inc) {
      RTCC_CHECK(dim_of(A0, sp.a, c) == dim_of(B0, sp.b, c), kEInval, std::string("extent mismatch in ") + specstr);
    }
  }
  for (char c : sp.b) {
    bool ina = sp.a.find(c) != std::string::npos, inc = sp.c.find(c) != std::string::npos;
    RTCC_CHECK(ina || inc, kEInval, std::string("summed-only index in ") + specstr);
  }
  RTCC_CHECK(C0.cplx() || (!A0.cplx() && !B0.cplx()), kEInval, std::string("complex into real in ") + specstr);
}

template <typename T>
void ein(Engine& E, double alpha, const char* specstr, const Ten<T>& A0, const Ten<T>& B0, const Ten<T>& C0,
         double beta) {
  Spec sp = parse3(specstr);
  check_spec(sp, specstr, A0, B0, C0);

  // batch axis: prepended as letter Z to every batched operand
  const bool bA = E.nb > 1 && A0.bs != 0, bB = E.nb > 1 && B0.bs != 0, bC = E.nb > 1 && C0.bs != 0;
  RTCC_CHECK(bC || (!bA && !bB), kEInval, std::string("batched operand into a shared output in ") + specstr);
  std::string sa = sp.a, sb = sp.b, sc = sp.c;
  Ten<T> A = bA ? batch_ext(A0, E.nb, &sa) : A0;
  Ten<T> B = bB ? batch_ext(B0, E.nb, &sb) : B0;
  Ten<T> C = bC ? batch_ext(C0, E.nb, &sc) : C0;

  // Z in both inputs: a batched GEMM. Z in one input: folded into M (or N) -- one GEMM against
  // the shared operand -- unless that needs more permuting than a batched GEMM with the shared
  // operand at batch stride 0. Z in the output only (both inputs shared): a batched GEMM.
  Plan pl;
  char hl = 'Z';  // the batch letter
  if (bC && bA == bB) {
    pl = plan_for(A, sa, B, sb, C, sc, "Z");
  } else {
    pl = plan_for(A, sa, B, sb, C, sc, "");
    if (bC && pl.cost > 0) {
      Plan pz = plan_for(A, sa, B, sb, C, sc, "Z");
      if (pz.cost < pl.cost) pl = pz;
    }
  }
  if (!bC && pl.cost > 0) {
    // Without a member batch, an output letter shared with one input (or both) may serve as the batch
    // letter of a batched GEMM when that needs less permuting -- but only for small products (below
    // the split-BF16 threshold, in every precision: a large product kept as one GEMM keeps its tiles
    // full, where a batch of thin slices pads every slice to whole tiles; in FP32 the split-BF16 kernel
    // takes single GEMMs only), and not for the GEMV kernels (M or N of 1).
    int64_t M0 = 1, N0 = 1, K0 = 1;
    for (char c : pl.m) M0 *= dim_of(C, sc, c);
    for (char c : pl.n) N0 *= dim_of(C, sc, c);
    for (char c : pl.k) K0 *= dim_of(A, sa, c);
    const bool large = 2.0 * M0 * N0 * K0 >= E.bf16_min_flops;
    if (!large && M0 > 1 && N0 > 1) {
      for (char x : sc) {
        if (sa.find(x) == std::string::npos && sb.find(x) == std::string::npos) continue;
        if (dim_of(C, sc, x) < 2 || dim_of(C, sc, x) > 65535) continue;
        Plan px = plan_for(A, sa, B, sb, C, sc, std::string(1, x));
        if (px.cost < pl.cost) {
          pl = px;
          hl = x;
        }
      }
    }
  }
  const std::string &bm = pl.m, &bn = pl.n, &bk = pl.k;
  const bool hb = !pl.h.empty();
  // the batch letter's presence in A and B (member batch: the operands' own batch flags)
  const bool zA = hl == 'Z' ? bA : sa.find(hl) != std::string::npos;
  const bool zB = hl == 'Z' ? bB : sb.find(hl) != std::string::npos;
  int64_t M = 1, N = 1, K = 1;
  for (char c : bm) M *= dim_of(C, sc, c);
  for (char c : bn) N *= dim_of(C, sc, c);
  for (char c : bk) K *= dim_of(A, sa, c);
  const int nbt = !hb ? 1 : hl == 'Z' ? E.nb : (int)dim_of(C, sc, hl);

  if (!hb && !bA && !bB && !bC && (M == 1) != (N == 1) && K > 1) {
    // a GEMV whose matrix operand would need a permute
    GemmOp<T> t;
    const bool wb = M == 1;  // W = B(k, n) (else W = A(m, k))
    if (wb ? !view2d(B, sb, bk, bn, &t) : !view2d(A, sa, bm, bk, &t)) {
      if (gemv_two_level<T>(E, alpha, wb ? A : B, wb ? sa : sb, wb ? B : A, wb ? sb : sa, C, sc, wb ? bn : bm, bk,
                            beta, specstr))
        return;
    }
  }

  if (E.trace) {
    GemmOp<T> xa, xb, xc;
    bool pa = !view2d(A, sa, bm, bk, &xa), pb = !view2d(B, sb, bk, bn, &xb), pc = !view2d(C, sc, bm, bn, &xc);
    fprintf(stderr, "[rtcc] ein %-22s M=%lld N=%lld K=%lld batch=%d permute:%s%s%s (A %lld, B %lld, C %lld elems)\n",
            specstr, (long long)M, (long long)N, (long long)K, nbt, pa ? " A" : "", pb ? " B" : "", pc ? " C" : "",
            (long long)A.size(), (long long)B.size(), (long long)C.size());
  }
  size_t mark = E.scratch.used;
  GemmOp<T> oa, ob, oc;
  Ten<T> Ap = A, Bp = B;
  const std::string ha = (hb && zA) ? std::string(1, hl) : "", hbb = (hb && zB) ? std::string(1, hl) : "";
  if (!view2d(A, sa, bm, bk, &oa)) {
    Ap = (A.konst && !bA && E.cache) ? cached_permute(E, A, sa, ha + bm + bk)
         : (!bA && memo_fixed(E, A.re)) ? memo_permute(E, A, sa, ha + bm + bk)
                                        : permuted_copy(E, A, sa, ha + bm + bk);
    sa = ha + bm + bk;
    view2d(Ap, sa, bm, bk, &oa);
  }
  if (!view2d(B, sb, bk, bn, &ob)) {
    Bp = (B.konst && !bB && E.cache) ? cached_permute(E, B, sb, hbb + bk + bn)
         : (!bB && memo_fixed(E, B.re)) ? memo_permute(E, B, sb, hbb + bk + bn)
                                        : permuted_copy(E, B, sb, hbb + bk + bn);
    sb = hbb + bk + bn;
    view2d(Bp, sb, bk, bn, &ob);
  }
  GemmBatch gb;
  gb.n = nbt;
  if (hb) {
    gb.a = zA ? str_of(Ap, sa, hl) : 0;
    gb.b = zB ? str_of(Bp, sb, hl) : 0;
    gb.c = str_of(C, sc, hl);
  }
  if (view2d(C, sc, bm, bn, &oc)) {
    if (oc.trans == 0) {
      gemm<T>(E, M, N, K, alpha, oa, ob, C.re, C.im, oc.ld, beta, gb);
    } else {
      // C^T(n,m) = B^T(n,k) A^T(k,m)
      GemmOp<T> bt = ob, at = oa;
      bt.trans ^= 1;
      at.trans ^= 1;
      std::swap(gb.a, gb.b);
      gemm<T>(E, N, M, K, alpha, bt, at, C.re, C.im, oc.ld, beta, gb);
    }
  } else {
    const int64_t nt = std::max<int64_t>(M * N * nbt, 1);
    T* tre = E.scratch.get<T>(nt);
    T* tim = C.im ? E.scratch.get<T>(nt) : nullptr;
    GemmBatch gt = gb;
    gt.c = M * N;
    gemm<T>(E, M, N, K, 1.0, oa, ob, tre, tim, N, 0.0, gt);
    // temp is row-major over letters (Z) bm bn; add into C
    std::string tl = pl.h + bm + bn;
    int64_t d[kMaxDim], is[kMaxDim], os[kMaxDim];
    int64_t st = 1;
    for (int i = (int)tl.size() - 1; i >= 0; --i) {
      d[i] = dim_of(C, sc, tl[i]);
      is[i] = st;
      st *= d[i];
      os[i] = str_of(C, sc, tl[i]);
    }
    permute_axpby<T>(E.stream, (int)tl.size(), d, tre, tim, is, C.re, C.im, os, alpha, beta);
  }
  E.scratch.reset(mark);
}

// Whether the memory of two tensors (either plane) intersects.
template <typename T>
bool overlaps(const Ten<T>& x, const Ten<T>& y) {
  auto span = [](const Ten<T>& t) {
    int64_t e = 1;
    for (int i = 0; i < t.nd; ++i) e += (t.d[i] - 1) * t.s[i];
    return e;
  };
  const int64_t ex = span(x), ey = span(y);
  for (const T* a : {x.re, x.im})
    for (const T* b : {y.re, y.im})
      if (a && b && a < b + ey && b < a + ex) return true;
  return false;
}

template <typename T>
bool ein_multi(Engine& E, const EinTerm<T>* terms, int n) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    if (!E.group_products || !E.bf16x3 || E.nb != 1 || E.force || E.bf16_kernel != 1 || n < 2 || n > 3) return false;
    // every term first checked without issuing anything
    Spec sp[3];
    Plan pl[3];
    int64_t M[3], N[3], K[3];
    for (int h = 0; h < n; ++h) {
      const EinTerm<T>& t = terms[h];
      sp[h] = parse3(t.spec);
      check_spec(sp[h], t.spec, *t.A, *t.B, *t.C);
      if (t.C->re == nullptr || !t.C->cplx()) return false;
      // independent: no output shares memory with another term's output or inputs
      for (int g = 0; g < n; ++g)
        if (g != h && (overlaps(*terms[g].C, *t.C) || overlaps(*terms[g].C, *t.A) || overlaps(*terms[g].C, *t.B)))
          return false;
      pl[h] = plan_for(*t.A, sp[h].a, *t.B, sp[h].b, *t.C, sp[h].c, "");
      M[h] = N[h] = K[h] = 1;
      for (char c : pl[h].m) M[h] *= dim_of(*t.C, sp[h].c, c);
      for (char c : pl[h].n) N[h] *= dim_of(*t.C, sp[h].c, c);
      for (char c : pl[h].k) K[h] *= dim_of(*t.A, sp[h].a, c);
      GemmOp<T> oc;
      if (M[h] < 2 || N[h] < 2 || 2.0 * M[h] * N[h] * K[h] < E.bf16_min_flops) return false;
      if (!view2d(*t.C, sp[h].c, pl[h].m, pl[h].n, &oc)) return false;
      if ((t.A->im != nullptr) != (terms[0].A->im != nullptr) || (t.B->im != nullptr) != (terms[0].B->im != nullptr))
        return false;
    }
    size_t mark = E.scratch.used;
    Bf16Job jobs[3];
    for (int h = 0; h < n; ++h) {
      const EinTerm<T>& t = terms[h];
      const Ten<T>&A = *t.A, &B = *t.B, &C = *t.C;
      const std::string &bm = pl[h].m, &bn = pl[h].n, &bk = pl[h].k;
      std::string sa = sp[h].a, sb = sp[h].b;
      GemmOp<T> oa, ob, oc;
      Ten<T> Ap = A, Bp = B;
      if (!view2d(A, sa, bm, bk, &oa)) {
        Ap = (A.konst && E.cache) ? cached_permute(E, A, sa, bm + bk)
             : memo_fixed(E, A.re) ? memo_permute(E, A, sa, bm + bk)
                                   : permuted_copy(E, A, sa, bm + bk);
        sa = bm + bk;
        view2d(Ap, sa, bm, bk, &oa);
      }
      if (!view2d(B, sb, bk, bn, &ob)) {
        Bp = (B.konst && E.cache) ? cached_permute(E, B, sb, bk + bn)
             : memo_fixed(E, B.re) ? memo_permute(E, B, sb, bk + bn)
                                   : permuted_copy(E, B, sb, bk + bn);
        sb = bk + bn;
        view2d(Bp, sb, bk, bn, &ob);
      }
      view2d(C, sp[h].c, bm, bn, &oc);
      if (E.trace)
        fprintf(stderr, "[rtcc] ein-multi %d/%d %-22s M=%lld N=%lld K=%lld\n", h + 1, n, t.spec, (long long)M[h],
                (long long)N[h], (long long)K[h]);
      if (oc.trans == 0) {
        jobs[h] = Bf16Job{M[h], N[h], K[h], t.alpha, oa, ob, C.re, C.im, oc.ld, t.beta};
      } else {
        // C^T(n, m) = B^T(n, k) A^T(k, m)
        GemmOp<T> at = oa, bt = ob;
        at.trans ^= 1;
        bt.trans ^= 1;
        jobs[h] = Bf16Job{N[h], M[h], K[h], t.alpha, bt, at, C.re, C.im, oc.ld, t.beta};
      }
    }
    bool tuned = false;
    for (int h = 0; h < n && E.use_tuning; ++h)
      tuned |= tuned_choice(2, jobs[h].M, jobs[h].N, jobs[h].K, jobs[h].A.im != nullptr, jobs[h].B.im != nullptr,
                            jobs[h].A.trans, jobs[h].B.trans).kind != 0;
    const bool done = !tuned && gemm_bf16x3_multi(E, jobs, n);
    if (!done) {
      // a product with a table entry of its own (or a kernel choice the launch cannot take): one by one
      for (int h = 0; h < n; ++h)
        gemm<T>(E, jobs[h].M, jobs[h].N, jobs[h].K, jobs[h].alpha, jobs[h].A, jobs[h].B, jobs[h].Cre, jobs[h].Cim,
                jobs[h].ldc, jobs[h].beta);
    }
    E.scratch.reset(mark);
    return true;
  }
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
  const bool bA = E.nb > 1 && A.bs != 0, bC = E.nb > 1 && C.bs != 0;
  RTCC_CHECK(bC || !bA, kEInval, std::string("batched operand into a shared output in ") + specstr);
  int64_t d[kMaxDim], is[kMaxDim], os[kMaxDim];
  int nd = 0;
  if (bC) {  // batch axis; a shared input is broadcast (stride 0)
    RTCC_CHECK(C.nd < kMaxDim, kEInval, std::string("batched permute of too many dimensions: ") + specstr);
    d[0] = E.nb;
    is[0] = bA ? A.bs : 0;
    os[0] = C.bs;
    nd = 1;
  }
  for (size_t i = 0; i < sc.size(); ++i) {
    size_t j = sa.find(sc[i]);
    RTCC_CHECK(j != std::string::npos && A.d[j] == C.d[i], kEInval, std::string("bad permute spec: ") + specstr);
    d[nd] = C.d[i];
    is[nd] = A.s[j];
    os[nd] = C.s[i];
    ++nd;
  }
  if (E.trace) fprintf(stderr, "[rtcc] padd %s\n", specstr);
  if (A.cplx() || !C.cplx()) {
    permute_axpby<T>(E.stream, nd, d, A.re, A.im, is, C.re, C.im, os, alpha, beta);
  } else {
    // real input into complex output: imaginary plane is scaled by beta only
    permute_axpby<T>(E.stream, nd, d, A.re, (const T*)nullptr, is, C.re, C.im, os, alpha, beta);
  }
}

template void ein<double>(Engine&, double, const char*, const Ten<double>&, const Ten<double>&, const Ten<double>&,
                          double);
template void ein<float>(Engine&, double, const char*, const Ten<float>&, const Ten<float>&, const Ten<float>&,
                         double);
template void padd<double>(Engine&, double, const char*, const Ten<double>&, const Ten<double>&, double);
template bool ein_multi<double>(Engine&, const EinTerm<double>*, int);
template bool ein_multi<float>(Engine&, const EinTerm<float>*, int);
template void padd<float>(Engine&, double, const char*, const Ten<float>&, const Ten<float>&, double);

}  // namespace rtcc
