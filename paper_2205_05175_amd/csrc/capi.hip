// C ABI: context lifetime, right-hand side, RK4 / Cash-Karp / general-tableau stepping, delta kick,
// dipole and ground state. See include/rtcc.h for the contract of every entry point.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rtcc.h"
#include "rhs.h"

using namespace rtcc;

namespace {

// Classical RK4 (paper: Eq. rk4truncation; c = 0, 1/2, 1/2, 1).
const double kRk4C[4] = {0.0, 0.5, 0.5, 1.0};
const double kRk4A[4][3] = {{0, 0, 0}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 1.0}};
const double kRk4B[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};

// Cash-Karp pair (Eqs. ck-k, ck-y). The printed c4, c5, a42 and a63 violate sum_j a_ij = c_i;
// Cash and Karp's values are used: c4 = 3/5, c5 = 1, a42 = -9/10, a63 = +575/13824.
const double kCkC[6] = {0.0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1.0, 7.0 / 8};
const double kCkA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0},
    {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
    {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
    {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}};
// fifth-order weights (the step advances with these) and the embedded fourth-order ones
const double kCkB5[6] = {37.0 / 378, 0.0, 250.0 / 621, 125.0 / 594, 0.0, 512.0 / 1771};
const double kCkB4[6] = {2825.0 / 27648, 0.0, 18575.0 / 48384, 13525.0 / 55296, 277.0 / 14336, 1.0 / 4};
// Fehlberg's 4(5) pair (the published coefficients); the step advances with the fourth-order weights.
const double kRkfC[6] = {0.0, 1.0 / 4, 3.0 / 8, 12.0 / 13, 1.0, 1.0 / 2};
const double kRkfA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4, 0, 0, 0, 0},
    {3.0 / 32, 9.0 / 32, 0, 0, 0},
    {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0},
    {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0},
    {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}};
const double kRkfB4[6] = {25.0 / 216, 0.0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0.0};
const double kRkfB5[6] = {16.0 / 135, 0.0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};
const double kSafety = 0.84, kFacMin = 0.1, kFacMax = 5.0;
const int kMaxBatchSystems = 64, kMaxBatchMembers = 4096;

thread_local std::string g_init_error;
std::atomic<uint64_t> g_serial{0};

}  // namespace

void rtcc::set_noctx_error(const std::string& msg) { g_init_error = msg; }

namespace rtcc {
// Workspace of one context for a batch of nb propagations of its system (rtcc_propagate_batch).
struct BatchWS {
  int nb = 0;
  uint64_t gen = 0;  // unique per allocation: a captured batch graph is keyed on it
  bool has32 = false;
  Arena arena;
  Engine E;          // nb members, the context's stream
  Work<double> W64;  // FP64 contractions and the density of every member
  Work<float> W32;   // FP32 / split-BF16 contractions
  void* k[4] = {nullptr, nullptr, nullptr, nullptr};  // RK4 stage derivatives, nb states each
  void* ytmp = nullptr;
  FieldDev* fdev = nullptr;  // the members' fields (device)
  std::vector<FieldDev> fhost;
  double* tdev = nullptr;     // start time of the current step (device)
  double* mu_slot = nullptr;  // nb * 6 dipole values written by a captured step
  double* red = nullptr;      // reduction partials (2 * 1024) and results
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ~BatchWS() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};
}  // namespace rtcc

struct rtcc_ctx {
  uint64_t id = 0;  // unique per context (never reused within a process)
  int o = 0, v = 0, n = 0, precision = RTCC_FP64;
  int64_t n1 = 0, n2 = 0, nstate = 0;  // complex entries
  hipStream_t stream = nullptr;
  std::string err;
  Engine E;
  Engine EB[2];  // branch engines of E (own streams and scratch)
  // engine of the dipole that a captured FP32 / split-BF16 step computes for its start state beside the
  // first right-hand side (own stream, scratch and reduction buffer; FP64 workspace W64, which those
  // right-hand sides do not touch)
  Engine ED;
  hipEvent_t ev_dfork = nullptr, ev_djoin = nullptr;
  double* red_d = nullptr;
  bool dip_overlap = true;
  Memo memo[3];  // per-call memos of E and EB
  Arena arena;        // integrals and workspaces
  Arena arena32;      // FP32 integrals and workspace (allocated on demand)
  bool have32 = false;
  double* f0 = nullptr;
  double* mu = nullptr;
  double* fdiag = nullptr;
  double mu_ref[3] = {0, 0, 0};
  double* mu_ref_dev = nullptr;
  Ints<double> I64;
  Work<double> W64;
  Ints<float> I32;
  Work<float> W32;
  std::vector<void*> k;  // RK stage derivatives (FP64 state-sized)
  void* ytmp = nullptr;
  void* y4 = nullptr;
  void* y5 = nullptr;
  double* red = nullptr;      // reduction partials
  double* redout = nullptr;   // reduction results (device)
  double* host_pinned = nullptr;
  std::vector<void*> diis_x, diis_e;
  void* diis_err = nullptr;
  size_t bytes = 0;
  int64_t last_flops = 0;
  // live timing of the particle-particle ladder GEMM (HIP events on the context stream)
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0.0, prof_flops = 0.0, prof_bytes = 0.0;
  // streams: all work runs on `stream` (owned), ordered with the caller's `ustream` by events
  hipStream_t ustream = nullptr;
  hipEvent_t e_in = nullptr, e_out = nullptr;
  double* tdev = nullptr;     // start time of the current step (device)
  double* mu_slot = nullptr;  // dipole written by a captured step
  // divergence guard: |T2| and the non-finite count of the state after a step (device), checked on the
  // host every guard_every steps when guard_limit > 0
  double* gslot = nullptr;
  double guard_limit = 0.0;
  int guard_every = 50;
  // captured RK4 step
  bool use_graph = true, capturing = false;
  hipGraphExec_t gexec = nullptr;
  struct Key {
    const void* y;
    double h;
    int prec, dip, prof, kind, guard;  // dip: 0 none, 1 end state, 2 start state (overlapped)
    double E0, omega, sigma, t0, n[3];
    bool operator==(const Key& o) const {
      return y == o.y && h == o.h && prec == o.prec && dip == o.dip && prof == o.prof && kind == o.kind &&
             guard == o.guard &&
             E0 == o.E0 && omega == o.omega && sigma == o.sigma && t0 == o.t0 && n[0] == o.n[0] &&
             n[1] == o.n[1] && n[2] == o.n[2];
    }
  } gkey{};
  // batched propagation: this context's batch workspace, and the multi-context step graph of the
  // calls in which this context comes first
  std::unique_ptr<BatchWS> batch;
  std::unique_ptr<BatchWS> adj;  // 4 members: the circle points of the Jacobian-vector product
  void* abuf[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // adjoint state buffers
  hipGraphExec_t bexec = nullptr;
  std::vector<uint64_t> bkey;
};

namespace {

__global__ void add_mu_ref(double* mu6, const double* ref) {
  if (threadIdx.x < 3) mu6[2 * threadIdx.x] += ref[threadIdx.x];
}

template <typename F>
int guarded(rtcc_ctx* c, F&& f) {
  try {
    if (c && c->e_in) {
      RTCC_HIP(hipEventRecord(c->e_in, c->ustream));
      RTCC_HIP(hipStreamWaitEvent(c->stream, c->e_in, 0));
    }
    f();
    if (c && c->e_out) {
      RTCC_HIP(hipEventRecord(c->e_out, c->stream));
      RTCC_HIP(hipStreamWaitEvent(c->ustream, c->e_out, 0));
    }
    return RTCC_OK;
  } catch (const Error& e) {
    if (c) c->err = e.what();
    else g_init_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    else g_init_error = e.what();
    return RTCC_EHIP;
  }
}

template <typename T>
Planes4<T> planes(Work<T>& w, bool inputs) {
  Planes4<T> P;
  if (inputs) {
    Ten<T>* ts[4] = {&w.t1, &w.t2, &w.l1, &w.l2};
    for (int i = 0; i < 4; ++i) {
      P.re[i] = ts[i]->re;
      P.im[i] = ts[i]->im;
      P.bs[i] = ts[i]->bs;
    }
  } else {
    Ten<T>* ts[4] = {&w.R1, &w.R2, &w.S1, &w.S2};
    for (int i = 0; i < 4; ++i) {
      P.re[i] = ts[i]->re;
      P.im[i] = ts[i]->im;
      P.bs[i] = ts[i]->bs;
    }
  }
  return P;
}

void ensure32(rtcc_ctx* c, const double* eri_dev) {
  if (c->have32) return;
  RTCC_CHECK(eri_dev != nullptr, kEInval, "FP32 integrals requested after initialisation without them");
  build_ints<float>(c->E, c->arena32, c->o, c->v, eri_dev, c->I32);
  build_work<float>(c->arena32, c->o, c->v, c->W32);
  c->have32 = true;
}

// out = scale * F(y) with F the RHS at field E (s0 = 1) or of the operator -E.mu alone (s0 = 0, twobody = false)
template <typename T>
void eval_rhs(rtcc_ctx* c, Ints<T>& I, Work<T>& w, const void* y, const double E[3], double s0, bool twobody,
              void* out, double scale) {
  field_fock<T>(c->stream, c->n, c->f0, c->mu, E, s0, w.f.re);
  unpack_state<T>(c->stream, y, c->o, c->v, planes(w, true));
  int64_t f0 = c->E.gemm_flops;
  residuals<T>(c->E, I, w, twobody, true);
  c->last_flops = c->E.gemm_flops - f0;
  pack_rhs<T>(c->stream, c->o, c->v, planes(w, false), out, scale);
}

// Add the durations of the recorded event pairs (each pair on one stream: the main stream or a branch
// engine's, which need not have been joined yet when the buffer fills mid-step) and free the buffer.
void prof_flush(rtcc_ctx* c) {
  if (c->ev_used == 0) return;
  for (int i = 0; i < c->ev_used; i += 2) {
    float ms = 0.f;
    RTCC_HIP(hipEventSynchronize(c->ev[i + 1]));
    RTCC_HIP(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    c->prof_ms += ms;
  }
  c->ev_used = 0;
}

void prof_mark(void* user, int phase, double flops, double bytes, hipStream_t st) {
  rtcc_ctx* c = (rtcc_ctx*)user;
  if (!c->prof) return;
  if (phase == 0 && c->ev_used + 2 > (int)c->ev.size()) prof_flush(c);
  RTCC_HIP(hipEventRecord(c->ev[c->ev_used++], st));
  if (phase == 1) {
    c->prof_launches++;
    c->prof_flops += flops;  // timed launches may differ in size
    c->prof_bytes += bytes;
  }
}

FieldDev to_dev(const rtcc_field* f) {
  FieldDev d{};
  if (f) {
    d.kind = f->kind;
    d.E0 = f->E0;
    d.omega = f->omega;
    d.sigma = f->sigma;
    d.t0 = f->t0;
    for (int i = 0; i < 3; ++i) d.n[i] = f->n[i];
  }
  return d;
}

// An RK stage input y + sum_j cs[j] ks[j] (nk terms; nk = 0: y itself).
struct StageIn {
  const void* y;
  int nk;
  const void* const* ks;
  const double* cs;
};

// out = F(stage input) at t = *tdev + toff, field evaluated on the device; the stage input is formed
// and converted to the contraction precision in one pass
template <typename T>
void eval_rhs_t(rtcc_ctx* c, Ints<T>& I, Work<T>& w, const StageIn& in, const FieldDev& fd, double toff, void* out) {
  field_fock_t<T>(c->stream, c->n, c->f0, c->mu, fd, c->tdev, toff, w.f.re);
  if (in.nk) combo_unpack<T>(c->stream, c->o, c->v, 1, in.y, in.nk, in.ks, in.cs, planes(w, true));
  else unpack_state<T>(c->stream, in.y, c->o, c->v, planes(w, true));
  residuals<T>(c->E, I, w, true, true);
  pack_rhs<T>(c->stream, c->o, c->v, planes(w, false), out, 1.0);
}

void rhs_t(rtcc_ctx* c, const StageIn& in, const FieldDev& fd, double toff, void* out) {
  if (c->precision == RTCC_FP64) {
    eval_rhs_t<double>(c, c->I64, c->W64, in, fd, toff, out);
  } else {
    c->E.bf16x3 = c->precision == RTCC_BF16X3;
    eval_rhs_t<float>(c, c->I32, c->W32, in, fd, toff, out);
    c->E.bf16x3 = false;
  }
}
void rhs_t(rtcc_ctx* c, const void* y, const FieldDev& fd, double toff, void* out) {
  rhs_t(c, StageIn{y, 0, nullptr, nullptr}, fd, toff, out);
}

void rhs_any(rtcc_ctx* c, const void* y, const double E[3], void* out, double scale) {
  if (c->precision == RTCC_FP64) {
    eval_rhs<double>(c, c->I64, c->W64, y, E, 1.0, true, out, scale);
  } else {
    c->E.bf16x3 = c->precision == RTCC_BF16X3;
    eval_rhs<float>(c, c->I32, c->W32, y, E, 1.0, true, out, scale);
    c->E.bf16x3 = false;
  }
}

// The FP64 density is not one of the launches kernel timing brackets: marks are off while it is issued.
struct NoMark {
  Engine& E;
  void (*m)(void*, int, double, double, hipStream_t);
  explicit NoMark(Engine& e) : E(e), m(e.mark) { e.mark = nullptr; }
  ~NoMark() { E.mark = m; }
};

void dipole_dev(rtcc_ctx* c, const void* y, double* out6) {
  Work<double>& w = c->W64;
  unpack_state<double>(c->stream, y, c->o, c->v, planes(w, true));
  {
    NoMark nm(c->E);
    density<double>(c->E, w);
  }
  int64_t nn = (int64_t)c->n * c->n;
  for (int a = 0; a < 3; ++a)
    dot_planar_real<double>(c->stream, nn, w.rho.re, w.rho.im, c->mu + a * nn, c->red, out6 + 2 * a);
  hipLaunchKernelGGL(add_mu_ref, dim3(1), dim3(64), 0, c->stream, out6, c->mu_ref_dev);
  RTCC_HIP(hipGetLastError());
}

// The dipole of y on the dipole engine's stream (the caller orders it with the main stream).
void dipole_dev_overlap(rtcc_ctx* c, const void* y, double* out6) {
  Engine& D = c->ED;
  D.cache = c->E.cache;
  D.trace = c->E.trace;
  D.use_tuning = c->E.use_tuning;
  D.nb = 1;
  Work<double>& w = c->W64;
  unpack_state<double>(D.stream, y, c->o, c->v, planes(w, true));
  density<double>(D, w);
  int64_t nn = (int64_t)c->n * c->n;
  for (int a = 0; a < 3; ++a)
    dot_planar_real<double>(D.stream, nn, w.rho.re, w.rho.im, c->mu + a * nn, c->red_d, out6 + 2 * a);
  hipLaunchKernelGGL(add_mu_ref, dim3(1), dim3(64), 0, D.stream, out6, c->mu_ref_dev);
  RTCC_HIP(hipGetLastError());
}

// |T2| and the non-finite count of y into c->gslot
void guard_dev(rtcc_ctx* c, const void* y) {
  state_guard(c->stream, c->nstate, c->n1, c->n1 + c->n2, y, c->red, c->gslot);
}

// Reads the guard values of the last step (synchronises) and throws RTCC_ENONFINITE when the state has
// a non-finite entry or |T2| exceeds the limit.
void guard_check(rtcc_ctx* c, int64_t step, double t);

// One RK4 step from t = *tdev; advances *tdev by h; optionally the dipole of the new state (dip_start:
// of the start state, on the dipole engine beside the right-hand sides; not in FP64, whose right-hand
// sides use the same workspace) and the guard values.
void rk4_step(rtcc_ctx* c, void* y, double h, const FieldDev& fd, double* dip, bool guard = false,
              bool dip_start = false) {
  RTCC_CHECK(!dip_start || (c->precision != RTCC_FP64 && c->ED.stream), kEInval,
             "rk4_step: no overlapped dipole for this context");
  if (dip && dip_start) {
    RTCC_HIP(hipEventRecord(c->ev_dfork, c->stream));
    RTCC_HIP(hipStreamWaitEvent(c->ED.stream, c->ev_dfork, 0));
    dipole_dev_overlap(c, y, dip);
    RTCC_HIP(hipEventRecord(c->ev_djoin, c->ED.stream));
  }
  for (int s = 0; s < 4; ++s) {
    const void* ks[3] = {c->k[0], c->k[1], c->k[2]};
    double cs[3] = {h * kRk4A[s][0], h * kRk4A[s][1], h * kRk4A[s][2]};
    rhs_t(c, StageIn{y, s, ks, cs}, fd, kRk4C[s] * h, c->k[s]);
  }
  // the dipole engine has finished reading y before y is overwritten
  if (dip && dip_start) RTCC_HIP(hipStreamWaitEvent(c->stream, c->ev_djoin, 0));
  const void* ks[4] = {c->k[0], c->k[1], c->k[2], c->k[3]};
  double cs[4] = {h * kRk4B[0], h * kRk4B[1], h * kRk4B[2], h * kRk4B[3]};
  state_combo(c->stream, c->nstate, y, 4, ks, cs, y);
  if (dip && !dip_start) dipole_dev(c, y, dip);
  if (guard) guard_dev(c, y);
  scalar_update(c->stream, c->tdev, h, true);
}

// Capture one RK4 step (with its dipole) as a graph; replayed while the key is unchanged.
void capture_step(rtcc_ctx* c, void* y, double h, const rtcc_field* field, bool dip, bool guard = false,
                  bool dip_start = false) {
  rtcc_ctx::Key key{};
  key.y = y;
  key.h = h;
  key.prec = c->precision;
  key.dip = dip ? (dip_start ? 2 : 1) : 0;
  key.guard = guard;
  key.prof = c->prof;
  FieldDev fd = to_dev(field);
  key.kind = fd.kind;
  key.E0 = fd.E0;
  key.omega = fd.omega;
  key.sigma = fd.sigma;
  key.t0 = fd.t0;
  for (int i = 0; i < 3; ++i) key.n[i] = fd.n[i];
  if (c->gexec && key == c->gkey) return;
  if (c->gexec) {
    // launches of the old graph may still be executing on this stream: let them finish first
    RTCC_HIP(hipStreamSynchronize(c->stream));
    RTCC_HIP(hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
  }
  RTCC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  c->capturing = true;
  hipGraph_t g = nullptr;
  try {
    rk4_step(c, y, h, fd, dip ? c->mu_slot : nullptr, guard, dip_start);
  } catch (...) {
    c->capturing = false;
    (void)hipStreamEndCapture(c->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  c->capturing = false;
  RTCC_HIP(hipStreamEndCapture(c->stream, &g));
  hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  RTCC_HIP(e);
  c->gkey = key;
}

// ---- batched propagation -------------------------------------------------------------------------
std::atomic<uint64_t> g_batch_gen{0};

void ensure_batch(rtcc_ctx* c, std::unique_ptr<BatchWS>& slot, int nb) {
  if (slot && slot->nb == nb && slot->has32 == c->have32) return;
  // the old workspace may be in use by a step graph launched on another context's stream
  if (slot) RTCC_HIP(hipDeviceSynchronize());
  slot.reset();
  auto B = std::make_unique<BatchWS>();
  B->nb = nb;
  B->gen = ++g_batch_gen;
  B->has32 = c->have32;
  B->E.stream = c->stream;
  B->E.cache = c->E.cache;
  B->E.nb = nb;
  B->E.trace = c->E.trace;
  B->E.bf16_min_flops = c->E.bf16_min_flops;
  B->E.bf16_kernel = c->E.bf16_kernel;
  B->E.group_products = c->E.group_products;
  B->E.split_wg = c->E.split_wg;
  B->E.group_wg = c->E.group_wg;
  B->E.tile_band = c->E.tile_band;
  B->E.sym_ladder = c->E.sym_ladder;
  B->E.ladder_lds = c->E.ladder_lds;
  B->E.pair_splits = c->E.pair_splits;
  B->E.scratch.cap = c->E.scratch.cap * (size_t)nb;
  B->E.scratch.base = B->arena.alloc<char>(B->E.scratch.cap);
  build_work<double>(B->arena, c->o, c->v, B->W64, nb);
  if (c->have32) build_work<float>(B->arena, c->o, c->v, B->W32, nb);
  const int64_t nst = (int64_t)nb * c->nstate;
  for (auto& p : B->k) p = B->arena.alloc<double>(2 * nst);
  B->ytmp = B->arena.alloc<double>(2 * nst);
  B->fdev = (FieldDev*)B->arena.alloc<char>((int64_t)nb * sizeof(FieldDev));
  B->fhost.resize(nb);
  B->tdev = B->arena.alloc<double>(1);
  B->mu_slot = B->arena.alloc<double>(6 * (int64_t)nb);
  B->red = B->arena.alloc<double>(2 * 1024 + 16);
  RTCC_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
  RTCC_HIP(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
  slot = std::move(B);
}
void ensure_batch(rtcc_ctx* c, int nb) { ensure_batch(c, c->batch, nb); }

template <typename T>
void eval_rhs_batch(rtcc_ctx* c, BatchWS& B, Ints<T>& I, Work<T>& w, const StageIn& in, double toff, void* out) {
  field_fock_tb<T>(B.E.stream, c->n, c->f0, c->mu, B.fdev, B.nb, B.tdev, toff, w.f.re, w.f.bs);
  if (in.nk) combo_unpack<T>(B.E.stream, c->o, c->v, B.nb, in.y, in.nk, in.ks, in.cs, planes(w, true));
  else unpack_state<T>(B.E.stream, in.y, c->o, c->v, planes(w, true), B.nb);
  residuals<T>(B.E, I, w, true, true);
  pack_rhs<T>(B.E.stream, c->o, c->v, planes(w, false), out, 1.0, B.nb);
}

void rhs_batch(rtcc_ctx* c, BatchWS& B, const StageIn& in, double toff, void* out) {
  if (c->precision == RTCC_FP64) {
    eval_rhs_batch<double>(c, B, c->I64, B.W64, in, toff, out);
  } else {
    B.E.bf16x3 = c->precision == RTCC_BF16X3;
    eval_rhs_batch<float>(c, B, c->I32, B.W32, in, toff, out);
    B.E.bf16x3 = false;
  }
}
void rhs_batch(rtcc_ctx* c, BatchWS& B, const void* y, double toff, void* out) {
  rhs_batch(c, B, StageIn{y, 0, nullptr, nullptr}, toff, out);
}

// dipoles of all members of y (FP64 density) into out[6 * nb]
void dipole_batch_dev(rtcc_ctx* c, const void* y, double* out) {
  BatchWS& B = *c->batch;
  Work<double>& w = B.W64;
  unpack_state<double>(B.E.stream, y, c->o, c->v, planes(w, true), B.nb);
  {
    NoMark nm(B.E);
    density<double>(B.E, w);
  }
  dipole_batch(B.E.stream, B.nb, (int64_t)c->n * c->n, w.rho.re, w.rho.im, w.rho.bs, c->mu, c->mu_ref_dev, out);
}

// One RK4 step of every member from t = *tdev (the members' own fields); advances *tdev by h.
void rk4_step_batch(rtcc_ctx* c, void* y, double h, double* dip) {
  BatchWS& B = *c->batch;
  const int64_t nst = (int64_t)B.nb * c->nstate;
  for (int s = 0; s < 4; ++s) {
    const void* ks[3] = {B.k[0], B.k[1], B.k[2]};
    double cs[3] = {h * kRk4A[s][0], h * kRk4A[s][1], h * kRk4A[s][2]};
    rhs_batch(c, B, StageIn{y, s, ks, cs}, kRk4C[s] * h, B.k[s]);
  }
  const void* ks[4] = {B.k[0], B.k[1], B.k[2], B.k[3]};
  double cs[4] = {h * kRk4B[0], h * kRk4B[1], h * kRk4B[2], h * kRk4B[3]};
  state_combo(B.E.stream, nst, y, 4, ks, cs, y);
  if (dip) dipole_batch_dev(c, y, dip);
  scalar_update(B.E.stream, B.tdev, h, true);
}

// Streams of ctxs[1..] wait for the work already on ctxs[0]'s stream.
void batch_fork(rtcc_ctx* const* ctxs, int nsys) {
  rtcc_ctx* c0 = ctxs[0];
  RTCC_HIP(hipEventRecord(c0->batch->ev_fork, c0->stream));
  for (int s = 1; s < nsys; ++s) RTCC_HIP(hipStreamWaitEvent(ctxs[s]->stream, c0->batch->ev_fork, 0));
}
// ctxs[0]'s stream waits for the work on the other contexts' streams.
void batch_join(rtcc_ctx* const* ctxs, int nsys) {
  for (int s = 1; s < nsys; ++s) {
    RTCC_HIP(hipEventRecord(ctxs[s]->batch->ev_join, ctxs[s]->stream));
    RTCC_HIP(hipStreamWaitEvent(ctxs[0]->stream, ctxs[s]->batch->ev_join, 0));
  }
}

// One RK4 step of every member of every system captured as one graph (a branch per system),
// replayed while the contexts, their workspaces, the states, h and the precisions are unchanged.
void capture_batch(rtcc_ctx* const* ctxs, int nsys, void* const* ys, double h, const bool* dip) {
  rtcc_ctx* c0 = ctxs[0];
  std::vector<uint64_t> key;
  uint64_t hb;
  std::memcpy(&hb, &h, sizeof hb);
  key.push_back((uint64_t)nsys);
  key.push_back(hb);
  for (int s = 0; s < nsys; ++s) {
    key.push_back(ctxs[s]->id);
    key.push_back(ctxs[s]->batch->gen);
    key.push_back((uint64_t)(uintptr_t)ys[s]);
    key.push_back((uint64_t)ctxs[s]->precision);
    key.push_back(dip[s] ? 1 : 0);
  }
  if (c0->bexec && key == c0->bkey) return;
  if (c0->bexec) {
    // launches of the old graph may still be executing on this stream: let them finish first
    RTCC_HIP(hipStreamSynchronize(c0->stream));
    RTCC_HIP(hipGraphExecDestroy(c0->bexec));
    c0->bexec = nullptr;
  }
  RTCC_HIP(hipStreamBeginCapture(c0->stream, hipStreamCaptureModeRelaxed));
  hipGraph_t g = nullptr;
  try {
    batch_fork(ctxs, nsys);
    for (int s = 0; s < nsys; ++s) rk4_step_batch(ctxs[s], ys[s], h, dip[s] ? ctxs[s]->batch->mu_slot : nullptr);
    batch_join(ctxs, nsys);
  } catch (...) {
    (void)hipStreamEndCapture(c0->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  RTCC_HIP(hipStreamEndCapture(c0->stream, &g));
  hipError_t e = hipGraphInstantiate(&c0->bexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  RTCC_HIP(e);
  c0->bkey = key;
}

// ---- adjoint ----------------------------------------------------------------------------------------
// The right-hand side F = S_hat grad L of the Lagrangian L = <0|(1+Lambda) Hbar|0> in closed-shell
// variables, S_hat = [[0, -i G^-1], [i G^-1, 0]] with the closed-shell metric G (singles 2, doubles
// 2 x_ijab - x_ijba), so the Jacobian J = S_hat Hess(L) has the bilinear transpose
// J^T w = -S_hat^-1 J (S_hat w): a vector-Jacobian product is a Jacobian-vector product between two
// swaps. F is a polynomial of degree 4 in the state, so J u is the first Taylor coefficient of
// F(y + eps u), extracted exactly from four points on a circle in the complex eps plane.
const int kCircleM = 4;
const double kCircleRho = 0.1;  // circle radius in units of 1 / max|u|

void ensure_adj(rtcc_ctx* c) {
  ensure_batch(c, c->adj, kCircleM);
  if (!c->abuf[0])
    for (auto& p : c->abuf) p = c->arena.alloc<double>(2 * c->nstate);
}

void set_adj_field(rtcc_ctx* c, const FieldDev& fd, double t) {
  BatchWS& A = *c->adj;
  for (auto& f : A.fhost) f = fd;
  upload_fields(c->stream, A.fhost.data(), A.nb, A.fdev);
  scalar_update(c->stream, A.tdev, t, false);
}

// out = J^H ybar (the gradient convention of a real loss: Re-part + i Im-part derivatives), J = dF/dy at y
// for the adjoint workspace's field at time *tdev + toff. out must not overlap ybar or y.
void rhs_vjp_dev(rtcc_ctx* c, const void* y, double toff, const void* ybar, void* out) {
  BatchWS& A = *c->adj;
  hipStream_t st = c->stream;
  void* u = c->abuf[0];
  void* Ju = c->abuf[1];
  double* maxu = A.red + 2048;
  // J^H ybar = conj(J^T conj(ybar)) = conj(-S_hat^-1 J S_hat conj(ybar))
  hamil_apply(st, c->o, c->v, ybar, nullptr, nullptr, false, true, false, 1.0, false, u);
  max_abs(st, c->nstate, u, A.red, maxu);
  circle_points(st, c->nstate, y, u, maxu, kCircleRho, kCircleM, A.ytmp);
  rhs_batch(c, A, A.ytmp, toff, A.k[0]);
  circle_coef1(st, c->nstate, A.k[0], maxu, kCircleRho, kCircleM, Ju);
  hamil_apply(st, c->o, c->v, Ju, nullptr, nullptr, true, false, true, -1.0, false, out);
}

// out = F[m . mu, 0](y): the right-hand side of the one-body operator m . mu alone (context precision)
void one_body_rhs(rtcc_ctx* c, const void* y, const double m[3], void* out, bool fp64) {
  const double E[3] = {-m[0], -m[1], -m[2]};
  if (fp64 || c->precision == RTCC_FP64) eval_rhs<double>(c, c->I64, c->W64, y, E, 0.0, false, out, 1.0);
  else eval_rhs<float>(c, c->I32, c->W32, y, E, 0.0, false, out, 1.0);
}

// Derivatives of the Gaussian pulse amplitude e(t) = -E0 exp(-x^2 / (2 sigma^2)) cos(omega x), x = t - t0,
// with respect to (E0, omega, sigma, t0).
void pulse_grad(const FieldDev& fd, double t, double g[4]) {
  const double x = t - fd.t0, s2 = fd.sigma * fd.sigma;
  const double env = std::exp(-0.5 * x * x / s2), cs = std::cos(fd.omega * x), sn = std::sin(fd.omega * x);
  g[0] = -env * cs;
  g[1] = fd.E0 * env * sn * x;
  g[2] = -fd.E0 * env * cs * x * x / (s2 * fd.sigma);
  g[3] = -fd.E0 * env * (x * cs / s2 + fd.omega * sn);
}

void sync_read(rtcc_ctx* c, const double* dev, double* host, int n) {
  RTCC_HIP(hipMemcpyAsync(c->host_pinned, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  RTCC_HIP(hipStreamSynchronize(c->stream));
  std::memcpy(host, c->host_pinned, n * sizeof(double));
}

bool solve_small(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (std::fabs(A[piv * n + col]) < 1e-300) return false;
    if (piv != col) {
      for (int j = 0; j < n; ++j) std::swap(A[col * n + j], A[piv * n + j]);
      std::swap(b[col], b[piv]);
    }
    for (int r = col + 1; r < n; ++r) {
      double f = A[r * n + col] / A[col * n + col];
      for (int j = col; j < n; ++j) A[r * n + j] -= f * A[col * n + j];
      b[r] -= f * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
    b[r] = s / A[r * n + r];
  }
  return true;
}

void guard_check(rtcc_ctx* c, int64_t step, double t) {
  double g[2];
  sync_read(c, c->gslot, g, 2);
  if (g[1] > 0.0 || !(g[0] <= c->guard_limit)) {
    char msg[200];
    if (g[1] > 0.0)
      snprintf(msg, sizeof msg, "divergence guard: %.0f non-finite state entries after step %lld (t = %.6g)", g[1],
               (long long)step, t);
    else
      snprintf(msg, sizeof msg, "divergence guard: |T2| = %.6g exceeds %.6g after step %lld (t = %.6g)", g[0],
               c->guard_limit, (long long)step, t);
    throw Error(kENonFinite, msg);
  }
}

// Step list of the mixed step-size RK4 propagation: (start time, step size) pairs from t0 to t_end,
// h1 while a Gaussian pulse is on (|t - t0_pulse| <= 5 sigma) and h2 elsewhere; every phase ends with a
// shorter step that lands on its boundary. Step sizes inside a phase are exactly h1 or h2 (start times
// are computed as phase start + k h, not accumulated).
std::vector<std::pair<double, double>> mixed_schedule(double t0, double t_end, double h1, double h2,
                                                       const rtcc_field* f) {
  std::vector<std::pair<double, double>> out;
  double on_lo = t_end, on_hi = t_end;
  if (f && f->kind == 1) {
    on_lo = std::min(std::max(t0, f->t0 - 5.0 * f->sigma), t_end);
    on_hi = std::min(std::max(t0, f->t0 + 5.0 * f->sigma), t_end);
  }
  const double bounds[4] = {t0, on_lo, on_hi, t_end};
  const double hs[3] = {h2, h1, h2};
  for (int ph = 0; ph < 3; ++ph) {
    const double a = bounds[ph], b = bounds[ph + 1], h = hs[ph];
    if (!(b > a)) continue;
    const double span = b - a;
    const int64_t nfull = (int64_t)std::floor(span / h * (1.0 + 1e-12));
    RTCC_CHECK(nfull < (int64_t)1 << 30, kEInval, "mixed RK4: too many steps");
    for (int64_t k = 0; k < nfull; ++k) out.emplace_back(a + (double)k * h, h);
    const double rem = span - (double)nfull * h;
    if (rem > 1e-9 * h) out.emplace_back(a + (double)nfull * h, rem);
  }
  return out;
}

bool tab_explicit(const rtcc_tableau& T) {
  for (int i = 0; i < T.stages; ++i)
    for (int j = i; j < T.stages; ++j)
      if (T.a[i][j] != 0.0) return false;
  return true;
}

// Shape and finiteness of a caller's tableau; implicit tableaux are limited by the six stage buffers
// (old and new derivatives of up to three stages).
void check_tab(const rtcc_tableau* T, bool need_embedded, const char* who) {
  RTCC_CHECK(T && T->stages >= 1 && T->stages <= RTCC_MAX_STAGES && T->err_order >= 0, kEInval,
             std::string(who) + ": invalid tableau");
  for (int i = 0; i < T->stages; ++i) {
    RTCC_CHECK(std::isfinite(T->b[i]) && std::isfinite(T->c[i]) && std::isfinite(T->b_err[i]), kEInval,
               std::string(who) + ": non-finite tableau entry");
    for (int j = 0; j < T->stages; ++j)
      RTCC_CHECK(std::isfinite(T->a[i][j]), kEInval, std::string(who) + ": non-finite tableau entry");
  }
  const bool ex = tab_explicit(*T);
  RTCC_CHECK(ex || T->stages <= 3, kEInval, std::string(who) + ": implicit tableaux are limited to 3 stages");
  RTCC_CHECK(!need_embedded || (ex && T->err_order > 0), kEInval,
             std::string(who) + ": needs an explicit tableau with an embedded solution (err_order > 0)");
}

// All stage derivatives k[0..s-1] of an explicit tableau for a step of size hh from the device time.
void explicit_stages(rtcc_ctx* c, const void* y, double hh, const rtcc_tableau& T, const FieldDev& fd) {
  for (int s = 0; s < T.stages; ++s) {
    const void* ks[RTCC_MAX_STAGES];
    double cs[RTCC_MAX_STAGES];
    for (int j = 0; j < s; ++j) {
      ks[j] = c->k[j];
      cs[j] = hh * T.a[s][j];
    }
    rhs_t(c, StageIn{y, s, ks, cs}, fd, T.c[s] * hh, c->k[s]);
  }
}

// One trial of an embedded explicit tableau of size hh from t (device time set here): the advancing
// solution into y5, the embedded one into y4, Delta = max|y5 - y4| into redout[0]; with mu6 also the
// dipole of y5 (redout[8..13]). Returns Delta (and the dipole) after one synchronisation.
double emb_trial(rtcc_ctx* c, const void* y, double t, double hh, const rtcc_tableau& T, const FieldDev& fd,
                 double* mu6) {
  scalar_update(c->stream, c->tdev, t, false);
  explicit_stages(c, y, hh, T, fd);
  const void* ks[RTCC_MAX_STAGES];
  double cb[RTCC_MAX_STAGES], ce[RTCC_MAX_STAGES];
  for (int j = 0; j < T.stages; ++j) {
    ks[j] = c->k[j];
    cb[j] = hh * T.b[j];
    ce[j] = hh * T.b_err[j];
  }
  state_combo(c->stream, c->nstate, y, T.stages, ks, cb, c->y5);
  state_combo(c->stream, c->nstate, y, T.stages, ks, ce, c->y4);
  max_abs_diff(c->stream, c->nstate, c->y5, c->y4, c->red, c->redout);
  if (mu6) {
    dipole_dev(c, c->y5, c->redout + 8);
    double d[14];
    sync_read(c, c->redout, d, 14);
    for (int i = 0; i < 6; ++i) mu6[i] = d[8 + i];
    return d[0];
  }
  double d[2];
  sync_read(c, c->redout, d, 2);
  return d[0];
}

// Controller of Eq. ck-h-final for a pair of lower order p (p = 4: exponents 1/5 and 1/4).
double ctl_factor(double eps, double dl, int p) {
  double fac;
  if (dl == 0.0) fac = kFacMax;
  else fac = kSafety * std::pow(eps / dl, dl <= eps ? 1.0 / (p + 1) : 1.0 / p);
  return std::min(std::max(fac, kFacMin), kFacMax);
}

void builtin_tableau(int id, rtcc_tableau& T) {
  T = rtcc_tableau{};
  if (id == RTCC_TAB_RK4) {
    T.stages = 4;
    for (int i = 0; i < 4; ++i) {
      T.c[i] = kRk4C[i];
      T.b[i] = kRk4B[i];
      for (int j = 0; j < 3; ++j) T.a[i][j] = kRk4A[i][j];
    }
  } else if (id == RTCC_TAB_CASHKARP || id == RTCC_TAB_RKF45) {
    const bool ck = id == RTCC_TAB_CASHKARP;
    T.stages = 6;
    T.err_order = 4;
    for (int i = 0; i < 6; ++i) {
      T.c[i] = ck ? kCkC[i] : kRkfC[i];
      T.b[i] = ck ? kCkB5[i] : kRkfB4[i];
      T.b_err[i] = ck ? kCkB4[i] : kRkfB5[i];
      for (int j = 0; j < 5; ++j) T.a[i][j] = ck ? kCkA[i][j] : kRkfA[i][j];
    }
  } else if (id == RTCC_TAB_GL2) {
    // Gauss-Legendre, two stages: nodes 1/2 -+ sqrt(3)/6 (order 4)
    const double r = std::sqrt(3.0) / 6.0;
    T.stages = 2;
    T.c[0] = 0.5 - r;
    T.c[1] = 0.5 + r;
    T.a[0][0] = 0.25;
    T.a[0][1] = 0.25 - r;
    T.a[1][0] = 0.25 + r;
    T.a[1][1] = 0.25;
    T.b[0] = T.b[1] = 0.5;
  } else if (id == RTCC_TAB_GL3) {
    // Gauss-Legendre, three stages: nodes 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10 (order 6)
    const double q = std::sqrt(15.0);
    T.stages = 3;
    T.c[0] = 0.5 - q / 10;
    T.c[1] = 0.5;
    T.c[2] = 0.5 + q / 10;
    const double a[3][3] = {{5.0 / 36, 2.0 / 9 - q / 15, 5.0 / 36 - q / 30},
                            {5.0 / 36 + q / 24, 2.0 / 9, 5.0 / 36 - q / 24},
                            {5.0 / 36 + q / 30, 2.0 / 9 + q / 15, 5.0 / 36}};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) T.a[i][j] = a[i][j];
    T.b[0] = T.b[2] = 5.0 / 18;
    T.b[1] = 4.0 / 9;
  } else {
    throw Error(kEInval, "rtcc_tableau_builtin: unknown tableau id");
  }
}

// Adaptive propagation with an embedded explicit tableau (shared by rtcc_propagate_cashkarp).
void propagate_embedded(rtcc_ctx* c, void* y, double t0, double t_end, double h0, double eps, const rtcc_tableau& T,
                        const rtcc_field* field, int max_trials, int cap, double* t_out, double* mu_out,
                        int* naccepted, int* nrejected, double* h_next, const char* who) {
  const FieldDev fd = to_dev(field);
  const bool rec = t_out || mu_out;
  double t = t0, h = h0;
  int trials = 0;
  while (t < t_end) {
    RTCC_CHECK(trials < max_trials, kENotConv, std::string(who) + ": trial limit reached before t_end");
    ++trials;
    const double hh = std::min(h, t_end - t);
    double mu6[6];
    const double dl = emb_trial(c, y, t, hh, T, fd, mu_out ? mu6 : nullptr);
    RTCC_CHECK(std::isfinite(dl), kENonFinite, std::string(who) + ": non-finite error estimate");
    const double fac = ctl_factor(eps, dl, T.err_order);
    if (dl <= eps) {
      RTCC_CHECK(!rec || *naccepted < cap, kEInval, std::string(who) + ": output capacity exceeded");
      RTCC_HIP(hipMemcpyAsync(y, c->y5, c->nstate * 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      t = (hh == t_end - t) ? t_end : t + hh;
      if (t_out) t_out[*naccepted] = t;
      if (mu_out)
        for (int i = 0; i < 6; ++i) mu_out[6 * (int64_t)(*naccepted) + i] = mu6[i];
      ++*naccepted;
    } else {
      ++*nrejected;
    }
    h = hh * fac;
  }
  if (h_next) *h_next = h;
}

// One implicit step (full A, s <= 3): Jacobi fixed-point sweeps over the stage derivatives, alternating
// between the buffer sets k[0..2] and k[3..5]; the first sweep reads k[0] = f(t, y) for every stage.
int implicit_step(rtcc_ctx* c, void* y, double t, double h, const rtcc_tableau& T, const FieldDev& fd, double tol,
                  int max_iter) {
  const int S = T.stages;
  scalar_update(c->stream, c->tdev, t, false);
  rhs_t(c, y, fd, 0.0, c->k[0]);
  const void* old[3] = {c->k[0], c->k[0], c->k[0]};
  int set = 1;  // the set the next sweep writes
  for (int it = 1; it <= max_iter; ++it) {
    void* nw[3] = {c->k[3 * set], c->k[3 * set + 1], c->k[3 * set + 2]};
    for (int i = 0; i < S; ++i) {
      double cs[3];
      for (int j = 0; j < S; ++j) cs[j] = h * T.a[i][j];
      rhs_t(c, StageIn{y, S, old, cs}, fd, T.c[i] * h, nw[i]);
    }
    for (int i = 0; i < S; ++i) max_abs_diff(c->stream, c->nstate, nw[i], old[i], c->red, c->redout + 2 * i);
    double d[6];
    sync_read(c, c->redout, d, 2 * S);
    double dmax = 0.0;
    for (int i = 0; i < S; ++i) {
      RTCC_CHECK(std::isfinite(d[2 * i]), kENonFinite, "rtcc_step_tableau: non-finite stage change");
      dmax = std::max(dmax, d[2 * i]);
    }
    for (int i = 0; i < S; ++i) old[i] = nw[i];
    set ^= 1;
    if (h * dmax <= tol) {
      double cb[3];
      for (int j = 0; j < S; ++j) cb[j] = h * T.b[j];
      state_combo(c->stream, c->nstate, y, S, old, cb, y);
      return it;
    }
  }
  throw Error(kENotConv, "rtcc_step_tableau: stage iteration did not converge within max_iter sweeps");
}

}  // namespace

extern "C" {

int rtcc_init(rtcc_ctx** out, int o, int v, const double* eri, const double* fock, const double* dipole,
              int precision, void* hip_stream) {
  if (!out) {
    g_init_error = "rtcc_init: ctx pointer is NULL";
    return RTCC_EINVAL;
  }
  *out = nullptr;
  if (o < 1 || v < 1 || !eri || !fock || !dipole ||
      (precision != RTCC_FP64 && precision != RTCC_FP32 && precision != RTCC_BF16X3)) {
    g_init_error = "rtcc_init: invalid arguments";
    return RTCC_EINVAL;
  }
  auto c = std::make_unique<rtcc_ctx>();
  int st = guarded(nullptr, [&] {
    c->id = ++g_serial;
    c->o = o;
    c->v = v;
    c->n = o + v;
    c->precision = precision;
    c->n1 = (int64_t)o * v;
    c->n2 = c->n1 * c->n1;
    c->nstate = 2 * (c->n1 + c->n2);
    c->ustream = (hipStream_t)hip_stream;
    RTCC_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    RTCC_HIP(hipEventCreateWithFlags(&c->e_in, hipEventDisableTiming));
    RTCC_HIP(hipEventCreateWithFlags(&c->e_out, hipEventDisableTiming));
    c->E.stream = c->stream;
    c->E.cache = const_cache_create();
    const char* bm = std::getenv("RTCC_BF16_MIN_FLOPS");
    if (bm && bm[0]) c->E.bf16_min_flops = std::atof(bm);
    const char* bk = std::getenv("RTCC_BF16_KERNEL");
    if (bk && bk[0]) c->E.bf16_kernel = std::atoi(bk);
    RTCC_CHECK(c->E.bf16_kernel >= 1 && c->E.bf16_kernel <= 4, kEInval, "RTCC_BF16_KERNEL must be 1 to 4");
    const char* lm = std::getenv("RTCC_LADDER");
    if (lm && lm[0]) {
      RTCC_CHECK(!std::strcmp(lm, "full") || !std::strcmp(lm, "symmetric") || !std::strcmp(lm, "symmetric-nolds"),
                 kEInval, "RTCC_LADDER must be full, symmetric or symmetric-nolds");
      c->E.sym_ladder = std::strcmp(lm, "full") != 0;
      c->E.ladder_lds = std::strcmp(lm, "symmetric-nolds") != 0;
    }
    const char* ps = std::getenv("RTCC_LADDER_PAIR_SPLITS");
    if (ps && ps[0]) c->E.pair_splits = std::atoi(ps);
    RTCC_CHECK(c->E.pair_splits >= -1 && c->E.pair_splits <= 16, kEInval,
               "RTCC_LADDER_PAIR_SPLITS must be -1 (no pairing) to 16");
    const char* ng = std::getenv("RTCC_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    const char* ngr = std::getenv("RTCC_NO_GROUP");
    c->E.group_products = !(ngr && ngr[0] == '1');
    const char* swg = std::getenv("RTCC_SPLIT_WG");
    if (swg && swg[0]) c->E.split_wg = std::atoi(swg);
    const char* gwg = std::getenv("RTCC_GROUP_WG");
    if (gwg && gwg[0]) c->E.group_wg = std::atoi(gwg);
    RTCC_CHECK(c->E.split_wg >= 1 && c->E.group_wg >= 1, kEInval, "RTCC_SPLIT_WG and RTCC_GROUP_WG must be positive");
    const char* tb = std::getenv("RTCC_TILE_BAND");
    if (tb && tb[0]) c->E.tile_band = std::atoi(tb);
    RTCC_CHECK(c->E.tile_band >= 1 && c->E.tile_band <= 64, kEInval, "RTCC_TILE_BAND must be 1 to 64");
    const char* tr = std::getenv("RTCC_TRACE");
    c->E.trace = tr && tr[0] == '1';
    const char* nbr = std::getenv("RTCC_NO_BRANCH");
    const bool branches = !(nbr && nbr[0] == '1');
    const int64_t n = c->n, nn = n * n, n4 = nn * nn;
    for (int64_t i = 0; i < nn; ++i)
      RTCC_CHECK(std::isfinite(fock[i]) && std::isfinite(dipole[i]) && std::isfinite(dipole[nn + i]) &&
                     std::isfinite(dipole[2 * nn + i]),
                 kEInval, "rtcc_init: non-finite Fock or dipole integrals");
    c->f0 = c->arena.alloc<double>(nn);
    c->mu = c->arena.alloc<double>(3 * nn);
    c->fdiag = c->arena.alloc<double>(n);
    c->mu_ref_dev = c->arena.alloc<double>(3);
    std::vector<double> diag(n);
    for (int i = 0; i < n; ++i) diag[i] = fock[i * n + i];
    for (int a = 0; a < 3; ++a) {
      c->mu_ref[a] = 0;
      for (int i = 0; i < o; ++i) c->mu_ref[a] += 2.0 * dipole[a * nn + i * n + i];
    }
    RTCC_HIP(hipMemcpy(c->f0, fock, nn * sizeof(double), hipMemcpyHostToDevice));
    RTCC_HIP(hipMemcpy(c->mu, dipole, 3 * nn * sizeof(double), hipMemcpyHostToDevice));
    RTCC_HIP(hipMemcpy(c->fdiag, diag.data(), n * sizeof(double), hipMemcpyHostToDevice));
    RTCC_HIP(hipMemcpy(c->mu_ref_dev, c->mu_ref, 3 * sizeof(double), hipMemcpyHostToDevice));
    double* eri_dev = nullptr;
    RTCC_HIP(hipMalloc(&eri_dev, n4 * sizeof(double)));
    std::unique_ptr<double, void (*)(double*)> guard(eri_dev, [](double* p) { (void)hipFree(p); });
    RTCC_HIP(hipMemcpy(eri_dev, eri, n4 * sizeof(double), hipMemcpyHostToDevice));
    // scratch: largest permuted operand or temporary output, twice, plus split-K partials
    int64_t big = std::max<int64_t>({(int64_t)o * v * v * v, 2 * c->n2, (int64_t)o * o * o * o, c->n2 * 2});
    c->E.scratch.cap = (size_t)(8 * big + (1 << 22)) * sizeof(double) * 2;
    c->E.scratch.base = c->arena.alloc<char>(c->E.scratch.cap);
    // per-call memo arenas (as large as the scratch) for the main and branch engines
    for (int k = 0; k < 3; ++k) {
      c->memo[k].cap = c->E.scratch.cap;
      c->memo[k].base = c->arena.alloc<char>(c->memo[k].cap);
    }
    c->E.memo = &c->memo[0];
    const char* dov = std::getenv("RTCC_DIPOLE_OVERLAP");
    c->dip_overlap = !(dov && dov[0] == '0');
    if (branches) {
      RTCC_HIP(hipStreamCreateWithFlags(&c->ED.stream, hipStreamNonBlocking));
      RTCC_HIP(hipEventCreateWithFlags(&c->ev_dfork, hipEventDisableTiming));
      RTCC_HIP(hipEventCreateWithFlags(&c->ev_djoin, hipEventDisableTiming));
      c->ED.scratch.cap = c->E.scratch.cap;
      c->ED.scratch.base = c->arena.alloc<char>(c->ED.scratch.cap);
      c->red_d = c->arena.alloc<double>(2 * 1024);
      RTCC_HIP(hipEventCreateWithFlags(&c->E.ev_fork, hipEventDisableTiming));
      for (int k = 0; k < 2; ++k) {
        Engine& b = c->EB[k];
        RTCC_HIP(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
        RTCC_HIP(hipEventCreateWithFlags(&c->E.ev_join[k], hipEventDisableTiming));
        b.scratch.cap = c->E.scratch.cap;
        b.scratch.base = c->arena.alloc<char>(b.scratch.cap);
        b.memo = &c->memo[1 + k];
        c->E.br[k] = &b;
      }
    }
    build_ints<double>(c->E, c->arena, o, v, eri_dev, c->I64);
    build_work<double>(c->arena, o, v, c->W64);
    if (precision != RTCC_FP64) ensure32(c.get(), eri_dev);
    c->k.resize(6);
    for (auto& p : c->k) p = c->arena.alloc<double>(2 * c->nstate);
    c->ytmp = c->arena.alloc<double>(2 * c->nstate);
    c->y4 = c->arena.alloc<double>(2 * c->nstate);
    c->y5 = c->arena.alloc<double>(2 * c->nstate);
    c->tdev = c->arena.alloc<double>(1);
    c->mu_slot = c->arena.alloc<double>(6);
    c->gslot = c->arena.alloc<double>(2);
    c->red = c->arena.alloc<double>(2 * 1024);
    c->redout = c->arena.alloc<double>(64);
    RTCC_HIP(hipHostMalloc((void**)&c->host_pinned, 64 * sizeof(double), hipHostMallocDefault));
    RTCC_HIP(hipStreamSynchronize(c->stream));
  });
  if (st != RTCC_OK) {
    const_cache_destroy(c->E.cache);
    c->E.cache = nullptr;
    for (int k = 0; k < 2; ++k) {
      if (c->EB[k].stream) (void)hipStreamDestroy(c->EB[k].stream);
      if (c->E.ev_join[k]) (void)hipEventDestroy(c->E.ev_join[k]);
    }
    if (c->E.ev_fork) (void)hipEventDestroy(c->E.ev_fork);
    if (c->ED.stream) (void)hipStreamDestroy(c->ED.stream);
    if (c->ev_dfork) (void)hipEventDestroy(c->ev_dfork);
    if (c->ev_djoin) (void)hipEventDestroy(c->ev_djoin);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->e_in) (void)hipEventDestroy(c->e_in);
    if (c->e_out) (void)hipEventDestroy(c->e_out);
    return st;
  }
  *out = c.release();
  return RTCC_OK;
}

int rtcc_set_precision(rtcc_ctx* c, int precision) {
  if (!c) return RTCC_EINVAL;
  if (precision != RTCC_FP64 && precision != RTCC_FP32 && precision != RTCC_BF16X3) {
    c->err = "rtcc_set_precision: unknown precision";
    return RTCC_EINVAL;
  }
  if (precision != RTCC_FP64 && !c->have32) {
    c->err = "rtcc_set_precision: context was created without FP32 integrals; create it with RTCC_FP32 or "
             "RTCC_BF16X3";
    return RTCC_EINVAL;
  }
  c->precision = precision;
  return RTCC_OK;
}

int rtcc_rhs(rtcc_ctx* c, const void* y, double t, const double E[3], void* dydt) {
  if (!c) return RTCC_EINVAL;
  if (!y || !dydt || !E || y == dydt || !std::isfinite(t) || !std::isfinite(E[0]) || !std::isfinite(E[1]) ||
      !std::isfinite(E[2])) {
    c->err = "rtcc_rhs: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] { rhs_any(c, y, E, dydt, 1.0); });
}

int rtcc_step_rk4(rtcc_ctx* c, void* y, double t, double h, const rtcc_field* field) {
  if (!c) return RTCC_EINVAL;
  if (!y || !std::isfinite(t) || !std::isfinite(h)) {
    c->err = "rtcc_step_rk4: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    scalar_update(c->stream, c->tdev, t, false);
    rk4_step(c, y, h, to_dev(field), nullptr);
  });
}

int rtcc_propagate_rk4(rtcc_ctx* c, void* y, double t0, double h, int nsteps, const rtcc_field* field,
                       double* mu_dev) {
  if (!c) return RTCC_EINVAL;
  if (!y || nsteps < 0 || !std::isfinite(t0) || !std::isfinite(h)) {
    c->err = "rtcc_propagate_rk4: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    scalar_update(c->stream, c->tdev, t0, false);
    const FieldDev fd = to_dev(field);
    // HIP cannot time events recorded inside a captured graph: profiling runs the eager launches
    const bool graph = c->use_graph && !c->prof;
    const bool guard = c->guard_limit > 0.0;
    // captured FP32 / split-BF16 steps compute the dipole of their start state beside the right-hand
    // sides; the final state's dipole follows the last step
    const bool overlap = graph && mu_dev && c->dip_overlap && c->precision != RTCC_FP64 && c->ED.stream;
    if (mu_dev && !overlap) dipole_dev(c, y, mu_dev);
    for (int s = 0; s < nsteps; ++s) {
      if (graph) {
        capture_step(c, y, h, field, mu_dev != nullptr, guard, overlap);
        RTCC_HIP(hipGraphLaunch(c->gexec, c->stream));
        if (mu_dev)
          RTCC_HIP(hipMemcpyAsync(mu_dev + 6 * (int64_t)(overlap ? s : s + 1), c->mu_slot, 6 * sizeof(double),
                                  hipMemcpyDeviceToDevice, c->stream));
      } else {
        rk4_step(c, y, h, fd, mu_dev ? mu_dev + 6 * (int64_t)(s + 1) : nullptr, guard);
      }
      if (guard && ((s + 1) % c->guard_every == 0 || s + 1 == nsteps)) guard_check(c, s + 1, t0 + (s + 1) * h);
    }
    if (overlap) dipole_dev(c, y, mu_dev + 6 * (int64_t)nsteps);
  });
}

int rtcc_set_guard(rtcc_ctx* c, double t2_limit, int check_every) {
  if (!c) return RTCC_EINVAL;
  if (std::isnan(t2_limit) || check_every < 1) {
    c->err = "rtcc_set_guard: invalid arguments";
    return RTCC_EINVAL;
  }
  c->guard_limit = t2_limit > 0.0 ? t2_limit : 0.0;
  c->guard_every = check_every;
  return RTCC_OK;
}

int rtcc_mixed_schedule(double t0, double t_end, double h1, double h2, const rtcc_field* field, int cap,
                        double* times, int* nsteps) {
  if (!nsteps || !std::isfinite(t0) || !std::isfinite(t_end) || !(t_end >= t0) || !(h1 > 0) || !(h2 > 0) ||
      !std::isfinite(h1) || !std::isfinite(h2) || (field && field->kind == 1 && !(field->sigma > 0)) ||
      (times && cap < 1)) {
    g_init_error = "rtcc_mixed_schedule: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(nullptr, [&] {
    const auto sch = mixed_schedule(t0, t_end, h1, h2, field);
    RTCC_CHECK(sch.size() < (size_t)INT32_MAX, kEInval, "rtcc_mixed_schedule: too many steps");
    *nsteps = (int)sch.size();
    if (times) {
      RTCC_CHECK((int64_t)sch.size() + 1 <= cap, kEInval, "rtcc_mixed_schedule: times[] too short");
      times[0] = t0;
      for (size_t k = 0; k < sch.size(); ++k) times[k + 1] = k + 1 < sch.size() ? sch[k + 1].first : t_end;
    }
  });
}

int rtcc_propagate_rk4_mixed(rtcc_ctx* c, void* y, double t0, double t_end, double h1, double h2,
                             const rtcc_field* field, double* mu_dev, double* t2norm_dev) {
  if (!c) return RTCC_EINVAL;
  if (!y || !std::isfinite(t0) || !std::isfinite(t_end) || !(t_end >= t0) || !(h1 > 0) || !(h2 > 0) ||
      !std::isfinite(h1) || !std::isfinite(h2) || (field && field->kind == 1 && !(field->sigma > 0))) {
    c->err = "rtcc_propagate_rk4_mixed: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    const auto sch = mixed_schedule(t0, t_end, h1, h2, field);
    const int64_t ns = (int64_t)sch.size();
    const FieldDev fd = to_dev(field);
    const bool graph = c->use_graph && !c->prof;
    const bool guard = c->guard_limit > 0.0 || t2norm_dev != nullptr;
    if (mu_dev) dipole_dev(c, y, mu_dev);
    if (t2norm_dev) {
      guard_dev(c, y);
      RTCC_HIP(hipMemcpyAsync(t2norm_dev, c->gslot, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    for (int64_t s = 0; s < ns; ++s) {
      const double ts = sch[s].first, h = sch[s].second;
      scalar_update(c->stream, c->tdev, ts, false);  // exact start time of every step
      if (graph) {
        capture_step(c, y, h, field, mu_dev != nullptr, guard);
        RTCC_HIP(hipGraphLaunch(c->gexec, c->stream));
        if (mu_dev)
          RTCC_HIP(hipMemcpyAsync(mu_dev + 6 * (s + 1), c->mu_slot, 6 * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
      } else {
        rk4_step(c, y, h, fd, mu_dev ? mu_dev + 6 * (s + 1) : nullptr, guard);
      }
      if (t2norm_dev)
        RTCC_HIP(hipMemcpyAsync(t2norm_dev + s + 1, c->gslot, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      if (c->guard_limit > 0.0 && ((s + 1) % c->guard_every == 0 || s + 1 == ns)) guard_check(c, s + 1, ts + h);
    }
  });
}

int rtcc_propagate_cashkarp(rtcc_ctx* c, void* y, double t0, double t_end, double h0, double eps,
                            const rtcc_field* field, int max_trials, int cap, double* t_out, double* mu_out,
                            int* naccepted, int* nrejected, double* h_next) {
  if (!c) return RTCC_EINVAL;
  if (!y || !std::isfinite(t0) || !std::isfinite(t_end) || !(t_end >= t0) || !(h0 > 0) || !std::isfinite(h0) ||
      !(eps > 0) || max_trials < 1 || ((t_out || mu_out) && cap < 1) || !naccepted || !nrejected) {
    c->err = "rtcc_propagate_cashkarp: invalid arguments";
    return RTCC_EINVAL;
  }
  *naccepted = 0;
  *nrejected = 0;
  return guarded(c, [&] {
    rtcc_tableau T;
    builtin_tableau(RTCC_TAB_CASHKARP, T);
    propagate_embedded(c, y, t0, t_end, h0, eps, T, field, max_trials, cap, t_out, mu_out, naccepted, nrejected,
                       h_next, "rtcc_propagate_cashkarp");
  });
}

int rtcc_propagate_embedded(rtcc_ctx* c, void* y, double t0, double t_end, double h0, double eps,
                            const rtcc_tableau* tab, const rtcc_field* field, int max_trials, int cap,
                            double* t_out, double* mu_out, int* naccepted, int* nrejected, double* h_next) {
  if (!c) return RTCC_EINVAL;
  if (!y || !std::isfinite(t0) || !std::isfinite(t_end) || !(t_end >= t0) || !(h0 > 0) || !std::isfinite(h0) ||
      !(eps > 0) || max_trials < 1 || ((t_out || mu_out) && cap < 1) || !naccepted || !nrejected || !tab) {
    c->err = "rtcc_propagate_embedded: invalid arguments";
    return RTCC_EINVAL;
  }
  *naccepted = 0;
  *nrejected = 0;
  return guarded(c, [&] {
    check_tab(tab, true, "rtcc_propagate_embedded");
    propagate_embedded(c, y, t0, t_end, h0, eps, *tab, field, max_trials, cap, t_out, mu_out, naccepted,
                       nrejected, h_next, "rtcc_propagate_embedded");
  });
}

int rtcc_tableau_builtin(int id, rtcc_tableau* out) {
  if (!out) {
    g_init_error = "rtcc_tableau_builtin: out is NULL";
    return RTCC_EINVAL;
  }
  return guarded(nullptr, [&] { builtin_tableau(id, *out); });
}

int rtcc_step_tableau(rtcc_ctx* c, void* y, double t, double h, const rtcc_tableau* tab, const rtcc_field* field,
                      double tol, int max_iter, double* delta, int* sweeps) {
  if (!c) return RTCC_EINVAL;
  if (!y || !tab || !std::isfinite(t) || !std::isfinite(h)) {
    c->err = "rtcc_step_tableau: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    check_tab(tab, false, "rtcc_step_tableau");
    const FieldDev fd = to_dev(field);
    const rtcc_tableau& T = *tab;
    if (!tab_explicit(T)) {
      RTCC_CHECK(tol > 0 && std::isfinite(tol) && max_iter >= 1, kEInval,
                 "rtcc_step_tableau: implicit tableaux need tol > 0 and max_iter >= 1");
      const int it = implicit_step(c, y, t, h, T, fd, tol, max_iter);
      if (sweeps) *sweeps = it;
      return;
    }
    scalar_update(c->stream, c->tdev, t, false);
    explicit_stages(c, y, h, T, fd);
    const void* ks[RTCC_MAX_STAGES];
    double cb[RTCC_MAX_STAGES], ce[RTCC_MAX_STAGES];
    for (int j = 0; j < T.stages; ++j) {
      ks[j] = c->k[j];
      cb[j] = h * T.b[j];
      ce[j] = h * T.b_err[j];
    }
    const bool est = T.err_order > 0 && delta;
    if (est) state_combo(c->stream, c->nstate, y, T.stages, ks, ce, c->y4);
    state_combo(c->stream, c->nstate, y, T.stages, ks, cb, y);
    if (est) {
      max_abs_diff(c->stream, c->nstate, y, c->y4, c->red, c->redout);
      double d[2];
      sync_read(c, c->redout, d, 2);
      *delta = d[0];
    }
    if (sweeps) *sweeps = 1;
  });
}

int rtcc_propagate_batch(rtcc_ctx* const* ctxs, int nsys, const int* nprop, void* const* ys,
                         const rtcc_field* fields, double t0, double h, int nsteps, double* const* mu_dev) {
  if (!ctxs || nsys < 1 || !ctxs[0]) {
    g_init_error = "rtcc_propagate_batch: no contexts";
    return RTCC_EINVAL;
  }
  rtcc_ctx* c0 = ctxs[0];
  auto bad = [&](const char* why) {
    c0->err = std::string("rtcc_propagate_batch: ") + why;
    return RTCC_EINVAL;
  };
  if (nsys > kMaxBatchSystems) return bad("too many systems");
  if (!nprop || !ys || !fields || nsteps < 0 || !std::isfinite(t0) || !std::isfinite(h)) return bad("invalid arguments");
  int total = 0;
  for (int s = 0; s < nsys; ++s) {
    if (!ctxs[s] || !ys[s]) return bad("null context or state");
    for (int r = 0; r < s; ++r)
      if (ctxs[r] == ctxs[s]) return bad("a context appears twice");
    if (nprop[s] < 1 || nprop[s] > kMaxBatchMembers) return bad("members per system out of range");
    total += nprop[s];
  }
  for (int m = 0; m < total; ++m) {
    const rtcc_field& f = fields[m];
    if (f.kind < 0 || f.kind > 2 || !std::isfinite(f.E0) || !std::isfinite(f.omega) || !std::isfinite(f.t0) ||
        !std::isfinite(f.n[0]) || !std::isfinite(f.n[1]) || !std::isfinite(f.n[2]) ||
        (f.kind == 1 && !(f.sigma > 0)))
      return bad("invalid field");
  }
  return guarded(c0, [&] {
    bool dip[kMaxBatchSystems];
    bool profiling = false;
    int off = 0;
    for (int s = 0; s < nsys; ++s) {
      rtcc_ctx* c = ctxs[s];
      ensure_batch(c, nprop[s]);
      BatchWS& B = *c->batch;
      for (int m = 0; m < nprop[s]; ++m) B.fhost[m] = to_dev(&fields[off + m]);
      off += nprop[s];
      upload_fields(c0->stream, B.fhost.data(), nprop[s], B.fdev);
      dip[s] = mu_dev && mu_dev[s];
      B.E.mark = c->E.mark;  // kernel timing of a profiling context
      B.E.mark_user = c;
      B.E.mark_mode = c->E.mark_mode;
      if (c->prof) profiling = true;
    }
    // initial time and dipoles on every system's stream
    batch_fork(ctxs, nsys);
    for (int s = 0; s < nsys; ++s) {
      rtcc_ctx* c = ctxs[s];
      scalar_update(c->stream, c->batch->tdev, t0, false);
      if (dip[s]) dipole_batch_dev(c, ys[s], mu_dev[s]);
    }
    // HIP cannot time events recorded inside a captured graph: profiling runs the eager launches. A
    // batch with an FP64 system also runs them: a captured FP64 batch step once ended its process in
    // a re-capture (with a since-removed change to the density) and no cause was shown, so that path
    // stays unused until one is.
    bool fp64 = false;
    for (int s = 0; s < nsys; ++s) fp64 |= ctxs[s]->precision == RTCC_FP64;
    if (!c0->use_graph || profiling || fp64) {
      for (int st = 0; st < nsteps; ++st)
        for (int s = 0; s < nsys; ++s)
          rk4_step_batch(ctxs[s], ys[s], h, dip[s] ? mu_dev[s] + (int64_t)6 * nprop[s] * (st + 1) : nullptr);
      batch_join(ctxs, nsys);
      return;
    }
    batch_join(ctxs, nsys);
    for (int st = 0; st < nsteps; ++st) {
      capture_batch(ctxs, nsys, ys, h, dip);
      RTCC_HIP(hipGraphLaunch(c0->bexec, c0->stream));
      for (int s = 0; s < nsys; ++s)
        if (dip[s])
          RTCC_HIP(hipMemcpyAsync(mu_dev[s] + (int64_t)6 * nprop[s] * (st + 1), ctxs[s]->batch->mu_slot,
                                  6 * nprop[s] * sizeof(double), hipMemcpyDeviceToDevice, c0->stream));
    }
  });
}

int rtcc_rhs_vjp(rtcc_ctx* c, const void* y, double t, const double E[3], const void* ybar, void* ybar_out,
                 double Ebar[3]) {
  if (!c) return RTCC_EINVAL;
  if (!y || !E || !ybar || !ybar_out || ybar_out == ybar || ybar_out == y || !std::isfinite(t) ||
      !std::isfinite(E[0]) || !std::isfinite(E[1]) || !std::isfinite(E[2])) {
    c->err = "rtcc_rhs_vjp: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    ensure_adj(c);
    FieldDev fd{};
    fd.kind = kFieldConstant;
    for (int a = 0; a < 3; ++a) fd.n[a] = E[a];
    set_adj_field(c, fd, t);
    rhs_vjp_dev(c, y, 0.0, ybar, ybar_out);
    if (Ebar) {
      // dF/dE_a = -F[mu_a, 0](y)
      for (int a = 0; a < 3; ++a) {
        double m[3] = {0, 0, 0};
        m[a] = 1.0;
        one_body_rhs(c, y, m, c->abuf[2], false);
        vdot(c->stream, c->nstate, ybar, c->abuf[2], c->red, c->redout + 40 + 2 * a);
      }
      double d[6];
      sync_read(c, c->redout + 40, d, 6);
      for (int a = 0; a < 3; ++a) Ebar[a] = -d[2 * a];
    }
  });
}

int rtcc_dipole_vjp(rtcc_ctx* c, const void* y, const double mubar[6], void* ybar) {
  if (!c) return RTCC_EINVAL;
  if (!y || !mubar || !ybar || ybar == y) {
    c->err = "rtcc_dipole_vjp: invalid arguments";
    return RTCC_EINVAL;
  }
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(mubar[i])) {
      c->err = "rtcc_dipole_vjp: non-finite cotangent";
      return RTCC_EINVAL;
    }
  return guarded(c, [&] {
    ensure_adj(c);
    // mu_a = mu_ref_a + L[mu_a, 0](y), so its bilinear gradient is S_hat^-1 F[mu_a, 0](y). With
    // g_a = mubar_a: ybar += sum_a conj(S_hat^-1 F[mu_a, 0]) g_a = conj(S_hat^-1 F[sum_a conj(g_a) mu_a, 0]),
    // F linear in the operator: F[Re c . mu] + i F[Im c . mu] with c = conj(g).
    const double mr[3] = {mubar[0], mubar[2], mubar[4]}, mi[3] = {-mubar[1], -mubar[3], -mubar[5]};
    one_body_rhs(c, y, mr, c->abuf[2], true);
    one_body_rhs(c, y, mi, c->abuf[3], true);
    const double ci[2] = {0.0, 1.0};
    hamil_apply(c->stream, c->o, c->v, c->abuf[2], c->abuf[3], ci, true, false, true, 1.0, true, ybar);
  });
}

int rtcc_step_rk4_vjp(rtcc_ctx* c, const void* y, double t, double h, const rtcc_field* field, void* ybar,
                      double pbar[4]) {
  if (!c) return RTCC_EINVAL;
  if (!y || !ybar || ybar == y || !std::isfinite(t) || !std::isfinite(h)) {
    c->err = "rtcc_step_rk4_vjp: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    ensure_adj(c);
    const FieldDev fd = to_dev(field);
    const bool pulse = fd.kind == 1;
    hipStream_t st = c->stream;
    const int64_t nst = c->nstate;
    // stage states of the step (recomputed): Y1 = y, Y2, Y3, Y4
    void* Ys[4] = {const_cast<void*>(y), c->y4, c->y5, c->ytmp};
    scalar_update(st, c->tdev, t, false);
    for (int s = 0; s < 3; ++s) {
      rhs_t(c, Ys[s], fd, kRk4C[s] * h, c->k[s]);
      const void* ks[1] = {c->k[s]};
      double cs[1] = {h * kRk4A[s + 1][s]};
      state_combo(st, nst, y, 1, ks, cs, Ys[s + 1]);
    }
    // reverse sweep: kbar_s = h b_s ybar + h a_{s+1,s} g_{s+1}, g_s = J_s^H kbar_s, ybar += sum_s g_s
    void* yb0 = c->k[5];
    void* kbar = c->k[4];
    void* g = c->k[3];
    void* Fn = c->k[0];
    RTCC_HIP(hipMemcpyAsync(yb0, ybar, nst * sizeof(double2), hipMemcpyDeviceToDevice, st));
    set_adj_field(c, fd, t);
    for (int s = 3; s >= 0; --s) {
      const void* ks[2] = {yb0, g};
      double cs[2] = {h * kRk4B[s], s < 3 ? h * kRk4A[s + 1][s] : 0.0};
      state_combo(st, nst, nullptr, 2, ks, cs, kbar);
      if (pulse) {
        one_body_rhs(c, Ys[s], fd.n, Fn, false);
        vdot(st, nst, kbar, Fn, c->red, c->redout + 48 + 2 * s);
      }
      rhs_vjp_dev(c, Ys[s], kRk4C[s] * h, kbar, g);
      const void* kg[1] = {g};
      double one[1] = {1.0};
      state_combo(st, nst, ybar, 1, kg, one, ybar);
    }
    if (pulse && pbar) {
      double d[8];
      sync_read(c, c->redout + 48, d, 8);
      for (int s = 0; s < 4; ++s) {
        double gp[4];
        pulse_grad(fd, t + kRk4C[s] * h, gp);
        for (int j = 0; j < 4; ++j) pbar[j] -= gp[j] * d[2 * s];
      }
    }
  });
}

int rtcc_step_cashkarp(rtcc_ctx* c, void* y, double* t, double* h, double eps, const rtcc_field* field,
                       int* accepted, double* delta) {
  if (!c) return RTCC_EINVAL;
  if (!y || !t || !h || !accepted || !(eps > 0) || !std::isfinite(*t) || !std::isfinite(*h) || !(*h > 0)) {
    c->err = "rtcc_step_cashkarp: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    const double hh = *h;
    rtcc_tableau T;
    builtin_tableau(RTCC_TAB_CASHKARP, T);
    const double dl = emb_trial(c, y, *t, hh, T, to_dev(field), nullptr);
    if (delta) *delta = dl;
    RTCC_CHECK(std::isfinite(dl), kENonFinite, "rtcc_step_cashkarp: non-finite error estimate");
    const double fac = ctl_factor(eps, dl, T.err_order);
    if (dl <= eps) {
      RTCC_HIP(hipMemcpyAsync(y, c->y5, c->nstate * 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      *t += hh;
      *accepted = 1;
    } else {
      *accepted = 0;
    }
    *h = hh * fac;
  });
}

int rtcc_dipole_dev(rtcc_ctx* c, const void* y, double* mu_dev) {
  if (!c) return RTCC_EINVAL;
  if (!y || !mu_dev) {
    c->err = "rtcc_dipole_dev: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] { dipole_dev(c, y, mu_dev); });
}

int rtcc_dipole(rtcc_ctx* c, const void* y, double mu[6]) {
  if (!c) return RTCC_EINVAL;
  if (!y || !mu) {
    c->err = "rtcc_dipole: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    dipole_dev(c, y, c->redout + 8);
    sync_read(c, c->redout + 8, mu, 6);
  });
}

int rtcc_kick(rtcc_ctx* c, void* y, double kappa, const double n[3]) {
  if (!c) return RTCC_EINVAL;
  if (!y || !n || !std::isfinite(kappa) || !std::isfinite(n[0]) || !std::isfinite(n[1]) || !std::isfinite(n[2])) {
    c->err = "rtcc_kick: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    // dy/ds = -kappa * F_m(y), F_m the right-hand side of m = n.mu alone: f <- n.mu (s0 = 0, E = -n)
    const int nsub = 100;
    const double hs = 1.0 / nsub;
    const double E[3] = {-n[0], -n[1], -n[2]};
    for (int it = 0; it < nsub; ++it) {
      for (int s = 0; s < 4; ++s) {
        const void* ys = y;
        if (s > 0) {
          const void* ks[3] = {c->k[0], c->k[1], c->k[2]};
          double cs[3] = {hs * kRk4A[s][0], hs * kRk4A[s][1], hs * kRk4A[s][2]};
          state_combo(c->stream, c->nstate, y, s, ks, cs, c->ytmp);
          ys = c->ytmp;
        }
        eval_rhs<double>(c, c->I64, c->W64, ys, E, 0.0, false, c->k[s], -kappa);
      }
      const void* ks[4] = {c->k[0], c->k[1], c->k[2], c->k[3]};
      double cs[4] = {hs * kRk4B[0], hs * kRk4B[1], hs * kRk4B[2], hs * kRk4B[3]};
      state_combo(c->stream, c->nstate, y, 4, ks, cs, y);
    }
  });
}

int rtcc_check_state(rtcc_ctx* c, const void* y, int64_t* nonfinite) {
  if (!c) return RTCC_EINVAL;
  if (!y || !nonfinite) {
    c->err = "rtcc_check_state: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    count_nonfinite(c->stream, c->nstate, y, c->red, c->redout);
    double d[2];
    sync_read(c, c->redout, d, 2);
    *nonfinite = (int64_t)d[0];
  });
}

int rtcc_ground_state(rtcc_ctx* c, void* y, double tol, int maxiter, double* e_corr) {
  if (!c) return RTCC_EINVAL;
  if (!y || !(tol > 0) || maxiter < 1) {
    c->err = "rtcc_ground_state: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(c, [&] {
    Work<double>& w = c->W64;
    const double E0[3] = {0, 0, 0};
    field_fock<double>(c->stream, c->n, c->f0, c->mu, E0, 1.0, w.f.re);
    const int64_t nsub = c->n1 + c->n2;
    const int kmax = 8;
    if (c->diis_x.empty()) {
      for (int i = 0; i < kmax; ++i) {
        c->diis_x.push_back(c->arena.alloc<double>(2 * nsub));
        c->diis_e.push_back(c->arena.alloc<double>(2 * nsub));
      }
      c->diis_err = c->arena.alloc<double>(2 * nsub);
    }
    double2* ybase = (double2*)y;
    for (int phase = 0; phase < 2; ++phase) {
      double2* x = ybase + phase * nsub;  // T part, then Lambda part
      if (phase == 1)
        RTCC_HIP(hipMemcpyAsync(x, ybase, nsub * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
      int count = 0, head = 0;
      bool conv = false;
      for (int it = 0; it < maxiter; ++it) {
        unpack_state<double>(c->stream, y, c->o, c->v, planes(w, true));
        residuals<double>(c->E, c->I64, w, true, phase == 1);
        const Ten<double>& r1 = phase ? w.S1 : w.R1;
        const Ten<double>& r2 = phase ? w.S2 : w.R2;
        maxabs_planar<double>(c->stream, c->n1, r1.re, r1.im, c->red, c->redout);
        maxabs_planar<double>(c->stream, c->n2, r2.re, r2.im, c->red + 1024, c->redout + 2);
        double m[4];
        sync_read(c, c->redout, m, 4);
        RTCC_CHECK(std::isfinite(m[0]) && std::isfinite(m[2]), kENonFinite, "ground state: non-finite residual");
        if (std::max(m[0], m[2]) <= tol) {
          conv = true;
          break;
        }
        double2* e = (double2*)c->diis_err;
        jacobi_update<double>(c->stream, c->o, c->v, c->fdiag, r1.re, r2.re, x, x + c->n1, e, e + c->n1);
        // DIIS on the updated vectors with the Jacobi steps as error vectors
        RTCC_HIP(hipMemcpyAsync(c->diis_x[head], x, nsub * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
        RTCC_HIP(hipMemcpyAsync(c->diis_e[head], e, nsub * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
        head = (head + 1) % kmax;
        count = std::min(count + 1, kmax);
        if (count >= 2) {
          std::vector<double> B((count + 1) * (count + 1), 0.0), rhsv(count + 1, 0.0);
          for (int i = 0; i < count; ++i)
            for (int j = i; j < count; ++j) {
              vdot(c->stream, nsub, c->diis_e[i], c->diis_e[j], c->red, c->redout + 16);
              double d[2];
              sync_read(c, c->redout + 16, d, 2);
              B[i * (count + 1) + j] = B[j * (count + 1) + i] = d[0];
            }
          for (int i = 0; i < count; ++i) {
            B[i * (count + 1) + count] = B[count * (count + 1) + i] = -1.0;
          }
          rhsv[count] = -1.0;
          if (solve_small(B, rhsv, count + 1)) {
            std::vector<const void*> ks(c->diis_x.begin(), c->diis_x.begin() + count);
            state_combo(c->stream, nsub, nullptr, count, ks.data(), rhsv.data(), x);
          }
        }
      }
      RTCC_CHECK(conv, kENotConv, phase == 0 ? "ground state: T equations did not converge"
                                             : "ground state: Lambda equations did not converge");
    }
    if (e_corr) {
      // E = 2 sum f_ia t_ia + sum_ijab L_ijab tau_ijab
      unpack_state<double>(c->stream, y, c->o, c->v, planes(w, true));
      Ten<double> s = make_ten<double>(c->redout + 32, c->redout + 33, {});
      padd<double>(c->E, 1, "ijab->ijab", w.t2, w.tau, 0);
      ein<double>(c->E, 1, "ia,jb->ijab", w.t1, w.t1, w.tau, 1);
      ein<double>(c->E, 2, "ia,ia->", w.fov, w.t1, s, 0);
      ein<double>(c->E, 1, "ijab,ijab->", c->I64.Loovv, w.tau, s, 1);
      double d[2];
      sync_read(c, c->redout + 32, d, 2);
      *e_corr = d[0];
    }
  });
}

int rtcc_profile(rtcc_ctx* c, int enable) {
  if (!c || enable < 0 || enable > 2) return RTCC_EINVAL;
  return guarded(c, [&] {
    if (c->ev.empty()) {
      c->ev.resize(1024);
      for (auto& e : c->ev) RTCC_HIP(hipEventCreate(&e));
    }
    if (enable) {
      prof_flush(c);
      c->prof_launches = 0;
      c->prof_ms = 0.0;
      c->prof_flops = 0.0;
      c->prof_bytes = 0.0;
    }
    c->prof = enable != 0;
    c->E.mark = enable ? prof_mark : nullptr;
    c->E.mark_user = c;
    if (enable) c->E.mark_mode = enable;
  });
}

int rtcc_profile_read(rtcc_ctx* c, int64_t* launches, double* total_ms, double* flops_per_launch,
                      double* bytes_per_launch) {
  if (!c || !launches || !total_ms || !flops_per_launch) return RTCC_EINVAL;
  return guarded(c, [&] {
    prof_flush(c);
    *launches = c->prof_launches;
    *total_ms = c->prof_ms;
    *flops_per_launch = c->prof_launches ? c->prof_flops / (double)c->prof_launches : 0.0;
    if (bytes_per_launch) *bytes_per_launch = c->prof_launches ? c->prof_bytes / (double)c->prof_launches : 0.0;
  });
}

int rtcc_info(rtcc_ctx* c, int64_t out[6]) {
  if (!c || !out) return RTCC_EINVAL;
  out[0] = c->o;
  out[1] = c->v;
  out[2] = c->nstate;
  out[3] = c->last_flops;
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  out[4] = (int64_t)(total_b - free_b);
  out[5] = c->precision;
  return RTCC_OK;
}

void rtcc_destroy(rtcc_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->batch) (void)hipDeviceSynchronize();  // batch buffers may be in use on another context's stream
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->bexec) (void)hipGraphExecDestroy(c->bexec);
  if (c->e_in) (void)hipEventDestroy(c->e_in);
  if (c->e_out) (void)hipEventDestroy(c->e_out);
  if (c->host_pinned) (void)hipHostFree(c->host_pinned);
  hipStream_t st = c->stream;
  ConstCache* cache = c->E.cache;
  hipStream_t bst[3] = {c->EB[0].stream, c->EB[1].stream, c->ED.stream};
  for (int k = 0; k < 3; ++k)
    if (bst[k]) (void)hipStreamSynchronize(bst[k]);
  for (int k = 0; k < 2; ++k)
    if (c->E.ev_join[k]) (void)hipEventDestroy(c->E.ev_join[k]);
  if (c->E.ev_fork) (void)hipEventDestroy(c->E.ev_fork);
  if (c->ev_dfork) (void)hipEventDestroy(c->ev_dfork);
  if (c->ev_djoin) (void)hipEventDestroy(c->ev_djoin);
  delete c;  // frees device memory first
  const_cache_destroy(cache);
  for (hipStream_t b : bst)
    if (b) (void)hipStreamDestroy(b);
  if (st) (void)hipStreamDestroy(st);
}

int rtcc_load_tuning(const char* path, int* nentries) {
  return guarded(nullptr, [&] {
    const int n = load_tuning(path);
    if (nentries) *nentries = n;
  });
}

int rtcc_gemm(int precision, int64_t M, int64_t N, int64_t K, double alpha, const void* a_re, const void* a_im,
              int64_t lda, int ta, const void* b_re, const void* b_im, int64_t ldb, int tb, double beta, void* c_re,
              void* c_im, int64_t ldc, const int* choice, int reps, float* ms, void* hip_stream) {
  if ((precision != RTCC_FP64 && precision != RTCC_FP32 && precision != RTCC_BF16X3) || M < 1 || N < 1 || K < 1 ||
      !a_re || !b_re || !c_re || ((a_im || b_im) && !c_im) || reps < 0 || (reps > 0 && !ms) ||
      lda < (ta ? M : K) || ldb < (tb ? K : N) || ldc < N || !std::isfinite(alpha) || !std::isfinite(beta)) {
    g_init_error = "rtcc_gemm: invalid arguments";
    return RTCC_EINVAL;
  }
  return guarded(nullptr, [&] {
    Engine E;
    E.stream = (hipStream_t)hip_stream;
    E.bf16x3 = precision == RTCC_BF16X3;
    GemmChoice ch;
    if (choice) {
      ch.kind = choice[0];
      ch.p1 = choice[1];
      ch.p2 = choice[2];
      ch.splits = choice[3];
      RTCC_CHECK(ch.kind >= 0 && ch.kind <= 2, kEInval, "rtcc_gemm: unknown kernel kind");
      if (ch.kind != 0) E.force = &ch;
    }
    // scratch: split-BF16 packs of both operands plus the split-K partial planes (the library's own rules
    // keep splits x M x N within 2^24 elements: at most ~1024-2048 workgroups of <= 128 x 128 outputs)
    const size_t elt = precision == RTCC_FP64 ? 8 : 4;
    const size_t packs = 2 * 2 * 2 * ((size_t)(M + 256) + (size_t)(N + 256)) * (size_t)(K + 32);
    const size_t mn = (size_t)M * (size_t)N;
    const size_t nsplit = ch.kind != 0 ? (size_t)std::max(ch.splits, 1) : 0;
    const size_t parts = 2 * elt * (nsplit ? nsplit * mn : std::min<size_t>(64 * mn, (size_t)1 << 24));
    E.scratch.cap = packs + parts + ((size_t)1 << 24);
    RTCC_HIP(hipMalloc((void**)&E.scratch.base, E.scratch.cap));
    std::unique_ptr<char, void (*)(char*)> sguard(E.scratch.base, [](char* p) { (void)hipFree(p); });
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto run = [&] {
      E.scratch.reset();
      if (precision == RTCC_FP64) {
        GemmOp<double> A{(const double*)a_re, (const double*)a_im, lda, ta};
        GemmOp<double> B{(const double*)b_re, (const double*)b_im, ldb, tb};
        gemm<double>(E, M, N, K, alpha, A, B, (double*)c_re, (double*)c_im, ldc, beta);
      } else {
        GemmOp<float> A{(const float*)a_re, (const float*)a_im, lda, ta};
        GemmOp<float> B{(const float*)b_re, (const float*)b_im, ldb, tb};
        gemm<float>(E, M, N, K, alpha, A, B, (float*)c_re, (float*)c_im, ldc, beta);
      }
    };
    try {
      run();
      if (reps > 0) {
        RTCC_HIP(hipEventCreate(&ev[0]));
        RTCC_HIP(hipEventCreate(&ev[1]));
        RTCC_HIP(hipEventRecord(ev[0], E.stream));
        for (int r = 0; r < reps; ++r) run();
        RTCC_HIP(hipEventRecord(ev[1], E.stream));
        RTCC_HIP(hipEventSynchronize(ev[1]));
        float t = 0.f;
        RTCC_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
        *ms = t / reps;
      }
      RTCC_HIP(hipStreamSynchronize(E.stream));  // the scratch is freed on return
    } catch (...) {
      (void)hipStreamSynchronize(E.stream);
      for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
      throw;
    }
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  });
}

const char* rtcc_last_error(const rtcc_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
