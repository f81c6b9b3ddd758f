// Tensor views and the two-operand contraction engine.
//
// Every coupled-cluster term is evaluated as  C[c] = alpha * sum_k A[a] B[b] + beta * C[c]
// with index strings in einsum notation ("ijef,abef->ijab"). Contracted letters appear in A
// and B only; free letters of C come from exactly one operand. An operand whose memory
// layout already groups its letters as one matrix (row- or column-major) is passed to the
// MFMA GEMM as a strided view; otherwise it is permuted into scratch first. Complex
// tensors are planar: separate real and imaginary planes.
#pragma once
#include <functional>
#include <map>
#include <string>
#include <vector>
#include "common.h"

namespace rtcc {

constexpr int kMaxDim = 6;

template <typename T>
struct Ten {
  T* re = nullptr;
  T* im = nullptr;  // nullptr: real tensor
  int nd = 0;
  int64_t d[kMaxDim] = {0};
  int64_t s[kMaxDim] = {0};  // element strides
  // Batch stride: 0 for a tensor shared by every member of a batch (the integrals), else the
  // element offset between consecutive members (both planes of a complex tensor).
  int64_t bs = 0;
  // A constant operand (an integral block): permuted layouts of it are cached by the engine.
  bool konst = false;
  bool cplx() const { return im != nullptr; }
  int64_t size() const {
    int64_t n = 1;
    for (int i = 0; i < nd; ++i) n *= d[i];
    return n;
  }
};

// Row-major view of a (possibly complex) contiguous buffer.
template <typename T>
Ten<T> make_ten(T* re, T* im, std::initializer_list<int64_t> dims) {
  Ten<T> t;
  t.re = re;
  t.im = im;
  t.nd = (int)dims.size();
  int i = 0;
  for (auto x : dims) t.d[i++] = x;
  int64_t st = 1;
  for (int k = t.nd - 1; k >= 0; --k) {
    t.s[k] = st;
    st *= t.d[k];
  }
  return t;
}

// Bump allocator for per-call temporaries (device memory owned by the context).
struct Scratch {
  char* base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  template <typename T>
  T* get(int64_t n) {
    size_t bytes = ((size_t)n * sizeof(T) + 255) & ~(size_t)255;
    RTCC_CHECK(used + bytes <= cap, kENoMem, "contraction scratch exhausted");
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    if (used > peak) peak = used;
    return p;
  }
  void reset(size_t mark = 0) { used = mark; }
};

// Permuted copies of constant operands, made once and kept (shared by the engines of a context).
struct ConstCache;
ConstCache* const_cache_create();
void const_cache_destroy(ConstCache* c);
size_t const_cache_bytes(const ConstCache* c);
// The buffer cached under `key`; on a miss `bytes` are allocated and fill(buffer, stream) is run on
// the cache's own stream and waited for.
void* const_cache_get(ConstCache* c, const std::string& key, size_t bytes,
                      const std::function<void(void*, hipStream_t)>& fill);

// Per-call memo of derived layouts (permuted copies, split-BF16 packs) of operands that stay fixed
// during one right-hand side. memo_begin clears it and registers the fixed tensors' base pointers;
// memo_end clears and disables it. Entries live in a device arena owned by the context. An engine
// reads only its own memo, so every entry is written and read on that engine's stream.
struct Memo {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool on = false;
  std::vector<const void*> fixed;
  std::map<std::string, void*> entries;
};

// A GEMM kernel choice, the unit the tile autotuner picks per product shape. kind 0: the library's
// own rule; 1: the FP32/FP64 tile kernel with a p1 / 1000 x p1 % 1000 output tile, k stage p2 and
// `splits` K splits; 2: the split-BF16 kernel (FP32 operands) with p1 waves along N (2: 128 x 128
// tiles, 4: 128 x 256), `splits` K splits (0: its cost model) and variant p2 (0: the engine's, 1:
// register-staged, 2: direct-to-LDS ring, 3: the ring with 128 x 128 tiles, two workgroups per CU).
struct GemmChoice {
  int kind = 0, p1 = 0, p2 = 0, splits = 0;
};
// Precision tags of the tuning table: 0 FP64, 1 FP32, 2 split-BF16 contexts.
// The tuned choice for a product of that shape (kind 0 when the table has none).
GemmChoice tuned_choice(int prec, int64_t M, int64_t N, int64_t K, bool ac, bool bc, int ta, int tb);
// Replace the tuning table with the entries of a text file (one "prec M N K ac bc ta tb kind p1 p2 splits"
// per line, '#' starts a comment); path == nullptr clears it. Returns the number of entries.
int load_tuning(const char* path);

struct Engine {
  hipStream_t stream = nullptr;
  ConstCache* cache = nullptr;
  Memo* memo = nullptr;  // nullptr: no memo (batched and adjoint workspaces)
  Scratch scratch;
  int64_t gemm_flops = 0;  // algorithmic real flops issued (accounting)
  // optional hook called before (phase 0) and after (phase 1) a timed launch with the launch's
  // algorithmic real flops and bytes and the stream it is issued on; mark_mode selects the launches:
  // 1 the ladder GEMM(s); 2 every complex x complex product with 2 M N K >= bf16_min_flops (the ring and
  // Lambda products), the GEMM kernel alone -- in the split-BF16 context only its register-staged
  // 128 x 256 kernel (gemm_bf16x3_nt<1, 1, 0, 4>), the kernel with the largest share of the step
  void (*mark)(void*, int, double, double, hipStream_t) = nullptr;
  void* mark_user = nullptr;
  int mark_mode = 1;
  // 1 while the ladder GEMM is issued: the split-BF16 path then launches its kernel under a name of
  // its own; with mark_mode 1 every path calls `mark` around the GEMM kernel alone
  int ladder = 0;
  double ladder_flops = 0.0;  // algorithmic real flops of the last ladder GEMM
  bool trace = false;         // print every contraction's layout decisions to stderr
  bool bf16x3 = false;        // FP32 GEMMs above bf16_min_flops use the split-BF16 three-term kernel
  double bf16_min_flops = 5e8;
  // particle-particle ladder in its symmetric / antisymmetric form (two GEMMs over pair triangles);
  // false: one GEMM over the full o^2 x v^2 x v^2 product
  bool sym_ladder = true;
  bool ladder_lds = true;
  int pair_splits = 0;  // K splits of the paired split-BF16 ladder launch (0: the cost model; -1: no pairing)  // LDS-staged fold / unfold of the symmetric ladder (false: element kernels)
  int bf16_kernel = 1;  // split-BF16 kernel: 1 register-staged, 2 direct-to-LDS ring, 3 the ring at 2 per CU,
                        // 4 wide waves (64 x 128 per wave)
  bool use_tuning = true;               // consult the tuning table (single, non-batched products)
  bool group_products = true;           // ein_multi may issue independent products as one launch
  int split_wg = 160;                   // split-BF16 K splits: workgroup cap of a single product
  int group_wg = 256;                   // ... of a grouped launch
  int tile_band = 8;                    // split-BF16 tile map: output-tile rows per band
  const GemmChoice* force = nullptr;    // this choice for every product (kernel tests, the autotuner)
  // Batch size of the tensors with bs != 0. Every contraction then runs for all members: a
  // member index carried by one operand only becomes part of the GEMM's M or N (one fat GEMM
  // against the shared integrals); one carried by both becomes a batched GEMM.
  int nb = 1;
  // Optional branch engines (own stream and scratch): independent parts of the right-hand side run
  // on them concurrently between fork() and join().
  Engine* br[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[2] = {nullptr, nullptr};
};

void memo_begin(Engine& E, std::initializer_list<const void*> fixed);
void memo_end(Engine& E);
bool memo_fixed(const Engine& E, const void* p);
// The memo buffer for `key` (*hit: it already holds the data), or nullptr when the arena is full.
void* memo_get(Engine& E, const std::string& key, size_t bytes, bool* hit);

// Branch engines take this engine's settings and wait for the work already on its stream.
void fork_branches(Engine& E);
// This engine's stream waits for the branches; their flop counts are added to this engine's.
void join_branches(Engine& E);


// C = alpha * contraction(A, B) + beta * C   (beta 0 or 1)
template <typename T>
void ein(Engine& E, double alpha, const char* spec, const Ten<T>& A, const Ten<T>& B, const Ten<T>& C,
         double beta);

// One contraction of a group issued together (ein_multi).
template <typename T>
struct EinTerm {
  double alpha;
  const char* spec;
  const Ten<T>* A;
  const Ten<T>* B;
  const Ten<T>* C;
  double beta;
};
// Two or three independent contractions into distinct outputs, each a single GEMM for the split-BF16
// kernel (FP32 context with the split enabled, no member batch, 2 M N K >= bf16_min_flops, an output the
// GEMM writes in place, no tuning-table entry of its own, operands of one kind): operands permuted as ein
// would, then one launch (gemm_bf16x3_multi). Returns false, with nothing issued, when any term does not
// qualify; the caller then issues them one by one.
template <typename T>
bool ein_multi(Engine& E, const EinTerm<T>* terms, int n);

// C = alpha * permute(A) + beta * C   ("ijab->jiba"; the identity spec is an axpby)
template <typename T>
void padd(Engine& E, double alpha, const char* spec, const Ten<T>& A, const Ten<T>& C, double beta);

// Raw GEMM entry (used by the engine and directly for the shared ladder):
// C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n)
// A(m,k) = transA ? A[k*lda + m] : A[m*lda + k];  B(k,n) = transB ? B[n*ldb + k] : B[k*ldb + n]
template <typename T>
struct GemmOp {
  const T* re;
  const T* im;
  int64_t ld;
  int trans;
  bool konst = false;  // constant operand: derived layouts of it may be cached
};
// Batched form: `n` independent products, operand X of product z at X + z * (batch stride of X);
// a stride of 0 shares the operand.
struct GemmBatch {
  int n = 1;
  int64_t a = 0, b = 0, c = 0;
};
template <typename T>
void gemm(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<T> A, GemmOp<T> B, T* Cre, T* Cim,
          int64_t ldc, double beta, GemmBatch bt = GemmBatch());

// force_wn (2 or 4), force_splits (>= 1) and force_kernel (1 register-staged, 2 direct-to-LDS ring, 3 the
// ring with 128 x 128 tiles and two workgroups per CU) replace the library's own choices when non-zero.
bool gemm_bf16x3(Engine& E, int64_t M, int64_t N, int64_t K, double alpha, GemmOp<float> A, GemmOp<float> B,
                 float* Cre, float* Cim, int64_t ldc, double beta, int force_wn = 0, int force_splits = 0,
                 int force_kernel = 0);

// One product of a pair issued together (gemm_bf16x3_pair).
struct Bf16Job {
  int64_t M, N, K;
  double alpha;
  GemmOp<float> A, B;
  float* Cre;
  float* Cim;
  int64_t ldc;
  double beta;
};
// The two products in one launch of the register-staged split-BF16 kernel (workgroups of the first, then
// of the second; one K split for both from the cost model over their summed tiles), each then reduced on
// its own. For complex x real pairs (the symmetric / antisymmetric ladder, issued while E.ladder is set and
// marked as one ladder launch); returns false (nothing launched) for other operand kinds or when the
// context selects another split-BF16 kernel.
bool gemm_bf16x3_pair(Engine& E, const Bf16Job (&jobs)[2]);
// Two or three independent products of the same operand kinds (complex output) in one launch of the
// register-staged 128 x 256 kernel, with one K split for all from the cost model over their summed tiles
// (within one workgroup per CU), each then reduced on its own; returns false (nothing launched) for other
// operand kinds or when the context selects another split-BF16 kernel.
bool gemm_bf16x3_multi(Engine& E, const Bf16Job* jobs, int n);

// y(n) = alpha * sum_k x(k) W(k, n) + beta * y(n) for n < N, k < K, with x(k) at k * incx, y(n) at n * incy
// and W(k, n) at (k / K2) sk1 + (k % K2) sk2 + (n / N2) sn1 + (n % N2) sn2 (two-level indices: a
// matrix operand that no single row and column stride describes). Planar complex or real.
template <typename T>
void gemv_strided(Engine& E, int64_t N, int64_t K, double alpha, const T* xre, const T* xim, int64_t incx,
                  const T* wre, const T* wim, int64_t N2, int64_t sn1, int64_t sn2, int64_t K2, int64_t sk1,
                  int64_t sk2, T* yre, T* yim, int64_t incy, double beta);

// Sum `splits` partial planes P[s][m][n] (plane stride M * N) into C = alpha * sum + beta * C, in a
// fixed order; nbatch members (member z's planes start at z * splits * M * N, its C at Cre + z * sc).
template <typename T>
void splitk_reduce_launch(hipStream_t st, const T* Pre, const T* Pim, int splits, int64_t M, int64_t N, T* Cre,
                          T* Cim, int64_t ldc, int64_t sc, int nbatch, double alpha, double beta);

// General strided permute-axpby on planar complex or real data (nd <= 6).
template <typename T>
void permute_axpby(hipStream_t st, int nd, const int64_t* dims, const T* inre, const T* inim,
                   const int64_t* instr, T* outre, T* outim, const int64_t* outstr, double alpha, double beta);

}  // namespace rtcc
