/*
 * rtcc.h -- C ABI of the MI355X (gfx950) real-time CCSD propagation library.
 *
 * The library evaluates the time derivatives of the coupled-cluster amplitudes
 * (T1, T2) and Lambda amplitudes (L1, L2) of real-time CCSD under a dipole
 * field and integrates them with explicit Runge-Kutta methods, after
 * Wang, Peyton and Crawford, "Accelerating real-time coupled cluster methods
 * with single-precision arithmetic and adaptive numerical integration"
 * (arXiv 2205.05175):
 *   - equations of motion: Theory section, Eq. derivT (dt/dt = -i <mu|Hbar|0>)
 *     and Eq. derivL (dlambda/dt = +i <0|(1+Lambda)[Hbar, tau_mu]|0>), with
 *     Hbar = e^{-T} H e^{T} (Eq. simtranH);
 *   - field coupling: V(t) = -mu.E(t) (linear-absorption subsection), entering
 *     only through the Fock matrix f(t) = f - sum_a E_a(t) mu_a;
 *   - Gaussian pulse: Eq. field; Dirac-delta kick: E(t) = kappa delta(t) n;
 *   - integrators: Eqs. rk_y/rk_k (Table tab:butcher), RK4 (Eq. rk4truncation),
 *     Cash-Karp (Eqs. ck-k, ck-y) with the controller of Eqs. ck-h/ck-h-final;
 *   - dipole: Eq. dipole, mu_a = Tr(rho mu_a) with the unrelaxed density.
 *
 * Closed-shell variables. With o doubly occupied and v virtual spatial orbitals
 * (occupied first), the state y is complex128 (interleaved Re, Im), row-major:
 *     y = [ T1 (o*v) | T2 (o*o*v*v) | L1 (o*v) | L2 (o*o*v*v) ]
 * where T1[i,a] = t_{i alpha}^{a alpha}, T2[i,j,a,b] = t_{i alpha, j beta}^{a alpha, b beta}
 * (so T2[i,j,a,b] == T2[j,i,b,a]) and Lambda uses the same map.
 *
 * Ownership and streams. rtcc_init copies the integrals; the context owns its
 * device copies and workspaces until rtcc_destroy. State and output buffers
 * (y, dydt, mu_dev) are caller-owned DEVICE memory; the library keeps no pointer
 * to them after a call returns. Work is enqueued on the stream given to
 * rtcc_init and is asynchronous, except for calls that return host values
 * (rtcc_dipole, rtcc_step_cashkarp, rtcc_ground_state, rtcc_check_state), which
 * synchronise that stream. A context is used by one host thread at a time.
 *
 * Errors. Every call returns RTCC_OK (0) or a negative code; the message is
 * available from rtcc_last_error(ctx) (or rtcc_last_error(NULL) for a failed
 * rtcc_init). No call aborts or throws across the ABI.
 */
#ifndef RTCC_H
#define RTCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtcc_ctx rtcc_ctx;

/* Contraction precision. The RK state, the stage updates, the dipole and the
 * ground-state iterations are always FP64.
 *   RTCC_FP64   : FP64 operands, v_mfma_f64_16x16x4f64.
 *   RTCC_FP32   : complex FP32 operands, v_mfma_f32_16x16x4f32, FP32 accumulation.
 *   RTCC_BF16X3 : FP32 operands; every complex product of more than 5e8 flops splits each
 *                 element into two BF16 halves (hi = bf16(x), lo = bf16(x - hi)) and forms
 *                 hi*hi + hi*lo + lo*hi with v_mfma_f32_32x32x16_bf16, FP32 accumulation;
 *                 smaller products as RTCC_FP32 (the threshold can be overridden by the
 *                 environment variable RTCC_BF16_MIN_FLOPS, read by rtcc_init). Independent
 *                 products of one part of the right-hand side (the three l2s x t2
 *                 intermediates of each of the two Lambda1 groups, the three Y3
 *                 intermediates, the two ring-formation products) go out as one launch with
 *                 one K split for all; RTCC_NO_GROUP=1, read by rtcc_init, issues them one
 *                 by one.
 *                 K splits are chosen within a workgroup cap, 160 for a single product and 256
 *                 for a grouped launch (RTCC_SPLIT_WG, RTCC_GROUP_WG); workgroups walk the
 *                 output tiles in bands of 8 tile rows (RTCC_TILE_BAND, 1 to 64). */
enum { RTCC_FP64 = 0, RTCC_FP32 = 1, RTCC_BF16X3 = 2 };

enum {
  RTCC_OK = 0,
  RTCC_EINVAL = -1,     /* bad argument (sizes, null pointers, non-finite scalars) */
  RTCC_ENOMEM = -2,     /* device allocation or scratch exhausted */
  RTCC_EHIP = -3,       /* HIP runtime error */
  RTCC_ENONFINITE = -4, /* non-finite values in the state */
  RTCC_ENOTCONV = -5    /* ground-state iterations did not converge */
};

/* External field. kind 0: none. kind 1: Gaussian pulse of Eq. field,
 * E(t) = -E0 exp(-(t-t0)^2/(2 sigma^2)) cos(omega (t-t0)) n. kind 2: Dirac-delta
 * kick of strength E0 along n at t = 0 -- apply it with rtcc_kick; the stepping
 * functions treat kind 2 as field-free. n need not be normalised (it is used as given). */
typedef struct {
  int kind;
  double E0, omega, sigma, t0;
  double n[3];
} rtcc_field;

/* Create a context.
 *   o, v     : occupied / virtual spatial orbitals (o >= 1, v >= 1), n = o + v.
 *   eri      : HOST, n^4 doubles, chemists' order (pq|rs), row-major, real, 8-fold symmetric.
 *   fock     : HOST, n*n doubles, real symmetric Fock matrix (occupied orbitals first).
 *   dipole   : HOST, 3*n*n doubles, real symmetric dipole integrals (x, y, z).
 *   precision: RTCC_FP64, RTCC_FP32 or RTCC_BF16X3 (contractions of rtcc_rhs and the steppers);
 *              a context created with RTCC_FP32 or RTCC_BF16X3 can switch among all three.
 *   hip_stream: hipStream_t to run on (NULL = default stream).
 * All host arrays are copied; the caller may free them on return. */
int rtcc_init(rtcc_ctx** ctx, int o, int v, const double* eri, const double* fock, const double* dipole,
              int precision, void* hip_stream);

/* Switch the contraction precision of an existing context (allocates FP32 copies on first use). */
int rtcc_set_precision(rtcc_ctx* ctx, int precision);

/* dydt = ( -i R_T(y; f - E.mu), +i R_L(y; f - E.mu) ): the right-hand side of
 * Eqs. derivT/derivL at the field value E[3] (HOST). y, dydt: DEVICE, state layout above;
 * they must not overlap. t is the time label (unused by the operator itself). */
int rtcc_rhs(rtcc_ctx* ctx, const void* y, double t, const double E[3], void* dydt);

/* One classical RK4 step of size h from time t; y (DEVICE) is updated in place. */
int rtcc_step_rk4(rtcc_ctx* ctx, void* y, double t, double h, const rtcc_field* field);

/* nsteps RK4 steps of size h from t0. If mu_dev (DEVICE, (nsteps+1)*6 doubles) is not NULL,
 * the complex dipole (Re x, Im x, Re y, Im y, Re z, Im z) at t0 and after every step is
 * written to it. Asynchronous. One step (its four right-hand sides, stage updates and dipole,
 * with the field evaluated on the device) is captured once as a HIP graph and replayed for every
 * step; the graph is rebuilt when y, h, the field or the precision change. Setting the environment
 * variable RTCC_NO_GRAPH=1 before rtcc_init selects plain launches. */
int rtcc_propagate_rk4(rtcc_ctx* ctx, void* y, double t0, double h, int nsteps, const rtcc_field* field,
                       double* mu_dev);

/* Batched RK4 propagation of several systems, each with several members (polarisations, field
 * strengths, pulses), as one graph per step.
 *   ctxs[s], s < nsys (1 <= nsys <= 64): distinct contexts, one per system (each uses its own
 *              precision); the call is ordered on the stream of ctxs[0] (the states must be ready
 *              there) and returns asynchronously.
 *   nprop[s]  : members of system s (1 ... 4096).
 *   ys[s]     : DEVICE, nprop[s] consecutive states of system s (state layout above), advanced in place.
 *   fields    : HOST, sum_s nprop[s] fields, system 0's members first; member m of system s uses
 *               fields[nprop[0] + ... + nprop[s-1] + m]. A kick (kind 2) is applied beforehand with
 *               rtcc_kick on the member's state; during the propagation it acts as no field.
 *   t0, h, nsteps: nsteps RK4 steps of size h from t0 for every member.
 *   mu_dev    : NULL, or per system NULL or DEVICE (nsteps+1) * nprop[s] * 6 doubles: the dipole of
 *               every member (6 values as in rtcc_dipole) at t0 and after every step, [step][member][6].
 * Each context's integrals are shared by its members: a contraction of an integral with the
 * members' amplitudes is one GEMM over all members; a contraction of two amplitude tensors is a
 * batched GEMM. Every member's result equals its own rtcc_propagate_rk4 up to the rounding order of
 * those sums. One step of all systems (a branch per system) is captured once as a HIP graph and
 * replayed; RTCC_NO_GRAPH=1 selects plain launches on each context's stream, and a batch with an FP64
 * system always uses them (its captured form is not in use). Workspaces for the
 * members are allocated by the first call with a given nprop[s] (a change reallocates them). */
int rtcc_propagate_batch(rtcc_ctx* const* ctxs, int nsys, const int* nprop, void* const* ys,
                         const rtcc_field* fields, double t0, double h, int nsteps, double* const* mu_dev);

/* Divergence guard (paper: Results, strong-field propagation, Fig. t2-mag: an RK4 step too long for
 * the field makes |T2| grow without bound). With t2_limit > 0, rtcc_propagate_rk4 and
 * rtcc_propagate_rk4_mixed form, after every step, the Frobenius norm |T2| of the closed-shell T2
 * block of y and the number of non-finite entries of y on the device; every check_every steps (and
 * after the last step) they synchronise and return RTCC_ENONFINITE, with the step and time in
 * rtcc_last_error, if an entry is non-finite or |T2| > t2_limit. y then holds the state of that step.
 * t2_limit <= 0 switches the guard off (the default; the calls then stay asynchronous). */
int rtcc_set_guard(rtcc_ctx* ctx, double t2_limit, int check_every);

/* Mixed step-size RK4 (paper: Results, "Comparison of numerical integrators", strong fields, Fig.
 * ms-results): steps of h1 while the Gaussian pulse of `field` is on, |t - t0_pulse| <= 5 sigma, and of
 * h2 elsewhere, from t0 to t_end; each of the (up to three) phases ends with a shorter step that lands on
 * its boundary. For other field kinds every step is h2. rtcc_mixed_schedule (no context, host only)
 * returns the number of steps and, if times (HOST, cap >= nsteps + 1 doubles) is not NULL, t0 and the
 * end time of every step. rtcc_propagate_rk4_mixed advances y (DEVICE) through that schedule; if
 * mu_dev (DEVICE, (nsteps+1)*6 doubles) is not NULL the dipole (as rtcc_dipole) at t0 and after every
 * step is written to it, and if t2norm_dev (DEVICE, nsteps+1 doubles) is not NULL |T2| likewise.
 * Asynchronous unless the guard is on. Steps of one size replay one captured graph. */
int rtcc_mixed_schedule(double t0, double t_end, double h1, double h2, const rtcc_field* field, int cap,
                        double* times, int* nsteps);
int rtcc_propagate_rk4_mixed(rtcc_ctx* ctx, void* y, double t0, double t_end, double h1, double h2,
                             const rtcc_field* field, double* mu_dev, double* t2norm_dev);

/* Adaptive Cash-Karp propagation of y (DEVICE) from t0 to t_end (Eqs. ck-k, ck-y, ck-h, ck-h-final):
 * trials of hh = min(h, t_end - t) starting from h = h0; a trial is accepted when the largest complex
 * modulus of y5 - y4 is <= eps (y advances with the fifth-order solution), and after every trial
 * h = hh * 0.84 (eps/Delta)^(1/5 accepted, 1/4 rejected), the factor clamped to [0.1, 5]. The last step
 * lands on t_end. If t_out / mu_out (HOST, cap and 6*cap doubles) are not NULL, the time and the dipole
 * (as rtcc_dipole) after every accepted step are written to them (RTCC_EINVAL if more than cap steps are
 * accepted). *naccepted, *nrejected (HOST) count the trials; *h_next (HOST, may be NULL) is the next
 * trial size. Returns RTCC_ENOTCONV after max_trials trials short of t_end and RTCC_ENONFINITE on a
 * non-finite error estimate. Synchronises once per trial. */
int rtcc_propagate_cashkarp(rtcc_ctx* ctx, void* y, double t0, double t_end, double h0, double eps,
                            const rtcc_field* field, int max_trials, int cap, double* t_out, double* mu_out,
                            int* naccepted, int* nrejected, double* h_next);

/* One Cash-Karp trial of size *h from *t with absolute tolerance eps on the largest complex
 * modulus of y5 - y4. If accepted (*accepted = 1) y advances by the fifth-order solution and
 * *t += h; otherwise y is unchanged. In both cases *h becomes the controller's next trial size
 * and *delta the error estimate. Synchronises. */
int rtcc_step_cashkarp(rtcc_ctx* ctx, void* y, double* t, double* h, double eps, const rtcc_field* field,
                       int* accepted, double* delta);

/* ---- General Runge-Kutta tableaux ---------------------------------------------------------------
 * Any Runge-Kutta method given by its Butcher tableau (Eqs. rk_y, rk_k; Table tab:butcher): explicit
 * (A strictly lower triangular), embedded (explicit with a second weight row, driven by the controller
 * of Eq. ck-h-final) and implicit (a full A; the Introduction's third type of integrator, here
 * Gauss-Legendre collocation), through the same stage machinery as RK4 and Cash-Karp: the stage input
 * y + h sum_j a_ij k_j is formed and converted to the contraction precision in one pass, all
 * combinations are FP64. The coefficients are a host struct owned by the caller. */
#define RTCC_MAX_STAGES 6
typedef struct {
  int stages;    /* s, 1..RTCC_MAX_STAGES (implicit tableaux: 1..3) */
  int err_order; /* p > 0: b_err is an embedded solution of order p, the controller takes exponents
                    1/(p+1) after an accepted and 1/p after a rejected trial (p = 4: the paper's 1/5,
                    1/4); 0: no embedded solution */
  double a[RTCC_MAX_STAGES][RTCC_MAX_STAGES]; /* a[i][j], i, j < stages; the rest is ignored */
  double b[RTCC_MAX_STAGES];                  /* weights of the solution the step advances with */
  double b_err[RTCC_MAX_STAGES];              /* weights of the embedded solution (err_order > 0) */
  double c[RTCC_MAX_STAGES];                  /* nodes: stage i is evaluated at t + c[i] h */
} rtcc_tableau;

/* Built-in tableaux. RK4: classical (Eq. rk4truncation). CASHKARP: the corrected Cash-Karp pair of
 * Eqs. ck-k/ck-y, advancing with the fifth-order weights, err_order 4. RKF45: Fehlberg's 4(5) pair
 * (Comparison of numerical integrators), advancing with the fourth-order weights, embedded fifth-order
 * weights, err_order 4. GL2, GL3: two- and three-stage Gauss-Legendre collocation (orders 4 and 6,
 * implicit). */
enum { RTCC_TAB_RK4 = 1, RTCC_TAB_CASHKARP = 2, RTCC_TAB_RKF45 = 3, RTCC_TAB_GL2 = 4, RTCC_TAB_GL3 = 5 };

/* Fill *out (HOST) with built-in tableau `id`. Needs no context or GPU; RTCC_EINVAL for an unknown id
 * (message via rtcc_last_error(NULL)). */
int rtcc_tableau_builtin(int id, rtcc_tableau* out);

/* One step of size h from t with tableau *tab (HOST); y (DEVICE) advances in place with the b weights.
 * Explicit tableau: s right-hand sides; if err_order > 0 and delta (HOST) is not NULL, *delta = the
 * largest complex modulus of the difference between the b and b_err solutions (synchronises).
 * Implicit tableau: the stage equations k_i = f(t + c_i h, y + h sum_j a_ij k_j) are solved by fixed-point
 * sweeps that start from k_i = f(t, y) and evaluate every stage from the previous sweep's k, until
 * h max_i max|k_i(new) - k_i(old)| <= tol (tol > 0); each sweep costs s right-hand sides and one
 * synchronisation. *sweeps (HOST, may be NULL) receives the number of sweeps; RTCC_ENOTCONV after
 * max_iter sweeps (y unchanged), RTCC_ENONFINITE on a non-finite change. tol and max_iter are ignored
 * for explicit tableaux. */
int rtcc_step_tableau(rtcc_ctx* ctx, void* y, double t, double h, const rtcc_tableau* tab,
                      const rtcc_field* field, double tol, int max_iter, double* delta, int* sweeps);

/* Adaptive propagation from t0 to t_end with an explicit embedded tableau (err_order > 0): the
 * trial / accept / controller loop of rtcc_propagate_cashkarp (same arguments, same outputs) with the
 * tableau's weights and exponents; with the built-in CASHKARP tableau it performs the same operations
 * as rtcc_propagate_cashkarp. */
int rtcc_propagate_embedded(rtcc_ctx* ctx, void* y, double t0, double t_end, double h0, double eps,
                            const rtcc_tableau* tab, const rtcc_field* field, int max_trials, int cap,
                            double* t_out, double* mu_out, int* naccepted, int* nrejected, double* h_next);

/* ---- Adjoint (vector-Jacobian products) -------------------------------------------------------
 * Gradients follow the convention for a real loss L of complex variables z: zbar = dL/dRe z + i dL/dIm z
 * (PyTorch's), so a map z -> w(z) holomorphic in z sends wbar to J^H wbar.
 *
 * Structure used (equations of motion Eqs. derivT/derivL): with the Lagrangian L = <0|(1+Lambda)Hbar|0>,
 * dt/dt = -i dL/dlambda and dlambda/dt = +i dL/dt; in the closed-shell variables of this ABI this reads
 * F = S grad L with S = [[0, -i G^-1], [i G^-1, 0]], G the closed-shell metric (singles: 2 x_ia; doubles:
 * 2 x_ijab - x_ijba). Hence the bilinear transpose of the Jacobian is J^T w = -S^-1 J (S w), and J u is
 * evaluated exactly as the first Taylor coefficient of the degree-4 polynomial F(y + eps u) from four
 * points on a circle in the complex eps plane (one batched evaluation of four right-hand sides).
 * All three calls run the right-hand sides in the context's precision (the dipole gradient in FP64) and
 * accumulate in FP64. The cotangents are DEVICE states (layout above) and must not overlap y. */

/* ybar_out = J^H ybar with J = dF/dy at (y, field E); if Ebar (HOST) is not NULL, Ebar[a] = d/dE_a of
 * Re <ybar, F> = -Re sum conj(ybar) F[mu_a, 0](y) (synchronises). ybar_out must not overlap ybar or y. */
int rtcc_rhs_vjp(rtcc_ctx* ctx, const void* y, double t, const double E[3], const void* ybar, void* ybar_out,
                 double Ebar[3]);

/* ybar += gradient of Re sum_a conj(mubar_a) mu_a(y) (mubar_a = mubar[2a] + i mubar[2a+1], HOST), i.e.
 * the adjoint of rtcc_dipole: with mu_a = mu_ref_a + L[mu_a, 0](y) its bilinear gradient is
 * S^-1 F[mu_a, 0](y), F[mu_a, 0] the right-hand side of the operator mu_a alone. Asynchronous. */
int rtcc_dipole_vjp(rtcc_ctx* ctx, const void* y, const double mubar[6], void* ybar);

/* Adjoint of one rtcc_step_rk4 from (y, t) with step h: on entry ybar is the gradient with respect to the
 * step's result, on return with respect to y (the discrete adjoint of the RK4 map: the four stage states
 * are recomputed from y, then J^H is applied stage by stage in reverse). For a Gaussian pulse (kind 1),
 * pbar[0..3] (HOST) += the gradient with respect to (E0, omega, sigma, t0) through
 * dF/dp = -(de/dp) F[n . mu, 0], e(t) the pulse amplitude (synchronises); other kinds leave pbar alone. */
int rtcc_step_rk4_vjp(rtcc_ctx* ctx, const void* y, double t, double h, const rtcc_field* field, void* ybar,
                      double pbar[4]);

/* Complex dipole expectation value (Eq. dipole), reference part included, into mu[6] (HOST):
 * (Re mu_x, Im mu_x, Re mu_y, Im mu_y, Re mu_z, Im mu_z). Computed in FP64. Synchronises. */
int rtcc_dipole(rtcc_ctx* ctx, const void* y, double mu[6]);

/* Same as rtcc_dipole but written to DEVICE memory mu_dev[6]; asynchronous. */
int rtcc_dipole_dev(rtcc_ctx* ctx, const void* y, double* mu_dev);

/* Ground state at zero field (the initial condition y0 of the propagation): Jacobi iterations
 * with orbital-energy denominators and DIIS, first T from the T part of y (zeros are fine),
 * then Lambda from lambda = t, each to max|R| <= tol. FP64. *e_corr (HOST, may be NULL)
 * receives the CCSD correlation energy. Returns RTCC_ENOTCONV after maxiter iterations. */
int rtcc_ground_state(rtcc_ctx* ctx, void* y, double tol, int maxiter, double* e_corr);

/* Dirac-delta kick E(t) = kappa delta(t) n applied to y in place: the flow of the dipole
 * operator n.mu alone over unit "time", integrated with 100 RK4 sub-steps. FP64. */
int rtcc_kick(rtcc_ctx* ctx, void* y, double kappa, const double n[3]);

/* *nonfinite (HOST) = number of non-finite complex entries of y. Synchronises. */
int rtcc_check_state(rtcc_ctx* ctx, const void* y, int64_t* nonfinite);

/* Live timing of one class of GEMM launches with HIP events recorded on the stream each launch is
 * issued on. rtcc_profile(ctx, 1) resets the statistics and times every subsequent launch of the
 * particle-particle ladder, the GEMM kernel alone without packing or split-K reduction (in the
 * split-BF16 path a kernel under a name of its own); rtcc_profile(ctx, 2) resets them and times every
 * complex x complex product with 2 M N K >= 5e8 (those RTCC_BF16X3 gives the split kernel: the ring and
 * Lambda products of the right-hand side, Eq. simtranH), the GEMM kernel alone without packing or split-K
 * reduction -- with RTCC_BF16X3 only the launches of the register-staged 128 x 256 split-BF16 kernel
 * (gemm_bf16x3_nt<1, 1, 0, 4>, one launch also where it carries several independent products), which
 * has the largest share of the split-BF16 step at o = 20, v = 76;
 * rtcc_profile(ctx, 0) stops; other values: RTCC_EINVAL. While profiling is on, rtcc_propagate_rk4 issues
 * its kernels one by one instead of replaying the captured step graph (events recorded inside a
 * captured graph cannot be timed); rtcc_propagate_batch does the same when any of its contexts
 * is profiling, and times that context's batched launches. rtcc_profile_read synchronises and returns
 * (HOST) the number of timed launches, their summed duration in ms, and per launch, averaged over the
 * timed launches, the algorithmic real flops (real x complex products: 4 flops per row, column and k;
 * complex x complex: 8) and -- bytes_per_launch may be NULL; 0 for the ladder -- the algorithmic HBM
 * bytes of the complex products: each operand read once and the output written once (read once more
 * when accumulated into), 8 bytes per complex FP32 (or packed hi / lo BF16) element, 16 per FP64.
 * The ladder is by default the two GEMMs of its symmetric / antisymmetric form, X+ V+ over the
 * (i <= j) x (e <= f) and X- V- over the (i < j) x (e < f) pair triangles (rows o(o+1) and o(o-1) per
 * member for tau and lambda2, K = N = v(v+1)/2 and v(v-1)/2), a quarter of the flops of the full
 * product of 2 o^2 rows with the v^2 x v^2 matrix <ab|ef>; the environment variable RTCC_LADDER=full,
 * read by rtcc_init, selects the full product (one launch, 4 * 2 o^2 * v^4 flops), and
 * RTCC_LADDER=symmetric-nolds the symmetric form with its element fold / unfold kernels (the LDS-staged
 * ones serve v <= 96). */
int rtcc_profile(rtcc_ctx* ctx, int enable);
int rtcc_profile_read(rtcc_ctx* ctx, int64_t* launches, double* total_ms, double* flops_per_launch,
                      double* bytes_per_launch);

/* Diagnostics: out[0] = o, out[1] = v, out[2] = state length (complex entries),
 * out[3] = real flops issued to the MFMA GEMMs by the last rtcc_rhs call,
 * out[4] = device bytes held by the context, out[5] = current precision. */
int rtcc_info(rtcc_ctx* ctx, int64_t out[6]);

/* ---- GEMM kernels and the tile autotuner ------------------------------------------------------
 * Every contraction of the right-hand side (Eqs. derivT, derivL; the ladder, ring and hole-hole terms)
 * is a GEMM C(m,n) = alpha sum_k A(m,k) B(k,n) + beta C(m,n) on planar complex or real operands.
 * rtcc_gemm runs one such product with the library's kernels on caller-owned DEVICE operands, for
 * kernel tests and for the autotuner (paper_2205_05175_amd/autotune.py), which times candidate kernels
 * per product shape and writes the table that rtcc_load_tuning reads.
 *   precision : RTCC_FP64 (double operands), RTCC_FP32 or RTCC_BF16X3 (float operands; BF16X3 lets
 *               products take the split-BF16 kernel as in a context of that precision).
 *   A(m,k) = ta ? a[k*lda + m] : a[m*lda + k];  B(k,n) = tb ? b[n*ldb + k] : b[k*ldb + n];  C(m,n) at
 *   c[m*ldc + n]. *_im == NULL: a real operand (C must be complex if A or B is).
 *   choice    : NULL or int[4] {kind, p1, p2, splits}: kind 0 the library's own choice; 1 the tile
 *               kernel with a (p1 / 1000) x (p1 % 1000) tile, k stage p2 and `splits` K splits; 2 the
 *               split-BF16 kernel with p1 (2 or 4) waves along N and `splits` K splits (0: its model).
 *               RTCC_EINVAL if that kernel cannot take the product.
 *   reps      : 0 runs the product once; > 0 runs it once more and then reps times between two HIP
 *               events and writes the mean duration to *ms (HOST) -- C is overwritten each time.
 * Allocates its own scratch (hipMalloc) and synchronises hip_stream before returning. */
int rtcc_gemm(int precision, int64_t M, int64_t N, int64_t K, double alpha, const void* a_re, const void* a_im,
              int64_t lda, int ta, const void* b_re, const void* b_im, int64_t ldb, int tb, double beta, void* c_re,
              void* c_im, int64_t ldc, const int* choice, int reps, float* ms, void* hip_stream);

/* Replace the process-wide tuning table with the text file at path (NULL: clear it). One entry per
 * line, "prec M N K ac bc ta tb kind p1 p2 splits" (prec 0 FP64, 1 FP32, 2 split-BF16 contexts; ac, bc:
 * complex A, B; the kernel choice as in rtcc_gemm); '#' starts a comment. Products of a listed shape
 * (not batched, M, N > 1) then use the listed kernel. *nentries (HOST, may be NULL) = entries read. */
int rtcc_load_tuning(const char* path, int* nentries);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the check of rtcc_check_state without a context and without
 * synchronising. For a state y (DEVICE, the layout above for o, v) it writes out_dev[0] = |T2| (the
 * Frobenius norm of the T2 block; NaN if y has a non-finite entry) and out_dev[1] = the number of
 * non-finite complex entries of y (out_dev: DEVICE, 2 doubles), enqueued on hip_stream. Nothing is
 * allocated: the only scratch, 8 KB of reduction partials, is a static device array of the library,
 * one copy per GPU, held until the process ends; its contents need no clearing (every call overwrites
 * the partials it reads), and calls that overlap on one GPU race on it. Returns RTCC_EINVAL for o or
 * v < 1, null pointers or o v > 2^20 (the message is rtcc_last_error(NULL)). */
int rtcc_check_state_noalloc(int o, int v, const void* y, double* out_dev, void* hip_stream);

/* Measured machine ceilings of the device the caller has current, for reading the kernels' roofline
 * fractions beside the datasheet figures. kind 0, 1, 2: the sustained rate of v_mfma_f64_16x16x4f64,
 * v_mfma_f32_16x16x4f32 and v_mfma_f32_32x32x16_bf16 (every wave of a 4096 x 256-thread grid runs
 * `size` rounds of independent accumulator chains, no memory traffic; 1 <= size <= 2^24), *value (HOST)
 * in TFLOP/s (2 M N K flops per instruction); kind 3: a plain device copy of `size` bytes (a multiple of
 * 16 KiB, at most 64 GiB) with 16-byte loads and stores, *value in GB/s counting bytes read plus bytes
 * written. Each measurement is the mean of several timed launches after an untimed one on a stream of its
 * own; the probe allocates and frees its buffers and synchronises. Returns RTCC_EINVAL for other
 * arguments (the message is rtcc_last_error(NULL)), RTCC_EHIP on a HIP error. */
int rtcc_peak_probe(int kind, int64_t size, double* value);

void rtcc_destroy(rtcc_ctx* ctx);
const char* rtcc_last_error(const rtcc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RTCC_H */
