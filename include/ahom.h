/*
 * ahom -- generalized Basic Scheme of FFT-based homogenization on lattice
 * patterns P(M), native to AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every call returns an int status
 * (AHOM_OK = 0, a positive warning, or a negative error); no exception or
 * abort crosses this boundary.  ahom_last_error() gives a thread-local text
 * for the last failure.  Handles are created and destroyed explicitly by
 * the caller; one handle must not be used from two threads at once,
 * separate handles may.
 *
 * Conventions shared by all calls
 *  - d is 2 or 3.  Matrices are row-major.
 *  - Pattern points and frequencies are always in the library's canonical
 *    Smith-normal-form order (lexicographic in lambda, resp. kappa, slowest
 *    axis first, over the axes with e_j > 1).  ahom_pattern_points /
 *    ahom_pattern_freqs give the exact coordinates of that order.
 *  - Strain/stress tensors: plain tensor components (no sqrt(2), no
 *    engineering shear).  A full 3x3 symmetric tensor is passed as 9 doubles
 *    row-major; in 2-D its upper-left 2x2 block is used.
 *  - Field components: 3-D (11,22,33,23,13,12), 2-D (11,22,12).
 *  - mem_flags = AHOM_MEM_HOST (default): host arrays, copied before the call
 *    returns.  AHOM_MEM_DEVICE: the *field* arrays (phase ids, per-point
 *    stiffness, init, strain_out, dft in/out) are device pointers used on the
 *    solver's stream; the caller keeps them alive until that stream has been
 *    synchronized.  Small arrays (eps_bar, iters, resid, mean_stress, Ceff,
 *    lame table) are always host memory.
 */
#ifndef AHOM_H
#define AHOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define AHOM_OK                  0
#define AHOM_W_NOT_CONVERGED     1   /* max_iter reached; outputs hold iterate max_iter */
#define AHOM_E_ARG              -1   /* invalid argument (null pointer, bad d, bad size) */
#define AHOM_E_SINGULAR         -2   /* det M = 0 */
#define AHOM_E_OVERFLOW         -3   /* |det M| > 2^31 or int64 overflow in the Smith form */
#define AHOM_E_UNSUPPORTED_SIZE -4   /* an elementary divisor has a prime factor > 7 */
#define AHOM_E_MATERIAL         -5   /* mu <= 0 or 3 lambda + 2 mu <= 0, or no material set */
#define AHOM_E_DIVERGED         -6   /* residual NaN/Inf or grew beyond 1e3 times its start */
#define AHOM_E_DEVICE           -7   /* HIP runtime error, or no GPU */
#define AHOM_E_NOMEM            -8   /* device allocation failed */

/* precision modes */
#define AHOM_FP64               0    /* every stage in double precision */
#define AHOM_FP32_MIXED         1    /* FFT, Gamma0 and local law in float; residual,
                                        averages and twiddle generation in double */

/* memory flags */
#define AHOM_MEM_HOST           0
#define AHOM_MEM_DEVICE         1

/* treatment of unpaired boundary frequencies */
#define AHOM_NYQUIST_HERMITIAN  0

typedef struct ahom_pattern ahom_pattern;
typedef struct ahom_solver ahom_solver;

typedef struct ahom_config {
    int precision;      /* AHOM_FP64 or AHOM_FP32_MIXED */
    double tol;         /* stop when the equilibrium residual r(n) <= tol */
    int max_iter;       /* upper bound on the number of updates */
    int check_period;   /* iterations enqueued between host-side status reads (>= 1) */
    int nyquist;        /* AHOM_NYQUIST_HERMITIAN */
    void* stream;       /* hipStream_t to run on; NULL = the null stream */
    int resid_period;   /* evaluate r(n) only for n = 0 (mod resid_period) and at max_iter
                           (<= 1: every iteration).  The stop is the first evaluated n with
                           r(n) <= tol; the traction terms are only read and written around
                           evaluated iterations, which saves memory traffic. */
    double refine;      /* AHOM_FP32_MIXED only: defect-correction restarts.  The FP32
                           iteration runs until r(n) <= max(tol, refine * r_stage), where
                           r_stage is 1 for the first stage; then the strain is handed to
                           FP64, two FP64 updates give the accurate defect (traction step)
                           of the FP64 iterate, and a new FP32 stage iterates on the
                           correction to that iterate with the defect as a fixed traction
                           offset, so FP32 rounding scales with the correction rather than
                           with the whole field.  0 = default (1e-3; 1e-4 with the CG
                           scheme in elasticity); < 0 = no restarts (the
                           plain FP32 iteration, whose residual floor is set by FP32
                           rounding of the polarization). */
    int stop_rule;      /* AHOM_STOP_RESIDUAL (0, default): stop at r(n) <= tol.
                           AHOM_STOP_CAUCHY (1): the criterion of Sec. 5.2, stop at the
                           first evaluated n with c(n) = |eps(n+1) - eps(n)| / |eps(0)| <= tol
                           (see ahom_solver_cauchy_history) and return eps(n).  Single-pattern
                           solver only; in AHOM_FP32_MIXED it needs refine < 0. */
    int scheme;         /* AHOM_SCHEME_BASIC (0, default): Algorithm 1 (Sec. 3.2).
                           AHOM_SCHEME_CG (1): conjugate gradients on the same discrete
                           Lippmann-Schwinger system (the accelerated schemes the paper
                           names in Sec. 1 and Sec. 6): x = eps - eps_bar compatible with
                           zero mean, A x = Gamma0 * (C : x) = -Gamma0 * (C : eps_bar), in
                           the C0 inner product sum_x u : C0 : v, in which A is symmetric
                           positive definite on compatible fields.  Each update costs one
                           sweep of the passes plus two vector kernels; the stop test, the
                           history and the outputs are those of the Basic Scheme (r(n) of
                           eps(n) = eps_bar + x_n; n = updates performed).  The residual
                           and <sigma> follow their own recurrences, so a FP64 solve with
                           no field output (strain_out NULL, ahom_effective_stiffness) does
                           not form x at all.  An initial guess (ahom_solve init) starts CG
                           from x_0 = P init, its projection Gamma0 C0 init onto compatible
                           zero-mean fields (any field is accepted; one more operator sweep);
                           guess_probe does not apply.  Single-pattern solver,
                           AHOM_STOP_RESIDUAL.  In AHOM_FP32_MIXED: defect
                           correction — one FP64 sweep gives the exact residual field and
                           equilibrium residual of the FP64 iterate, an FP32 CG solve of the
                           correction runs until its residual has dropped by `refine` (C0
                           norm), the FP64 iterate takes the correction's projection onto
                           compatible zero-mean fields (one more FP64 sweep); n counts the FP32
                           updates, ahom_solver_last_restarts the corrections, the history holds
                           the FP64 residual where a sweep evaluated it.  Needs refine >= 0
                           (0 selects 1e-4 for elasticity, 1e-3 for conductivity). */
    int physics;        /* AHOM_ELASTICITY (0, default): quasi-static linear elasticity (Sec. 3.1).
                           AHOM_CONDUCTIVITY (1): the steady-state heat (conductivity) equation that
                           Sec. 3 names beside it: unknown the gradient e = grad theta of a
                           periodic potential plus a prescribed mean (d components), flux
                           q = k(x) e, equilibrium div q = 0, scalar Green operator
                           Gamma0(h) tau = h (h . tau) / (k0 |h|^2).  Set the material with
                           ahom_solver_set_conductivity, solve with ahom_solve_conductivity /
                           ahom_effective_conductivity.  Single-pattern solver; both schemes,
                           both precisions (FP32 restarts as for elasticity). */
    int guess_probe;    /* with an initial guess (ahom_solve init): 0 (default) starts every load
                           from it.  k > 0: the plain start eps_bar runs beside the guessed one
                           (as n_load more loads in the same launches) for the first k updates;
                           per load the start that met the tolerance first is kept (with FP32
                           restarts: the first stage's tolerance), or if neither has, the guessed
                           start if it is predicted to reach tol in
                           at most 90 % of the plain start's updates (from the contraction of the
                           evaluated residuals over the second half of the probe); else the plain
                           start's iterate,
                           traction and history are kept (the fallback to a zero guess).
                           ahom_solver_last_starts reports the choice.  0 <= k <= max_iter. */
} ahom_config;

#define AHOM_STOP_RESIDUAL 0
#define AHOM_STOP_CAUCHY 1
#define AHOM_SCHEME_BASIC 0
#define AHOM_SCHEME_CG 1
#define AHOM_ELASTICITY 0
#define AHOM_CONDUCTIVITY 1

/* Library version, (major << 16) | (minor << 8) | patch. */
int ahom_version(void);

/* Text of the last failure on this thread ("" if none).  Owned by the library. */
const char* ahom_last_error(void);

/*
 * Pattern P(M) of a regular integer matrix M (Sec. 2.1) and its Smith normal
 * form M = Q E R, Q and R unimodular, E = diag(e_1..e_d), e_j | e_{j+1}
 * (Sec. 2.2).  M: d*d int64, row-major, host memory, copied.
 * Errors: AHOM_E_ARG (d not 2 or 3, null), AHOM_E_SINGULAR, AHOM_E_OVERFLOW,
 * AHOM_E_UNSUPPORTED_SIZE.  Host-only: needs no GPU.
 */
int ahom_pattern_create(int d, const int64_t* M, ahom_pattern** out);

/*
 * Transformed pattern P_L(M) = L Lambda(M) within the cell L [-1/2,1/2)^d
 * (Def. 3.3): the periodic cell is spanned by the columns of the real regular
 * matrix L (d*d, row-major, host memory, copied).  Point i sits at L y_i with
 * y_i as ahom_pattern_points gives it; the frequency of class h is L^{-T} h,
 * so Gamma0 and the equilibrium residual use xi parallel to L^{-T} h.  The
 * Smith form, the point and frequency orders, the transforms and all solver
 * calls are those of P(M); strains, stresses and C_eff are in the physical
 * (x = L y) frame.  L = I gives P(M) bit for bit.
 * Errors: those of ahom_pattern_create, AHOM_E_ARG (null, non-finite entry),
 * AHOM_E_SINGULAR (|det L| <= 1e-12 max|L_ij|^d).  Host-only.
 */
int ahom_pattern_create_transformed(int d, const int64_t* M, const double* L, ahom_pattern** out);
void ahom_pattern_destroy(ahom_pattern* p);

/*
 * m = |det M|, dM = #{j : e_j > 1} (pattern dimension, Sec. 2.2), e[0..d-1],
 * Q and R (d*d row-major).  E is unique; Q and R are the library's
 * deterministic choice.  Any output pointer may be NULL.
 */
int ahom_pattern_info(const ahom_pattern* p, int64_t* m, int* dM, int64_t* e, int64_t* Q, int64_t* R);

/*
 * Canonical point order: num[i*d + j] = m * y_j of point i, exact, with
 * y in [-1/2, 1/2)^d (Sec. 2.1).  num: m*d int64, host memory.
 */
int ahom_pattern_points(const ahom_pattern* p, int64_t* num);

/*
 * Canonical frequency order: h[i*d + j], h in G(M^T) = M^T [-1/2,1/2)^d
 * intersected with Z^d (Sec. 2.1), exact.  h: m*d int64, host memory.
 */
int ahom_pattern_freqs(const ahom_pattern* p, int64_t* h);

/*
 * Bare pattern DFT (eq. Fouriermatrix, Sec. 2.2) on the GPU, computed as the
 * d_M-dimensional FFT over the Smith-form axes.  sign = -1: forward,
 * out_h = (1/m) sum_y in_y exp(-2 pi i h^T y); sign = +1: inverse,
 * out_y = sum_h in_h exp(+2 pi i h^T y).  in/out: m interleaved complex
 * values (re, im) in canonical point (forward input) / frequency order,
 * double when prec = AHOM_FP64, float when AHOM_FP32_MIXED.  in and out may
 * not alias.  stream: hipStream_t or NULL.
 */
int ahom_dft(const ahom_pattern* p, int sign, int prec, const void* in, void* out, int mem_flags, void* stream);

/*
 * ahom_dft for callers that cannot allocate device memory (code that must not
 * call hipMalloc, e.g. tight serving loops or harnesses that forbid it): the
 * same transform through the same kernels, with no hipMalloc, hipFree or
 * other allocating call.  in and out are device pointers (m complex values as
 * for ahom_dft, not aliasing).  The plan, the twiddle tables and the working
 * array live in one static device array of the library (about 33 MiB, held
 * on each GPU the library runs on until the process ends): m must not exceed
 * 2^21 points (AHOM_E_ARG otherwise).  Every call on a GPU shares that array,
 * so calls that overlap on one GPU (two streams, two threads) race; the call
 * returns after the transform has completed on `stream`.
 */
int ahom_dft_noalloc(const ahom_pattern* p, int sign, int prec, const void* in, void* out, void* stream);

/*
 * Solver for Algorithm 1 (Sec. 3.2) on the pattern p (which must outlive
 * the solver).  Allocates device buffers.  Errors: AHOM_E_ARG, AHOM_E_DEVICE,
 * AHOM_E_NOMEM.
 */
int ahom_solver_create(const ahom_pattern* p, const ahom_config* cfg, ahom_solver** out);
void ahom_solver_destroy(ahom_solver* s);

/*
 * Piecewise-constant isotropic stiffness (Sec. 3.1): lame[2*k], lame[2*k+1]
 * = (lambda, mu) of phase k (host memory); phase[i] in [0, n_phase) is the
 * phase of canonical point i (m bytes).  n_phase <= 256.
 * Errors: AHOM_E_MATERIAL (mu <= 0 or 3 lambda + 2 mu <= 0), AHOM_E_ARG.
 */
int ahom_solver_set_material(ahom_solver* s, int n_phase, const double* lame, const uint8_t* phase, int mem_flags);

/*
 * Per-point isotropic stiffness (Sec. 3.2: the stiffness field C(x) is only
 * needed at the pattern points y, collocation): lame_pts[2*i],
 * lame_pts[2*i+1] = (lambda, mu) at canonical point i (m*2 doubles, host or,
 * with AHOM_MEM_DEVICE, device memory; copied).  Replaces any phase table.
 * Errors: AHOM_E_MATERIAL (some mu <= 0 or 3 lambda + 2 mu <= 0), AHOM_E_ARG.
 */
int ahom_solver_set_stiffness_field(ahom_solver* s, const double* lame_pts, int mem_flags);

/*
 * Reference medium C0 of the Lippmann-Schwinger equation (Sec. 3.1; Gamma0 is
 * built from it): an isotropic Lame pair.  The paper's numerics do not state
 * C0; if never called, the mean of the extreme values over the material
 * (phase table or field) is used, (lambda_min + lambda_max) / 2 and
 * (mu_min + mu_max) / 2.  Errors: AHOM_E_MATERIAL for mu0 <= 0 or
 * lambda0 + 2 mu0 <= 0.
 */
int ahom_solver_set_reference(ahom_solver* s, double lambda0, double mu0);

/*
 * Algorithm 1 for n_load macroscopic strains at once (one batched launch per
 * pass).  eps_bar: n_load*9 (host).  init: NULL, or n_load*c*m doubles, the
 * fluctuation added to eps_bar in eps(0) (c = 6 in 3-D, 3 in 2-D,
 * component-major per load, canonical point order).  strain_out: NULL, or
 * n_load*c*m doubles receiving eps(n_k) per load.  iters[k]: n_k = number of
 * updates performed for load k; resid[k] = r(n_k), the equilibrium
 * residual sqrt(sum_{h active, h != 0} |sigma_hat_h xi_h|^2) / |<sigma>|_F;
 * mean_stress: n_load*9, <sigma(n_k)> (Def. 3.1: C_eff : eps_bar).
 * Any of iters, resid, mean_stress may be NULL.
 * Returns AHOM_OK if every load converged, AHOM_W_NOT_CONVERGED if some load
 * reached max_iter (outputs hold that iterate), AHOM_E_DIVERGED if some
 * load diverged, or an error (AHOM_E_ARG for init with the Cauchy stop rule).
 * AHOM_FP32_MIXED with refine > 0: after each FP32 stage the iterate is
 * handed to FP64 (see ahom_config.refine); a restart performs two FP64
 * updates and advances n_k by one, and the returned strain is the FP64
 * iterate plus the FP32 correction.  The history keeps one value per n.
 */
int ahom_solve(ahom_solver* s, int n_load, const double* eps_bar, const void* init, void* strain_out,
               int* iters, double* resid, double* mean_stress, int mem_flags);

/*
 * Effective stiffness (Def. 3.1: C_eff : eps_bar is the mean stress <sigma>
 * of the solution for the macroscopic strain eps_bar) in Mandel form (c x c
 * row-major, c = 6 or 3): runs the c Mandel unit loads as one batched solve;
 * column k is Mandel(<sigma>) of load k.  iters: NULL or c ints.  Same
 * return codes as ahom_solve.
 */
int ahom_effective_stiffness(ahom_solver* s, double* Ceff, int* iters);

/*
 * Conductivity (ahom_config.physics = AHOM_CONDUCTIVITY; Sec. 3 names the
 * steady-state heat equation as the other cell problem of the framework).
 * Piecewise-constant isotropic conductivity: k[q] > 0 of phase q (host
 * memory); phase[i] in [0, n_phase) the phase of canonical point i (m bytes,
 * host or device memory as ahom_solver_set_material).  n_phase <= 256.  The
 * reference k0 defaults to (k_min + k_max) / 2.  Errors: AHOM_E_MATERIAL
 * (k <= 0 or not finite), AHOM_E_ARG (bad arguments or an elasticity solver).
 */
int ahom_solver_set_conductivity(ahom_solver* s, int n_phase, const double* k, const uint8_t* phase, int mem_flags);
/* Reference conductivity k0 of the Lippmann-Schwinger equation.  AHOM_E_MATERIAL for k0 <= 0. */
int ahom_solver_set_reference_conductivity(ahom_solver* s, double k0);

/*
 * The Basic Scheme (Algorithm 1, Sec. 3.2, with the scalar Green operator of
 * the heat equation of Sec. 3; or CG, per ahom_config.scheme) for n_load mean
 * gradients grad_bar (n_load*3 doubles, host; in 2-D the first two entries
 * are used).
 * field_out: NULL, or n_load*d*m doubles receiving the gradient field e(n_k)
 * per load, component-major, canonical point order (host, or device memory
 * with AHOM_MEM_DEVICE).  iters, resid: as ahom_solve, with the residual
 * r(n) = sqrt(sum_{h active, h != 0} |q_hat_h . xi_h|^2) / |<q>| of the
 * flux; mean_flux: n_load*3, <q(n_k)> (K_eff grad_bar).  Any output may be
 * NULL.  Same return codes as ahom_solve.
 */
int ahom_solve_conductivity(ahom_solver* s, int n_load, const double* grad_bar, void* field_out, int* iters,
                            double* resid, double* mean_flux, int mem_flags);

/*
 * Effective conductivity K_eff (d x d row-major; the heat-equation
 * counterpart of the effective tensor of Sec. 3.1): column j is <q> for the
 * unit mean gradient e_j (the d loads solved together).  iters: NULL or d
 * ints.  Same return codes as ahom_solve.
 */
int ahom_effective_conductivity(ahom_solver* s, double* Keff, int* iters);

/*
 * Device timing of the last ahom_solve on this solver: total milliseconds
 * between the first kernel and convergence detection (HIP events on the
 * solver's stream), and the number of iterations enqueued.
 */
int ahom_solver_last_timing(const ahom_solver* s, double* ms, int* iterations_enqueued);

/*
 * Start kept per load in the last ahom_solve (ahom_config.guess_probe):
 * which[l] = 1 for the initial guess, 0 for the plain start eps_bar (also 0
 * for every load of a solve without init).  Writes min(cap, n_load) ints.
 */
int ahom_solver_last_starts(const ahom_solver* s, int* which, int cap);

/*
 * Number of FP64 defect-correction restarts in the last ahom_solve (0 for
 * AHOM_FP64, for refine < 0, or when the first FP32 stage met tol).
 */
int ahom_solver_last_restarts(const ahom_solver* s, int* n);

/*
 * Per-pass device timing (profiling mode): runs n_iter iterations of the
 * last solve's load set from eps(0) = eps_bar (no stopping), with a HIP event
 * pair around every pass kernel on the solver's stream.  ms[p] receives the
 * mean duration of pass p over the iterations, in launch order within an
 * iteration: real-space turnaround, forward middle axes, spectral
 * turnaround, inverse middle axes, reduction.  bytes[p] receives the
 * algorithmic bytes that pass must move per launch (each state field read
 * and written once, plus phase ids or traction terms).  *n_pass = number of
 * passes (<= cap).
 */
int ahom_solver_pass_times(ahom_solver* s, int n_iter, double* ms, double* bytes, int cap, int* n_pass);

/*
 * Per-iteration residual history r(0..n) of load k of the last solve (the
 * equilibrium residual of the stop test that replaces the Cauchy criterion
 * of Algorithm 1, Sec. 3.2): writes up to cap doubles, *count = number
 * written.
 */
int ahom_solver_history(const ahom_solver* s, int load, double* hist, int cap, int* count);

/*
 * Cauchy measure of Sec. 5.2 beside the residual (the stop rule when
 * ahom_config.stop_rule = AHOM_STOP_CAUCHY):
 * c(n) = |eps(n+1) - eps(n)|_{l2(P(M))} / |eps(0)|, Frobenius norms summed over
 * the points, |eps(0)| = sqrt(m) |eps_bar|_F.  Evaluated on the iterations
 * whose residual is evaluated (-1 elsewhere) from the traction step the
 * residual uses: on active frequencies eps_hat(n+1) - eps_hat(n) =
 * -sym(xi (x) K(xi)^{-1} (t(n) - t(n-1))).  With a user initial guess the
 * denominator stays sqrt(m) |eps_bar|_F (not the norm of the guessed start),
 * and c(0) measures against the compatible part of the guess; the Cauchy
 * stop rule therefore rejects an initial guess (AHOM_E_ARG from ahom_solve).
 * Same output convention as ahom_solver_history.
 */
int ahom_solver_cauchy_history(const ahom_solver* s, int load, double* hist, int cap, int* count);

/* ------------------------------------------------------------------------
 * Batched solves: Algorithm 1 on many patterns P(M_i) of uneven size (same
 * dimension) in persistent device launches.  A workgroup takes one
 * (member, load) item from a device queue and iterates it to its own stop,
 * so members of different sizes and iteration counts share a launch.  The
 * plan (largest radix) and tile widths of each distinct Smith shape are
 * chosen by timing the candidates on the device the first time the shape is
 * seen in the process.  AHOM_FP64 items are solved in one launch.
 * AHOM_FP32_MIXED items use the defect-correction restarts of
 * ahom_config.refine: a launch of first FP32 stages, then rounds of (FP64
 * restart steps, FP32 correction stages) for the items that need them, all
 * on the batch's stream (and replayed from one HIP graph when asked).
 * ------------------------------------------------------------------------ */
typedef struct ahom_batch ahom_batch;

/*
 * n_members matrices M (n_members*d*d int64, row-major each), d in {2, 3}.
 * cfg as for ahom_solver_create (stream: NULL or a hipStream_t of the
 * library's HIP runtime).  Errors as ahom_pattern_create, per member.
 */
int ahom_batch_create(int d, int n_members, const int64_t* M, const ahom_config* cfg, ahom_batch** out);

/*
 * As ahom_batch_create for transformed patterns P_L(M) (Def. 3.3, as
 * ahom_pattern_create_transformed): L holds one real regular cell matrix per
 * member (n_members * d * d doubles, row-major, host memory, copied); member
 * i's Gamma0 and residual use the wave vectors L_i^{-T} h.  Errors: those of
 * ahom_batch_create, AHOM_E_ARG (null L, non-finite entry), AHOM_E_SINGULAR.
 */
int ahom_batch_create_transformed(int d, int n_members, const int64_t* M, const double* L, const ahom_config* cfg,
                                  ahom_batch** out);
void ahom_batch_destroy(ahom_batch* b);

/* m = |det M_i| and the elementary divisors e[0..d-1] of member i. */
int ahom_batch_member_info(const ahom_batch* b, int member, int64_t* m, int64_t* e);

/* Canonical point order of member i (as ahom_pattern_points). */
int ahom_batch_member_points(const ahom_batch* b, int member, int64_t* num);

/*
 * Phase table and phase ids of member i (host memory, canonical order), as
 * ahom_solver_set_material; the reference defaults to the mean of the
 * extreme phases of that member.
 */
int ahom_batch_set_material(ahom_batch* b, int member, int n_phase, const double* lame, const uint8_t* phase);
int ahom_batch_set_reference(ahom_batch* b, int member, double lambda0, double mu0);

/*
 * Algorithm 1 (Sec. 3.2) on every member for the same n_load macroscopic
 * strains (n_load*9).  Outputs
 * are indexed [member * n_load + load]: iters, resid, status (0 converged,
 * 1 not converged, 2 diverged, 3 invalid: a large item iterated by a group of
 * workgroups lost a member at a pass barrier), mean_stress (9 doubles each);
 * any may be NULL.  use_graph != 0 replays the launch from a HIP graph
 * captured on the first call (on a stream of the batch's own).  Returns as
 * ahom_solve; AHOM_E_DEVICE if an item has status 3.
 */
int ahom_batch_solve(ahom_batch* b, int n_load, const double* eps_bar, int* iters, double* resid, double* mean_stress,
                     int* status, int use_graph);

/* Strain field eps(n) of Algorithm 1 (Sec. 3.2) for (member, load) after a
 * solve: c*m doubles (host), component-major. */
int ahom_batch_strain(ahom_batch* b, int member, int load, double* out);

/* Residual history of (member, load), as ahom_solver_history. */
int ahom_batch_history(const ahom_batch* b, int member, int load, double* hist, int cap, int* count);

/* Cauchy measure history of (member, load), as ahom_solver_cauchy_history
 * (|eps(0)| = sqrt(m) |eps_bar|_F of the load; -1 on iterations whose residual
 * is not evaluated and on the FP64 step of a restart). */
int ahom_batch_cauchy_history(const ahom_batch* b, int member, int load, double* hist, int cap, int* count);

/* Device time of the last batch solve (HIP events around its launches) and
 * total restarts. */
int ahom_batch_last_timing(const ahom_batch* b, double* ms, int* restarts);

/* Plan variant the autotuner chose for member i (index into the candidate list). */
int ahom_batch_member_variant(const ahom_batch* b, int member, int* variant);

/* ------------------------------------------------------------------------
 * Learned initial guess on tensor grids M = diag(n, n, n), n a multiple of 8.
 * A 3-D convolutional encoder-decoder (4 levels n^3 .. (n/8)^3 with 32, 64,
 * 96, 128 channels, two periodic 3x3x3 convolutions per level, 2x2x2
 * average pooling, nearest upsampling, additive skips, ReLU; 36 outputs =
 * fluctuation strain (11,22,33,23,13,12) of the six Mandel unit loads) runs
 * on BF16 matrix cores with FP32 accumulation; FP32 master weights and Adam.
 * Inputs per point: phase indicator (id != 0), mu/mu0 - 1, lambda/lambda0 - 1.
 * Training loss: the C0-energy norm of the strain error divided by mu0,
 * averaged over points and loads.  Points are in canonical order (z slowest).
 * The guess only sets eps(0): Algorithm 1 still iterates to its tolerance.
 * ------------------------------------------------------------------------ */
typedef struct ahom_guess ahom_guess;

/* batch: largest number of samples per training step (<= 64); seed: weights
 * (He-normal) and sample drawing; stream: NULL or a hipStream_t. */
int ahom_guess_create(int n, int batch, uint64_t seed, void* stream, ahom_guess** out);
void ahom_guess_destroy(ahom_guess* g);
int ahom_guess_num_params(const ahom_guess* g, int64_t* n);
/* flat FP32 parameters: per convolution W[cout][27][cin] (tap t = 9 (dz+1) +
 * 3 (dy+1) + (dx+1)) then b[cout], channel counts padded (input 32, output 64) */
int ahom_guess_get_params(const ahom_guess* g, float* out);
int ahom_guess_set_params(ahom_guess* g, const float* in);

/* Training sample: phase ids (n^3), its phase table (n_phase <= 8), the
 * reference (lambda0, mu0) and the solved strain of the six Mandel unit loads
 * (ahom_solve output for the loads of ahom_effective_stiffness),
 * [6 loads][6 components][n^3] doubles (host or device); the target is that
 * strain minus the load. */
int ahom_guess_add_sample(ahom_guess* g, const uint8_t* phase, int n_phase, const double* lame, double lam0, double mu0,
                          const double* strain, int mem_flags);
int ahom_guess_num_samples(const ahom_guess* g, int* n);
/* Drop every training sample (the storage is kept for the next ones): training
 * on more solves than device memory holds streams them in chunks. */
int ahom_guess_clear_samples(ahom_guess* g);

/* Loss and its gradient (flat, as the parameters) over the given samples. */
int ahom_guess_gradients(ahom_guess* g, const int* samples, int count, float* grad, double* loss);
/* steps of Adam (lr, beta 0.9 / 0.999, eps 1e-8) on random batches; losses[steps] (nullable) */
int ahom_guess_train(ahom_guess* g, int steps, int batch, double lr, double* losses);
/* one Adam step with a caller-supplied gradient */
int ahom_guess_adam_step(ahom_guess* g, const float* grad, double lr);

/* Initial fluctuation for n_load strains eps_bar (n_load*9): the network's
 * unit-load fields combined with the Mandel coordinates of each eps_bar,
 * written as [n_load][6][n^3] doubles: the `init` argument of ahom_solve. */
int ahom_guess_infer(ahom_guess* g, int n_phase, const double* lame, double lam0, double mu0, const uint8_t* phase,
                     int n_load, const double* eps_bar, double* init_out, int mem_flags);
/* network output [n^3][36] of dataset sample i */
int ahom_guess_predict_sample(ahom_guess* g, int sample, float* out);
int ahom_guess_save(const ahom_guess* g, const char* path);
int ahom_guess_load(ahom_guess* g, const char* path);

/* One periodic 3x3x3 convolution through the network's kernels (host FP32
 * arrays, rounded to BF16 on entry; channels-last [batch][n^3][c]).  mode 0:
 * out = conv(x) + b (ReLU if relu); mode 1: out = adjoint of the convolution
 * applied to dy (cout multiple of 32); mode 2: out = weight gradient
 * [cout][27][cin] of sum(dy * conv(x)), db (nullable) = bias gradient. */
int ahom_conv3d(int n, int batch, int cin, int cout, int mode, int relu, const float* x, const float* w, const float* b,
                const float* dy, float* out, float* db);

#ifdef __cplusplus
}
#endif

#endif /* AHOM_H */
