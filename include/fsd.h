/*
 * fsd.h - C ABI of the MI355X (gfx950) solver for the Crank-Nicolson
 * finite-volume scheme of the 2D/3D conservative space-fractional diffusion
 * equation with the sine-transform (tau) preconditioner
 * (Qu, Lei, Hon, Huang, arXiv 2511.21198).
 *
 * The model (Section 1): u_t - d_x D_x^alpha u - d_y D_y^beta u - d_z D_z^gamma u = f
 * on a box, u = 0 outside, with D_x^alpha = k_{1,+} d^{1-alpha}_x - k_{1,-} d^{1-alpha}_{-x}
 * (two-sided Riemann-Liouville derivatives) and 0 < alpha, beta, gamma < 1.
 *
 * Each Crank-Nicolson step solves the dense multilevel Toeplitz system of
 * Section 2 (``linear_sys``):
 *   A u^m = b^m,  A = A_N + sum_i eta_i (A (x) .. (x) B_i (x) .. (x) A),
 *   b^m = (A_N - sum_i eta_i (..B_i..)) u^{m-1} + dt F^{m-1/2},
 * with A_n = tridiag(1,6,1)/8, B_i = k_{i,+} T_i + k_{i,-} T_i^T, T_i the
 * lower-Hessenberg Toeplitz matrix of the q_k coefficients, and
 * eta_i = dt / (2 Gamma(delta_i+1) h_i^(2-delta_i)).
 * It is solved by PCG (symmetric case, k_{i,+} = k_{i,-} on every axis) or
 * left-preconditioned restarted GMRES (otherwise) with the preconditioner
 * P = S_N Lambda S_N of Section 3 (``pre_definition``, ``diag_tau_pre``).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid functions are dense float64 device arrays of n_1*n_2(*n_3) values,
 *    x index fastest, then y, then z (the vector ordering of Section 2).
 *  - The caller owns all device memory.  The library never allocates device
 *    memory: fsd_workspace_bytes() says how much scratch it needs and
 *    fsd_bind() hands it a caller-allocated buffer (e.g. a torch uint8
 *    tensor).  The workspace must stay alive and unmodified while the
 *    problem is used.
 *  - All device work is enqueued on the stream given to fsd_bind().  Entry
 *    points whose stats argument is NULL return after enqueueing, except the
 *    Krylov solvers, which synchronise the stream to read their convergence
 *    flag (a few times per solve).
 *  - No C++ exception crosses the ABI.  Every entry point returns an
 *    fsd_status; fsd_last_error() gives a thread-local message for the last
 *    failure on the calling thread.
 *  - Sizes: the fast transforms need n_i + 1 = 2^a or 3 * 2^a with
 *    4 <= 2(n_i+1) <= 8192 (n_i in {1,2,3,5,7,11,15,23,31,47,63,95,127,191,
 *    255,383,511,767,1023,1535,2047,3071,4095}); other sizes return
 *    FSD_EUNSUPPORTED (the circulant comparators: n_i <= 1024).
 */
#ifndef FSD_H
#define FSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSD_OK = 0,
    FSD_EINVAL = 1,        /* invalid argument (message in fsd_last_error) */
    FSD_ENOTCONV = 2,      /* solver hit maxit; the output holds the last iterate */
    FSD_EBREAKDOWN = 3,    /* Krylov breakdown, e.g. (p, Ap) <= 0 in PCG */
    FSD_ENONFINITE = 4,    /* NaN or Inf in an input or in the residual */
    FSD_ESMALLWS = 5,      /* workspace smaller than fsd_workspace_bytes() */
    FSD_EHIP = 6,          /* a HIP runtime call failed */
    FSD_EUNSUPPORTED = 7,  /* grid size without a transform plan */
    FSD_ENOTBOUND = 8      /* fsd_bind() has not been called */
} fsd_status;

typedef enum {
    FSD_SOLVER_AUTO = 0,   /* PCG iff k_{i,+} == k_{i,-} on every axis */
    FSD_SOLVER_PCG = 1,
    FSD_SOLVER_PGMRES = 2, /* left-preconditioned restarted GMRES */
    FSD_SOLVER_PGMRES2 = 3 /* restarted GMRES on the two-sided system
                              P^{-1/2} A P^{-1/2} v = P^{-1/2} b, u = P^{-1/2} v
                              (Section 3.2, the system Theorem 3.2 bounds); stops
                              when ||P^{-1/2}(b - A u)|| <= tol ||P^{-1/2} b|| */
} fsd_solver;

typedef enum {
    FSD_PREC_FP64 = 0,     /* every vector, transform and reduction in float64 */
    FSD_PREC_MIXED = 1     /* float32 inner Krylov solve (float64 reductions)
                              inside a float64 defect-correction loop */
} fsd_precision;

typedef enum {
    FSD_X0_PREV = 0,       /* initial guess u^{m-1} */
    FSD_X0_ZERO = 1,       /* initial guess 0 (the setting that reproduces the
                              paper's iteration counts) */
    FSD_X0_EXTERNAL = 2,   /* initial guess passed to fsd_cn_step */
    FSD_X0_EXTRAP = 3,     /* 2 u^{m-1} - u^{m-2}: linear extrapolation in time
                              from the previous call's u_prev (the history is
                              kept in the workspace; u^{m-1} on the first call
                              after fsd_bind or fsd_reset_history) */
    FSD_X0_GUARDED = 4     /* d_guess (e.g. the network of fsd_nn.h) unless its
                              float64 residual ||b - A guess|| exceeds that of
                              u^{m-1}; then u^{m-1} (fsd_stats.x0_fallback = 1).
                              Costs two extra float64 matvecs. */
} fsd_x0_mode;

typedef enum {
    FSD_PC_TAU = 0,        /* the sine-transform preconditioner P = S Lambda S
                              (Section 3): the method, and the default */
    FSD_PC_NONE = 1,       /* no preconditioner (P = I): the CG / GMRES columns
                              of the comparisons in Section 4 */
    FSD_PC_TCHAN = 2,      /* comparator of Section 4: every Toeplitz factor
                              (A_i and B_i) replaced by T. Chan's optimal
                              circulant, c_j = ((n-j) t_j + j t_{j-n}) / n;
                              P^{-1} applied by DFTs of length n_i.  float64
                              precision and the one-sided solvers only */
    FSD_PC_STRANG = 3      /* as FSD_PC_TCHAN with Strang's circulant, which
                              keeps the central diagonals: s_j = t_j for
                              j <= n/2, t_{j-n} above */
} fsd_precond;

/* Problem parameters.  Fill with fsd_default_params() first. */
typedef struct {
    int dim;               /* 2 or 3 */
    int n[3];              /* interior nodes per axis (n[2] ignored for dim 2) */
    double a[3], b[3];     /* domain (a_i, b_i); default (0, 1) */
    double delta[3];       /* (alpha, beta, gamma), each in (0, 1) */
    double kplus[3];       /* k_{i,+} > 0 */
    double kminus[3];      /* k_{i,-} > 0 */
    int M;                 /* number of time steps (dt = T/M) */
    double T;              /* final time */
    int solver;            /* fsd_solver */
    int restart;           /* GMRES restart length (default 20; <= 64) */
    double tol;            /* relative tolerance (default 1e-9) */
    long maxit;            /* max Krylov iterations per solve; 0 = prod(n) */
    int precision;         /* fsd_precision */
    double inner_tol;      /* relative tolerance of the float32 inner solve
                              (mixed precision only; default 1e-5) */
    int max_outer;         /* max defect-correction steps (default 8) */
    int x0_mode;           /* fsd_x0_mode */
    int allow_delta_zero;  /* test builds: accept delta = 0 (classical limit) */
    int dst_mfma;          /* mixed precision: the float32 preconditioner applies
                              DST-I as a bf16 matrix-core product on axes with
                              n <= 256 (1) or by FFT (0, default: faster as
                              measured at 255^3) */
    double reorth_eta2;    /* GMRES reorthogonalisation test: a second
                              Gram-Schmidt pass when ||w'||^2 <= reorth_eta2
                              ||w||^2 after the first (0: never; 1 or more:
                              always).  Negative (default): 0, one pass (the
                              preconditioned operator is close to the
                              identity and the pass works on w - v_j; the
                              paper's iteration counts are reproduced with
                              it); 0.5 is the Daniel-Gragg-Kaufman-Stewart
                              test. */
    int precond;           /* fsd_precond (default FSD_PC_TAU) */
} fsd_params;

/* Per-solve statistics. */
typedef struct {
    long iters;            /* Krylov iterations (summed over inner solves) */
    int outer_iters;       /* defect-correction steps (1 for FSD_PREC_FP64) */
    int converged;         /* 1 if the stopping test was met */
    double relres;         /* final ||b - A x||_2 / ||b||_2 in float64 */
    double solver_relres;  /* the solver's own stopping quantity at exit */
    int status;            /* fsd_status of the solve */
    int x0_fallback;       /* FSD_X0_GUARDED: 1 if u^{m-1} replaced the guess */
} fsd_stats;

typedef struct fsd_problem_s* fsd_problem;

/* Fill p with defaults: dim 3, n = 63, domain (0,1), delta 0.5, k = 1,
 * M = 1, T = 1, AUTO solver, restart 20, tol 1e-9, maxit 0, FP64,
 * inner_tol 1e-5, max_outer 8, x0 PREV, dst_mfma 0, reorth_eta2 -1. */
fsd_status fsd_default_params(fsd_params* p);

/* Validate p and build the host-side plan (Section 2 coefficients s_k, q_k,
 * eta_i; circulant spectra of the Toeplitz factors; Lambda factors of
 * Section 3).  Host only: no device work.  *out receives a handle owned by
 * the caller (release with fsd_destroy).
 * Errors: FSD_EINVAL (dim not 2/3, n < 1, delta outside (0,1), k <= 0,
 * T <= 0, M < 1, tol <= 0, restart outside [1, 64]), FSD_EUNSUPPORTED. */
fsd_status fsd_init_problem(const fsd_params* p, fsd_problem* out);

/* Release host state.  Does not touch the caller's workspace. */
void fsd_destroy(fsd_problem prob);

/* Bytes of device workspace the problem needs (depends on dim, n,
 * solver, restart and precision).  Returns 0 for a NULL handle. */
size_t fsd_workspace_bytes(fsd_problem prob);

/* Attach a device workspace (at least fsd_workspace_bytes(), 256-byte
 * aligned) and a HIP stream (hipStream_t passed as void*; NULL = default
 * stream) to the problem and upload its tables.  Must be called with the
 * device that owns d_ws current.  Errors: FSD_ESMALLWS, FSD_EINVAL
 * (misaligned), FSD_EHIP. */
fsd_status fsd_bind(fsd_problem prob, void* d_ws, size_t bytes, void* stream);

/* y = A x  (Section 2, ``linear_sys``, left-hand operator).  x, y: dense
 * device arrays of N doubles; must not alias. */
fsd_status fsd_apply_A(fsd_problem prob, const double* d_x, double* d_y);

/* b = (A_N - K) u + dt F  (right-hand side of ``linear_sys``; the source
 * factor printed as tau is the time step dt).  d_F may be NULL (f = 0).
 * d_u and d_b must not alias. */
fsd_status fsd_apply_rhs(fsd_problem prob, const double* d_u, const double* d_F,
                         double* d_b);

/* y = A x exactly as fsd_apply_A computes it (same kernels, bitwise equal
 * results), for callers that cannot allocate device memory: the packed
 * input and output and the pass intermediates are not taken from the
 * problem's workspace but from a library-owned static device array of
 * fsd_noalloc_scratch_bytes() bytes (64 MiB), one per GPU, held until the
 * process ends.  The call allocates nothing (no hipMalloc, no allocating
 * library routine); it still needs a bound problem (its tables and stream).
 * Limit: six padded vectors of n1' n2 (n3) doubles must fit the array
 * (n1' = n1 rounded up to 32; about 1.39 million values, e.g. 95^3 or
 * 1023 x 1023); larger grids return FSD_EUNSUPPORTED.  Each call clears the
 * part it uses, so calls are independent; calls that overlap on one GPU
 * (several streams or threads) share the array and race.  Errors as
 * fsd_apply_A. */
fsd_status fsd_apply_A_noalloc(fsd_problem prob, const double* d_x, double* d_y);

/* Bytes of the static scratch array behind fsd_apply_A_noalloc. */
size_t fsd_noalloc_scratch_bytes(void);

/* z = P^{-1} r = S_N Lambda^{-1} S_N r  (Section 3, ``diag_tau_pre``). */
fsd_status fsd_apply_Pinv(fsd_problem prob, const double* d_r, double* d_z);

/* y = A x as the float32 inner solve of a FSD_PREC_MIXED problem applies it
 * (Section 2, ``linear_sys``): x rounded to float32, the three float32
 * Toeplitz line passes (float32 twiddles and circulant spectra, float32
 * arithmetic), y widened to float64.  x, y: dense device arrays of N
 * doubles; must not alias.  Errors: FSD_EINVAL for a float64-only problem
 * or a null vector, FSD_ENOTBOUND, FSD_EHIP. */
fsd_status fsd_apply_A32(fsd_problem prob, const double* d_x, double* d_y);

/* z = P^{-1} r as the float32 inner solve of a FSD_PREC_MIXED problem
 * applies it: r rounded to float32, the float32 passes (DST-I by FFT, or by
 * the bf16 matrix-core product on axes with n <= 256 when dst_mfma is set),
 * z widened to float64.  Errors: FSD_EINVAL for a float64-only problem. */
fsd_status fsd_apply_Pinv32(fsd_problem prob, const double* d_r, double* d_z);

/* Solve A x = b with the configured solver and precision.  d_x holds the
 * initial guess on entry and the solution on exit.  st may be NULL.
 * Returns FSD_OK, FSD_ENOTCONV, FSD_EBREAKDOWN or FSD_ENONFINITE (d_x then
 * holds the last iterate). */
fsd_status fsd_solve(fsd_problem prob, const double* d_b, double* d_x, fsd_stats* st);

/* One Crank-Nicolson step (Section 2, ``CN`` / ``linear_sys``):
 * b = (A_N - K) u_prev + dt F, then solve A u_next = b from the initial
 * guess selected by x0_mode (u_prev, 0 or d_guess).  d_F may be NULL
 * (f = 0); d_guess is read only in FSD_X0_EXTERNAL and FSD_X0_GUARDED
 * modes.  d_u_prev may
 * equal d_u_next.  st may be NULL. */
fsd_status fsd_cn_step(fsd_problem prob, const double* d_u_prev, const double* d_F,
                       const double* d_guess, double* d_u_next, fsd_stats* st);

/* Engines (tile shapes) of the line passes.  Every pass of the matvec and
 * of the preconditioner can run on more than one engine: the wave engine
 * (lengths 64..512; for float32 also with one line per lane group instead
 * of two, FSD_ENGINE_WAVE1, which launches twice the wavefronts), the
 * column engine (float32 strided passes of length 512; for DST passes with
 * the DST-I by the odd extension or by the half-length algorithm), and the
 * LDS-stage engine with its default tile or half of it (its last-axis
 * DST-Lambda-DST pass by the half-length DST-I).  All give the same
 * operator to rounding.  FSD_ENGINE_AUTO is the built-in choice per
 * length. */
enum {
    FSD_ENGINE_AUTO = 0, FSD_ENGINE_WAVE = 1, FSD_ENGINE_COL = 2, FSD_ENGINE_COLH = 3,
    FSD_ENGINE_STAGE = 4, FSD_ENGINE_STAGE_HALF = 5, FSD_ENGINE_WAVE1 = 6
};
/* Passes: Toeplitz x / y / z, DST x / y, and the DST-Lambda-DST pass of the
 * last axis (y in 2D, z in 3D). */
enum {
    FSD_PASS_TOEP_X = 0, FSD_PASS_TOEP_Y = 1, FSD_PASS_TOEP_Z = 2, FSD_PASS_DST_X = 3,
    FSD_PASS_DST_Y = 4, FSD_PASS_DSTS_LAST = 5, FSD_PASS_COUNT = 6
};

/* Set the engine of one pass for the float64 operators (precision
 * FSD_PREC_FP64) or the float32 ones of mixed precision (FSD_PREC_MIXED).
 * Errors: FSD_EINVAL (no such pass in this dimension, unknown engine),
 * FSD_EUNSUPPORTED (the engine does not run that pass at its length). */
fsd_status fsd_set_engine(fsd_problem prob, int precision, int pass, int engine);

/* Autotuner: time every engine of every pass of the problem (float64 and,
 * for mixed precision, float32) on the bound workspace and stream, five
 * launches each after two untimed ones, and keep the fastest (the built-in
 * choice unless another engine is more than 5% faster).  Synchronises
 * the stream; overwrites the workspace's scratch vectors (call between CN
 * steps, not inside a solve).  Results change only by rounding. */
fsd_status fsd_autotune(fsd_problem prob);

/* The engine of every pass as "pass_prec(L=..)=engine,...", written to buf
 * (at most len - 1 characters and a terminating zero); returns the full
 * length, or -1 on error. */
int fsd_engines(fsd_problem prob, char* buf, int len);

/* Launch graphs (default off).  When on, each chunk of Krylov iterations
 * the host enqueues between two convergence checks (every PCG chunk, and
 * the first chunk of every GMRES cycle) is captured once into a HIP graph on
 * the bound stream and replayed with a single launch afterwards; results
 * are bitwise those of the direct launches.  Pays off where kernel launches
 * dominate (small grids).  Graphs are not used with the kernel profiler on
 * or on the null stream; they are dropped by fsd_bind and when turned off.
 * The problem keeps its graphs (a few per precision and chunk length) until
 * fsd_destroy. */
fsd_status fsd_set_graphs(fsd_problem prob, int on);

/* Forget the time history used by FSD_X0_EXTRAP (call when the next
 * fsd_cn_step does not continue the previous trajectory). */
fsd_status fsd_reset_history(fsd_problem prob);

/* Host copies of the per-axis coefficients (axis 0 = x):
 * q[0..n]   q_k of Section 2 (``coef_expression``), n+1 values;
 * lam[0..n-1] eigenvalues of tau(H(T)) (Lemma 3.2), n values;
 * eta       eta_i.  Any pointer may be NULL. */
fsd_status fsd_get_coefficients(fsd_problem prob, int axis, double* q, double* lam,
                                double* eta);

/* Kernel timing.  When enabled, the library records a pair of hipEvents on
 * the bound stream around every line-pass and multi-vector kernel launch
 * (adding two event records per launch).  fsd_profile_read() synchronises
 * the stream, aggregates the records per kernel kind into at most `max`
 * entries of `out`, clears them, and returns the number of kinds (or -1 on
 * error).  `bytes` is the algorithmic traffic summed over the launches: the
 * interior values each launch must read and write (padding excluded).
 * Launches of a Krylov iteration that was enqueued ahead of the convergence
 * test and found the solve already stopped (they return without work) are
 * not counted. */
typedef struct {
    char name[32];     /* e.g. "toep_z_f32", "dsts_z_f64", "gm_maxpy_f32" */
    long launches;
    double total_ms;   /* summed hipEvent durations */
    double bytes;      /* summed algorithmic bytes */
} fsd_profile_entry;

fsd_status fsd_profile_enable(fsd_problem prob, int on);
int fsd_profile_read(fsd_problem prob, fsd_profile_entry* out, int max);

/* Streaming device-to-device copy of `bytes` bytes (16-byte vector loads and
 * stores, four in flight per thread) on `stream` (hipStream_t as void*;
 * NULL = default stream).  Not part of the method: a plain copy of known
 * size that measures the HBM bandwidth this device attains (the measured
 * peak the line passes are compared with, next to the datasheet figure) and
 * calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE counters.  bytes and both
 * addresses must be multiples of 16 and the buffers must not overlap
 * (FSD_EINVAL otherwise).  Returns after enqueueing. */
fsd_status fsd_hbm_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* Messages. */
const char* fsd_status_string(fsd_status s);
const char* fsd_last_error(void);

/* Library version string. */
const char* fsd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FSD_H */
