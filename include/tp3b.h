/*
 * tp3b.h - tensor-product three-body eigensolver for AMD Instinct MI355X (gfx950).
 *
 * Implements the hot path of the tensor-product scheme of Thies, Hof, Zimmermann
 * and Efremov ("Tensor Product Scheme for Computing Bound States of the Quantum
 * Mechanical Three-Body Problem"): the pseudospectral three-body Hamiltonian
 * applied in tensor form (Sec. 3.2-3.3, eqs. (9)-(11)), the kinetic-only shifted
 * Sylvester preconditioner (Sec. 4.2, eq. (14)), block orthogonalisation and a
 * block Jacobi-Davidson QR eigensolver (Sec. 4.1, eqs. (12)-(13)).
 *
 * Conventions shared by every call
 *  - Every function returns a tp3b_status: 0 on success, a negative code on
 *    failure.  No function aborts or exits; tp3b_last_error() returns a message
 *    for the calling thread's last failure.  No C++ exception leaves the
 *    library: a failed host allocation returns TP3B_ENOMEM, any other host
 *    exception TP3B_EDEVICE with its message.
 *  - Vectors are 2d-mode tensors stored with the x modes slowest: 1D
 *    psi[i][j] at i*n_y + j (eq. (6)); 2D psi[x1][x2][y1][y2].  N is the product
 *    of the mode sizes.
 *  - A block of nvec vectors is a column-major N x nvec array with leading
 *    dimension ld >= N: vector v starts at X + v*ld.
 *  - Device pointers are HIP device (or managed) memory owned by the caller;
 *    the library never frees or reallocates them.  Host pointers are ordinary
 *    host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    apply/prec calls are stream-ordered and asynchronous; create, block_orth
 *    and the eigensolver calls are synchronous.
 *  - Buffers handed to TP3B_FP64 calls hold doubles; buffers handed to
 *    TP3B_FP32 / TP3B_BF16X3 calls hold floats (storage follows the compute
 *    precision).
 *  - One handle per thread; distinct handles are independent.
 */
#ifndef TP3B_H
#define TP3B_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TP3B_OK = 0,
  TP3B_EINVAL = -1,     /* bad argument, shape or descriptor (checked before any launch) */
  TP3B_ENOMEM = -2,     /* device or host allocation failed, or above the workspace cap */
  TP3B_EDEVICE = -3,    /* a HIP call failed; the message carries the HIP error string */
  TP3B_ENOCONV = -4,    /* eigensolver stopped before nev pairs converged */
  TP3B_ENOTSUP = -5,    /* valid request that the library does not support */
  TP3B_ENONFINITE = -6  /* NaN or Inf found in an input (when checking is enabled) */
} tp3b_status;

/* Compute precision of the mode products.  FP64: MFMA f64.  FP32: MFMA f32 with
 * FP32 accumulation.  BF16X3: each FP32 operand split into bf16 hi + lo, the
 * product formed as hi*hi + hi*lo + lo*hi on bf16 MFMA with FP32 accumulation
 * (about 16 significant bits per product; the potential term and the
 * preconditioner's divide stay FP32).  Mode products with an output tile of
 * 32 x 32 run as 64 x 64 in BF16X3. */
typedef enum { TP3B_FP64 = 0, TP3B_FP32 = 1, TP3B_BF16X3 = 2 } tp3b_prec;

/* Pair potential u(r) between the light particle and one heavy particle; the
 * three-body potential is V = u(|y - x/2|) + u(|y + x/2|) (eq. (3), read with x
 * the heavy-heavy and y the light-particle Jacobi coordinate). */
typedef enum {
  TP3B_POT_GAUSS = 0,       /* -v0 exp(-r^2 / (2 width^2))          */
  TP3B_POT_GAUSS_PAPER = 1, /* -v0 exp(-r^2)            (eq. (4))   */
  TP3B_POT_LORENTZ3 = 2,    /* -v0 / (1 + r^2)^3        (eq. (5))   */
  TP3B_POT_HARMONIC = 3,    /* +v0 r^2 / 2  (closed-form test case) */
  TP3B_POT_TABLE = 4        /* V given point by point in V_table     */
} tp3b_pot;

typedef struct tp3b_op_s* tp3b_op;

/* Grid of each mode (Sec. 3.1). */
typedef enum {
  TP3B_GRID_CGL = 0,    /* n[k] interior Gauss-Lobatto points of [-L[k], L[k]],
                           homogeneous Dirichlet conditions (end points removed) */
  TP3B_GRID_MAPPED = 1  /* the paper's grid: roots of T_N carried to the whole real
                           line by the algebraic map x = L[k] t / sqrt(1 - t^2)
                           (no boundary condition) */
} tp3b_grid;

/* Problem descriptor (Sec. 2-3).  H = -c_x Lap_x - c_y Lap_y + V, discretised on
 * n[k] unknowns per mode on the grid selected by `grid` (default: Gauss-Lobatto
 * points of [-L[k], L[k]] with Dirichlet conditions). */
typedef struct {
  int32_t ndim;            /* 1 (two modes x, y) or 2 (four modes x1, x2, y1, y2) */
  int32_t n[4];            /* points per mode, order x1,(x2),y1,(y2); each >= 2 */
  double L[4];             /* half-widths of the intervals, > 0 */
  double c_x, c_y;         /* kinetic coefficients, > 0 */
  int32_t pot;             /* tp3b_pot */
  double v0, width;        /* potential depth and (TP3B_POT_GAUSS) width */
  const double* V_table;   /* TP3B_POT_TABLE: N host values in vector layout, copied */
  const double* D2[4];     /* optional host n_k x n_k row-major second-derivative
                              matrices (the operator form of eq. (9)); NULL selects
                              the Chebyshev-Gauss-Lobatto matrix; copied */
  double sigma;            /* preconditioner shift; NaN selects the two-body ground
                              energy on the y grid with reduced mass mu_hl */
  double mu_hl;            /* heavy-light reduced mass for the default shift */
  int32_t grid;            /* a tp3b_grid value; 0 = Gauss-Lobatto with Dirichlet conditions */
  int32_t parity[4];       /* TP3B_GRID_MAPPED only, per mode: 0 = full grid of n[k]
                              points; +1 / -1 = functions even / odd under x -> -x
                              (the parity selection rule of Sec. 5.1): a 2 n[k]-point
                              grid of which the n[k] positive nodes carry the
                              unknowns.  1D: parity[0] = +1 / -1 selects bosonic /
                              fermionic heavy particles (heavy exchange is x -> -x) */
} tp3b_problem_desc;

/* Creates an operator: builds the second-derivative matrices, the potential
 * table, the preconditioner's eigen-factors of every mode and uploads them to
 * the current HIP device (in FP64 and FP32, and for modes whose size is a
 * multiple of 32 also split into bf16 hi and lo for the BF16x3 products: 4 n^2
 * bytes for each of the mode's six n x n matrices, 24 n^2 per mode).
 * Synchronous.  *out receives the handle. */
tp3b_status tp3b_create(const tp3b_problem_desc* desc, void* stream, tp3b_op* out);
tp3b_status tp3b_destroy(tp3b_op op);

/* Sizes and derived quantities of an operator (any pointer may be NULL):
 * N, the preconditioner shift sigma, and the smallest |denominator| of the
 * preconditioner's eigenbasis divide. */
tp3b_status tp3b_op_info(tp3b_op op, int64_t* N, double* sigma, double* lambda_min_kinetic);

/* Copies mode k's n_k x n_k second-derivative matrix (row-major) or the N
 * potential values (vector layout) to host memory. */
tp3b_status tp3b_get_D2(tp3b_op op, int32_t mode, double* host_out);
tp3b_status tp3b_get_V(tp3b_op op, double* host_out);

/* Y = H X for nvec vectors (eqs. (10), (11)): one dense product per tensor mode,
 * all modes summed, plus V o X fused into the epilogue.  X and Y must not
 * overlap.  `shifts`, if not NULL, is a device array of nvec doubles s_v and the
 * call returns Y = (H - s_v I) X instead. */
tp3b_status tp3b_apply_H(tp3b_op op, int32_t prec, int32_t nvec, const void* X, int64_t ldx,
                         void* Y, int64_t ldy, void* stream);
tp3b_status tp3b_apply_H_shifted(tp3b_op op, int32_t prec, int32_t nvec, const void* X,
                                 int64_t ldx, void* Y, int64_t ldy, const double* shifts,
                                 void* stream);

/* Y = (K - sigma I)^{-1} X with K the kinetic Kronecker sum (eq. (14)).  1D:
 * per vector the Sylvester equation (K_x - s_x I) Z + Z (K_y - s_y I)^T = B,
 * s_x + s_y = sigma, split in proportion to c_x and c_y, solved in the
 * eigenbasis of K_x and K_y (four mode products and a pointwise divide), which
 * is exact, as the paper's Bartels-Stewart solve is.  2D (the paper has no 2D
 * preconditioner; this extends the same construction): the four-mode sum
 * K_x1 + K_x2 + K_y1 + K_y2 - sigma is inverted in the eigenbases of the four
 * mode operators (eight mode products and a divide).  TP3B_ENOTSUP if a mode
 * operator has a complex spectrum or a denominator vanishes.  X and Y may not
 * overlap. */
tp3b_status tp3b_apply_prec(tp3b_op op, int32_t prec, int32_t nvec, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, void* stream);

/* Block orthogonalisation in FP64.  Q: device N x nq with orthonormal columns
 * (nq may be 0); X: device N x nx, overwritten by an orthonormal basis of the
 * part of span(X) orthogonal to Q.  Two classical Gram-Schmidt passes against Q,
 * then Cholesky-QR applied twice.  On return, if *rank == nx,
 * X_in = Q C_qx + X_out R_xx with R_xx upper triangular, positive diagonal.
 * C_qx (device nq x nx, column-major, ld nq) and R_xx (device nx x nx,
 * column-major) may be NULL.  A column whose norm after projection falls below
 * 1e-7 of its input norm is replaced by a pseudo-random vector (seeded by
 * `seed`) orthogonalised in its place, and *rank counts only the independent
 * columns.  nx <= 32.  Synchronous.  ENONFINITE if X holds NaN/Inf. */
tp3b_status tp3b_block_orth(int64_t N, int32_t nq, const double* Q, int64_t ldq, int32_t nx,
                            double* X, int64_t ldx, double* C_qx, double* R_xx, int32_t* rank,
                            uint64_t seed, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): tp3b_block_orth without
 * the factors, with its scratch (the partial sums of the block dots, the small
 * Gram and Cholesky factors and the dependence flags) taken from a fixed array
 * of 16.25 MiB that the library holds in device memory, one per GPU, until the
 * process ends.  The call allocates nothing; the caller passes Q and X as for
 * tp3b_block_orth, and the result is what tp3b_block_orth with
 * C_qx = R_xx = NULL computes (the same kernels in the same order while no
 * column is dependent).  A dependent column is replaced by a pseudo-random
 * vector and the queued sequence is run again.  Sizes: nx <= 32 and nq such
 * that the partial sums fit (nq <= 64 always does); larger requests return
 * TP3B_ENOMEM before any launch.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (other threads, other streams) race and must be serialised by the caller.
 * Synchronous (one read-back of the dependence flags). */
tp3b_status tp3b_block_orth_noalloc(int64_t N, int32_t nq, const double* Q, int64_t ldq, int32_t nx,
                                    double* X, int64_t ldx, int32_t* rank, uint64_t seed,
                                    void* stream);

/* Eigensolver options (Sec. 4.1).  Zero/negative fields select defaults
 * (except stall_tol; start from tp3b_jdqr_default_opts). */
typedef struct {
  int32_t nev;          /* wanted eigenpairs (smallest real part) */
  int32_t block;        /* block size b (vectors added per outer iteration) */
  int32_t m_min, m_max; /* restart sizes; default m_max = max(4b, 2(nev+b)) rounded
                           up to a multiple of b, m_min = m_max/2 */
  int32_t gmres_steps;  /* fixed GMRES steps per correction equation, default 10 */
  int32_t max_outer;    /* outer iteration cap, default 1000 */
  int32_t precond;      /* 0: none, 1: kinetic preconditioner (tp3b_apply_prec) */
  int32_t inner_prec;   /* tp3b_prec of the GMRES applies; outer work is FP64 */
  double tol;           /* lock when ||r|| <= tol max(|theta|, 1); default 1e-12 */
  double switch_tol;    /* use `target` as the correction shift while
                           ||r|| > switch_tol |theta|; default 1e-2 */
  double target;        /* NaN: the preconditioner shift sigma */
  uint64_t seed;        /* start block and rank-repair vectors */
  int32_t check_finite; /* reject NaN/Inf in X0 */
  int32_t verbose;      /* print one line per outer iteration to stderr */
  int32_t profile;      /* time the mode-product launches with HIP events (stats) */
  int32_t graph;        /* capture the GMRES inner iteration (right-hand side and
                           the fixed steps) as a HIP graph and replay it every
                           outer iteration; the single-instance solver keeps one
                           graph per projection width and block width
                           (0 = launch eagerly) */
  double stall_tol;     /* when nothing locks, lock the leading pair once its
                           residual is <= stall_tol max(|theta|, 1) and has stayed
                           within 10% of its previous value for three outer
                           iterations (the FP64 rounding floor of the residual
                           grows with ||H||); default 1e-8, <= 0 disables */
  int32_t low_start;    /* in the first low_start outer iterations, while no pair
                           has locked, the correction shift of unconverged
                           columns is a lower bound of the spectrum (min V + the
                           smallest eigenvalue of each kinetic mode operator)
                           instead of `target`, so that a ground state far below
                           the target is not passed over (default 3; 0 = off) */
  int32_t test_dup_column; /* testing hook (single-instance solver): at this outer
                           iteration the second correction column is made a copy
                           of the first before the basis is extended, which
                           exercises the replacement of dependent columns
                           (0 = off, the default) */
} tp3b_jdqr_opts;

typedef struct {
  int32_t n_conv, n_outer, n_restart, n_lock_events;
  int64_t n_apply_H_fp64, n_apply_H_low, n_apply_prec;
  double t_apply, t_prec, t_orth, t_rr, t_gmres, t_total; /* seconds */
  /* with opts.profile: device time (s), launch-group count and vectors of the
     timed launch groups of
     [0] FP64 H applies, [1] low-precision H applies,
     [2] FP64 preconditioner applies, [3] low-precision preconditioner applies.
     Launches replayed from a captured graph (opts.graph) are not timed. */
  double t_kernel[4];
  int64_t n_kernel[4];
  int64_t v_kernel[4];
  int32_t n_stall_lock;    /* pairs locked by the stagnation rule (opts.stall_tol)
                              rather than by the residual tolerance */
  int32_t n_dep_replaced;  /* dependent expansion columns replaced by random
                              vectors */
} tp3b_jdqr_stats;

tp3b_status tp3b_jdqr_default_opts(tp3b_jdqr_opts* opts);

/* Partial Schur form H Q = Q R for the nev eigenvalues of smallest real part
 * (eq. (12)) by block JDQR with GMRES on the correction equation (eq. (13)).
 * X0: optional device N x b0 start block (NULL: seeded normal block).
 * evals: host nev, ascending by real part (real parts; complex pairs are not
 * expected for these operators and are reported by their real part).
 * Q: optional device N x nev (ld N) Schur vectors; R: optional host nev x nev
 * column-major; resnorm: optional host nev residual norms at locking.
 * Synchronous.  ENOCONV: fewer than nev converged within max_outer; the
 * converged prefix (stats->n_conv) is returned. */
tp3b_status tp3b_jdqr_solve(tp3b_op op, const tp3b_jdqr_opts* opts, const double* X0, int32_t b0,
                            double* evals, double* Q, double* R, double* resnorm,
                            tp3b_jdqr_stats* stats);

/* ---- The paper's procedure over binding energies (Sec. 2; Sec. 5.1, 5.2).
 *
 * Depth v0 of the pair potential -v0 f(|xi|) for which the heavy-light
 * two-body Hamiltonian -(1/(2 mu_hl)) Lap - v0 f has the eigenvalue -E0
 * (eq. (1)), i.e. the smallest positive eigenvalue of the generalized problem
 * (-(1/(2 mu_hl)) Lap + E0) psi = v0 F psi, F = diag f(|xi|).  The relative
 * coordinate lives on the descriptor's light-particle modes: mode 1 for
 * ndim = 1 (xi on that grid, |xi| = |y|), modes 2 and 3 for ndim = 2 (their
 * Cartesian product, |xi| = hypot(y1, y2)), with the descriptor's grid,
 * parity and D2 overrides; f is the shape of desc->pot (TP3B_POT_GAUSS with
 * desc->width, TP3B_POT_GAUSS_PAPER or TP3B_POT_LORENTZ3; others: ENOTSUP);
 * desc->v0 and the heavy-particle modes are ignored.  E0 > 0.  Light-particle
 * mode sizes at most 1024.  Host computation (no device work, no stream);
 * ENOCONV if the iteration does not settle or no bound state exists. */
tp3b_status tp3b_two_body_depth(const tp3b_problem_desc* desc, double E0, double* v0);

/* The whole procedure for count binding energies E0[0], E0[1], ... (in the
 * paper: decreasing): for each, v0[i] = tp3b_two_body_depth(two_body or, if
 * NULL, desc; E0[i]); the three-body operator of desc with depth v0[i] and, if
 * desc->sigma is NaN, the preconditioner shift -E0[i] (the two-body
 * threshold); and tp3b_jdqr_solve with opts.  Every solve after the first
 * starts from the previous solve's nev Schur vectors (homotopy, Sec. 5.2).
 * Outputs are host arrays, each may be NULL: v0[count], evals[count * nev] and
 * resnorm[count * nev] (row i for E0[i]), n_outer[count].  Synchronous; stops
 * at the first failing step and returns its status (earlier rows are valid). */
tp3b_status tp3b_homotopy_solve(const tp3b_problem_desc* desc, const tp3b_problem_desc* two_body,
                                const tp3b_jdqr_opts* opts, int32_t count, const double* E0,
                                double* v0, double* evals, double* resnorm, int32_t* n_outer);

/* ---- Batched forms: many independent 1D operators (instances) at once.
 * Every step of the method runs as one grouped, persistent launch over all
 * instances (one launch per tile shape in use): a device job table holds one
 * job per instance, and each workgroup loops over its share of the tiles.
 * Instances may differ in grid size, coefficients and potential.  All ops must
 * be 1D and live on the current device; `count` >= 1. */

/* Y_i = H_i X_i (or (H_i - s) X_i with shifts[i] a device array of nvec
 * doubles, if shifts is not NULL) for i < count.  X[i], Y[i]: device blocks of
 * nvec vectors of op i (column-major N_i x nvec, leading dimensions ldx[i],
 * ldy[i] >= N_i); X, Y, ldx, ldy (and shifts) are host arrays of count entries.
 * Precision and storage as for tp3b_apply_H.  Stream-ordered; the job tables
 * are staged through the library's pinned buffer, so the call waits for the
 * previous batched call on the same thread to have consumed its tables. */
tp3b_status tp3b_apply_H_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                 const void* const* X, const int64_t* ldx, void* const* Y,
                                 const int64_t* ldy, const double* const* shifts, void* stream);

/* Y_i = (K_i - sigma_i I)^{-1} X_i for i < count (tp3b_apply_prec per
 * instance, four grouped mode-product launches).  nvec <= 64. */
tp3b_status tp3b_apply_prec_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                    const void* const* X, const int64_t* ldx, void* const* Y,
                                    const int64_t* ldy, void* stream);

/* Autotuner for a batch: instances are grouped by grid size (n_x, n_y); for
 * every group and tile shape the grouped Hamiltonian and preconditioner applies
 * of that group are timed (`reps` repetitions, HIP events), and the fastest
 * shape is stored in every operator of the group (as tp3b_autotune does for
 * one operator).  Synchronous; allocates and frees scratch blocks. */
tp3b_status tp3b_autotune_batched(const tp3b_op* ops, int32_t count, int32_t prec, int32_t nvec,
                                  int32_t reps);

/* Block JDQR on `count` independent instances at once (tp3b_jdqr_solve per
 * instance, same options for all).  The instances advance together: each
 * outer iteration performs the Rayleigh-Ritz step, the residuals, locking and
 * restart of every unconverged instance, then the correction equations of all
 * instances that did not lock, every device step as one grouped launch.  Seeds:
 * instance i starts from the counter-based block of seed opts->seed + i.
 * evals: host count x nev (row i = instance i, ascending); resnorm: host
 * count x nev or NULL; n_conv, n_outer: host arrays of count or NULL; Q: NULL
 * or a host array of count device pointers (each NULL or N_i x nev) receiving
 * the Schur vectors; stats: totals over the batch (n_outer = the largest).
 * Synchronous.  The instances' small dense problems (the ordered Schur forms
 * of their projected matrices) are solved on up to 8 host threads that the
 * call starts and joins; their results do not depend on the thread count.
 * ENOCONV if any instance stopped short of nev pairs (its converged prefix is
 * returned, the rest of its row is NaN). */
tp3b_status tp3b_jdqr_solve_batched(const tp3b_op* ops, int32_t count, const tp3b_jdqr_opts* opts,
                                    double* evals, double* resnorm, int32_t* n_conv,
                                    int32_t* n_outer, double* const* Q, tp3b_jdqr_stats* stats);

/* Mode-product tile shape used by this operator's applies: 0 = 32x32,
 * 1 = 64x64, 2 = 128x128, 3 = 64x128 output tile per 256-thread workgroup,
 * 4 = 32x32 per 512-thread workgroup (the contraction split over eight
 * wavefronts); -1 restores the built-in choice (or the autotuned one, see
 * below).  BF16x3 applies run tiles 0 and 4 as tile 1.  EINVAL outside -1..4. */
tp3b_status tp3b_set_tile(tp3b_op op, int32_t tile);

/* Autotuner: times every tile shape for the Hamiltonian apply and the
 * preconditioner of this operator at `nvec` vectors in precision `prec` on
 * scratch blocks (HIP events, `reps` repetitions each) and keeps the fastest
 * per (precision, apply kind).  Synchronous; allocates and frees its scratch
 * blocks.  best_ms (optional, host 2 doubles) receives the winning times. */
tp3b_status tp3b_autotune(tp3b_op op, int32_t prec, int32_t nvec, int32_t reps, double* best_ms);

/* Library-internal dense host routine exposed for host-side testing: real Schur
 * form of a small n x n row-major matrix A (overwritten by T), Schur vectors Z
 * (row-major, may be NULL), eigenvalue real/imaginary parts wr, wi. */
tp3b_status tp3b_host_schur(int32_t n, double* A, double* Z, double* wr, double* wi);

const char* tp3b_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TP3B_H */
