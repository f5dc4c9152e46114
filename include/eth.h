/*
 * eth.h -- C ABI of the MI355X (gfx950) solvers for the enriched Taylor-Hood
 * discretisation of Pestana & Silvester, "Fast solution of incompressible flow
 * problems with two-level pressure approximation" (arXiv 2303.10233).
 *
 * Discrete problem (Sec. 2, eq:stokes_fe / eq:saddle_point; Sec. 3,
 * eq:oseen-system): on a uniform n x n mesh of square Q2 elements, find
 * x = [u; p] with K x = b, where
 *     K = [ F  B^T ]     F = nu*A (Stokes) or nu*A + N(w) (Oseen),
 *         [ B   0  ]     A: vector Q2 Laplacian, N(w): Q2 convection by the
 *                        nodal Q2 wind w, B: -int q div u,
 * and the pressure is given in the frame Q1 + P0 (eq:eth_spec): n_k = (n+1)^2
 * Q1 coefficients followed by n_0 = n^2 element coefficients.  The frame null
 * vector k = [1; -1] (eq:pressure_null_vector) lies in null(B^T)
 * (rem:Bnull) and in null(M_Q) (prop:Qnull); for enclosed flow null(K) is
 * spanned by [0; 1_{n_k}; 0] and [0; 0; 1_{n_0}].
 *
 * VECTOR LAYOUT (all vectors FP64, device memory, caller-owned):
 *     [ u_x on all (2n+1)^2 Q2 nodes | u_y (same) | p_k (n+1)^2 | p_0 n^2 ]
 * Node (I,J) of an m x m grid is entry J*m + I (x fastest); element (ex,ey) is
 * entry ey*n + ex.  N = eth_vector_length() = 2(2n+1)^2 + (n+1)^2 + n^2.
 * A batch of `batch` vectors is stored with stride `ld` >= N (elements).
 * The velocity on boundary nodes is Dirichlet data: the operator acts on the
 * interior velocity x all pressure coefficients.
 *
 * ERRORS: every int-returning call returns 0 on success, a negative ETH_E*
 * code on failure (nothing is written to outputs unless stated) and a
 * positive ETH_W* code for a warning.  eth_last_error() gives a message.
 * Calls are ordered on the stream given at setup; handles are not thread-safe.
 */
#ifndef ETH_H
#define ETH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ETH_OK             0
#define ETH_EINVAL        -1  /* invalid argument (size, pointer, option)          */
#define ETH_EDEVICE       -2  /* a HIP runtime error                                */
#define ETH_ENOMEM        -3  /* device allocation failed during setup              */
#define ETH_EINCONSISTENT -4  /* enclosed-flow RHS not orthogonal to null(K^T)      */
#define ETH_EBREAKDOWN    -5  /* Krylov breakdown (gamma^2 < 0, NaN or Inf)         */
#define ETH_EUNSUPPORTED  -6  /* option combination not available                   */
#define ETH_WMAXIT         1  /* iteration limit reached; x holds the last iterate  */
#define ETH_WNOPROGRESS    2  /* FGMRES ended with a true residual above that of the
                                 initial guess; x holds the initial guess           */

typedef struct eth_problem eth_problem;

typedef enum { ETH_STOKES = 0, ETH_OSEEN = 1 } eth_kind;
typedef enum { ETH_FP64 = 0, ETH_MIXED = 1 } eth_precision;
/* velocity block of the preconditioner */
typedef enum { ETH_VEL_GMG = 0, ETH_VEL_EXACT = 1 } eth_velocity_mode;
/* pressure block: M_S in the bordered system [[M_S, k], [k^T, 0]] (Sec. 2.2).
 * ETH_MQ_SCHUR_GMG: elimination of the P0 block (Q_0 = h^2 I, Sec. 2.3),
 * z_k = B (r_k - R^T Q_0^{-1} r_0), z_0 = Q_0^{-1}(r_0 - R z_k), with B one Q1
 * multigrid V-cycle for S_k = Q_k - R^T Q_0^{-1} R and k-projection of input
 * and output: mesh independent, unlike the Chebyshev-SGS solve. */
typedef enum { ETH_MQ_DIAG = 1, ETH_MQ_CHEB_SGS = 2, ETH_MQ_SCHUR_GMG = 3 } eth_mq_mode;
typedef enum { ETH_MINRES = 0, ETH_FGMRES = 1, ETH_TWO_STAGE = 2 } eth_method;

/*
 * Problem description.  Zero-initialise, then set what you need; a zero in an
 * optional field selects the documented default.
 */
typedef struct {
  int32_t n;                 /* Q2 elements per side, >= 2                         */
  double x0, x1, y0, y1;     /* square domain (x1-x0 == y1-y0)                      */
  int32_t kind;              /* eth_kind                                            */
  double nu;                 /* viscosity, > 0 (Stokes: -nu Lap u + grad p = f)     */
  const double* wind;        /* Oseen: device, 2(2n+1)^2 nodal Q2 wind [w_x|w_y]    */
  double lid_u;              /* tangential lid velocity on y = y1                   */
  int32_t corner_mode;       /* 0: top corners get 0 (watertight); 1: lid value;
                                2: regularised lid lid_u (1 - xi^4), xi in [-1, 1]
                                across the top wall (the enclosed-flow example of
                                Sec. 3)                                           */
  int32_t velocity_mode;     /* eth_velocity_mode; EXACT needs (2n-1)^2 <= 4096     */
  int32_t mq_mode;           /* eth_mq_mode (default ETH_MQ_CHEB_SGS)               */
  int32_t mq_steps;          /* Chebyshev steps for ETH_MQ_CHEB_SGS (default 20)    */
  double mq_cheb_lo;         /* eigen-interval of M_SGS^{-1} M_Q (default min(0.01, 0.4/n)) */
  double mq_cheb_hi;         /*   (default 1, the SGS bound)                        */
  int32_t gmg_coarse_n;      /* halve while n even and n > gmg_coarse_n (default 4;
                                the coarsest level is solved with a dense inverse,
                                so n = m 2^k needs an odd factor m <= 49;
                                Oseen 32: coarse levels of the unstabilised F must
                                keep a moderate cell Peclet number)                 */
  int32_t gmg_degree;        /* smoothing steps pre and post (default 2): Chebyshev
                                degree (Stokes) or damped-Jacobi sweeps (Oseen)     */
  double gmg_lo_frac;        /* smoother interval [lo_frac, hi_frac] * lambda_max    */
  double gmg_hi_frac;        /*   (defaults 0.3, 1.1)                               */
  const double* gmg_lambda;  /* host, optional: lambda_max(D^{-1}A) per smoothing
                                level (levels-1 values); NULL: Lanczos at setup     */
  int32_t precision;         /* eth_precision: preconditioner in FP64 or FP32       */
  int32_t max_batch;         /* largest batch passed to any call (default 1)        */
  void* stream;              /* hipStream_t for every call (NULL: default stream)   */
  /* Oseen (kind = ETH_OSEEN) preconditioners, Sec. 3 */
  double gmg_omega;          /* damped-Jacobi weight of the F multigrid (0.7)       */
  int32_t pcd_q1_steps;      /* Chebyshev-Jacobi steps for Q_1^{-1} in PCD (10)     */
  int32_t gmres_restart;     /* largest FGMRES restart length, <= 63 (50)          */
  int32_t mq_tile;           /* ETH_MQ_CHEB_SGS: Q1 nodes per side of the blocks of
                                the fused Chebyshev step, 8, 16, 24, 32 or 64 (64
                                with ETH_MIXED only); 0: the fastest, timed at
                                setup                                           */
  int32_t mq_fuse_steps;     /* Chebyshev steps per launch, 1 or 2 (2 needs tile
                                16 or 24 and ETH_MIXED); 0: 1 when mq_tile is
                                given, else timed at setup                      */
  double gmg_peclet_max;     /* Oseen: > 0 caps the element Peclet number of every
                                level of the F multigrid: level l smooths and
                                solves nu_l A + N(w) with nu_l = max(nu,
                                max|w| h_l / (2 gmg_peclet_max)); the Krylov
                                method still solves the Galerkin F.  Keeps the
                                damped-Jacobi cycle a contraction where the
                                unstabilised F is convection dominated (element
                                Peclet >= 8, e.g. nu = 1/1000 on 256^2).  0: off */
  int32_t oseen_schur;       /* Oseen: Schur block of the full-system preconditioner
                                [F~ B^T; 0 -M_S] used by ETH_FGMRES and stage II:
                                0: M_1, M_S = M_Q / nu (eq:nse-precon-ref);
                                1: M_2, the two-field PCD approximation M_S =
                                   diag(Q_1,Q_0) diag(F_1,F_0)^{-1} B M^{-1} B^T
                                   (eq:twofield-pcd) with F_0 the jump-based P0
                                   convection-diffusion operator;
                                2: M_3, the least-squares commutator M_S =
                                   (B M^{-1} B^T)(B M^{-1} F M^{-1} B^T)^{-1}
                                   (B M^{-1} B^T) (eq:lsc-definition, boundary
                                   scaling D = I).  M = diag of the velocity mass.
                                1 and 2 (comparison preconditioners of Sec. 3.1
                                and 3.2) need max_batch 1, invert B M^{-1} B^T by
                                conjugate gradients on its range, synchronise
                                with the host inside and so run without graph
                                replay, and have no transposed form              */
  double schur_cg_tol;       /* relative tolerance of that CG (default 1e-10)       */
  int32_t schur_cg_maxit;    /* its iteration limit (default 2000)                  */
} eth_problem_desc;

typedef struct {
  int32_t method;            /* eth_method (default ETH_MINRES)                     */
  double rtol;               /* MINRES: |eta|/gamma_1 (P^{-1}-norm, alg:minres);
                                GMRES: ||b-Kx||_2/||b||_2 (eq:residual-norm)       */
  int32_t maxit;             /* iteration limit (default 1000)                      */
  int32_t restart;           /* FGMRES restart length (default 50)                  */
  double c_factor;           /* two-stage: stage-I factor c (default 10)           */
  int32_t canonicalize;      /* 1: subtract the means of p_k and p_0 (default); 0:
                                the pressure is one representative of its class
                                modulo null(K) (MINRES may leave a multiple of
                                the frame null vector k in it)                    */
  int32_t use_x0;            /* 1: x holds the initial guess on entry               */
  int32_t use_graph;         /* 1: replay the iteration as a captured hipGraph;
                                2 (eth_batch_solve only): one graph holds eight
                                MINRES iterations of every member of the ragged
                                batch, replayed until no member is active (no
                                refinement restarts)                               */
  int32_t true_residual;     /* 1: compute ||b - K x||/||b|| into info (default 0)   */
  int32_t refine;            /* MINRES: at most this many FP64 defect-correction
                                restarts (default 0).  When the recurrence has met
                                rtol, the residual b - K x is formed again in FP64
                                and MINRES restarts from x until the P^{-1}-norm of
                                that true residual is <= rtol * gamma_1 (gamma_1 of
                                the first start).  With an FP32 preconditioner the
                                recurrence's |eta| and the true residual part below
                                about 1e-7; the restarts close that gap.           */
  double* residual_history;  /* host, batch x history_len doubles, or NULL: per
                                right-hand side the stopping quantity before the
                                first and after every iteration -- MINRES
                                |eta_j|/gamma_1 (a refinement restart continues the
                                sequence with the P^{-1}-norm of its FP64 residual
                                over gamma_1); FGMRES the Arnoldi estimate of
                                ||b-Kx_j||_2/||b||_2; TWO_STAGE the stage-I
                                sequence (reduced system) followed by the stage-II
                                one, whose first entry is the full residual of the
                                stage-I iterate (Sec. 3.1: it jumps up where the
                                P0 rows enter).  Entries past the end are -1.     */
  int32_t history_len;       /* entries per right-hand side of residual_history     */
} eth_solve_opts;

typedef struct {
  int32_t status;            /* per-RHS status code                                 */
  int32_t iterations;        /* Krylov iterations (both stages for TWO_STAGE)      */
  int32_t stage1_iterations; /* TWO_STAGE only                                       */
  double rel_residual_est;   /* the stopping quantity at exit                       */
  double rel_residual_true;  /* ||b-Kx||_2/||b||_2 if requested, else -1           */
} eth_solve_info;

/* Set up a problem: allocates every workspace (solves never allocate), builds
 * the multigrid hierarchy, diagonals and smoother bounds.  On success *out is
 * a new handle; on failure *out is NULL and the code is returned. */
int eth_setup(const eth_problem_desc* desc, eth_problem** out);
int eth_destroy(eth_problem* p);

/* N = 2(2n+1)^2 + (n+1)^2 + n^2 */
int64_t eth_vector_length(const eth_problem* p);
/* number of multigrid levels and the smoother lambda_max per level (host
 * array of size >= levels-1); either pointer may be NULL */
int eth_get_levels(const eth_problem* p, int32_t* levels, double* lambdas);

/* Lifted right-hand side (Sec. 2, eq:stokes_fe with the boundary velocity):
 * interior velocity rows (M_v f)_I - F_IB u_B, pressure rows -B_{:,B} u_B,
 * boundary velocity rows the Dirichlet values u_B (lid per desc).
 * f_nodal: device, 2(2n+1)^2 nodal forces [f_x|f_y] per batch entry with
 * stride ld_f (>= 2(2n+1)^2), or NULL for f = 0.  b: device, batch x ld. */
int eth_assemble_rhs(eth_problem* p, const double* f_nodal, int64_t ld_f,
                     double* b, int64_t batch, int64_t ld);

/* y = K x (transpose = 0) or K^T x (transpose = 1) on the full layout:
 * boundary velocity entries of x are ignored, those of y are set to 0. */
int eth_apply_operator(eth_problem* p, int transpose, const double* x, double* y,
                       int64_t batch, int64_t ld);

/* z = P^{-1} r.  Stokes: block-diagonal diag(nu A~, M~_S/nu) (eq:stokes_pre)
 * with the bordered pressure solve of Sec. 2.2 (z_p orthogonal to k).
 * Oseen: block upper-triangular M_1 = [F~, B^T; 0, -M~_Q/nu]
 * (eq:nse-precon-ref): z_p = -nu M~_Q^+ r_p, z_u = F~^{-1}(r_u - B^T z_p);
 * transpose = 1 gives the same preconditioner for the transposed system
 * K^T = [F^T B^T; B 0], i.e. with F~^{-T} (one multigrid cycle on F^T) in
 * place of F~^{-1} -- the preconditioner of eth_solve_adjoint.  Stokes: the
 * preconditioner is symmetric and transpose is ignored.
 * Boundary velocity entries of z are set to 0. */
int eth_apply_preconditioner(eth_problem* p, int transpose, const double* r, double* z,
                             int64_t batch, int64_t ld);

/* Solve K x = b (b from eth_assemble_rhs).  x receives the boundary data on
 * boundary rows, the Krylov solution elsewhere, the pressure canonicalised if
 * opts->canonicalize.  info: host array of `batch` entries, or NULL.
 * Consistency (Sec. 2.2): the flow is enclosed (Dirichlet velocity on the
 * whole boundary), so null(K^T) = span{[0; 1_{n_k}; 0], [0; 0; 1_{n_0}]} and
 * K x = b is solvable only if both pressure blocks of b sum to zero.  Before
 * iterating, every right-hand side is checked: when the component of the
 * interior b in that null space exceeds 1e-12 ||b_interior||_2 the call
 * returns ETH_EINCONSISTENT, and when b holds a NaN or Inf it returns
 * ETH_EINVAL; x is then not written and info (if given) receives the status
 * of every right-hand side with zero iterations.
 * Methods: ETH_MINRES (Stokes; alg:minres with P), ETH_FGMRES (Oseen, right
 * preconditioned by M_1, restarted), ETH_TWO_STAGE (Oseen, Sec. 3.1: stage I
 * FGMRES on the reduced system with PCD until ||r|| <= c*rtol*||b||, stage II
 * FGMRES on the full system with M_1 from [u_1; q_1; 0] until rtol*||b||).
 * Returns the worst per-RHS status. */
int eth_solve(eth_problem* p, const eth_solve_opts* opts, const double* b, double* x,
              int64_t batch, int64_t ld, eth_solve_info* info);

/* Oseen only: the stage-I PCD preconditioner of the reduced Taylor-Hood
 * system (Sec. 3.1, eq:reduced-system, eq:discrete-commutator1x):
 * z_pk = -A_p^+ F_1 Q_1^{-1} r_pk, z_p0 = 0, z_u = F~^{-1}(r_u - B_1^T z_pk),
 * with A_p = B_1 diag(M_v)^{-1} B_1^T; the p_0 part of r is ignored.
 * transpose = 1: the same construction for the transposed reduced system
 * [F^T B_1^T; B_1 0] (stage I of the adjoint): the Schur complement S^T is
 * approximated by A_p F_1^{-T} Q_1, so z_pk = -Q_1^{-1} F_1^T A_p^+ r_pk and
 * z_u = F~^{-T}(r_u - B_1^T z_pk). */
int eth_apply_pcd(eth_problem* p, int transpose, const double* r, double* z, int64_t batch,
                  int64_t ld);
/* The Q1 multigrid of the problem -- A_p inside PCD (Oseen) or S_k of
 * ETH_MQ_SCHUR_GMG (Stokes) -- : number of levels and the Chebyshev bounds
 * lambda_max(D^{-1} A_l) per smoothing level (levels-1 values); either pointer
 * may be NULL.  ETH_EUNSUPPORTED when the problem has none. */
int eth_get_q1_levels(const eth_problem* p, int32_t* levels, double* lambdas);
/* Variant of the fused Chebyshev step of ETH_MQ_CHEB_SGS in use for one
 * right-hand side (tile side tile_1, Chebyshev steps per launch steps_1) and
 * for max_batch of them (tile_max, steps_max); any pointer may be NULL.
 * ETH_EUNSUPPORTED for other mq_mode values. */
int eth_get_mq_tile(const eth_problem* p, int32_t* tile_1, int32_t* tile_max, int32_t* steps_1,
                    int32_t* steps_max);

/* Set-up choices made by timing (the fused Chebyshev step's variant for one
 * and for max_batch right-hand sides, the V(2,2) smoothing launch pattern):
 * how many were timed during this set-up and how many were read from the
 * set-up cache instead.  The cache is a text file of "key value" lines keyed
 * by device (architecture, compute units), kernel or launch pattern, storage
 * type, mesh size and batch: $ETH_TUNE_CACHE (empty: no cache), default
 * $HOME/.cache/eth_tune.txt.  Either pointer may be NULL. */
int eth_tuning_source(const eth_problem* p, int32_t* timed, int32_t* cached);

/* Replace the nodal Q2 wind of an Oseen problem (device, 2(2n+1)^2
 * [w_x|w_y], the w_h of eq:generic-conv-diff) and rebuild what depends on it:
 * the wind and the F diagonal of every multigrid level and the dense inverse
 * of the coarsest F.  Allocates nothing; stream-ordered; the wind is copied.
 * ETH_EUNSUPPORTED for Stokes problems. */
int eth_set_wind(eth_problem* p, const double* wind);

/* Picard iteration for the steady Navier-Stokes equations (Sec. 3: the wind
 * is the velocity of the most recent nonlinear iterate).  x (device, full
 * layout, one right-hand side) holds the current iterate on entry, e.g. the
 * Stokes solution with the same boundary data; each of `steps` steps sets the
 * wind to the velocity of x (eth_set_wind), lifts the right-hand side
 * (eth_assemble_rhs with f_nodal, NULL: f = 0) and solves the Oseen system
 * with x as the initial guess (opts->use_x0 is forced to 1; opts NULL:
 * ETH_TWO_STAGE, canonicalize = 1).  On return x is the last iterate and the
 * problem holds its wind, so eth_solve then solves the Oseen system of the
 * next step.  info: NULL or `steps` entries, one per step.  Returns the worst
 * status; a negative status ends the iteration at once. */
int eth_picard(eth_problem* p, const eth_solve_opts* opts, int32_t steps, const double* f_nodal,
               double* x, eth_solve_info* info);

/* Discrete adjoint (K^T lambda = g) of a solve, for gradients of
 * J(x(f, nu)) through the lifted system (eq:saddle_point, eq:oseen-system).
 * g: device, batch x ld, dJ/dx on the full layout; its boundary velocity
 * rows are ignored and the means of its p_k and p_0 blocks are removed
 * first (that component lies in null(K) and has no adjoint).  lambda
 * receives the adjoint with zero boundary velocity rows, the pressure
 * canonicalised if opts->canonicalize.  Stokes: MINRES with the forward
 * preconditioner (K is symmetric).  Oseen: K^T = [F^T B^T; B 0] has the
 * structure of K with F^T for F, and is solved like K: ETH_TWO_STAGE (the
 * default) runs stage I with the transposed PCD (eth_apply_pcd, transpose =
 * 1) and stage II with [F~^T B^T; 0 -M~_Q/nu]; ETH_FGMRES only the latter.
 * opts NULL: defaults with canonicalize = 1.  Returns the worst per-RHS
 * status. */
int eth_solve_adjoint(eth_problem* p, const eth_solve_opts* opts, const double* g,
                      double* lambda, int64_t batch, int64_t ld, eth_solve_info* info);
/* dJ/df = M_v lambda~ on all 2(2n+1)^2 nodal forces, lambda~ = the velocity of
 * lambda with its boundary rows zeroed (b_u = (M_v f)_I).  dJdf: device,
 * batch x ld_f (ld_f >= 2(2n+1)^2 when batch > 1). */
int eth_grad_forcing(eth_problem* p, const double* lambda, int64_t ld, double* dJdf,
                     int64_t ld_f, int64_t batch);
/* dJ/dnu = -lambda_u^T (A u)_I per RHS, u = the full velocity of x (boundary
 * values included: K depends on nu through nu A_II, b through -nu A_IB u_B).
 * lambda and x: batch x ld; dJdnu: device, batch doubles. */
int eth_grad_viscosity(eth_problem* p, const double* lambda, const double* x, double* dJdnu,
                       int64_t batch, int64_t ld);
/* J = 1/2 (u - u_t)^T M_v (u - u_t) over all velocity nodes, u and u_t the
 * velocities of x and x_target (batch x ld).  J: device, batch doubles.
 * grad (device, batch x ld, or NULL): dJ/dx = [M_v (u - u_t); 0]. */
int eth_misfit(eth_problem* p, const double* x, const double* x_target, double* J,
               double* grad, int64_t batch, int64_t ld);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): eth_misfit
 * without a problem handle.  desc supplies n, the domain (square) and the
 * stream; every other field is ignored.  x, x_target, J, grad as for
 * eth_misfit (grad may be NULL).  Allocates nothing: the partial sums of the
 * reduction go to a fixed 2 MiB device array of the library (one per GPU,
 * held until the process ends), so batch * 2 * ceil((2n+1)^2 / 256) must not
 * exceed 262144 (one right-hand side up to n = 2048, eight at n = 1024);
 * larger calls return ETH_EINVAL with a message in eth_last_error(NULL).
 * The current device must be the one holding the vectors and the stream.
 * Calls that overlap in time on one GPU share that array and race: order
 * them on one stream (the array keeps the last call's partial sums). */
int eth_misfit_noalloc(const eth_problem_desc* desc, const double* x, const double* x_target,
                       double* J, double* grad, int64_t batch, int64_t ld);

/* Ragged batches: several Stokes problems of different sizes (e.g. cavities
 * of 32..256 elements per side) solved together.  Every problem gets its own
 * stream and workspaces; eth_batch_solve starts all MINRES solves, keeps each
 * one's iteration chunks (hipGraph replays) queued on its own stream and
 * polls their device-side convergence flags without blocking, so the
 * problems run concurrently on the GPU.  descs[i] as for eth_setup (kind must
 * be ETH_STOKES); descs[0].stream is the caller's stream: eth_batch_solve
 * waits for the work already queued on it and makes it wait for the results.
 * Each problem takes one right-hand side.  Members run their preconditioner
 * blocks one after the other (the batch itself is the concurrency), and
 * mq_fuse_steps = 0 means one Chebyshev step per launch here. */
typedef struct eth_batch eth_batch;
int eth_batch_setup(const eth_problem_desc* descs, int32_t count, eth_batch** out);
int eth_batch_count(const eth_batch* b);
/* borrowed handle of problem i (for eth_assemble_rhs, eth_apply_operator, ...);
 * owned by the batch, valid until eth_batch_destroy.  Calls on it are ordered
 * on the problem's own stream. */
int eth_batch_problem(eth_batch* b, int32_t i, eth_problem** out);
/* b[i], x[i]: device vectors of problem i (length eth_vector_length of it);
 * opts as for eth_solve (method ETH_MINRES); infos: host array of count
 * entries or NULL.  Returns the worst status. */
int eth_batch_solve(eth_batch* b, const eth_solve_opts* opts, const double* const* bvecs,
                    double* const* xvecs, eth_solve_info* infos);
const char* eth_batch_last_error(const eth_batch* b);
int eth_batch_destroy(eth_batch* b);

/* EST-MINRES estimate of the discrete inf-sup constant (Sec. 2.4,
 * eq:inf-sup_eig) from the last MINRES solve of right-hand side `rhs`
 * (Stokes): the Lanczos scalars delta_j, gamma_j of alg:minres are recorded
 * on the device during the solve; the harmonic Ritz values theta of the
 * preconditioned matrix follow from them, and with the negative theta closest
 * to zero gamma^2 = theta (theta - 1) (the eigenvalues (1 +- sqrt(1 + 4
 * sigma))/2 of diag(A, M_Q)^{-1} K).  The estimate is of the preconditioned
 * operator actually used (exact blocks give the inf-sup constant itself).
 * gamma2, theta (may be NULL), steps (may be NULL): host outputs. */
int eth_infsup_estimate(eth_problem* p, int64_t rhs, double* gamma2, double* theta, int32_t* steps);

/* Kernel timing for roofline reporting.  Launches `reps` times the kernel
 * `kernel` (ETH_K_*) exactly as one Krylov iteration launches it (same grid,
 * same workspaces, finest level where a hierarchy is involved), between two
 * HIP events recorded on the problem's stream, after a prior eth_solve has
 * filled the workspaces.  Returns the average duration of one launch in
 * *avg_ms and the algorithmic bytes one launch must move (reads + writes of
 * the vectors it touches, without halo re-reads) in *bytes. */
#define ETH_K_SADDLE_APPLY   0   /* a1: K x with the fused <Kx, x> partials          */
#define ETH_K_CHEB_STEP      1   /* a3: one Chebyshev smoothing step, finest level    */
#define ETH_K_RESTRICT       2   /* a3: fused residual + restriction, finest level    */
#define ETH_K_PROLONG        3   /* a3: prolongation + correction, finest level       */
#define ETH_K_MQ_CHEB_STEP   4   /* a4: one fused Chebyshev-SGS step (9 colour passes)*/
#define ETH_K_DOT            5   /* a6: deterministic dot product over N              */
#define ETH_K_MINRES_V       6   /* a6: Lanczos vector update                         */
#define ETH_K_MINRES_WX      7   /* a6: w / x update                                  */
#define ETH_K_OSEEN_APPLY    8   /* a2: K x for Oseen, fused <Kx, x> partials          */
#define ETH_K_CD_STEP        9   /* a3: damped-Jacobi step on F, finest level          */
#define ETH_K_GM_MDOT       10   /* a7: CGS multi-dot against m/2 Arnoldi vectors      */
#define ETH_K_GM_MAXPY      11   /* a7: CGS update with m/2 Arnoldi vectors            */
#define ETH_K_COPY          12   /* plain copy of N doubles (calibrates byte counters)  */
#define ETH_K_SYNC_GRAPH    13   /* one step of a ring dependency over one block per CU
                                    per launch, reps launches replayed as one graph     */
#define ETH_K_SYNC_GRID     14   /* the same steps inside one cooperative launch,
                                    separated by grid-wide barriers (persistent form)   */
int eth_profile_kernel(eth_problem* p, int kernel, int reps, int64_t batch, double* avg_ms,
                       double* bytes);

/* ---------------------------------------------------------------------------
 * Flow over a step (Sec. 3, the inflow-outflow example): the domain
 * [-1, 0) x [0, 1] union [0, L] x [-1, 1] (L = 5 in the paper), fixed walls,
 * the parabolic inflow u_x = 4 y (1 - y) on x = -1 and the natural outflow
 * condition on x = L, squares of side h = 1/m.  With an outflow the pressure
 * function is unique: null(K) is spanned by [0; k] alone (Sec. 2, the frame
 * null vector k = [1_{n_k}; -1_{n_0}]).
 *
 * Layout of a state vector (length N, device, FP64): [u_x (n_v) | u_y (n_v) |
 * p_1 (n_k) | p_0 (n_0)] over the Q2 nodes, Q1 nodes and elements of the
 * bounding box [-1, L] x [-1, 1] that belong to the domain, each counted row
 * by row (y outer, x inner); eth_step_host_layout gives their grid indices.
 * Velocity rows of Dirichlet nodes (walls, inflow) carry the boundary values
 * in a right-hand side and in a solution; the operator ignores them.
 *
 * The geometry is not one square, so the operators are assembled on the host
 * at set-up (and again for every new wind) and applied on the GPU as
 * sliced-ELL sparse matrices; every Krylov iteration runs in kernels.
 * Solves: ETH_TWO_STAGE (Sec. 3.1: stage I FGMRES on the reduced system with
 * PCD, stage II FGMRES with M_1 of eq:nse-precon-ref) or ETH_FGMRES (M_1
 * only).  The PCD matrix F_1 carries the inflow term -int (w.n) psi_j psi_i
 * ds (without it F_1 annihilates constants while A_p does not, and stage I
 * stalls); pcd_inflow_bc = 1 leaves it out.  Pressure mass solves: Chebyshev
 * semi-iteration based on multicolour symmetric Gauss-Seidel (Sec. 2.3).
 * One right-hand side per call. */
typedef struct eth_step eth_step;

typedef struct {
  int32_t m;                 /* elements per unit length, h = 1/m                  */
  int32_t length;            /* L: the channel ends at x = L (0: 5)                 */
  int32_t channel;           /* 1: the strip [-1, L] x [0, 1] without the step      */
  double nu;                 /* viscosity (the paper: 1/50)                        */
  int32_t precision;         /* eth_precision of the preconditioner                 */
  int32_t coarse_m;          /* multigrid levels m, m/2, ... while even and above
                                coarse_m (0: 4); the last is solved densely        */
  double gmg_omega;          /* damped-Jacobi weight of the F multigrid (0: 0.7)     */
  double gmg_peclet_max;     /* >0: level viscosity max(nu, |w|_max h/(2 Pe_max))    */
  int32_t pcd_q1_steps;      /* Chebyshev-Jacobi steps for Q_1^{-1} (0: 10)          */
  int32_t pcd_inflow_bc;     /* 0: inflow term in F_1 (default); 1: none             */
  int32_t mq_steps;          /* Chebyshev-SGS steps for M_Q (0: 20)                  */
  double mq_cheb_lo;         /* lower end of the SGS interval (0: min(0.01,
                                0.4 / (m (1 + L))))                                 */
  int32_t gmres_restart;     /* FGMRES restart length, <= 63 (0: 50)                 */
  void* stream;              /* hipStream_t for every call, or NULL (own stream)   */
} eth_step_desc;

/* Host-only inspection (no GPU needed): sizes[4] = {n_v, n_k, n_0, N}; the
 * grid indices (I, J) of every Q2 node (half grid, x = -1 + I h/2), Q1 node
 * and element (lower-left corner), and the Dirichlet flag of every Q2 node.
 * Any output may be NULL. */
int eth_step_host_layout(int32_t m, int32_t length, int32_t channel, int64_t* sizes, int32_t* q2_ij,
                         int32_t* q1_ij, int32_t* el_ij, uint8_t* dirichlet);
/* Host-only assembly of one matrix in CSR form (no GPU needed): call with
 * ptr/col/val NULL for rows, cols, nnz, then again with arrays of rows+1,
 * nnz, nnz entries.  wind: host, 2 n_v nodal values, or NULL.  which: */
#define ETH_STEP_K    0   /* the saddle operator K (N x N; Dirichlet rows and columns empty) */
#define ETH_STEP_MQ   1   /* pressure mass [Q_k R^T; R Q_0] (Sec. 2.3)                       */
#define ETH_STEP_Q1   2   /* Q_1 (Sec. 3.1)                                                  */
#define ETH_STEP_F1   3   /* F_1 with the inflow term (Sec. 3.1)                             */
#define ETH_STEP_AP   4   /* A_p = B_1 diag(M_v)^{-1} B_1^T over the free velocity nodes     */
#define ETH_STEP_P    5   /* Q2 prolongation from mesh m/2 (free rows and columns)           */
#define ETH_STEP_PQ   6   /* Q1 prolongation from mesh m/2                                   */
#define ETH_STEP_RHS  7   /* the lifted right-hand side (one column of N rows)              */
int eth_step_host_matrix(int32_t m, int32_t length, int32_t channel, double nu, const double* wind,
                         int32_t which, int64_t* rows, int64_t* cols, int64_t* nnz, int64_t* ptr,
                         int32_t* col, double* val);

/* Set up: host assembly, multigrid hierarchies, smoother bounds, coarse
 * inverses and every workspace; the operator starts without a wind (Stokes). */
int eth_step_setup(const eth_step_desc* desc, eth_step** out);
int eth_step_destroy(eth_step* p);
int eth_step_sizes(const eth_step* p, int64_t* nv, int64_t* nk, int64_t* n0, int64_t* N);
/* levels of the hierarchies, m of each, and lambda_max(D^{-1} A_p) of every
 * level but the coarsest (host arrays; any may be NULL) */
int eth_step_levels(const eth_step* p, int32_t* levels, int32_t* m_per_level, double* ap_lambdas);
/* wind: device, 2 n_v nodal values (the Picard iterate's velocity, Sec. 3.1
 * text after eq:generic-conv-diff), or NULL for none; re-assembles F on every
 * level, K and F_1 on the host */
int eth_step_set_wind(eth_step* p, const double* wind);
/* b (device, N): the lifted right-hand side with the inflow data, f = 0 */
int eth_step_rhs(eth_step* p, double* b);
/* y = K x (device, N) */
int eth_step_apply(eth_step* p, const double* x, double* y);
/* z = P^{-1} r (device, N): which 1 = M_1 (stage II), 2 = stage-I PCD
 * (the p_0 part of z is zero) */
int eth_step_apply_preconditioner(eth_step* p, int32_t which, const double* r, double* z);
/* opts as for eth_solve (method ETH_TWO_STAGE or ETH_FGMRES); canonicalize
 * shifts the pressure along k so that the element pressures have mean zero.
 * b must be consistent with null(K^T) = span{[0; k]}: ETH_EINCONSISTENT when
 * |k . b_p| > 1e-10 sqrt(n_k + n_0) ||b|| (the lifted right-hand side of
 * eth_step_rhs satisfies it to rounding), ETH_EINVAL for a NaN or Inf in b. */
int eth_step_solve(eth_step* p, const eth_solve_opts* opts, const double* b, double* x, eth_solve_info* info);
/* The Stokes solution (FGMRES with M_1) followed by `steps` Picard steps, each
 * an Oseen solve by opts->method whose wind is the velocity of the previous
 * iterate, started from it.  x (device, N): the last iterate; info: host
 * array of steps + 1 entries or NULL.  The problem keeps the last wind. */
int eth_step_picard(eth_step* p, const eth_solve_opts* opts, int32_t steps, double* x, eth_solve_info* info);
const char* eth_step_last_error(const eth_step* p);

const char* eth_status_string(int status);
/* message of the last failing call on this handle (or of the last failing
 * eth_setup when p is NULL); valid until the next call */
const char* eth_last_error(const eth_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* ETH_H */
