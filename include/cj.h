/*
 * cj.h -- C ABI of libcj.so, the Chebyshev-Jacobi method (CJM) for the 2D
 * finite-difference Poisson problem on AMD Instinct MI355X (gfx950).
 *
 * The method (Adsuara et al., "Speeding up a few orders of magnitude the
 * Jacobi method: high order Chebyshev-Jacobi over GPUs", §2.1): a weighted
 * Jacobi iteration u <- u + omega_n D^{-1} (f - A u) whose weights omega_n are
 * the reciprocals of the zeros of a Chebyshev polynomial mapped onto the
 * interval [kappa_min, kappa_max] that bounds the spectrum of D^{-1} A.  The
 * bounds are the paper's closed forms (§2.1, Eqs. for kappa^(9), kappa^(17);
 * the 5-point bounds follow from the stencil symbol).  The weights are
 * computed once per plan on the host in FP64 and applied in a fixed order.
 *
 * Problem.  nx x ny interior unknowns u(i, j), 1 <= i <= nx, 1 <= j <= ny, at
 * x_i = i h, y_j = j h on a uniform mesh.  The paper's N_x, N_y (number of
 * intervals) are nx + 1 and ny + 1; the default mesh spacing is
 * h = 1 / max(nx + 1, ny + 1).  Dirichlet data on the boundary nodes
 * i in {0, nx + 1}, j in {0, ny + 1}.  The system solved is A u = f
 * with A = -Delta_h, Delta_h the chosen stencil (§2.1, Eq. "9-points" and
 * Eq. "17-points"; Table "tab:ste2" for the classical 5-point stencil).  The
 * 17-point stencil reaches one node beyond the boundary.
 *
 * Boundary data (cj_bc).
 *   CJ_BC_DIRICHLET0: homogeneous data; the node beyond the boundary holds the
 *     odd reflection of the interior (u(-1, j) = -u(1, j), likewise on every
 *     side), which keeps the sine modes exact eigenvectors.
 *   CJ_BC_DIRICHLET_FRAME: arbitrary data carried by u itself, as in the
 *     paper's test problem (§3, boundaries from the analytic solution): u is
 *     the (nx + 2G) x (ny + 2G) array over nodes 1-G .. n+G with the interior
 *     inside a frame of width G = 1 (5-, 9-point) or G = 2 (17-point, whose
 *     second layer holds prescribed ghost values).  The frame is read, never
 *     written.  The relative residual is measured against the residual of the
 *     zero interior, i.e. the norm of the lifted right-hand side
 *     f - A_IB u_B.
 *
 * Arrays.  f is a device pointer to nx*ny doubles, row-major with x fastest:
 * element (i, j) at index (j - 1) * nx + (i - 1).  u has the same layout
 * (CJ_BC_DIRICHLET0) or the frame layout above, element (i, j) at index
 * (j - 1 + G) * (nx + 2G) + (i - 1 + G).  Arrays must be 8-byte aligned.  The
 * caller owns them; the library never frees them.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  All device work of a call is enqueued on that stream.  cj_solve,
 * cj_sweeps, cj_residual and cj_apply return after that work has completed.
 *
 * Errors.  Every call returns a cj_status; nothing aborts or throws across
 * the ABI.  cj_last_error() gives a message for the calling thread's last
 * failure.  Device pointers are checked for NULL and alignment only.  A plan
 * may be used by one thread at a time; separate plans are independent.
 */
#ifndef CJ_H
#define CJ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cj_plan_s* cj_plan_t;

typedef enum {
    CJ_OK = 0,                  /* converged: relative residual <= tol */
    CJ_STAGNATED = 1,           /* stopped at the FP64 floor (see cj_solve) */
    CJ_ERR_ARG = -1,            /* invalid argument */
    CJ_ERR_NOMEM = -2,          /* device or host allocation failed */
    CJ_ERR_HIP = -3,            /* a HIP runtime call failed */
    CJ_ERR_NOT_CONVERGED = -4,  /* max_cycles reached above tol */
    CJ_ERR_NONFINITE = -5,      /* NaN or Inf in f, u or the residual */
    CJ_ERR_DEVICE = -6          /* plan used on a device other than its first */
} cj_status;

typedef enum { CJ_STENCIL_5 = 5, CJ_STENCIL_9 = 9, CJ_STENCIL_17 = 17 } cj_stencil;

typedef enum { CJ_BC_DIRICHLET0 = 0, CJ_BC_DIRICHLET_FRAME = 1 } cj_bc;

/* Iteration (cj_options.method).
 * CJ_METHOD_CHEBYSHEV: the Chebyshev-Jacobi method (§2.1).
 * CJ_METHOD_JACOBI: plain Jacobi, omega = 1 (the paper's reference method,
 *   §3).  M is then the interval between residual tests: 0 selects the
 *   largest power of two not above n_J / 32, where n_J sweeps meet tol under
 *   the bound (1 - kappa_min)^n; the predicted cycle count is ceil(n_J / M).
 *   FP64 only. */
typedef enum { CJ_METHOD_CHEBYSHEV = 0, CJ_METHOD_JACOBI = 1 } cj_method;

/* Working precision of a plan.
 * CJ_PRECISION_F64: FP64 sweeps, the method as stated (§2.1).
 * CJ_PRECISION_F32_REFINE: iterative refinement; every outer step forms the
 *   residual r = f - A u in FP64, approximately solves A d = r with one cycle
 *   of FP32 weighted sweeps from d = 0 (the same Chebyshev schedule, weights
 *   rounded to FP32), and adds d to u in FP64.  The stopping test is the FP64
 *   relative residual.  Each FP32 sweep moves half the bytes of an FP64 one;
 *   the contraction per outer step is limited by eps32 * kmax / kmin, so on
 *   grids where that product is large the inner cycles run in FP64 instead
 *   (cj_inner_precision). */
typedef enum { CJ_PRECISION_F64 = 0, CJ_PRECISION_F32_REFINE = 1 } cj_precision;

/* Inner cycles of a CJ_PRECISION_F32_REFINE plan (cj_options.inner_precision).
 * CJ_INNER_AUTO: FP32, unless eps32 * kappa_max / kappa_min > 4 (for example
 *   16384^2, 9-point: 8.6; 8192^2: 2.2), where FP32 cycles barely contract
 *   the correction and FP64 cycles of the plan's schedule take their place.
 * CJ_INNER_F32, CJ_INNER_F64: forced.  With FP64 inner cycles the plan sweeps
 *   in FP64 everywhere (cj_sweeps, cj_plan_launch_info) and its workspace
 *   holds three more padded FP64 arrays instead of the FP32 ones. */
typedef enum { CJ_INNER_AUTO = 0, CJ_INNER_F32 = 1, CJ_INNER_F64 = 2 } cj_inner_precision;

/* Tuning and schedule options for cj_plan_ex.  Zero means "automatic". */
typedef struct {
    int    M;                  /* cycle length; 0 = the power of two 2^p that minimises
                                  (predicted cycles x M), ties to the smaller; else a
                                  power of two, 1 <= M <= 2^24 */
    int    max_cycles;         /* 0 = predicted cycles + 4 (CJ_PRECISION_F32_REFINE: the
                                  maximum number of outer steps, 0 = 50) */
    int    sweeps_per_launch;  /* temporal-blocking depth K of the sweep kernel: sweeps fused
                                  into one launch; 0 = automatic (FP64: 5- and 9-point 10 on
                                  grids of more than 2^22 points, else 8; 17-point 4.
                                  FP32: 8, 17-point 4); FP64 1, 2, 3, 4, 6, 8, 10
                                  (5/9-point) or 1, 2, 3, 4 (17-point); FP32 1, 2, 4, 8
                                  (5/9-point) or 1, 2, 3, 4 (17-point) */
    int    tile_rows;          /* rows per workgroup tile of the sweep kernel; 0 = automatic:
                                  the first cj_solve chooses it, on grids of more than 2^18
                                  points by timing the blocked kernel at several heights on
                                  the device, on smaller ones from a model of its row
                                  pipeline (results do not depend on it) */
    double h;                  /* mesh spacing; 0 = 1 / max(nx + 1, ny + 1) */
    int    precision;          /* cj_precision; 0 = CJ_PRECISION_F64 */
    int    inner_M;            /* CJ_PRECISION_F32_REFINE: inner cycle length (a power of
                                  two); 0 = the automatic M.  Must be 0 otherwise. */
    int    graph;              /* FP64 solves: replay each cycle's plain launches as one HIP
                                  graph; 0 = automatic (grids of at most 2^22 points, where
                                  launch overhead matters), 1 = always, -1 = never */
    int    method;             /* cj_method; 0 = CJ_METHOD_CHEBYSHEV */
    int    inner_precision;    /* cj_inner_precision of a CJ_PRECISION_F32_REFINE plan; must be
                                  0 otherwise */
    int    single_workgroup;   /* FP64 5- and 9-point plans whose padded grid fits in one CU's LDS
                                  (at most 1024 columns and 16 rows per lane of a 1024-lane
                                  workgroup, e.g. 128^2): run the whole solve in one launch of one
                                  workgroup holding the grid in LDS (the same iterates; the residual
                                  is summed in another order); 0 = automatic (where one CU
                                  outpaced the launched cycles: bands of at most 4 rows per lane,
                                  e.g. 64^2; of at most 8 rows for 5 points, and for 9 points on
                                  grids of at most 4096 points), 1 = required (CJ_ERR_ARG if it
                                  does not fit), -1 = never */
    int    reserved[2];        /* must be zero */
} cj_options;

/* Outcome of a solve. */
typedef struct {
    int       status;          /* the cj_status returned */
    int       cycles;          /* completed weight cycles (refinement: outer steps) */
    long long sweeps;          /* cycles * M (refinement: FP32 sweeps) */
    double    rel_residual;    /* ||f - A u||_2 / ||f||_2 of the returned u */
    double    floor_estimate;  /* on CJ_STAGNATED: the residual level successive cycles
                                  stopped improving on; 0 otherwise */
    double    seconds;         /* host wall time of the call */
    double    sweep_seconds;   /* device time of the plain sweep launches (those not fused
                                  with the residual), timed with HIP events on `stream` */
    long long sweep_launches;  /* number of launches sweep_seconds covers */
} cj_result;

/* Fills *opt with zeros (all automatic). */
void cj_options_init(cj_options* opt);

/* Builds a plan on the host (no device work): kappa_min/kappa_max from the
 * closed forms with N = n + 1 (§2.1), the cycle length M, and the M weights
 * omega_j = 2 / ((kmax + kmin) - (kmax - kmin) cos(theta_j pi / (2M))), with
 * theta_j running over the odd integers 1 .. 2M - 1 in the recursive
 * symmetric-pair order S_1 = [1], S_2m = [s_1, 4m - s_1, s_2, 4m - s_2, ...]
 * (keeps every tail product of the cycle polynomial bounded by one).
 * nx, ny >= 1; stencil in {5, 9, 17}; bc a cj_bc (CJ_BC_DIRICHLET_FRAME
 * with CJ_PRECISION_F64 or CJ_PRECISION_F32_REFINE); tol > 0.
 * On success *out owns the plan; release it with cj_plan_destroy. */
cj_status cj_plan(int nx, int ny, int stencil, int bc, double tol, cj_plan_t* out);
cj_status cj_plan_ex(int nx, int ny, int stencil, int bc, double tol,
                     const cj_options* opt, cj_plan_t* out);

/* Reads a plan.  Any output pointer may be NULL.  *weights_host points to the
 * plan's M weights in applied order (owned by the plan, valid until destroy);
 * for CJ_PRECISION_F32_REFINE plans M, cycles_pred and the weights are those
 * of the inner cycle.
 * *workspace_bytes is the device memory cj_solve allocates on first use:
 * two padded iterates, the padded scaled right-hand side, the weights and
 * the reduction buffers. */
cj_status cj_plan_info(cj_plan_t p, double* kmin, double* kmax, int* M, int* cycles_pred,
                       const double** weights_host, size_t* workspace_bytes);

/* Launch geometry of the plan's sweep kernel: sweeps fused per launch
 * (temporal-blocking depth K), output rows per workgroup tile and
 * workgroups per launch.  With tile_rows = 0 the tile height is the one the
 * first cj_solve chose; before that solve this reports the default.  Any
 * output pointer may be NULL. */
cj_status cj_plan_launch_info(cj_plan_t p, int* sweeps_per_launch, int* tile_rows, int* workgroups);

/* Solves A u = f.  u is read as the initial guess and overwritten with the
 * solution (CJ_BC_DIRICHLET_FRAME: its interior; the frame is the data).
 * Cycles of M sweeps are run; the relative residual ||f - A u||_2 / ||f||_2
 * (frame: over the lifted right-hand side) is tested at cycle ends only (the paper stops at a
 * prescribed tolerance, §3.4; mid-cycle iterates are not meaningful).  Stops
 * with CJ_OK when it is <= tol; with CJ_STAGNATED when, at or after the
 * predicted cycle count, a cycle fails to halve it (the FP64 floor of large
 * grids; cj_solve_dd meets tolerances below it); with CJ_ERR_NOT_CONVERGED
 * after max_cycles.  In each of these cases
 * u holds the last cycle-end iterate.  f = 0 gives u = 0 and CJ_OK.
 * CJ_ERR_NONFINITE if f or an iterate has a NaN or Inf.  The device
 * workspace is allocated on the first call and kept by the plan.
 * res may be NULL. */
cj_status cj_solve(cj_plan_t p, const double* f, double* u, void* stream, cj_result* res);

/* cj_solve with the iterate carried as a double-double u + u_lo: iterative
 * refinement whose residual ||f - A (u + u_lo)|| / ||f|| is limited by
 * neither the rounding of an FP64 iterate nor its evaluation, so tolerances
 * below the FP64 floor of large grids can be met.  Each outer step evaluates
 * the residual of u + u_lo (error-free transformations), solves the
 * correction equation A d = r approximately and adds d into the pair.  The
 * correction is the Chebyshev-weighted Jacobi iteration of §2.1:
 *   CJ_PRECISION_F32_REFINE plans: one inner FP32 cycle, as in cj_solve;
 *   CJ_PRECISION_F64 plans: one FP64 cycle of the plan's own schedule (no
 *     limit from FP32 rounding on the largest grids; the first call
 *     allocates three more padded FP64 arrays, kept by the plan).
 * f, u: as in cj_solve (u in: the FP64 initial guess; out: the high parts).
 * u_lo: device array of u's shape, written only: the low parts, with
 * |u_lo| <= ulp(u) / 2, so u alone is the solution rounded to FP64; with
 * CJ_BC_DIRICHLET_FRAME its frame is set to zero.  u_lo must not overlap f
 * or u.  Status as in cj_solve; CJ_STAGNATED: two outer steps in a row
 * reduced the residual by less than 10%; CJ_ERR_NOT_CONVERGED after
 * max_cycles outer steps.  CJ_ERR_ARG for a CJ_METHOD_JACOBI plan or a NULL
 * array. */
cj_status cj_solve_dd(cj_plan_t p, const double* f, double* u, double* u_lo, void* stream, cj_result* res);

/* Applies the first n_sweeps weighted sweeps of the plan's schedule (weights
 * taken cyclically) to the guess u, with no residual test; u is overwritten.
 * Same kernels and launch configuration as cj_solve.  n_sweeps >= 0.
 * CJ_PRECISION_F32_REFINE plans with FP32 inner cycles sweep in FP32: u and
 * D^{-1} f are rounded to FP32, the sweeps run in FP32 and the result is
 * widened back. */
cj_status cj_sweeps(cj_plan_t p, const double* f, double* u, long long n_sweeps, void* stream);

/* *rel_residual = ||f - A u||_2 / ||f||_2 (0 when f = 0; frame: over the
 * lifted right-hand side), FP64 with a deterministic reduction order. */
cj_status cj_residual(cj_plan_t p, const double* f, const double* u, void* stream,
                      double* rel_residual);

/* Allocation-free form of cj_residual, for callers that cannot allocate
 * device memory or wait on the host: code under HIP graph capture, serving
 * loops that must not call hipMalloc.  The value is cj_residual's, from the
 * same partial sums in the same order, but read straight from the caller's f
 * and u (no staging copy, no plan workspace) and written to the DEVICE
 * address rel_residual (one double) on `stream`; the call returns once the
 * work is enqueued.  A NaN or Inf in f or u gives a non-finite value (there is
 * no status for it).  It allocates nothing: the per-tile partial sums live in
 * a fixed scratch array in the library, one per device (1 MiB, held until the
 * process ends), which limits the grid to at most 65536 tiles of the plan's
 * residual geometry (256 columns by 16 rows on large grids, e.g. 16384^2);
 * larger grids give CJ_ERR_ARG.  Calls that overlap on one device share that
 * array and race: order them on one stream.  The plan is only read (it need
 * not have a workspace, and is not bound to the device). */
cj_status cj_residual_noalloc(cj_plan_t p, const double* f, const double* u, double* rel_residual, void* stream);

/* au = A u = -Delta_h u (the stencil apply) on the interior; au has the
 * nx*ny layout of f.  With CJ_BC_DIRICHLET_FRAME the frame values enter the
 * stencil as they stand. */
cj_status cj_apply(cj_plan_t p, const double* u, double* au, void* stream);

/* ------------------------------------------------------------------ batches
 * Many independent problems of uneven size solved together (FP32 sweeps
 * inside FP64 refinement, as CJ_PRECISION_F32_REFINE, per problem).  Each
 * problem has its own schedule from the paper's closed forms for its nx, ny
 * (§2.1).  One launch runs K sweeps of every active problem (one workgroup
 * per problem tile); problems whose inner cycle ends are corrected, their
 * FP64 residuals formed and reduced together, and the host decides for each
 * as cj_solve does.  Results per problem match cj_solve on a
 * CJ_PRECISION_F32_REFINE plan of the same problem up to the order of the
 * residual reductions. */
typedef struct cj_batch_s* cj_batch_t;

typedef struct {
    int       supersteps;      /* batched sweep launches per stencil group */
    long long launches;        /* batched sweep launches in all */
    long long points;          /* sum of nx*ny */
    double    updates;         /* sum of nx*ny*sweeps (FP32 grid-point updates) */
    double    seconds;         /* host wall time of cj_batch_solve */
    int       sweeps_per_launch[3];   /* blocked depth K the 5-, 9- and 17-point problems ran at
                                         (0: no such problem) */
    int       tile_rows[3];           /* and their tile height (chosen by the autotuner when
                                         sweeps_per_launch and tile_rows are automatic) */
    int       reserved[2];
} cj_batch_stats;

/* n problems; nx, ny, stencil, tol are arrays of length n (read during the
 * call only).  opt: precision must be CJ_PRECISION_F32_REFINE; M, inner_M and
 * h must be 0; sweeps_per_launch 0 (automatic), 2, 4 or 8 (17-point at most
 * 4); tile_rows and max_cycles (outer steps per problem, 0 = 50) apply to
 * all.  With sweeps_per_launch and
 * tile_rows both automatic, the first solve times every (K in {8, 4, 2},
 * tile rows in {16, 32, 64, 128}) per stencil group on the problems
 * themselves before their first inner cycle and keeps the fastest per sweep
 * (results do not depend on it); cj_batch_info and cj_batch_stats report the
 * choice.  Host only; the device workspace is allocated by the first solve. */
cj_status cj_batch_create(int n, const int* nx, const int* ny, const int* stencil, const double* tol,
                          const cj_options* opt, cj_batch_t* out);

/* Problem i's longest inner cycle M, its sweeps per launch (after the first
 * solve: the autotuner's choice), and the batch's device workspace in bytes.
 * Any output pointer may be NULL. */
cj_status cj_batch_info(cj_batch_t b, int i, int* M, int* sweeps_per_launch, size_t* workspace_bytes);

/* Solves all problems: f[i], u[i] are device pointers laid out as in
 * cj_solve (u[i] in: guess, out: solution).  results (length n) and stats may
 * be NULL.  Returns CJ_OK if every problem converged, else the status of the
 * first problem that did not (per-problem statuses are in results).  Runs on
 * `stream` and returns when done. */
cj_status cj_batch_solve(cj_batch_t b, const double* const* f, double* const* u, void* stream,
                         cj_result* results, cj_batch_stats* stats);

void cj_batch_destroy(cj_batch_t b);

/* ------------------------------------------------------------------ serving
 * Continuous batching: requests are submitted at any time and join the
 * running batch as HBM budget frees up; each is admitted when its device
 * arrays fit in the server's pool, runs in the shared launches of the
 * batched solver (as described above), and leaves when finished.  A
 * request's arithmetic does not depend on which other requests share its
 * launches, so its result is the same alone and in the mix.
 * The server does work only inside cj_server_step. */
typedef struct cj_server_s* cj_server_t;

/* opt as for cj_batch_create.  hbm_budget_bytes: the device pool that
 * admission draws from (allocated at the first step).  stream: all work of
 * the server runs on it (hipStream_t as void*). */
cj_status cj_server_create(const cj_options* opt, size_t hbm_budget_bytes, void* stream, cj_server_t* out);

/* Queues a request.  f, u: device arrays as in cj_solve, owned by the caller
 * and left untouched by the caller until the request is reported done (u is
 * the initial guess and receives the solution).  *ticket identifies it.
 * CJ_ERR_NOMEM if the request alone exceeds the HBM budget. */
cj_status cj_server_submit(cj_server_t s, int nx, int ny, int stencil, double tol, const double* f, double* u,
                           long long* ticket);

/* Admits what fits, advances every admitted request by batched launches up
 * to the first inner-cycle end among them (at most 32 launches of K sweeps),
 * does the cycle-end work that is due, and reports up to max_done finished
 * requests (tickets and results; results[].seconds is the time from submit
 * to completion).  *n_done receives their number. */
cj_status cj_server_step(cj_server_t s, long long* done_tickets, cj_result* done_results, int max_done,
                         int* n_done);

/* Requests admitted and not finished, requests waiting, pool bytes in use. */
cj_status cj_server_stats(cj_server_t s, int* active, int* queued, size_t* bytes_in_use);

void cj_server_destroy(cj_server_t s);

/* Frees the plan and its device workspace.  NULL is ignored. */
void cj_plan_destroy(cj_plan_t p);

/* Static text for a status code. */
const char* cj_status_string(int status);

/* Message for the calling thread's last failed call ("" if none). */
const char* cj_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CJ_H */
