/*
 * bchar.h -- C ABI of the B-char transfer build and apply on AMD MI355X.
 *
 * Method: Cheng & Droniou, "An efficient implementation of mass conserving
 * characteristic-based schemes in 2D and 3D" (arXiv:1908.05834).  The
 * problem is the pure advection equation phi dc/dt + div(u c) = 0 on a
 * box with u.n = 0 on its boundary (Sec. 1.1, eq. advection); cells carry a
 * piecewise-constant porosity phi > 0 and one concentration value each
 * (Sec. 1.2).  One time step computes the transfer matrix A whose entry
 * (K, M) approximates |M cap F_{-dt}(K)|_phi, and applies it:
 *     |K|_phi c_K^{n+1} = sum_M A_{K,M} c_M^n        (Sec. 2, eq. phys-inter-ELLAM)
 * A is built by Algorithm 1 (Sec. 3.3): balls per cell (Sec. 3), backward
 * tracking of their centres (eq. charac), ball-ball intersection volumes
 * combined into V (Sec. 3.1, eq. ball_int), N alternating column/row
 * scalings (Sec. 3.2, eq. volAdj) and the least-change bounded problem
 * (Sec. 3.2, eq. opti_masscons), so that every row sums to |K|_phi and
 * every column to |M|_phi (local and global mass conservation).
 *
 * Conventions
 *  - Every pointer argument documented "device" is a HIP device address on
 *    the current device; "host" is ordinary host memory.  The library
 *    never frees caller memory.
 *  - Handles own all device memory they allocate; *_destroy frees it.
 *    Destroying NULL is a no-op; destroying twice is a caller error.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device
 *    work is ordered on it.  Calls that return host values or statistics
 *    synchronise that stream before returning.
 *  - Errors are returned as bchar_status and never abort; no C++
 *    exception crosses this interface.  bchar_last_error() returns a
 *    thread-local message describing the most recent failure.  On error,
 *    output handles are set to NULL.
 *  - Handles are not safe for concurrent use from several threads.
 *  - Cells are numbered x-fastest: id = i + n0*(j + n1*k).  Nodal velocity
 *    lattices are stored the same way.  Sparse matrices are CSR with
 *    strictly ascending columns in each row.
 */
#ifndef BCHAR_H
#define BCHAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BCHAR_OK = 0,
  BCHAR_E_INVALID_ARG = 1,      /* a size, pointer or value is out of range     */
  BCHAR_E_OUT_OF_MEMORY = 2,    /* device allocation failed                     */
  BCHAR_E_DEVICE = 3,           /* a HIP runtime call failed                    */
  BCHAR_E_VOID_ROW = 4,         /* a tracked ball overlaps no residing ball:
                                   the denominator of eq. fracMaterial is 0    */
  BCHAR_E_VOID_COLUMN = 5,      /* a column of V sums to 0 (Sec. 3.2): no
                                   tracked ball reaches that residing cell     */
  BCHAR_E_QP_INFEASIBLE = 6,    /* eq. opti_masscons has no solution in the box
                                   allowed by the box policy                   */
  BCHAR_E_QP_NOT_CONVERGED = 7, /* the solver of eq. opti_masscons stopped
                                   before reaching the tolerance               */
  BCHAR_E_UNSUPPORTED = 8       /* a configuration outside what is built       */
} bchar_status;

/* Ball layouts: which balls B_{K,s} represent a cell (Sec. 3: "we choose
 * n_K points C_{K,s}" strictly inside K; Sec. 4 uses 4 balls per square and
 * 8 per cube).
 *   SUBCELL       Cartesian: 2^d balls at the centres of the 2^d half-size
 *                 sub-cells, radius min(h)/4 (disjoint, one quarter of the
 *                 smallest face)
 *   INSCRIBED     Cartesian: one ball at the centroid, radius min(h)/2
 *   EQUAL_MEASURE one ball at the centroid with |B| = |K| (overlaps its
 *                 neighbours)
 *   CUSTOM        the caller's balls (bchar_mesh_desc.n_balls, balls,
 *                 ball_cell), any number per cell, on either mesh kind
 *   PACKED        simplices: dim + 2 disjoint balls strictly inside each
 *                 cell (the paper leaves the packing of generic cells open,
 *                 Sec. 5).  In this order: the inscribed ball (centre the
 *                 incentre sum_i w_i v_i / sum_i w_i, w_i the measure of
 *                 the facet opposite vertex v_i; radius r = dim |K| /
 *                 sum_i w_i), then per vertex the ball tangent to the dim
 *                 facets through v_i and to the inscribed ball (centre
 *                 v_i + t (I - v_i), radius t r, t = (L - r) / (L + r),
 *                 L = |v_i - I|); every radius times 7/8, centres kept.  A
 *                 cell whose balls would still overlap keeps the inscribed
 *                 ball alone.  rho_K as for CUSTOM.                      */
enum { BCHAR_LAYOUT_SUBCELL = 0, BCHAR_LAYOUT_INSCRIBED = 1, BCHAR_LAYOUT_EQUAL_MEASURE = 2,
       BCHAR_LAYOUT_CUSTOM = 3, BCHAR_LAYOUT_PACKED = 4 };

/* Precision of the geometric part.  FP64: everything in binary64.
 * FP32_VOLUME: tracking, the overlap predicate and the lens volumes in
 * binary32; the weights, V, the scalings, the QP, the update and the mass
 * stay in binary64 (compensated sums where they accumulate).  Needs a
 * constant porosity: where phi varies, the speed u/phi jumps on cell faces
 * and the cardinal points of eq. rTrackedBall start on faces, so binary32
 * rounding would take the neighbouring cell's phi (BCHAR_E_UNSUPPORTED).
 * FP32_LENS: tracking in binary64, the predicate and the lens in binary32,
 * the rest in binary64 (any porosity).                                  */
enum { BCHAR_FP64 = 0, BCHAR_FP32_VOLUME = 1, BCHAR_FP32_LENS = 2 };

/* What to do when the box of eq. opti_masscons (0 <= 1 + x <= 2) admits no
 * solution.  PAPER_THEN_RELAX: drop the upper cap (level 1, volumes stay
 * non-negative), then keep the equalities alone (level 2).  STRICT: return
 * BCHAR_E_QP_INFEASIBLE.                                                 */
enum { BCHAR_BOX_PAPER_THEN_RELAX = 0, BCHAR_BOX_STRICT = 1 };

/* Last stage of Algorithm 1 to run (for inspection).  PAIRS: candidate
 * pairs only; V: A^(0) = V; SCALING: A^(N); ALL: the final matrix.        */
enum { BCHAR_STAGE_PAIRS = 1, BCHAR_STAGE_V = 2, BCHAR_STAGE_SCALING = 3, BCHAR_STAGE_ALL = 4 };

enum { BCHAR_MEM_HOST = 0, BCHAR_MEM_DEVICE = 1 };

/* The velocity field (Sec. 3.2, Remark on non-solenoidal fields).  FREE:
 * div u = 0 is assumed, so the porous volume of a tracked ball is that of
 * the ball (eq. expPhiB) and the row targets are |K|_phi (eq.
 * exactVol_traceback).  GENERAL: any u.  The generalised Liouville formula
 * (eq. genLiouville), with div u over a carried ball taken as its value at
 * the ball's centre times the ball's volume, makes the porous volume of
 * the ball B_{K,s} tracked back over dt equal to phi_K |B_{K,s}| exp(lam),
 * lam = -int (div u / phi)(X(t)) dt along the tracked centre X, div u that
 * of the Q1 interpolant, integrated by the centre's own RK4 stages
 * (exact where div u / phi is constant).  That mass, times rho_K, is the
 * ball's mass in eq. ball_int; r_hat comes from the tracked cardinal
 * points (eq. rTrackedBall) whatever phi; the row targets are eq.
 * volTracked's T_K = sum_s rho_K phi_K |B_{K,s}| exp(lam_{K,s}), rescaled
 * on every connected component of the bipartite graph of V's pattern
 * (row K -- column M per entry) by sum_{M in it} |M|_phi /
 * sum_{K in it} T_K: the trace-back regions cover the domain once, so the
 * two sides of eq. opti_masscons must total the same on each set of cells
 * that exchange material only among themselves (usually one component,
 * the whole domain).  The column targets stay |M|_phi and the update
 * still divides by |K|_phi (eq. phys-inter-ELLAM), so a compressing flow
 * concentrates c.  Tracking runs in binary64 (FP32_VOLUME is
 * UNSUPPORTED).                                                          */
enum { BCHAR_DIV_FREE = 0, BCHAR_DIV_GENERAL = 1 };

typedef struct bchar_mesh_s* bchar_mesh;
typedef struct bchar_transfer_s* bchar_transfer;

/* Cartesian mesh of the box [origin, origin + n*h] (Sec. 1.2).          */
/* Mesh kinds.  CARTESIAN: n[a] cells of size h[a] from origin (cell ids
 * x-fastest).  SIMPLEX: triangles (2D) or tetrahedra (3D) given by their
 * vertices; the domain is the bounding box of the vertices, which the cells
 * must cover; the paper gives no ball packing for such cells, each gets one
 * ball at its centroid (((v0 + v1) + v2) (+ v3)) / (dim + 1) with |B| = |K|
 * (layout EQUAL_MEASURE only), |K| = |det(v1 - v0, ...)| / dim!.  phi(x)
 * during tracking is phi of the cell holding x clamped into the domain box:
 * among the cells whose bounding box holds x, the lowest-numbered one whose
 * orientation tests (each vertex replaced by x) all agree in sign with the
 * cell's own orientation or vanish; if rounding leaves none, the one whose
 * centroid is nearest (lowest number on ties).                          */
enum { BCHAR_MESH_CARTESIAN = 0, BCHAR_MESH_SIMPLEX = 1 };

typedef struct {
  int dim;               /* 2 or 3                                        */
  int64_t n[3];          /* CARTESIAN: cells per axis (n[2] ignored in 2D),
                            each >= 1                                     */
  double origin[3];      /* CARTESIAN: lower corner                       */
  double h[3];           /* CARTESIAN: cell size per axis, > 0            */
  const double* phi;     /* porosity per cell (n0*n1*n2 or n_simplices
                            values), each finite and > 0 (Sec. 1.2);
                            copied at creation                            */
  int phi_mem;           /* BCHAR_MEM_HOST or BCHAR_MEM_DEVICE            */
  int layout;            /* BCHAR_LAYOUT_*                                */
  int kind;              /* BCHAR_MESH_CARTESIAN (0) or BCHAR_MESH_SIMPLEX */
  int64_t n_vertices;    /* SIMPLEX: vertices, >= dim + 1                 */
  int64_t n_simplices;   /* SIMPLEX: cells, >= 1                          */
  const double* vertices;/* SIMPLEX, host: n_vertices * dim coordinates,
                            vertex-major (x, y[, z] of vertex 0, ...);
                            copied at creation                            */
  const int32_t* cells;  /* SIMPLEX, host: n_simplices * (dim + 1) vertex
                            ids, each in [0, n_vertices), non-degenerate
                            cells; copied at creation                     */
  int geom_mem;          /* BCHAR_MEM_HOST (0) or BCHAR_MEM_DEVICE: where
                            vertices, cells, balls and ball_cell live     */
  int64_t n_balls;       /* CUSTOM: number of balls, >= number of cells   */
  const double* balls;   /* CUSTOM: n_balls * (dim + 1) values, ball-major:
                            centre x, y[, z], radius > 0; copied          */
  const int32_t* ball_cell; /* CUSTOM: cell of every ball, non-decreasing
                            (a cell's balls are consecutive), every cell
                            with at least one ball and at most 256; rho_K
                            is |K| / sum of the measures of K's balls
                            (eq. def:porous.density); copied              */
  int64_t n_ghost;       /* CARTESIAN: layers of ghost cells on every side
                            (Sec. 3.2, Remark on inflow and outflow, option
                            b), 0 (default) for none; n[a] > 2 n_ghost.  The
                            grid described by n, origin, h includes them.
                            Ghost cells carry balls and are tracked like
                            the others, but their rows and columns have no
                            target: the scaling leaves them alone, the
                            least-change problem constrains the interior
                            cells' rows and columns only (the ghost cells'
                            multipliers stay 0), and a ghost ball tracked
                            into nothing or a ghost column nothing reaches
                            is no void.  Material enters the interior from
                            ghost cells, whose concentrations the caller
                            sets to the inflow data before every update,
                            and leaves it into ghost cells.  bchar_mass
                            sums the interior cells; the ghost entries of
                            an update's output mean nothing.  Solenoidal
                            steps only (DIV_GENERAL: UNSUPPORTED)         */
  double hash_scale;     /* side of the spatial hash's buckets as a multiple
                            of 2 r_max (r_max: the largest residing ball):
                            0 (default) means 1, else within [0.25, 4].
                            Every side finds the same overlapping pairs
                            (the searched block of buckets widens or
                            narrows with it); it trades buckets visited
                            against balls tested per bucket, a tuning
                            knob for the candidate search (Sec. 3.1)      */
} bchar_mesh_desc;

/* Velocity u^{(n+1)} frozen over the time step (Sec. 1.2, eq. hyp:un) as
 * a nodal lattice with multilinear (Q1) interpolation; queries outside the
 * lattice box are clamped onto it.  For a Cartesian mesh the natural
 * lattice is its vertices (m = n + 1, spacing = h).                     */
typedef struct {
  int64_t m[3];          /* nodes per axis, each >= 2                     */
  double origin[3];      /* first node                                    */
  double spacing[3];     /* node spacing, > 0                             */
  const double* u[3];    /* device, one component each, m0*m1*m2 values,
                            x-fastest; u[2] unused in 2D                  */
} bchar_velocity;

typedef struct {
  int precision;         /* BCHAR_FP64 (default) or BCHAR_FP32_VOLUME      */
  int n_sweeps;          /* N scaling sweeps of eq. volAdj, default 10 (Sec. 4) */
  int rk_substeps;       /* RK4 sub-steps per time step, default 1         */
  int box_policy;        /* BCHAR_BOX_*, default PAPER_THEN_RELAX          */
  int stop_after;        /* BCHAR_STAGE_*, default ALL                     */
  double qp_tol;         /* bound on max |A_hat(1+x) - b| / max |K|_phi,
                            default 1e-13                                 */
  int qp_max_newton;     /* Newton iterations per box level, default 500   */
  int qp_max_cg;         /* CG iterations per Newton step, default 400     */
  int keep_pairs;        /* non-zero: keep the candidate pairs for export  */
  int warm_start;        /* non-zero (default): a rebuild starts the least-
                            change solve from the multipliers of the
                            transfer's previous solve (same mesh); the
                            solution is unique, only the iteration count
                            changes; a failed warm start is retried cold */
  int max_halvings;      /* a build that meets a void row or column (no
                            tracked ball in a residing cell, or none
                            overlapping a tracked ball) is repeated with
                            half the time step, at most this many times
                            (default 0: report the void); the transfer then
                            covers dt in 2^h sub-steps of dt / 2^h, which
                            bchar_step applies in turn (stats.dt_halvings
                            = h)                                         */
  int cg_graphs;         /* non-zero (default): the conjugate-gradient
                            iterations of the least-change solve are
                            captured once per solve as HIP graphs of four
                            iterations and replayed (same kernels, same
                            results bit for bit; fewer host launches)    */
  int cycle_skip;        /* non-zero: the preconditioner's multigrid cycle
                            visits every other level of the pairwise
                            hierarchy (aggregates of about four nodes,
                            exact Galerkin operators): half the launches
                            per cycle, a weaker cycle.  Default 0 (every
                            level); the same solution either way, only
                            the iteration count and time change          */
  int lds_stage;         /* non-zero: the assembly stages the residing
                            balls of each tile's search block in LDS when
                            they fit; 0 (default): every search reads the
                            hash through the caches (measured faster on
                            the 64^3 swirl: the staging area costs a
                            workgroup per CU).  The same transfer bit for
                            bit either way                               */
  int halve_on_level2;   /* non-zero: with max_halvings, a build whose
                            least-change problem would need level 2 (the
                            equalities alone: volumes may turn negative and
                            repeated updates grow without bound) is
                            repeated with half the time step instead; the
                            last allowed attempt may still take level 2 */
  int z_fuse_max_cells;  /* the fine level of the preconditioner runs its
                            first two smoothing sweeps as one pass on meshes
                            of at most this many cells (default 2^20: one
                            launch fewer where launches cost, wider gathers
                            than they save beyond); the same answer either
                            way up to the solver's tolerance             */
  int divergence;        /* BCHAR_DIV_FREE (default) or BCHAR_DIV_GENERAL  */
  int tile_aspect;       /* Cartesian meshes: shape of the assembly's tiles
                            of 256 / balls-per-cell cells.  0 (default): the
                            most cubic power-of-two box (32 cells: 4x4x2,
                            64 in 2D: 8x8); a in [-4, 4]: the last axis's
                            extent divided (a > 0) or multiplied (a < 0)
                            by 2^|a| and the others refitted (32 cells:
                            a = 1 gives 8x4x1, a = -1 4x2x4).  The same
                            transfer bit for bit; only the assembly's
                            speed changes (a tuning knob)               */
} bchar_opts;

typedef struct {
  int64_t n_balls;             /* tracked balls                           */
  int64_t n_pairs;             /* overlapping (tracked, residing) pairs   */
  int64_t nnz;                 /* entries of the transfer matrix          */
  int64_t first_void;          /* ball (void row) or cell (void column)
                                  that failed, else -1                    */
  double scaling_max_col_err;  /* max_j |sum_i a_ij^(N) / |M_j|_phi - 1|  */
  double qp_residual;          /* max |A_hat(1+x) - b| / max |K|_phi      */
  int qp_level;                /* box level used: 0 paper, 1 no cap, 2 none */
  int qp_newton;               /* Newton iterations (all levels)          */
  int qp_cg;                   /* CG iterations (all levels)              */
  int64_t n_at_lower;          /* entries with 1 + x = 0                  */
  int64_t n_at_upper;          /* entries with 1 + x = 2                  */
  int qp_ipm;                  /* interior-point iterations (all levels)  */
  int64_t qp_coarse_bytes;     /* bytes one cycle over the coarsest levels
                                  of the preconditioner (one workgroup)
                                  reads or writes at least              */
  int64_t qp_smooth_bytes;     /* bytes one Jacobi sweep of a launched
                                  multigrid level reads or writes at least,
                                  mean over the sweeps of one cycle       */
  int dt_halvings;             /* times the time step was halved after a
                                  void (opts.max_halvings)                */
  int64_t n_void_rows;         /* tracked cells with a ball that overlaps
                                  no residing ball (eq. fracMaterial has
                                  denominator 0)                         */
  int64_t n_void_cols;         /* residing cells that no tracked ball
                                  reaches (a zero column of V, Sec. 3.2) */
  int trace_precision;         /* precision the tracking ran in: BCHAR_FP64
                                  or BCHAR_FP32_VOLUME                    */
  int64_t device_bytes;        /* device memory the transfer holds after
                                  the build (kept for the next rebuild)   */
  double row_target_scale;     /* DIV_GENERAL: sum_M |M|_phi / sum_K T_K
                                  over the whole domain (the factor on
                                  eq. volTracked's T_K when V's pattern is
                                  connected); 1 for DIV_FREE             */
  int64_t n_target_groups;     /* DIV_GENERAL: connected components of V's
                                  pattern, each rescaled on its own; 0 for
                                  DIV_FREE                                */
  int qp_corrected;            /* 1 when the least-change answer is an
                                  interior point that stalled just short of
                                  the tolerance, put onto the row and column
                                  sums by a least-norm correction: the sums
                                  hold to qp_tol, but entries on the box
                                  may leave it by their share of the
                                  correction (n_at_lower / n_at_upper count
                                  those on or beyond a bound); else 0      */
} bchar_stats;

/* Fill *opts with the defaults listed above.                            */
void bchar_opts_default(bchar_opts* opts);

/* Create the mesh-static data: the balls of every cell and their porous
 * density rho_K with rho_K sum_s |B_{K,s}|_phi = |K|_phi (Sec. 3, eq.
 * def:porous.density), the porous volumes |K|_phi, and a uniform-grid
 * spatial hash of the balls.  Errors: INVALID_ARG (bad dims, sizes, phi
 * not finite or <= 0), OUT_OF_MEMORY, DEVICE.                           */
bchar_status bchar_mesh_create(const bchar_mesh_desc* desc, void* stream, bchar_mesh* out);
bchar_status bchar_mesh_destroy(bchar_mesh mesh);

/* Number of cells and balls of a mesh (host outputs, may be NULL).       */
bchar_status bchar_mesh_info(bchar_mesh mesh, int64_t* n_cells, int64_t* n_balls,
                             int* balls_per_cell);

/* Build the transfer of one time step dt > 0 with velocity u (Algorithm 1,
 * Sec. 3.3).  Allocates *out.  If `stats` is non-NULL it is filled.  The
 * call synchronises `stream` (the scaling and the QP iterate under host
 * control).  Errors: INVALID_ARG, VOID_ROW, VOID_COLUMN, QP_INFEASIBLE
 * (STRICT policy, or no level feasible), QP_NOT_CONVERGED, OUT_OF_MEMORY,
 * DEVICE.  On a VOID_* error stats->first_void names the culprit.       */
bchar_status bchar_build_transfer(bchar_mesh mesh, const bchar_velocity* u, double dt,
                                  const bchar_opts* opts, void* stream, bchar_transfer* out,
                                  bchar_stats* stats);

/* As bchar_build_transfer, but rebuild into an existing transfer of the
 * same mesh, reusing its device memory where it is large enough.        */
bchar_status bchar_rebuild_transfer(bchar_transfer t, const bchar_velocity* u, double dt,
                                    const bchar_opts* opts, void* stream, bchar_stats* stats);

/* As bchar_build_transfer, with the tracked centres and radii given
 * instead of computed (for callers that track the balls themselves).
 * `tracked` is device memory holding dim arrays of n_balls binary64
 * values (x coordinates, then y, then z), balls in mesh order; `r_hat` is
 * device memory with n_balls radii.  dt is not used.                    */
bchar_status bchar_build_transfer_tracked(bchar_mesh mesh, const double* tracked,
                                          const double* r_hat, const bchar_opts* opts,
                                          void* stream, bchar_transfer* out,
                                          bchar_stats* stats);

bchar_status bchar_transfer_destroy(bchar_transfer t);

/* One job of bchar_build_transfer_batch: the transfer of one time step of
 * one problem.                                                          */
typedef struct {
  bchar_transfer transfer;     /* in: a transfer to rebuild (its mesh is
                                  used), or NULL to create one on `mesh`;
                                  out: the transfer (NULL if a creation
                                  failed)                                */
  bchar_mesh mesh;             /* used when transfer is NULL              */
  const bchar_velocity* u;     /* as for bchar_build_transfer             */
  double dt;
  bchar_transfer warm_from;    /* optional, rebuilds only: a transfer of
                                  the same mesh whose last solve (ended
                                  before the call) gives the warm start
                                  instead of the job's own, e.g. the
                                  latest interval already built; taken
                                  before any job of the batch runs        */
  bchar_status status;         /* out: the job's own status              */
  bchar_stats stats;           /* out                                    */
} bchar_build_job;

/* Build the transfers of n_jobs independent jobs at once (Algorithm 1 for
 * each, exactly as bchar_build_transfer / bchar_rebuild_transfer would):
 * min(n_streams, n_jobs) workers, worker w on streams[w] and a host thread
 * of its own, each take the next job (in index order) whenever they are
 * free, so that the latency-bound launches of several builds overlap on
 * the device.  Jobs are
 * independent problems, or time intervals of one problem whose velocity
 * is prescribed ahead (the transfer of an interval depends on its
 * velocity, not on the concentration).  Jobs may share a mesh (read only
 * during builds); a transfer may appear in at most one job.  A rebuilt
 * transfer warm-starts from its own previous solve.  Returns once every
 * job has ended and every stream is synchronised: BCHAR_OK if all jobs
 * succeeded, else the status of the first failed job (its message is the
 * one bchar_last_error returns); every job's status is in its job.
 * Errors: INVALID_ARG (NULL arrays, n_streams < 1, a transfer in two
 * jobs), then the errors of bchar_build_transfer per job.              */
bchar_status bchar_build_transfer_batch(bchar_build_job* jobs, int n_jobs,
                                        const bchar_opts* opts, void* const* streams,
                                        int n_streams);

/* Autotuning of the options for a workload: which of n_candidates option
 * sets builds the given jobs fastest, measured.  The jobs (mesh, u, dt;
 * transfer and warm_from must be NULL, nothing is written to them) are
 * built once untimed, then `rounds` times per candidate as
 * bchar_build_transfer_batch would on the same streams (new transfers,
 * destroyed again), the candidates' order reversed every other round;
 * the host clock times each batch, GPU work included (destroying a batch's
 * transfers synchronises the device, so concurrent work of the caller on
 * the same device waits and is timed too).  On return *best is
 * the candidate with the least summed time and seconds[c] (may be NULL)
 * that sum, +inf for a candidate whose builds failed.  Every candidate
 * yields the same transfers up to the solver's tolerance; only the time
 * differs (e.g. cycle_skip, cg_graphs, precision).  Errors: INVALID_ARG
 * (NULL arrays, a count < 1, a job with a transfer or without a mesh or
 * velocity, an invalid candidate), the first failure if every candidate
 * fails.                                                               */
bchar_status bchar_tune_options(const bchar_build_job* jobs, int n_jobs,
                                const bchar_opts* candidates, int n_candidates, int rounds,
                                void* const* streams, int n_streams, int* best,
                                double* seconds);

/* ---- serving: a queue of independent requests ---------------------- */

typedef struct bchar_server_s* bchar_server;

/* One request: build the transfer of one time step dt of `mesh` with
 * velocity u and apply it `steps` times to c_in; the result is written to
 * c_out.  c_in, c_out and c_tmp are device arrays of n_cells binary64
 * values that must not overlap; c_tmp (scratch) may be NULL when steps
 * is 1; c_in is not written.  Everything the request points to must stay
 * valid until the request has been waited for.                         */
typedef struct {
  bchar_mesh mesh;
  const bchar_velocity* u;
  double dt;
  int steps;                   /* >= 1                                   */
  const double* c_in;
  double* c_out;
  double* c_tmp;
  int64_t bytes;               /* device memory the request may take
                                  (admission); 0: 900 bytes per ball    */
} bchar_request;

typedef struct {
  bchar_status status;         /* of the build (BCHAR_OK: c_out written) */
  bchar_stats stats;
  double t_submit, t_start, t_done;  /* host steady-clock seconds        */
} bchar_request_result;

/* A server with n_workers worker threads, worker w on streams[w] with a
 * transfer of its own that every request it takes rebuilds (its buffers
 * are kept between requests: no device allocation once the largest
 * request has been seen).  Requests are taken in submission order.
 * Admission counts the device memory the workers hold: a worker's own
 * (measured after each of its requests, stats.device_bytes) and, while it
 * serves a request, at least that request's `bytes`.  The oldest waiting
 * request starts only when the memory held with it stays within
 * mem_budget bytes (0: no limit); while it waits, idle workers that hold
 * memory release their buffers; a request larger than the budget starts
 * alone, once nothing else runs or is held.  A `bytes` below what the
 * build really takes lets the held memory exceed the budget by the
 * difference.  Errors: INVALID_ARG.                                     */
bchar_status bchar_server_create(int n_workers, void* const* streams, int64_t mem_budget,
                                 const bchar_opts* opts, bchar_server* out);

/* Queue a request (copied); *ticket identifies it.  Never blocks on the
 * device.  Errors: INVALID_ARG (NULL pointers, steps < 1, c_tmp NULL with
 * steps > 1, a server being destroyed).                                */
bchar_status bchar_server_submit(bchar_server srv, const bchar_request* req, int64_t* ticket);

/* Wait until request `ticket` has ended (its c_out is then final) and
 * fill *res; a ticket can be waited for once.  Errors: INVALID_ARG
 * (unknown ticket).                                                     */
bchar_status bchar_server_wait(bchar_server srv, int64_t ticket, bchar_request_result* res);

/* Finish the queued requests, stop the workers and free the server (the
 * results not yet waited for are dropped).  NULL is a no-op.            */
bchar_status bchar_server_destroy(bchar_server srv);

/* One update (Sec. 2, eq. phys-inter-ELLAM): c_out = diag(|K|_phi)^-1 A c_in,
 * applied 2^h times when the build halved the time step h times.
 * c_in, c_out: device, n_cells binary64 each, must not overlap.  Needs a
 * transfer built to BCHAR_STAGE_ALL.  Asynchronous on `stream`.         */
bchar_status bchar_step(bchar_transfer t, const double* c_in, double* c_out, void* stream);

/* Porous mass sum_K phi_K |K| c_K (Sec. 2.1) of a device vector c of
 * n_cells values, summed in binary64 with compensation in a fixed order;
 * the result is written to *host_out after synchronising `stream`.      */
bchar_status bchar_mass(bchar_mesh mesh, const double* c, void* stream, double* host_out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops): the porous mass of bchar_mass, the same kernels and the
 * same bits, written to device memory d_out (one binary64) in the order of
 * `stream`, without synchronising and without allocating anything.  The
 * block partials live in a device array of the library (8 KiB, one per
 * GPU, held until the process ends) that every call on a GPU shares: calls
 * that overlap on one GPU race, so order them on one stream (or
 * synchronise between them).  Nothing carries over from one call to the
 * next.  c: device, n_cells binary64.  Errors: INVALID_ARG (NULL, a mesh
 * of more than 2^31 - 1 cells), DEVICE.                                   */
bchar_status bchar_mass_into(bchar_mesh mesh, const double* c, double* d_out, void* stream);

const char* bchar_status_string(bchar_status s);
const char* bchar_last_error(void);

/* ---- inspection: copies to caller host buffers; synchronises -------- */

/* Sizes of a built transfer.                                           */
bchar_status bchar_transfer_info(bchar_transfer t, int64_t* n_rows, int64_t* nnz,
                                 int64_t* n_pairs, int* stage);

/* CSR of a stage (BCHAR_STAGE_V, _SCALING or _ALL; the pattern is shared):
 * row_ptr n_rows+1, col nnz, val nnz.  Any pointer may be NULL.          */
bchar_status bchar_transfer_export_csr(bchar_transfer t, int stage, int64_t* row_ptr,
                                       int32_t* col, double* val);

/* Candidate pairs (needs opts.keep_pairs): tracked ball ids and residing
 * ball ids, n_pairs each, sorted by (tracked, residing).                */
bchar_status bchar_transfer_export_pairs(bchar_transfer t, int32_t* tracked, int32_t* residing);

/* Tracked centres (dim arrays of n_balls, x then y then z) and radii.   */
bchar_status bchar_transfer_export_tracked(bchar_transfer t, double* tracked, double* r_hat);

/* Per-ball log growth lam (n_balls) and row targets (n_rows) of the last
 * build (host arrays, either may be NULL): DIV_GENERAL's values (see
 * BCHAR_DIV_GENERAL), or 0 and |K|_phi for DIV_FREE.  Synchronises the
 * device.                                                               */
bchar_status bchar_transfer_export_targets(bchar_transfer t, double* lam, double* b_row);

/* Solution of eq. opti_masscons: x (nnz) and the multipliers of the row
 * and column constraints (n_rows each, in units of 1 / max |K|_phi).    */
bchar_status bchar_transfer_export_qp(bchar_transfer t, double* x, double* mu, double* nu);

/* The multipliers of the last solve of eq. opti_masscons in the per-cell
 * coordinates the solver works in (host arrays of n_rows values, any may
 * be NULL): mu_K = s_K + g_K / 2 and nu_M = -(s_M - g_M / 2), so that
 * t_k = a_k (mu_K + nu_M) = a_k ((s_K - s_M) + (g_K + g_M) / 2) for an
 * entry off the diagonal and a_k g_K on it, a in units of max |K|_phi, and
 * the answer is x = clip(t) to the box.  Each multiplier is the sum of a
 * leading part (s, g) and what its rounding lost (s_lo, g_lo): cells that
 * barely move carry multipliers of 1e9 and more whose differences stay
 * small, so that t can be re-formed, and x = clip(t) checked entry by
 * entry, to double-double accuracy.                                     */
bchar_status bchar_transfer_export_qp_dual(bchar_transfer t, double* s, double* g,
                                           double* s_lo, double* g_lo);

/* ---- kernel timing (instrumentation) ------------------------------- */

/* Time every later launch of the kernel called `name` (NULL or "" turns
 * timing off): each launch is bracketed by two HIP events recorded on the
 * stream it is launched on.  Resets the accumulated figures.  Meant for
 * benchmarks; a kernel that is not being timed pays nothing.            */
bchar_status bchar_profile_kernel(const char* name);

/* As bchar_profile_kernel, but time only every `every`-th launch of the
 * kernel (every >= 1), so that a kernel launched very often can be timed
 * with little disturbance; bchar_profile_read then counts the timed
 * launches only.  Errors: INVALID_ARG (every < 1).                      */
bchar_status bchar_profile_kernel_sampled(const char* name, int every);

/* Launches timed since bchar_profile_kernel and their summed duration in
 * milliseconds (waits for the recorded events).                         */
bchar_status bchar_profile_read(int64_t* launches, double* total_ms);

/* Balls of the mesh: centres (dim arrays of n_balls), radii, cell ids.  */
bchar_status bchar_mesh_export_balls(bchar_mesh mesh, double* centres, double* radii,
                                     int32_t* cell);

#ifdef __cplusplus
}
#endif

#endif /* BCHAR_H */
