/*
 * fcgmg — restricted additive smoothing and geometric multigrid for finite cell Stokes problems
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: Saberi & Vogel, "A restricted additive smoother for finite cell flow problems"
 * (arXiv 2403.11636). The library implements the hot path of its geometric multigrid solver on a
 * uniform Cartesian background grid of the unit box [0,1]^d (d = 2, 3):
 *   - the finite cell Stokes operator L of Eq. (12): Q1-Q1 velocity/pressure with the local L2
 *     projection stabilisation of Eq. (10)-(11), the fictitious-domain weight alpha of Eq. (5)-(7)
 *     integrated on cut cells by a quadtree/octree, symmetric Nitsche terms on Dirichlet walls;
 *   - the restricted additive smoother of Eq. (14)-(15) under the three cache policies of
 *     Sec. 3.1.2 (cache_inverse, cache_matrix, cache_none);
 *   - the grid transfers of Eq. (13) (one GPU: T = identity, R = P^T), the coarsest direct solve,
 *     the V-cycle and the standalone solver settings of Sec. 4.
 *
 * Conventions for every call
 *   - Vectors (x, b, r, ...) are caller-owned DEVICE buffers of FP64, contiguous, laid out as d+1
 *     fields [u_x | u_y | (u_z) | p] of (n_l+1)^d values each, nodes numbered lexicographically
 *     with x fastest; n_l = n_cells >> (n_levels-1-l) cells per axis on level l (level 0 is the
 *     coarsest, level n_levels-1 the finest). The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = default stream). Calls are asynchronous on that stream
 *     unless stated otherwise; inputs must stay valid until the stream reaches the call.
 *   - Return value: FCGMG_OK or a negative FCGMG_E_* code; fcgmg_last_error() gives a message
 *     (thread-local). No exception crosses the interface.
 *   - A handle is not thread-safe; distinct handles may be used concurrently on distinct streams.
 */
#ifndef FCGMG_H
#define FCGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcgmg_ctx* fcgmg_h;

/* Cache policies of Sec. 3.1.2. */
enum {
  FCGMG_CACHE_INVERSE = 0, /* store the d+1 kept rows of L_i^{-1} (shared per regular patch class) */
  FCGMG_CACHE_MATRIX = 1,  /* store L_i (sparse pattern values), factorise at every application    */
  FCGMG_CACHE_NONE = 2     /* retrieve L_i from the operator rows at every application, factorise,
                              solve; nothing is stored beyond the operator itself (2D: the rows the
                              residual applies; 3D and the immersed-boundary case: the element
                              matrices of the window cells, cut cells integrated on the fly)      */
};

/* Face codes, faces ordered x-, x+, y-, y+, z-, z+. */
enum {
  FCGMG_BC_NOSLIP = 0,  /* Dirichlet (Nitsche), w = 0                                  */
  FCGMG_BC_INFLOW = 1,  /* Dirichlet (Nitsche), parabolic inflow of Eq. (16), H = 1     */
  FCGMG_BC_NEUMANN = 2  /* pseudo-traction h = 0 ("do-nothing")                         */
};

enum {
  FCGMG_OK = 0,
  FCGMG_E_ARG = -1,      /* invalid argument                                                  */
  FCGMG_E_NOMEM = -2,    /* device allocation failed                                          */
  FCGMG_E_HIP = -3,      /* HIP runtime error                                                 */
  FCGMG_E_SINGULAR = -4, /* a local block L_i or the coarsest operator is singular             */
  FCGMG_E_NOCONV = -5,   /* solve: max_iter reached (x holds the last iterate)                */
  FCGMG_E_NAN = -6       /* solve: non-finite residual                                        */
};

typedef struct {
  int dim;           /* 2 or 3                                                                 */
  int n_cells;       /* finest-level cells per axis; divisible by 2^(n_levels-1)               */
  int n_levels;      /* levels of the hierarchy (Algorithm 1, uniform case: full coarsening)    */
  int quad_depth;    /* space-tree depth for cut-cell integration                              */
  int cache_policy;  /* FCGMG_CACHE_*                                                          */
  int nu_pre;        /* pre-smoothing sweeps per V-cycle                                       */
  int nu_post;       /* post-smoothing sweeps per V-cycle                                      */
  int force;         /* body force: 0 none, 1 manufactured (curl of x^2(1-x)^2 y^2(1-y)^2 ...)  */
  int bc[6];         /* FCGMG_BC_* per face                                                    */
  double eta;        /* viscosity                                                              */
  double alpha_fict; /* alpha in the fictitious part, Eq. (7)                                  */
  double nitsche_beta; /* Nitsche parameter: lambda = beta * eta / h_l                         */
  double omega;      /* damping, omega_i = omega * I in Eq. (15)                                */
  double ubar;       /* inflow amplitude, Eq. (16)                                             */
  int precision;     /* FCGMG_PREC_*: arithmetic of fcgmg_solve's V-cycles                       */
  int solver;        /* FCGMG_SOLVER_*: outer iteration of fcgmg_solve                            */
  int krylov_restart; /* FGMRES restart length m, 1..63 (ignored by FCGMG_SOLVER_GMG)              */
  int immersed_nitsche; /* 1: the obstacle surfaces are no-slip Dirichlet boundaries (Eq. 5, Gamma_D),
                           imposed by the Nitsche forms of the walls on the circle arcs (2D) or
                           sphere pieces (3D) through the cut cells. The local blocks may then be
                           indefinite and are factorised by a dense LU with partial pivoting: in 2D
                           under every cache policy, in 3D at set-up for cache_inverse, the only
                           policy 3D accepts with it (E_ARG otherwise). 0: obstacles are fictitious
                           regions only.                                                             */
} fcgmg_params;

/* Outer iteration of fcgmg_solve. GMG: the standalone multigrid of Sec. 4, x <- V(x, b) until the
 * stopping test. FGMRES: flexible GMRES(m) in FP64 with one V-cycle from a zero guess as the right
 * preconditioner (FP32 cycle under FCGMG_PREC_MIXED), classical Gram-Schmidt applied twice, the
 * Arnoldi residual estimate as stopping test and the true residual checked at every restart; GMG
 * used as a Krylov preconditioner, which also converges where the standalone cycle does not. The
 * set-up holds 2m + 2 extra finest-level vectors. Iteration counts are V-cycles in both cases. */
enum { FCGMG_SOLVER_GMG = 0, FCGMG_SOLVER_FGMRES = 1 };

/* Precision of fcgmg_solve. FP64: every operation in FP64. MIXED (cache_inverse only): set-up,
 * including every patch factorisation, stays FP64; the inverse rows, stored stencils and coarse
 * inverse are then rounded to FP32, and each V-cycle runs in FP32 on the residual equation
 * A e = r. The outer loop is FP64 iterative refinement: r = b - A x in FP64, e from one FP32
 * V-cycle with a zero guess, x += e. The single-step calls (smooth, vcycle, ...) stay FP64. */
enum { FCGMG_PREC_FP64 = 0, FCGMG_PREC_MIXED = 1 };

typedef struct {
  int64_t n_cells_axis;   /* n_l                                                                */
  int64_t n_nodes;        /* (n_l+1)^d                                                          */
  int64_t n_cut_cells;    /* cells cut by an obstacle surface                                   */
  int64_t n_fict_cells;   /* cells entirely inside obstacles                                    */
  int64_t n_classes;      /* regular patch classes (one shared local block each)                */
  int64_t n_irregular;    /* patches with an individual local block                             */
  int64_t irregular_cols; /* sum of |S_i| over irregular patches                                */
  int64_t cached_bytes;   /* device bytes of policy-cached patch data on this level             */
  int64_t n_stencils;     /* nodes whose operator row is stored (not a uniform neighbourhood)    */
} fcgmg_level_stats;

/* Build the hierarchy of Algorithm 1 (uniform case: every level fully coarsened), classify cells,
 * integrate cut cells, classify vertex patches (Eq. 15 subdomains) into shared regular classes and
 * individual patches, and set up the chosen cache policy (Sec. 3.1.2) and the coarsest-grid direct
 * solver (Sec. 3). `balls` is a HOST array of n_balls x 4 doubles (centre x, y, z, radius; z
 * ignored in 2D): the fictitious part of Eq. (7) is the union of the closed balls.
 * Synchronises `stream`. Errors: E_ARG (bad sizes), E_NOMEM, E_HIP, E_SINGULAR (names the patch). */
int fcgmg_setup_hierarchy(const fcgmg_params* prm, const double* balls, int n_balls, void* stream,
                          fcgmg_h* out);

/* Number of levels / FP64 values of one vector on `level` ((d+1)*(n_l+1)^d). */
int fcgmg_num_levels(fcgmg_h h, int* n_levels);
int fcgmg_num_dofs(fcgmg_h h, int level, int64_t* n_dof);

/* Statistics of one level (host struct). */
int fcgmg_level_stats_get(fcgmg_h h, int level, fcgmg_level_stats* out);

/* Right-hand side b = (f, g) of Eq. (9) on `level` (body force weighted by alpha, Nitsche data
 * terms of the Dirichlet walls, h = 0 on Neumann walls). Writes (d+1)*(n_l+1)^d values to b. */
int fcgmg_rhs(fcgmg_h h, int level, double* b, void* stream);

/* r = b - L x on `level` (Eq. 12, 14). x, b read; r written; r must not alias x or b. */
int fcgmg_residual(fcgmg_h h, int level, const double* x, const double* b, double* r, void* stream);

/* `sweeps` applications of Eq. (14) with the smoother S of Eq. (15):
 *   x <- x + sum_i R~_i^T omega L_i^{-1} R_i (b - L x),
 * every subdomain reading the same residual and writing only the DoFs of its own node (restricted
 * prolongation R~_i). x is updated in place; b is read. */
int fcgmg_smooth(fcgmg_h h, int level, double* x, const double* b, int sweeps, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): fcgmg_smooth with the same kernels and arithmetic (x ends bitwise
 * equal), whose scratch (the residual and, 2D cache_inverse, the second iterate of the fused sweep
 * pairs) lives in a static device array of 96 MiB per GPU, held until the process ends, instead of
 * the level's own buffers. The call allocates nothing. The array's device address is looked up once
 * per device on the first call there (hipGetSymbolAddress, with that device current). Every call on
 * one GPU shares that array and leaves the last call's contents in it; nothing in it needs to start
 * at zero (each sweep writes its scratch before reading it). Calls that overlap on one GPU (other
 * streams, other threads) race on it. The level's scratch, (d+1) N_l doubles padded to a multiple of
 * 32 plus another (d+1) N_l for the 2D cache_inverse second iterate, must fit the 12,582,912 doubles
 * of the array: up to 1,447 cells per axis for 2D cache_inverse, 2,047 for the other 2D policies,
 * 145 in 3D. E_ARG for a larger level, or a bad level or pointer. */
int fcgmg_smooth_noalloc(fcgmg_h h, int level, double* x, const double* b, int sweeps, void* stream);

/* Stacked right-hand sides (several problems on one geometry): `sweeps` sweeps of Eq. (14)-(15) on
 * level `level` for nrhs (1..8) vectors at once. x and b hold nrhs vectors of (d+1) N_l doubles,
 * one after another (vector k at offset k (d+1) N_l); r is caller-owned scratch of the same size (3D:
 * it holds the residuals of the last sweep on return; 2D: the second iterate of the fused sweeps). In
 * 3D the inverse rows of every streamed patch are read once per sweep for all right-hand sides; in 2D
 * one fused launch sweeps every vector (the vector is the launch's second grid index; levels from
 * 2^21 nodes take one launch per vector). Each x_k ends bitwise equal to fcgmg_smooth on x_k, b_k.
 * cache_inverse only.
 * Asynchronous on `stream`; E_ARG for a bad level, pointer, nrhs or policy. */
int fcgmg_smooth_multi(fcgmg_h h, int level, double* x, const double* b, double* r, int nrhs, int sweeps,
                       void* stream);

/* One V-cycle (as fcgmg_vcycle) for each of nrhs right-hand sides of one geometry: x and b hold nrhs
 * finest-level vectors one after another (device, FP64, each (d+1) N_fine). cache_inverse only.
 * Every result is bitwise that of fcgmg_vcycle on its vector. In 3D each sweep of every level
 * streams the individual patches' inverse rows once for all vectors (as fcgmg_smooth_multi); in 2D
 * every level smooths all vectors as fcgmg_smooth_multi does, and the residual + restriction and the
 * coarsest solve also take all vectors in one launch. The first call allocates a workspace of 8 vectors of r per level and
 * of x and b per coarse level, kept by the handle (counted by fcgmg_device_bytes, not by
 * fcgmg_footprint_bytes). Errors: E_ARG (nrhs outside 1..8, another policy),
 * E_NOMEM, E_HIP. */
int fcgmg_vcycle_multi(fcgmg_h h, double* x, const double* b, int nrhs, void* stream);

/* b_coarse = R r_fine with R = P^T (Eq. 13, T = identity): level `fine_level` to fine_level-1. */
int fcgmg_restrict(fcgmg_h h, int fine_level, const double* r_fine, double* b_coarse, void* stream);

/* x_fine += P e_coarse (Q1 interpolation, Sec. 3): level fine_level-1 to `fine_level`. */
int fcgmg_prolongate_add(fcgmg_h h, int fine_level, const double* e_coarse, double* x_fine, void* stream);

/* x = L_0^{-1} b on the coarsest level (direct solver, Sec. 3; bordered with sum(p) = 0 when the
 * constant pressure is in the kernel). */
int fcgmg_coarse_solve(fcgmg_h h, const double* b, double* x, void* stream);

/* One V-cycle on the finest level (Sec. 3, 4): nu_pre sweeps, residual restriction, recursive
 * coarse correction from a zero guess, prolongation, nu_post sweeps. x updated in place. */
int fcgmg_vcycle(fcgmg_h h, double* x, const double* b, void* stream);

/* Mixed precision only: e = V(0, r), one V-cycle in FP32 on the residual equation of the finest
 * level from a zero guess. r (read) and e (written) are FP64 device vectors of the finest level;
 * r is rounded to FP32 on entry, e widened on exit. E_ARG when the hierarchy is not MIXED. */
int fcgmg_vcycle_fp32(fcgmg_h h, const double* r, double* e, void* stream);

/* Standalone GMG (Sec. 4): V-cycles until ||b - L x||_2 <= rtol ||b - L x0||_2 (Euclidean norm
 * over all DoFs) or max_iter cycles; with FCGMG_PREC_MIXED, FP64 iterative refinement around FP32
 * V-cycles (see FCGMG_PREC_*). Synchronises `stream` once per cycle to read the norm.
 * *iters, *rel_res receive the cycle count and final ratio (also on E_NOCONV / E_NAN).
 * res_hist (optional HOST array of max_iter+1 doubles) receives the residual norms. */
int fcgmg_solve(fcgmg_h h, double* x, const double* b, double rtol, int max_iter, int* iters,
                double* rel_res, double* res_hist, void* stream);

/* ||v||_2 of a level vector, written to *out (host) after synchronising `stream`. */
int fcgmg_norm(fcgmg_h h, int level, const double* v, double* out, void* stream);

/* Kernel kinds for the event profiler. */
enum {
  FCGMG_K_RESIDUAL = 0,      /* r = b - L x                                                     */
  FCGMG_K_APPLY_REGULAR = 1, /* cache_inverse: shared-row patches (LDS residual tile)            */
  FCGMG_K_APPLY_IRREGULAR = 2, /* cache_inverse: individual rows streamed from HBM              */
  FCGMG_K_PATCH_SOLVE = 3,   /* cache_matrix / cache_none: factorise + solve per patch           */
  FCGMG_K_RESTRICT = 4,
  FCGMG_K_PROLONG = 5,
  FCGMG_K_COARSE = 6,        /* coarsest-grid solve                                              */
  FCGMG_K_ZERO = 7,
  FCGMG_K_SWEEP_FUSED = 8,   /* cache_inverse, 2D: residual + all patch corrections in one kernel */
  FCGMG_K_RESIDUAL_RESTRICT = 9, /* 2D V-cycle: fine residual and its restriction in one kernel    */
  FCGMG_K_COUNT = 10
};

/* Event profiler (tracing): while enabled, every kernel launch of the handle is bracketed by a
 * pair of HIP events on the launch stream. fcgmg_profile_read synchronises those events and returns
 * the accumulated kernel time (ms) and launch count of one kind on one level since the last reset.
 * Enabling adds two event records per launch; leave it off for production timing. */
int fcgmg_profile_enable(fcgmg_h h, int on);
int fcgmg_profile_reset(fcgmg_h h);
int fcgmg_profile_read(fcgmg_h h, int kind, int level, double* total_ms, int64_t* launches);

/* Tile-shape autotuner of the fused 2D sweep (FCGMG_K_SWEEP_FUSED; 2D cache_inverse only). The
 * sweep covers the level's nodes in tiles of tile_x x tile_y nodes, one workgroup of `threads` per
 * tile plus extra workgroups for tiles with many individually stored patches, compiled for at least
 * `waves_per_simd` resident wavefronts per SIMD (which bounds its registers per lane);
 * fcgmg_fused_shape(k, ...) gives these four numbers of shape k, for k in [0, 8). Set-up picks a
 * shape by level size.
 * fcgmg_autotune times `reps` (1..1000) pairs of fused sweeps with every shape on every level above
 * the coarsest (on scratch vectors it allocates and frees; the level's own vectors are untouched),
 * keeps the fastest shape per level and rebuilds that level's extra-workgroup plan. Every shape
 * computes the same numbers in the same order: results are bitwise those of the default shapes.
 * shape_out: host array of n_levels ints, the shape index per level afterwards (-1 = default by
 * size; levels without the fused sweep keep -1). us_out: NULL or a host array of n_levels * 8
 * doubles, microseconds per sweep of level l with shape k at [l * 8 + k] (-1 where not timed).
 * Synchronises `stream`; must not overlap other work on the handle. The plan buffer may grow, so
 * fcgmg_device_bytes can exceed fcgmg_footprint_bytes afterwards by a few KiB.
 * Errors: E_ARG (bad handle, pointer or reps), E_NOMEM, E_HIP. */
int fcgmg_autotune(fcgmg_h h, int reps, int* shape_out, double* us_out, void* stream);
int fcgmg_fused_shape(int k, int* tile_x, int* tile_y, int* threads, int* waves_per_simd);
/* Apply a stored choice: shape k (-1 = default by size) on one level, plan rebuilt. Synchronises
 * `stream`. Errors: E_ARG (bad level or k, or a level without the fused sweep), E_NOMEM, E_HIP. */
int fcgmg_set_fused_shape(fcgmg_h h, int level, int k, void* stream);

/* How cache_none obtains each patch block L_i at every application (Sec. 3.1.2). integrate = 0
 * (default): read from the operator rows that the residual applies, as the policy retrieves the
 * block from the global operator; 1: assembled from the element integrals of the patch's cell
 * window, every cut cell of the window integrated on the fly by its space tree (no operator data
 * read; several times slower). Both give L_i = R_i L R_i^T to rounding. The immersed-boundary blocks
 * are always assembled. Errors: E_ARG (bad handle or mode, or a hierarchy of another policy). */
int fcgmg_set_cache_none_assembly(fcgmg_h h, int integrate);

/* Device bytes held by the handle (all levels, all policy data). */
int fcgmg_device_bytes(fcgmg_h h, size_t* bytes);

/* Device bytes fcgmg_setup_hierarchy would hold for these arguments (equal to fcgmg_device_bytes
 * after that set-up), computed on the host without touching the device: the cell kinds by the same
 * ball-box test, then the sizes of every level's vectors, operator data and policy cache (Sec.
 * 3.1.2: cache_inverse > cache_matrix > cache_none in general). For admission by memory footprint.
 * Cost: one pass over the cells of every level. Errors: E_ARG as set-up. */
int fcgmg_footprint_bytes(const fcgmg_params* prm, const double* balls, int n_balls, size_t* bytes);

/* ---- Batched cycles: many independent 2D problems per launch ---------------------------------
 * The hierarchies (2D, cache_inverse, FP64, equal even nu_pre and nu_post >= 2, each at most once)
 * stay owned by the caller and must outlive the batch. Every step of the V-cycle of Sec. 3 runs as
 * one launch over all problems taking part: depth d of the cycle works on level n_levels - 1 - d of
 * each problem, and the coarsest solves of all problems share one launch. Each problem's result is
 * bitwise the one of fcgmg_vcycle on its own. x, b: HOST arrays of `count` device pointers to the
 * finest-level vectors of the problems, in the order of hs. */
typedef struct fcgmg_batch* fcgmg_batch_h;
int fcgmg_batch_create(const fcgmg_h* hs, int count, fcgmg_batch_h* out);
/* One V-cycle on every problem; x updated in place. */
int fcgmg_batch_vcycle(fcgmg_batch_h bt, double* const* x, const double* const* b, void* stream);
/* Standalone GMG on every problem (as fcgmg_solve with the GMG solver), with the residual norms of
 * all problems from one launch and one synchronisation per cycle; a problem leaves the batch when it
 * meets its stopping test. iters, rel_res: HOST arrays of `count`. E_NOCONV if any problem did not
 * converge in max_iter cycles (the others are converged and their x final). */
int fcgmg_batch_solve(fcgmg_batch_h bt, double* const* x, const double* const* b, double rtol, int max_iter,
                      int* iters, double* rel_res, void* stream);
/* on = 1: every fused sweep of the batched cycle (fcgmg_batch_vcycle, fcgmg_batch_solve) runs as one
 * persistent launch, as many workgroups as the device holds at once, each taking every G-th tile of
 * the launch (G workgroups) over all problems; on = 0 (default): one workgroup per tile. The results
 * are the same bits either way. E_ARG: null handle, on not 0 or 1. */
int fcgmg_batch_set_persistent(fcgmg_batch_h bt, int on);
int fcgmg_batch_destroy(fcgmg_batch_h bt);

/* ---- Solve server: concurrent solves with device-resident hierarchies ------------------------
 * Worker threads (one HIP stream each) take requests in arrival order. A request runs on a resident
 * hierarchy of the same problem when one is idle; otherwise it is admitted once its footprint
 * (fcgmg_footprint_bytes plus its right-hand side) fits the memory budget, after evicting idle
 * hierarchies least recently used first. With cache_policy = -1 the server picks the fastest policy
 * of Sec. 3.1.2 that fits (cache_inverse, then cache_matrix, then cache_none). A request that can
 * never fit completes with E_NOMEM. Each solve is standalone GMG (or FGMRES) from x = 0 on the
 * problem's own right-hand side (fcgmg_rhs).
 * Continuous batching (continuous_batching = 1): a request that the batched cycle takes (2D,
 * cache_inverse, FP64, GMG, V(2,2)) is set up by a worker and then joins the running batch: one
 * engine thread advances every such request by one V-cycle per step, all of them in the launches
 * of fcgmg_batch_vcycle, with their residual norms from one launch; requests join as their set-up
 * finishes and leave when they meet their stopping test (or the cycle limit). Each problem's cycle
 * and norm are computed by workgroups of its own, so a result is bit for bit the same alone and in
 * any mix; against fcgmg_solve its norms are summed in another order (iterations within one). The
 * other requests run fcgmg_solve on their worker. */
typedef struct fcgmg_server* fcgmg_server_h;

typedef struct {
  int workers;             /* concurrent set-ups and unbatched solves, 1..16                      */
  int max_iter;            /* cycle limit of every solve                                          */
  int64_t hbm_budget;      /* device bytes for resident hierarchies; 0: 80% of the free memory     */
  int continuous_batching; /* 1: batchable requests share the batched cycle (see above); 0: off   */
} fcgmg_server_params;

typedef struct {
  int status;          /* FCGMG_OK or the error of the request (E_NOMEM: never fits the budget)     */
  int policy;          /* cache policy it ran with                                                */
  int iters;           /* V-cycles                                                                */
  int cache_hit;       /* 1: ran on a resident hierarchy                                          */
  double rel_res;      /* final relative residual                                                 */
  double t_queue_ms;   /* submit to start                                                         */
  double t_setup_ms;   /* hierarchy set-up (0 on a hit)                                           */
  double t_solve_ms;   /* solve, including the final stream synchronisation                       */
  double t_total_ms;   /* submit to completion                                                    */
  int64_t footprint;   /* device bytes of its hierarchy and right-hand side                       */
} fcgmg_request_result;

int fcgmg_server_create(const fcgmg_server_params* sp, fcgmg_server_h* out);
/* Queue a solve of the problem (prm, balls as for fcgmg_setup_hierarchy; prm->cache_policy may be
 * -1). x_out: caller-owned device buffer of (d+1)(n_cells+1)^d doubles, written before the request
 * completes; it must stay valid until fcgmg_server_wait returns for *request_id. */
int fcgmg_server_submit(fcgmg_server_h srv, const fcgmg_params* prm, const double* balls, int n_balls,
                        double rtol, double* x_out, int64_t* request_id);
/* Block until the request completes; fills *res and forgets the id. */
int fcgmg_server_wait(fcgmg_server_h srv, int64_t request_id, fcgmg_request_result* res);
/* Device bytes and number of hierarchies currently resident. */
int fcgmg_server_resident_bytes(fcgmg_server_h srv, int64_t* bytes, int* hierarchies);
/* Continuous batching so far: batched cycle steps run, and the sum over those steps of the number of
 * requests each advanced (their ratio is the mean batch size), and the largest batch. */
int fcgmg_server_stats(fcgmg_server_h srv, int64_t* steps, int64_t* request_cycles, int* max_batch);
/* Finish queued requests, join the workers, free every resident hierarchy. */
int fcgmg_server_destroy(fcgmg_server_h srv);

/* Release every device buffer of the handle. NULL is accepted. */
void fcgmg_destroy(fcgmg_h h);

/* Message of the last error on the calling thread ("" if none). */
const char* fcgmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FCGMG_H */
