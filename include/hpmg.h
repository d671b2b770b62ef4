/*
 * hpmg.h — C ABI of libhpmg.so: matrix-free hp-multigrid for symmetric
 * interior penalty DG (SIPG) discretisations of -div(kappa grad u) = f on
 * the unit box with homogeneous Dirichlet conditions, on AMD MI355X (gfx950).
 *
 * Method: arXiv 2510.00998 ("Implementation techniques for multigrid
 * solvers for high-order Discontinuous Galerkin methods").  The smoother is
 * the single-touch block-Jacobi sweep with auxiliary facet (trace)
 * variables and shift-and-fuse (Section 4.2, technique shift-and-fuse and
 * Algorithm BlockJacobi with loop fusion); the multigrid cycle follows
 * Section 5 (Algorithms CoarseGridCorrection and MGMult, hp-multigrid of
 * Section 5.2) with a gradual p-coarsening to continuous Q1 and
 * h-coarsening by two.
 *
 * Conventions (all entry points):
 *  - Vectors are DEVICE pointers owned by the caller, cell-major: cell
 *    c = cx + n*cy (+ n^2*cz), local node i = a + N*b (+ N^2*c), N = p+1,
 *    x fastest, Gauss-Lobatto nodes (Gauss-Legendre with options.basis =
 *    1).  `nrhs` right-hand sides are stacked back to back ([rhs][dof]).
 *  - All work is enqueued on `stream` (0 = the null stream).  The solvers
 *    (hpmg_solve, hpmg_mgmult, hpmg_batch_solve) synchronise it and read a
 *    few scalars per iteration back to the host.
 *  - No function throws; each returns a status.  A message describing the
 *    last failure of the calling thread is available from hpmg_last_error.
 *  - Right-hand sides are load vectors b_i = int f phi_i, not samples of f.
 */
#ifndef HPMG_H
#define HPMG_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hpmg_ctx* hpmg_handle; /* opaque, owned by the library */

typedef enum {
  HPMG_OK = 0,
  HPMG_E_INVALID = 1,       /* bad argument (null pointer, size, unsupported range) */
  HPMG_E_NOMEM = 2,         /* device or host allocation failed */
  HPMG_E_DEVICE = 3,        /* a HIP call failed (no device, launch failure, ...) */
  HPMG_E_NOT_CONVERGED = 4, /* hpmg_solve reached maxit before rtol */
  HPMG_E_BREAKDOWN = 5,     /* non-finite value met in hpmg_solve (e.g. NaN in b) */
  HPMG_E_UNSUPPORTED = 6    /* valid request the library does not implement */
} hpmg_status;

/* Element type of the vectors a call reads and writes.  F16 (IEEE binary16)
 * and BF16 are storage formats of the finest level only: the arithmetic,
 * the operator tables and the coarser levels are FP32 (16-bit operands,
 * FP32 accumulation).  hpmg_apply_A takes F64 and F32 only. */
typedef enum { HPMG_F64 = 0, HPMG_F32 = 1, HPMG_F16 = 2, HPMG_BF16 = 3 } hpmg_dtype;

/* Precision of the multigrid cycle used inside hpmg_solve.  F64: everything
 * in double.  F32: smoother, transfers and coarse levels in float inside the
 * FP64 outer iteration (fine residual, update and coarsest solve in double).
 * F16 / BF16: as F32, with the finest level's cycle vectors and traces stored
 * in 16 bits (half the bytes of its sweeps); the residual handed to the
 * cycle is scaled to mean square lambda = dim pi^2 kappa_min (h/(p+1))^dim
 * before the cast, which keeps it and the cycle's output (about r/lambda)
 * inside the FP16 range. */
typedef enum { HPMG_PREC_F64 = 0, HPMG_PREC_F32 = 1, HPMG_PREC_F16 = 2, HPMG_PREC_BF16 = 3 } hpmg_precision;

/* Unit box [0,1]^dim with n[0] cells per axis (n[1], n[2] must equal n[0]).
 * dim in {2, 3}, n >= 2. */
typedef struct { int dim; int n[3]; } hpmg_mesh;

/* Diffusion coefficient, piecewise constant per cell.  per_cell = 0: the
 * value kappa_const (> 0) everywhere.  per_cell = 1: kappa points to n^dim
 * HOST doubles (> 0, finite), copied during setup. */
typedef struct { int per_cell; double kappa_const; const double* kappa; } hpmg_coeff;

typedef struct {
  double sigma0;      /* penalty sigma = sigma0 (p+1)^2 / h on interior facets, 2 sigma on boundary facets (default 2) */
  double omega_dg;    /* block-Jacobi relaxation on DG levels, 0 < omega <= 1 (default 0.7) */
  double omega_cg;    /* point-Jacobi relaxation on Q1 levels (default 2/3) */
  int nu_pre;         /* block-Jacobi steps on DG levels before the coarse correction (default 2) */
  int nu_post;        /* block-Jacobi steps on DG levels after it (default 2; Algorithm MGMult of
                         Section 5.1: nu_pre = nu, nu_post = 0) */
  int coarsest_n;     /* stop h-coarsening once n <= coarsest_n (default 4) */
  int precision;      /* hpmg_precision of the cycle inside hpmg_solve (default F32) */
  int max_rhs;        /* largest nrhs any call will use (default 1) */
  int p_coarsening;   /* 0: halve p while >= 2, then Q1 (default); 1: DG_p -> Q1 in one step
                         (the paper's two-grid hp scheme, Section 5.2) */
  int h_factor;       /* Q1 h-coarsening factor, 2 (default) or 3 (the paper's 3^k meshes) */
  int basis;          /* DG nodes: 0 Gauss-Lobatto (default), 1 Gauss-Legendre (diagonal mass, dense
                         facet value functionals; Section 4.1 remark on the two bases) */
  int block_recompute; /* variable kappa only.  0 (default): the fast-diagonalisation data of every cell
                         block is built once at setup (on the device, by a Jacobi eigensolve per cell and
                         axis) and streamed in each traversal.  1: rebuilt inside every traversal from
                         kappa (the same eigensolve in the sweep/apply kernels), the paper's "recompute
                         the block inverse per cell" variant that mimics inhomogeneous problems (Section
                         7, single-core measurements); setup stores no per-cell data.  2: split and
                         postpone (Section 4.3): every finest-level sweep of hpmg_smooth / hpmg_sweep
                         reads stored records while the records of the next traversal are rebuilt from
                         kappa on a second stream of the handle into a second buffer (overlapping the
                         compute-bound rebuild with the memory-bound sweep); other calls read the
                         current records.  Same operator and iterates up to rounding in all three.  1 or
                         2 with constant kappa is HPMG_E_INVALID. */
  int nu_pre_cg;      /* point-Jacobi steps on Q1 levels before their coarse correction (-1, the
                         default: nu_pre); the h-multigrid of Section 5.2 pre- and post-smooths */
  int nu_post_cg;     /* point-Jacobi steps on Q1 levels after it (-1, the default: nu_post) */
  int block_variant;  /* block-Jacobi block on DG levels: 0 (default) the exact cell block A_{K<-K};
                         1 the block of an interior cell for every cell (Section 4.1, technique
                         approximate boundary operators: one stored block inverse; the operator A and
                         the fixed point are unchanged).  1 needs constant kappa and n >= 3. */
  int p_schedule[8];  /* explicit degrees of the p-coarse DG levels after the finest one, strictly
                         decreasing, each >= 2, terminated by 0 (Q1 follows the last); p_schedule[0]
                         = 0 (the default) takes the schedule from p_coarsening */
  void* (*alloc)(size_t bytes, void* ctx); /* device allocator for every buffer the handle (and a batch
                         of handles) holds, NULL (default): hipMalloc.  Must return memory of the
                         current device aligned to 256 bytes, or NULL on failure (HPMG_E_NOMEM). */
  void (*free)(void* ptr, void* ctx);      /* releases what alloc returned (hpmg_destroy, batch destroy) */
  void* alloc_ctx;    /* passed to alloc and free */
  int mfma;           /* 16-bit storage (F16 / BF16) sweeps in 3D: 0 (default) run the contractions of
                         the block solve on the vector units in FP32; 1 run its six volume contractions
                         on the matrix cores (v_mfma_f32_16x16x16 with FP16 or BF16 operands, FP32
                         accumulation; the operands of every contraction are rounded to the storage
                         format).  Facet transforms, lifts and updates stay in FP32.  1 needs dim 3. */
  int spacetree_levels; /* adaptive meshes (hpmg_setup_adaptive): 1 (default) coarsens the last DG degree of
                         the p-coarsening along the spacetree (the deepest leaves merged into their parents,
                         one level at a time, down to the base mesh; each level rediscretised with the fine
                         penalty factor, transfers by the parents' polynomials) before the Q1 level of the base
                         mesh; 0 goes from that degree straight to Q1 on the base mesh.  Ignored on uniform
                         meshes. */
} hpmg_options;

/* Fill *opt with the defaults listed above. */
void hpmg_default_options(hpmg_options* opt);

/* Build the level hierarchy on the current HIP device: 1D reference data,
 * fast-diagonalisation data of the cell blocks A_{K<-K} (per boundary class
 * for constant kappa, per cell for variable kappa), Q1 coarse operators by
 * Galerkin products, device buffers.  1 <= p <= 8.  The result is written to
 * *out; release it with hpmg_destroy.  Paper: Section 4.1 (Schur complement
 * block A_{K<-K}, technique precompute-block-inverse), Section 5.2. */
hpmg_status hpmg_setup(const hpmg_mesh* mesh, int p, const hpmg_coeff* coeff,
                       const hpmg_options* opt, hipStream_t stream, hpmg_handle* out);

/* Adaptive mesh: the leaves of a spacetree over the unit box (Section 2.1,
 * hierarchical Cartesian meshes).  The n^dim base cells (width 1/n) form
 * level 0; a refined cell of level l splits every axis into `refine` parts
 * (2, or 3 as the paper's spacetree), giving r^dim cells of level l + 1 and
 * width 1/(n r^(l+1)).  leaves: HOST array of nleaf rows (level, x_0, ..,
 * x_{dim-1}), integer coordinates at the leaf's level (0 <= x_k < n r^l),
 * copied during setup; the row order is the cell order of every vector.
 * The leaves must cover the box without overlap, and leaves that share a
 * facet must be at most one level apart (facet balance), so that a facet
 * is conforming or the coarse facet of a "hanging" facet covered by
 * r^(dim-1) finer leaves.  level <= 12, n r^level <= 2^20. */
typedef struct {
  int dim;
  int n;              /* base cells per axis, >= 2 */
  int refine;         /* subdivision factor r: 2 or 3 */
  int nleaf;
  const int* leaves;  /* [nleaf][1 + dim] */
} hpmg_adaptive_mesh;

/* hpmg_setup on an adaptive mesh: the SIPG operator of eq. weak_form_IP on
 * the leaves, with the penalty of a piece of the skeleton taken from the
 * finer of its two cells (sigma0 (p+1)^2 / min(h-, h+); 2 sigma0 (p+1)^2 /
 * h_K on the boundary).  The cell kernels read the neighbour-side traces of
 * each facet through a slot table; after every traversal that writes
 * traces, a remap kernel turns the traces at hanging facets into each
 * side's view (the coarse facet polynomial restricted to each fine facet;
 * the L2 projection of the fine traces onto the coarse facet), so that the
 * fused sweep stays one traversal per step.  Multigrid: the DG levels of
 * lower degree on the same leaves, then (options.spacetree_levels) the last
 * degree on the coarser levels of the spacetree down to the base mesh, then
 * continuous Q1 on the base mesh (transfer by evaluating its trilinear
 * functions at the nodes), then the h-levels of the base mesh.
 * Constant kappa only (coeff->per_cell = 0), Gauss-Lobatto or Gauss-Legendre
 * nodes, exact blocks (block_variant 0, block_recompute 0, mfma 0), FP64
 * or FP32 vectors and cycles (F16 / BF16: HPMG_E_UNSUPPORTED); every other
 * entry point works on the handle (not hpmg_batch_create).  HPMG_E_INVALID
 * for a mesh that breaks the rules above. */
hpmg_status hpmg_setup_adaptive(const hpmg_adaptive_mesh* mesh, int p, const hpmg_coeff* coeff,
                                const hpmg_options* opt, hipStream_t stream, hpmg_handle* out);

/* Number of DG degrees of freedom n^dim (p+1)^dim (adaptive meshes: nleaf
 * (p+1)^dim) of one right-hand side. */
size_t hpmg_ndof(hpmg_handle h);

/* Load vector b_i = int f phi_i ((p+3)-point Gauss per direction) for a
 * built-in f: kind 0: f = params[0] (constant); kind 1: f = -Laplace of
 * prod_i sin(params[0] pi x_i) (i.e. dim params[0]^2 pi^2 prod sin); kind 2
 * (dim 2 only): f = -Laplace of the two-peak solution of Section 6
 * (x(1-x)y(1-y)(2 e1 - e2), Gaussians e_i centred at (0.3, 0.4) and
 * (0.8, 0.6) with widths 0.2 and 0.1; params unused); b is a device FP64
 * vector of hpmg_ndof entries.  Paper: Section 2.3.1, b(v). */
hpmg_status hpmg_load_vector(hpmg_handle h, int kind, const double* params, double* b,
                             hipStream_t stream);

/* y = A u for the SIPG operator A of eq. weak_form_IP (matrix-free:
 * trace projection then one fused cell traversal).  dtype selects double or
 * float vectors; u and y must not overlap. */
hpmg_status hpmg_apply_A(hpmg_handle h, hpmg_dtype dtype, const void* u, void* y, int nrhs,
                         hipStream_t stream);

/* nsweeps block-Jacobi steps u <- u + omega A_{K<-K}^{-1} (b - A u) in
 * place (Algorithm BlockJacobi with loop fusion: one projection traversal,
 * then one fused traversal per step).  nsweeps >= 0. */
hpmg_status hpmg_smooth(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps,
                        int nrhs, hipStream_t stream);

/* Warm-up projection of Algorithm BlockJacobi (loop-fused form): writes
 * the facet traces of u (value and outward normal derivative on every
 * facet, technique projection-variables) into the handle's trace buffer for
 * dtype.  Enables hpmg_sweep on the same u. */
hpmg_status hpmg_project(hpmg_handle h, hpmg_dtype dtype, const void* u, int nrhs, hipStream_t stream);

/* nsweeps fused single-touch block-Jacobi sweeps (one traversal each,
 * technique shift-and-fuse) on u in place, reading the traces held by the
 * handle and replacing them with those of the updated u.  Requires that the
 * previous call on this handle and dtype was hpmg_project, hpmg_smooth or
 * hpmg_sweep on the same u with the same nrhs and that u was not modified in
 * between (HPMG_E_INVALID if no such state exists). */
hpmg_status hpmg_sweep(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps, int nrhs,
                       hipStream_t stream);

/* One V-cycle of the hp-multigrid in place on u (Algorithm MGMult body with
 * CoarseGridCorrection; nu_pre / nu_post block-Jacobi steps on the DG
 * levels, nu_pre_cg / nu_post_cg point-Jacobi steps on the Q1 levels,
 * p-coarsening, Q1, h-coarsening, dense coarsest solve) for each of the nrhs
 * stacked right-hand sides (1 <= nrhs <= max_rhs): the DG levels run every
 * column in one launch per traversal, the Q1 levels column after column. */
hpmg_status hpmg_vcycle(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nrhs,
                        hipStream_t stream);

typedef struct {
  int iterations;            /* outer iterations done */
  double initial_residual;   /* ||b - A u0||_2 */
  double final_residual;     /* true ||b - A u||_2 of the returned u (FP64) */
  double residual_history[256]; /* relative residuals, entry k after iteration k */
  double seconds;            /* wall time of the call */
} hpmg_solve_info;

/* Solve A u = b to ||b - A u||_2 <= rtol ||b - A u0||_2 (the true residual,
 * recomputed whenever the recurrence converges; the iteration restarts from
 * it if it misses rtol, at most 3 times per right-hand side: a true residual
 * still above rtol after that has met the FP64 rounding floor of b - A u and
 * the call returns HPMG_E_NOT_CONVERGED with final_residual set) with flexible CG
 * preconditioned by one V-cycle (precision from the options) in FP64.  u
 * holds the initial guess on entry.  info may be NULL (host pointer).
 * Returns HPMG_E_NOT_CONVERGED after maxit iterations, HPMG_E_BREAKDOWN on a
 * non-finite residual.  The caller's stream is synchronised first; the
 * iteration (one outer step, captured once per handle and cycle precision as
 * a HIP graph) then runs on an internal stream of the handle, and the call
 * returns when u holds the result.  Paper: Section 5 (MGMult, exit
 * criterion), with the unpreconditioned residual as exit test.  nrhs > 1
 * solves the stacked right-hand sides one after another (info: the last). */
hpmg_status hpmg_solve(hpmg_handle h, double* u, const double* b, int nrhs, double rtol,
                       int maxit, hpmg_solve_info* info, hipStream_t stream);

/* Stationary multigrid iteration u <- V(u, b) in FP64 (Algorithm MGMult with
 * the handle's V(nu_pre, nu_post) cycle; with precision F32/F16/BF16 each
 * step is u <- u + V(0, b - A u) with the reduced-precision cycle), from the
 * initial guess in u, until the relative residual of kind `exit_kind` is
 * <= rtol: 0 = unpreconditioned ||b - A u_k||_2 / ||b - A u_0||_2, 1 =
 * preconditioned ||u_k - u_{k-1}||_2 / ||u_1 - u_0||_2 (Section 5.1.1).
 * info->iterations = cycles done, residual_history[k] = relative residual of
 * that kind after cycle k+1 (first 256), final_residual = true ||b - A u||_2.
 * nrhs = 1.  HPMG_E_NOT_CONVERGED after maxit cycles. */
hpmg_status hpmg_mgmult(hpmg_handle h, double* u, const double* b, double rtol, int maxit, int exit_kind,
                        hpmg_solve_info* info, hipStream_t stream);

/* Size in bytes of the static device array that hpmg_smooth_noalloc keeps its
 * trace buffers in (one array per GPU, held until the process ends). */
#define HPMG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* hpmg_smooth without any device allocation, for callers that cannot
 * allocate device memory during the call (code under HIP stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result as hpmg_smooth (same kernels: the results are identical), but the
 * two ping-pong trace buffers live in a file-scope device array of
 * HPMG_NOALLOC_SCRATCH_BYTES bytes whose address hpmg_setup resolved for the
 * handle's device, instead of in memory owned by the handle; no hipMalloc,
 * hipFree or other allocating call is made (the 16-bit types included, for
 * which hpmg_smooth allocates traces on first use).  The handle's device must
 * be current.  Returns HPMG_E_INVALID when 2 x the traces of nrhs right-hand
 * sides (2 dim n^dim (p+1)^(dim-1) values each, in dtype, rounded up to 256
 * bytes) exceed the array.  Every call on one GPU shares that GPU's array and
 * leaves its last contents there; the projection writes every trace a sweep
 * reads, so nothing needs clearing, but calls that overlap in time on one GPU
 * (different streams, threads or handles) race on the array and must be
 * serialised by the caller.  The handle's own trace state is invalidated (as
 * u changes), so hpmg_sweep needs a new hpmg_project afterwards. */
hpmg_status hpmg_smooth_noalloc(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps, int nrhs,
                                hipStream_t stream);

/* Release every resource of the handle (NULL is ignored). */
void hpmg_destroy(hpmg_handle h);

/* ---------------------------------------------------------------- batches
 * Many independent problems (each set up by hpmg_setup, with its own mesh
 * size and degree) solved together.  Every phase of the V-cycle (sweeps,
 * residual + restriction, prolongation, Q1 levels, coarsest solve) runs as
 * one persistent launch over a work list of (problem, cell block,
 * right-hand side) items covering every problem at that level, so small
 * and large problems share the chip instead of running one after another;
 * one outer iteration of all problems is captured once as a HIP graph and
 * replayed.  This is the GPU counterpart of the task-based execution that
 * the paper uses to absorb uneven subdomain sizes (Section 7, subsections
 * on task-based realisation and on imbalanced domain decomposition): here
 * the uneven units are whole problems, merged into shared launches.
 */
typedef struct hpmg_batch_ctx* hpmg_batch; /* opaque, owned by the library */

/* Group `count` handles into a batch (*out; release with
 * hpmg_batch_destroy).  The handles must stay alive while the batch is
 * used, must be distinct, and must all be 3D with constant kappa,
 * 1 <= p <= 5, nu_pre >= 1, equal smoothing counts (DG and Q1), the
 * default p- and h-coarsening, the Gauss-Lobatto basis and the exact block
 * (HPMG_E_INVALID otherwise).  The batch's own workspace comes from the
 * first handle's allocator (options.alloc).  The batch uses the handles' level data and workspaces:
 * calls on a handle must not overlap a batch solve that contains it, and a
 * batch solve invalidates the handle's trace state (as hpmg_solve does). */
hpmg_status hpmg_batch_create(const hpmg_handle* hs, int count, hpmg_batch* out);

/* Solve every problem of the batch like hpmg_solve with the F32 cycle:
 * flexible CG in FP64 preconditioned by one FP32 V-cycle, until the true
 * residual satisfies ||b_j - A_j u_j||_2 <= rtol ||b_j - A_j u_j0||_2 for
 * every problem j and right-hand side.  u[j], b[j] (host array of count
 * DEVICE pointers each) hold nrhs stacked vectors of problem j
 * (nrhs <= its max_rhs); u[j] is the initial guess on entry.  Converged
 * segments stop changing while the others iterate.  infos (host, count
 * entries, may be NULL) receives per problem the largest iteration count,
 * initial and final true residual over its right-hand sides
 * (residual_history is left zero).  The first call for a given nrhs builds
 * the work lists, picks the persistent grid size and whether to launch
 * per polynomial degree by timing the V-cycle of the batch (autotuning),
 * and captures the iteration graph; later calls with the same
 * nrhs reuse them.  Work runs on an internal stream of the batch after the
 * caller's `stream` is synchronised; the call returns when done.
 * HPMG_E_NOT_CONVERGED after maxit iterations or when a segment's true
 * residual stays above rtol after 3 restarts (as in hpmg_solve),
 * HPMG_E_BREAKDOWN if a segment met a non-finite value.  A batch of one
 * problem solved for one right-hand side whose handle has precision
 * HPMG_F32 runs hpmg_solve on it (the same iteration without work lists;
 * infos[0] then carries its residual history). */
hpmg_status hpmg_batch_solve(hpmg_batch b, double* const* u, const double* const* rhs, int nrhs, double rtol,
                             int maxit, hpmg_solve_info* infos, hipStream_t stream);

/* Block-Jacobi smoothing of every problem of the batch on its finest level,
 * like hpmg_smooth: projection of the traces of u, then nsweeps fused
 * sweeps (Section 4.2, Algorithm BlockJacobi with loop fusion), each one
 * launch over all problems and right-hand sides.  u[j], b[j]: host array
 * of count DEVICE pointers to nrhs stacked vectors of problem j in dtype
 * (u updated in place).  Enqueued on `stream`; successive calls on one
 * batch must use one stream (they share an argument table).  The first
 * call for a dtype and nrhs tunes the launch grid on internal vectors.
 * Invalidates the handles' trace state. */
hpmg_status hpmg_batch_smooth(hpmg_batch b, hpmg_dtype dtype, void* const* u, const void* const* rhs,
                              int nsweeps, int nrhs, hipStream_t stream);

/* Launch configuration the autotuner chose for the batch's current number
 * of right-hand sides: out[0] grid cap (workgroups) of the V-cycle
 * launches: a persistent grid, or a cap at least the number of work items
 * of every launch (1 << 30 from the V-cycle tuner, the total item count
 * from the smoothing tuner): one workgroup per item, which runs loop-free
 * one-degree kernels; out[1] 1 if they run one launch per polynomial degree (else
 * one launch over all degrees), out[2..3] the same for FP32
 * hpmg_batch_smooth, out[4..5] for FP64, out[6..8] the tile masks of the
 * V-cycle, FP32 and FP64 smoothing launches: bit N (N = p + 1) set if the
 * degree-p launches use half the cells per workgroup (about 128 instead of
 * 256 threads).  0 where not tuned yet.  out: host array of 9 ints. */
hpmg_status hpmg_batch_tuning(hpmg_batch b, int* out);

/* Replace the launch configuration of the batch's current plan (the one
 * built by the last hpmg_batch_solve or hpmg_batch_smooth call): cfg (host,
 * 9 ints) as returned by hpmg_batch_tuning; a part whose grid entry
 * (cfg[0], cfg[2], cfg[4]) is 0 is left unchanged.  A tile mask may only
 * name degrees 1 <= p <= 5 and needs split 1.  For callers that reuse a
 * configuration tuned earlier, or compare configurations; all do the same
 * arithmetic per cell and agree to rounding.  HPMG_E_INVALID without a
 * plan or with an entry out of range. */
hpmg_status hpmg_batch_set_tuning(hpmg_batch b, const int* cfg);

/* Release the batch (not its handles; NULL is ignored). */
void hpmg_batch_destroy(hpmg_batch b);

const char* hpmg_status_string(hpmg_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char* hpmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HPMG_H */
