/*
 * regmg — regional (semi-structured) multigrid preconditioned CG on one MI355X.
 *
 * Method: Mayr, Berger-Vergiat, Ohm, Tuminaro, "Non-invasive multigrid for
 * semi-structured grids" (arXiv 2103.11962).  The domain is a set of boxes
 * ("regions", Section 3.1) of grid nodes that overlap only on shared
 * interface nodes.  Every region holds its own copy of its interface nodes and
 * its own regional matrix A^(k); the composite matrix is A = sum_k
 * Psi_k A^(k) Psi_k^T (eq. "extraction sum", Lemma on Psi [[A]] Psi^T = A).
 * A regional V-cycle (Section 3.6 figure, applied recursively) with Chebyshev
 * smoothing (Section 3.4, Algorithm 2), rate-3 linear transfers (Section 3.2),
 * per-region Galerkin products (eq. "RegionalGalerkinProduct") and a dense
 * direct solve of the coarsest composite operator (Section 3.5) preconditions
 * FP64 conjugate gradients.
 *
 * Conventions for every call:
 *  - All entry points return rmg_status; RMG_OK is 0.  On error the library
 *    stores a message retrievable with rmg_last_error() (thread-local) and
 *    leaves the handle usable unless the status is RMG_ERR_DEVICE.
 *  - Every argument is validated on the host before any kernel is launched.
 *  - Device pointers are HIP device addresses on the handle's device; "host"
 *    pointers are ordinary host memory.  Caller buffers are borrowed for the
 *    duration of the call only; the library never frees caller memory.
 *  - All device work is ordered on the stream given to rmg_create; calls
 *    that return results to the host synchronise that stream.
 *  - Coordinates are (x, y[, z]); arrays over nodes are x-fastest.  A
 *    COMPOSITE vector holds one value per composite dof (node-major, dof-minor);
 *    a REGIONAL vector holds region 0's nodes, then region 1's, ... (each
 *    region x-fastest, dof-minor), with interface nodes replicated (the
 *    regional layout [[v]] of Section 3.1).
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef REGMG_H
#define REGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RMG_OK = 0,
  RMG_ERR_ARG = 1,           /* bad argument value / null pointer / unsupported option */
  RMG_ERR_SHAPE = 2,         /* region boxes do not tile the domain, or cannot be coarsened */
  RMG_ERR_NUMERIC = 3,       /* NaN/Inf in input, non-positive diagonal, singular coarse matrix */
  RMG_ERR_DEVICE = 4,        /* a HIP runtime call failed */
  RMG_ERR_OOM = 5,           /* device allocation failed */
  RMG_ERR_NOT_SETUP = 6,     /* call made before the required earlier phase */
  RMG_ERR_BREAKDOWN = 7,     /* CG breakdown: p^T A p <= 0 or (r, z) <= 0 or non-finite */
  RMG_ERR_NOT_CONVERGED = 8  /* maxit reached; x holds the last iterate */
} rmg_status;

typedef enum { RMG_LAYOUT_COMPOSITE = 0, RMG_LAYOUT_REGIONAL = 1 } rmg_layout;

typedef enum {
  RMG_PDE_LAPLACE = 0,   /* Q1 Laplacian, element matrix scaled by h */
  RMG_PDE_DIFFUSION = 1, /* Q1 Laplacian times a per-element coefficient */
  RMG_PDE_ELASTICITY = 2 /* Q1 isotropic elasticity, Young's modulus per region */
} rmg_pde;

typedef enum {
  RMG_PREC_FP64 = 0,        /* whole V-cycle in FP64 */
  RMG_PREC_FP32 = 1,        /* V-cycle in FP32 inside FP64 CG */
  RMG_PREC_FP32_BF16 = 2,   /* FP32 V-cycle, finest-level stencil off-diagonals in BF16 */
  RMG_PREC_FP32_BF16_AUTO = 3 /* FP32 V-cycle; each smoothed level's stencil off-diagonals in BF16
                                where the measured convergence factor allows it: setup measures the
                                factor of bf16_cycles stationary V-cycles (rmg_convergence_factor)
                                with every level in FP32, then, finest level first, switches one
                                level at a time to BF16 and keeps it there when the factor stays
                                within (1 + bf16_tolerance) of the FP32 one (rmg_level_precision
                                reports the choice and both factors) */
} rmg_precision;

typedef struct rmg_handle rmg_handle;

/* Hierarchy options (Section 3.2 setup, Section 3.4 Chebyshev parameters). */
typedef struct {
  int nlevels;        /* region levels, >= 2; the last one is solved directly */
  int cheb_degree;    /* Chebyshev degree K >= 1, applied once before and once after */
  double eig_ratio;   /* eta: lower end of the interval = lambda / eta (default 20) */
  double boost;       /* kappa: upper end = kappa * lambda (default 1.1) */
  int power_iters;    /* power iterations for lambda_max(D~^-1 A) (default 10) */
  uint64_t seed;      /* seed of the counter-based power-method start vector */
  int precision;      /* rmg_precision */
  int stencil_kernel; /* 3D stencil kernel: 0 auto (2.5D tiles on levels with >= 2048 tiles of
                         21 planes; FP64 tiles are 41 planes deep where that still leaves >= 1024),
                         1 node-parallel, 2 2.5D plane-marching tiles (one block per tile),
                         3 the same tiles in a persistent grid (blocks stride over the tiles) */
  int autotune;       /* 1: at setup, time the scalar 3D stencil variants (node-parallel; 2.5D tiles
                         11/21/41 planes deep, one block per tile or a persistent grid striding
                         over the tile list) on every level and keep the fastest; overrides
                         stencil_kernel */
  int use_graph;      /* 1: rmg_solve captures the two halves of a CG iteration (around the
                         host convergence check) as HIP graphs once and replays them */
  const char* autotune_cache; /* text file of autotuner choices keyed by level shape and
                         precision; read before tuning, appended after (NULL: no file) */
  int smoother;       /* 0 (default): Chebyshev of degree cheb_degree (Section 3.4, Algorithm 2);
                         1: damped Jacobi, cheb_degree sweeps of u += jacobi_omega D~^-1 r
                         (Section 3.4, the smoother of Table 1);
                         2: region-local Gauss-Seidel (Section 3.4, Algorithm 1), cheb_degree
                         sweeps before and after the coarse correction: per sweep the composite
                         residual, then each region solves (D~/omega + L_k) delta = r with the
                         lower triangle L_k of its own matrix in lexicographic order (x fastest,
                         dofs of a node in order); the copies of an interface dof then take the
                         average of their corrections;
                         3: as 2, with the post-smoothing sweeps backward (upper triangle,
                         reverse order);
                         4: symmetric Gauss-Seidel: each of the cheb_degree iterations, before
                         and after the coarse correction, is a forward sweep then a backward sweep.
                         2, 3 and 4 need precision RMG_PREC_FP64 and cannot produce training
                         errors for the interpolation network (rmg_mlp_add_samples) */
  double jacobi_omega; /* damping omega of the Jacobi and Gauss-Seidel smoothers (default 0.6) */
  int symmetric;      /* 1 (default): on scalar 27-point 3D levels whose operator is symmetric to
                         rounding, the 2.5D kernel keeps only the upper half of each stencil
                         (14 coefficients per node) and reads a lower coupling from the
                         neighbour's record; 0: always the full 27-point stencil */
  int batched;        /* 1 (default): each stencil operation is one launch over the block or tile
                         list of all regions; 0: one node-parallel launch per region (the
                         region-by-region baseline of the batched form; no tiles, no autotuning) */
  int judge_cycles;   /* learned interpolation only: > 0 measures the convergence factor of
                         this many stationary V-cycles (rmg_convergence_factor) with the learned
                         and with the geometric interpolation at setup and keeps the better
                         hierarchy (default 10); 0 keeps the learned one whenever it is valid */
  int hybrid;         /* 1: the hierarchy of the structured/unstructured mesh hybrid (Table 5):
                         piecewise-constant transfers over aggregates, structured regions
                         aggregating every node to its nearest rate-3 coarse point, unstructured
                         regions (rmg_set_region_kinds) by staged plain aggregation whose first
                         stage aggregates their interface nodes by the structured rule; every
                         level's region matrices are sparse (Galerkin product per region); scalar
                         FP64 problems, smoother 1, 2 or 4.  0 (default): geometric linear
                         transfers on stencil levels */
  int cycle_gamma;    /* coarse cycles per visit of a level: 1 (default) V-cycle, 2 W-cycle
                         (hybrid hierarchy only) */
  int coarse_amg;     /* coarse solver of the region hierarchy (Section 3.5): 0 (default) the
                         dense inverse of Abar (at most 20,000 composite dofs); 1: one V-cycle of
                         smoothed-aggregation AMG on Abar (geometric region hierarchy; scalar
                         problems and 3D elasticity): staged plain aggregation of the free rows
                         (roots, joins, leftovers) -- for elasticity of the free nodes, on the graph
                         of blocks with Frobenius norm > 1e-12 sqrt(||A_II|| ||A_JJ||) --, the
                         tentative prolongator (a 1 per aggregated row; for elasticity a thin QR
                         per aggregate of the six rigid-body modes at the coarsest nodes' positions
                         on the finest lattice, the coarse nodes being the aggregates with six dofs
                         each), P = (I - omega D^-1 A) T with omega = 4 / (3 rho) and rho the
                         Gershgorin bound max_i sum_j |a_ij| / a_ii, coarse operators P^T A P, the
                         degree-cheb_degree Chebyshev smoother on [rho / eig_ratio, rho] before and
                         after each coarse correction, and a dense inverse on the first AMG level
                         with at most amg_coarse_size rows */
  int amg_coarse_size; /* rows of the directly solved AMG level, in [1, 20000] (default 2000) */
  int region_table;   /* 1 (default): on symmetric 27-point FP64 levels of the FP64 V-cycle (scalar
                         levels on 768-thread 2.5D tiles or node blocks, 3-dof levels on node
                         blocks; the FP32 V-cycle always streams), setup sorts every region's nodes
                         into 125 classes (per axis: the two low layers, the inside, the two high
                         layers) and compares each node's 27 couplings (its stored upper ones and
                         its neighbours' mirrored ones; 3 x 3 blocks on 3-dof levels) with those of
                         its class's first node; where all are equal bit for bit (a region whose
                         operator is the same everywhere inside, as the structured regions of the
                         Q1 Laplacian, the per-region diffusion and elasticity problems give), the
                         region's couplings come from its 125 x 27 class table (whole-row tiles on
                         tiled levels, each node's class row on node blocks) instead of being
                         streamed from memory.  Results are bit for bit those of 0, which always
                         streams them */
  int tile_planes;    /* planes per 2.5D tile: 0 (default) chooses (41 on FP64 levels that keep at
                         least 1024 such tiles, else 21); 21 or 41 forces that depth on every
                         tiled level, so that a problem small enough for the oracle runs the launch
                         shape of the large ones (used by the parity tests) */
  int galerkin_generic; /* 0 (default): on scalar 3D levels with the geometric interpolation the
                         per-region Galerkin product P^T A P runs as three one-axis products (P is
                         the tensor product of one rate-3 interpolation per axis); 1: the generic
                         product of every coarse node over its 5 x 5 x 5 fine window (also used for
                         2D, elasticity and stored weights) */
  double bf16_tolerance; /* RMG_PREC_FP32_BF16_AUTO: relative rise of the measured convergence
                         factor over the all-FP32 one that a BF16 level may cause (default 0.05) */
  int bf16_cycles;    /* RMG_PREC_FP32_BF16_AUTO: stationary V-cycles per measured factor, in
                         [1, 1000] (default 10) */
  int block_diag;     /* D~ of a 3-dof system (Section 3.2 smoother setup): 0 (default) the point
                         diagonal; 1 the 3 x 3 nodal blocks of [[A]]'s centre stencil summed over
                         each node's copies, inverted per node and applied wherever D~^-1 enters
                         (power method, Chebyshev and Jacobi smoothers, FP64 and low-precision
                         V-cycles).  Needs ndof 3 and smoother 0 or 1 (RMG_ERR_ARG otherwise);
                         RMG_ERR_NUMERIC if a summed block is not positive definite */
  int transfer_rows;  /* geometric restriction and prolongation (Section 3.3): 1 (default) by rows and
                         planes (a block owns whole rows of a region and walks its planes, staging
                         the values it reads in LDS) wherever every region's rows fit a block
                         (coarse and fine rows of at most 256 nodes); 0 one thread per node.  Both
                         give the same results bit for bit */
} rmg_options;

/* Filled by rmg_options_default with the values above. */
void rmg_options_default(rmg_options* opt);

typedef struct {
  int iterations;        /* number of A p products */
  int converged;         /* 1 if ||r||/||b|| <= rtol */
  double relres;         /* recursive relative residual at exit */
  double true_relres;    /* ||b - A x|| / ||b|| recomputed at exit */
  double solve_ms;       /* wall time of the CG loop on the stream (HIP events) */
  double* history;       /* caller-owned host array or NULL: relres per iteration, [0] = 1 */
  int history_cap;       /* capacity of history */
  int history_len;       /* entries written */
  double setup_ms;       /* host wall time of the last rmg_setup_hierarchy (stream synchronised) */
  double level_ms[12];   /* with rmg_profile on and no graph replay: device time of each region
                            level's share of the preconditioner over this solve (HIP events around
                            its smoothing, residual and transfers; on the last level the coarse
                            solve, the AMG V-cycle included); 0 otherwise and beyond nlevels (and
                            for the hybrid hierarchy) */
} rmg_solve_info;

/* Device memory provider for a handle (optional).  alloc(bytes, ctx) returns at least `bytes` of
   device memory on the handle's device usable on its stream, or NULL; free(ptr, ctx) takes back a
   pointer alloc returned.  Both are called only from inside this library's entry points for that
   handle (never from a kernel or a stream callback); every buffer is returned to the provider that
   gave it.  The caller keeps the functions and ctx valid until rmg_destroy of the handle returns. */
typedef struct rmg_allocator {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} rmg_allocator;

/* Create a handle on HIP device `device`; all work goes to `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *out owned by the library.  `alloc` (may be
 * NULL: hipMalloc/hipFree) provides every device buffer the handle's entry points allocate; the
 * struct is copied. */
rmg_status rmg_create(rmg_handle** out, int device, void* hip_stream, const rmg_allocator* alloc);

/* Release all device memory of the handle.  NULL is accepted. */
rmg_status rmg_destroy(rmg_handle* h);

/* Last error message of the calling thread ("" if none). */
const char* rmg_last_error(void);

/* Region description supplied by the application (Section 4): for each
 * region its node extent and the composite coordinates of its first node.
 * extent, origin: host int32 arrays [nreg][dim].  dim 2 or 3, ndof 1 or 3
 * (3 only with dim 3).  dirichlet_mask bit 2d / 2d+1 marks the low / high
 * domain face along axis d as homogeneous Dirichlet.  The boxes must tile the
 * bounding box of the domain, overlapping only on shared node planes
 * (RMG_ERR_SHAPE otherwise).  Discards any previous regions and hierarchy. */
rmg_status rmg_build_regions(rmg_handle* h, int dim, int ndof, int nreg, const int32_t* extent,
                             const int32_t* origin, uint32_t dirichlet_mask);

/* Finest-level regional matrix A^(k) of one region as a stencil
 * (block diagonal region matrix, Section 3.1).  coef is FP64, structure of
 * arrays: coef[s * nnodes + i] is the coupling of region node i to its
 * neighbour at stencil offset s, i x-fastest over the region's nnodes.
 * Offsets: npts 27 (3D): s = (dz+1)*9 + (dy+1)*3 + (dx+1); npts 9 (2D):
 * s = (dy+1)*3 + (dx+1); npts 5 (2D): (0,-1), (-1,0), (0,0), (1,0), (0,1).
 * Scalar problems only.  Couplings that point outside the region box are
 * ignored (set to zero).  on_device: coef is a device (1) or host (0) pointer.
 * RMG_ERR_NUMERIC on NaN/Inf. */
rmg_status rmg_set_region_stencil(rmg_handle* h, int region, int npts, const double* coef, int on_device);

/* Non-invasive construction (Section 4): split an assembled composite operator,
 * given as a composite stencil, into region matrices.  coef: FP64 structure of
 * arrays [npts][n_composite nodes] (x fastest, offsets as in
 * rmg_set_region_stencil); couplings that leave the domain must be zero.  An
 * off-diagonal entry is divided by the number of regions containing both of
 * its nodes; each region's diagonal is the row sum of A divided by the node's
 * multiplicity minus that region's split off-diagonals (zero row sums are
 * kept).  Needs a tensor-product region layout (RMG_ERR_SHAPE otherwise).
 * on_device: coef is a device (1) or host (0) pointer. */
rmg_status rmg_set_composite_stencil(rmg_handle* h, int npts, const double* coef, int on_device);

/* The same non-invasive split from an assembled composite matrix in CSR form
 * (Section 4: the application hands over its assembled matrix and the region
 * layout).  Rows and columns are composite nodes in x-fastest order
 * (n_composite rows); rowptr int64 [n+1] (0 .. nnz, non-decreasing, checked on
 * the host), colind int32 [nnz], values FP64 [nnz]; duplicate entries add up.
 * Every entry must couple nodes within the npts neighbourhood (RMG_ERR_SHAPE
 * otherwise; out-of-range columns RMG_ERR_ARG, NaN/Inf RMG_ERR_NUMERIC).
 * on_device: the three arrays are device (1) or host (0) pointers. */
rmg_status rmg_set_composite_csr(rmg_handle* h, int npts, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                                 const double* values, int on_device);

/* Assemble every region's matrix on the device from Q1 hexahedral elements of
 * side h inside that region (one admissible split of A, Section 3.1), with
 * symmetric elimination of Dirichlet nodes (identity rows split 1/mult).
 * elem_coef: device FP64 array over the composite element grid
 * ((nx-1)(ny-1)(nz-1), x fastest) for RMG_PDE_DIFFUSION, else NULL.
 * youngs: host FP64 [nreg] for RMG_PDE_ELASTICITY (with Poisson ratio nu), else NULL. */
rmg_status rmg_assemble_q1(rmg_handle* h, int pde, double hsize, const double* elem_coef,
                           const double* youngs, double nu);

/* Build the regional hierarchy (Section 3.2): composite diagonal
 * D~ = Psi^T Psi diag([[A]]), lambda_max(D~^-1 A) by power iteration, rate-3
 * linear interpolation with interface-replicated rows, per-region Galerkin
 * products [[Abar]] = R^(r) [[A]] P^(r) on the device, and on the last level the
 * composite operator Abar = Psi-bar [[Abar]] Psi-bar^T and its inverse.
 * Coarsening: along each axis a region keeps every third node from its first
 * one and its last node ((e + 1) / 3 + 1 of e nodes), interpolating linearly
 * over the actual spacing, so any extent >= 2 coarsens; the composite coarse
 * lattice is the union of the regions' coarse points.  RMG_ERR_SHAPE if two
 * regions' coarse points disagree on a shared interface (possible only when the
 * boxes do not form a tensor-product layout), or, with stored interpolation
 * weights, if some region extent-1 or origin is not divisible by 3^(nlevels-1);
 * the hybrid hierarchy (opt->hybrid) needs every aggregated level's composite
 * extent - 1 divisible by 3 and at least 6.  RMG_ERR_NUMERIC if a diagonal is not positive or the coarse
 * matrix is singular. */
rmg_status rmg_setup_hierarchy(rmg_handle* h, const rmg_options* opt);

/* z = V(r): one regional V-cycle with zero initial guess (device FP64 vectors in `layout`), the
 * cycle of Section 3.3 (the regional V-cycle figure and the regional residual and restriction
 * formulas): degree-K Chebyshev pre-smoothing (Algorithm 2), residual b - Psi^T Psi [[A]] u,
 * restriction of the residual divided by multiplicity with the coarse interface sum, the coarse
 * level's cycle (the direct solve of Section 3.5 at the bottom), interpolation added without an
 * interface sum, post-smoothing.  r and z may not alias.  Asynchronous on the stream. */
rmg_status rmg_apply_vcycle(rmg_handle* h, const double* r, double* z, int layout);

/* Preconditioned CG for A x = b (device FP64 vectors in `layout`; x holds x0
 * on entry, the solution on exit) with one rmg_apply_vcycle per iteration as the
 * preconditioner: the paper's experiments run the V-cycle as a solver and note that
 * applications use it inside a Krylov method (Section 6.2); every product is the
 * regional matrix-vector product of the Lemma on Psi [[A]] Psi^T (Section 3.1) and every inner
 * product counts each composite dof once.  Stops when the recursive residual satisfies
 * ||r_k|| / ||b|| <= rtol and the true residual ||b - A x_k|| / ||b|| does too (otherwise
 * CG continues from the true residual), or after maxit iterations (RMG_ERR_NOT_CONVERGED,
 * x = last iterate); RMG_ERR_BREAKDOWN if (p, A p) or (r, z) is not positive.  info may be
 * NULL.  Synchronises. */
rmg_status rmg_solve(rmg_handle* h, const double* b, double* x, int layout, double rtol, int maxit,
                     rmg_solve_info* info);

/* Multigrid as a solver (the paper's experiments, Section 6): x <- x + V(b - A x)
 * until ||b - A x|| / ||b|| <= rtol or maxit cycles (RMG_ERR_NOT_CONVERGED, x =
 * last iterate).  Vectors and info as in rmg_solve (iterations = cycles, history
 * = relative residual after each cycle, [0] = ||b - A x0|| / ||b||).  Synchronises. */
rmg_status rmg_mg_solve(rmg_handle* h, const double* b, double* x, int layout, double rtol, int maxit,
                        rmg_solve_info* info);

/* ---- conversions and per-step entry points (used by parity tests) ---- */

/* [[v]] = Psi^T v on level `level` (device FP64). */
rmg_status rmg_to_regional(rmg_handle* h, int level, const double* comp, double* reg);
/* v = owner copy of each composite dof (average = 0) or the average of the
 * copies (average = 1, (Psi Psi^T)^-1 Psi [[v]]). */
rmg_status rmg_to_composite(rmg_handle* h, int level, const double* reg, double* comp, int average);
/* z = Psi^T Psi [[A]] v on level `level` (RegMatVec). */
rmg_status rmg_regional_matvec(rmg_handle* h, int level, const double* v, double* z);
/* w = Psi^T Psi v (interface summation). */
rmg_status rmg_interface_sum(rmg_handle* h, int level, const double* v, double* w);
/* Coarse w = Psi-bar^T Psi-bar R^(r) [[Psi Psi^T]]^-1 r from level to level+1 (Section 3.3). */
rmg_status rmg_restrict(rmg_handle* h, int level, const double* r, double* w);
/* Fine u += P^(r) ubar from level+1 to level (Section 3.3). */
rmg_status rmg_prolongate_add(rmg_handle* h, int level, const double* ubar, double* u);
/* u = S(b): one degree-K Chebyshev application with zero initial guess.  b must be
 * consistent (every copy of a composite dof holds the same value), as the cycle's
 * right-hand sides are: the update of a shared dof is computed once, from the
 * copy in the lowest region, and written to every copy. */
rmg_status rmg_smooth(rmg_handle* h, int level, const double* b, double* u);

/* Level data.  n_regional / n_composite count dofs. */
rmg_status rmg_level_info(rmg_handle* h, int level, int64_t* n_regional, int64_t* n_composite,
                          int* npts, double* lambda_max);
/* How level `level`'s stencil operations run: kernel 0 node-parallel, 1 2.5D
 * tiles (one block per tile), 2 2.5D tiles in a persistent grid, 3 node-parallel
 * with one launch per region; coefs = stencil coefficients streamed per node by
 * the FP64 operations (npts x ndof^2, or 14 for the stored upper half of a
 * symmetric 27-point stencil); coefs_lo = the same for the low-precision
 * V-cycle copy (0 when there is none).  Any output may be NULL. */
rmg_status rmg_level_kernel(rmg_handle* h, int level, int* kernel, int* coefs, int* coefs_lo);
/* Storage of level `level`'s stencil in the low-precision V-cycle (Section 3.4 smoother, the
 * mixed-precision variant): coef_type 0 FP64 (no low-precision copy: precision RMG_PREC_FP64, or the
 * coarsest level), 1 FP32, 2 BF16 off-diagonals with FP32 centre blocks.  With
 * RMG_PREC_FP32_BF16_AUTO, rho_fp32 is the convergence factor measured with every level in FP32
 * and rho_bf16 the factor measured with this level switched to BF16 (and the finer levels as
 * decided); -1 where the level was not tried.  Any output may be NULL. */
rmg_status rmg_level_precision(rmg_handle* h, int level, int* coef_type, double* rho_fp32, double* rho_bf16);
/* Kernel launches this library has issued in the process so far (every handle and trainer, every
 * thread; a replayed HIP graph counts once per captured launch when it was recorded, not when
 * replayed).  The difference around a call is that call's launch count. */
rmg_status rmg_kernel_launches(int64_t* count);
/* 2.5D tile shape of `level`: the number of tiles, threads per tile block and planes per tile
 * (all 0 where the level runs node-parallel kernels).  Any output may be NULL. */
rmg_status rmg_level_tiles(rmg_handle* h, int level, int* ntiles, int* threads, int* planes);
/* Tiles of the transfers between `level` and the next coarser one (rmg_options.transfer_rows): the
 * restriction's and the prolongation's blocks, 0 where they run one thread per node (and on the
 * coarsest level).  Any output may be NULL. */
rmg_status rmg_level_transfer_tiles(rmg_handle* h, int level, int* restriction_tiles, int* prolongation_tiles);
/* Regions of `level` whose couplings the 2.5D kernels take from the region's class table
 * (rmg_options.region_table); 0 where no table was built.  Output may be NULL. */
rmg_status rmg_level_table_regions(rmg_handle* h, int level, int* nregions);
/* Copy region `region`'s stencil on `level` to host memory in the layout of
 * rmg_set_region_stencil (npts 27 in 3D, 9 in 2D, all levels). */
rmg_status rmg_get_level_stencil(rmg_handle* h, int level, int region, double* host_out);
/* Dense composite operator of the coarsest level (host, n_composite^2, row-major). */
rmg_status rmg_get_coarse_matrix(rmg_handle* h, double* host_out);

/* ---- structured/unstructured mesh hybrid (the paper's hybrid section, Table 5) ---- */
/* Kind of every finest-level region for rmg_options.hybrid = 1: kinds[k] = 0 structured (default),
   1 unstructured.  Host array of nreg entries; takes effect at the next rmg_setup_hierarchy. */
rmg_status rmg_set_region_kinds(rmg_handle* h, const int32_t* kinds);
/* Sizes of level `level` of the hybrid hierarchy: regional rows, composite nodes, stored nonzeros
   of the region matrices.  RMG_ERR_NOT_SETUP without a hybrid hierarchy. */
rmg_status rmg_hybrid_level_info(rmg_handle* h, int level, int64_t* n_regional, int64_t* n_composite,
                                 int64_t* nnz);
/* Aggregate of every regional row of level `level` (< nlevels - 1): the regional row of its coarse
   node on level + 1, or -1 for a Dirichlet row.  Host array of n_regional entries. */
rmg_status rmg_hybrid_aggregates(rmg_handle* h, int level, int32_t* agg);
/* Composite node of every regional row of level `level` (finest level: the composite lattice
   index; coarser levels: numbered by first sight, regions in order).  Host array of n_regional. */
rmg_status rmg_hybrid_composite_ids(rmg_handle* h, int level, int64_t* comp);
/* The region matrices of level `level` as one block-diagonal CSR matrix over the regional rows
   (host arrays: rowptr n_regional + 1, colind and values nnz; columns ascending per row). */
rmg_status rmg_hybrid_matrix(rmg_handle* h, int level, int64_t* rowptr, int32_t* colind, double* values);

/* Levels of the AMG coarse solver of the current hierarchy (coarse_amg = 1), 0 without one.  Level
 * 0 is the coarsest region level's composite operator Abar (rows in composite node order). */
rmg_status rmg_amg_levels(rmg_handle* h, int* nlevels);

/* Rows of AMG level `level`, nonzeros of its matrix, nonzeros of its prolongator to the next level
 * (0 on the directly solved last level).  RMG_ERR_ARG for a level out of range. */
rmg_status rmg_amg_level_info(rmg_handle* h, int level, int64_t* n, int64_t* nnz_a, int64_t* nnz_p);

/* The level's matrix (which = 0, n x n) or prolongator to the next level (which = 1, n x n_next)
 * in CSR with ascending columns, copied into caller host arrays sized by rmg_amg_level_info
 * (rowptr: n + 1 entries). */
rmg_status rmg_amg_matrix(rmg_handle* h, int level, int which, int64_t* rowptr, int32_t* colind, double* values);

/* ---- kernel timing (for roofline measurements) ---- */

/* Timed kernels: 0 = finest-level fused Chebyshev step (stencil product,
 * residual, direction and iterate update; excludes the first step of a
 * smoothing pass), 1 = finest-level CG product q = A p with its (p, q) partial
 * sums.  Only the stencil kernel is timed, not the interface-group kernel. */
#define RMG_TIMED_CHEB 0
#define RMG_TIMED_CG_MATVEC 1

/* Enable (1) or disable (0) HIP-event timing of the kernels above and reset
 * the counters.  Timing adds an event pair per timed launch. */
rmg_status rmg_profile(rmg_handle* h, int enable);
/* Text of the autotuner's choices (one line per level: level, mode, depth, grid, time), copied
 * into buf (NUL-terminated, truncated to cap bytes). */
rmg_status rmg_tune_report(rmg_handle* h, char* buf, int cap);
/* Launch count and summed duration (ms) of a timed kernel since the last reset. */
rmg_status rmg_profile_query(rmg_handle* h, int kernel, int64_t* launches, double* total_ms);

/* ---- stored and learned interpolation (finest level -> level 1) ----
 *
 * Operator-dependent interpolation in the spirit of the black-box multigrid
 * transfers that Section 3.2 names as needing interface averaging: the rows of
 * P for shared interface nodes must be identical in every region holding a
 * copy (the interpolation condition behind the Theorem on per-region Galerkin
 * products).  Scalar 3D problems only.
 *
 * Stored weights: 8 FP64 values per regional node of the finest level
 * ([n_regional][8]), for the corners (ix, iy, iz) of the node's canonical
 * coarse cell c = min(x / 3, coarse extent - 2) per axis (region-local
 * coordinates), slot ix + 2 iy + 4 iz.  Valid weights (checked at setup):
 * finite; non-zero only towards corners on the node's own coarse face, edge or
 * point; zero from a Dirichlet coarse node to a free fine node; summing to one
 * unless such a Dirichlet weight was dropped; equal on all copies of a shared
 * node (per composite coarse node). */

/* Weight-validity flags (rmg_prolongator_info) and the judge's verdict. */
#define RMG_PW_NONFINITE 1
#define RMG_PW_SUPPORT 2
#define RMG_PW_DIRICHLET 4
#define RMG_PW_COPIES 8
#define RMG_PW_SUM 16
#define RMG_PW_JUDGED_WORSE 32

/* Kinds of finest-level interpolation. */
#define RMG_P_GEOMETRIC 0
#define RMG_P_STORED 1
#define RMG_P_LEARNED 2

/* Caller weights for the next rmg_setup_hierarchy (copied; w: host or device
 * FP64 [n_regional][8] as above, on_device selects).  NULL restores the
 * geometric interpolation.  Invalid weights make the setup fail with
 * RMG_ERR_ARG.  Needs regions of a scalar 3D problem; rmg_build_regions
 * clears the weights. */
rmg_status rmg_set_prolongator_weights(rmg_handle* h, const double* w, int on_device);

/* MLP of the learned interpolation: 27 inputs (log of the coefficients of a
 * coarse cell's 3 x 3 x 3 fine elements, x fastest, minus their mean), two
 * hidden layers of 64 with ReLU, 208 outputs: one logit per (fine node,
 * admissible coarse corner) for the cell's 56 non-corner nodes in x-fastest
 * order over the 4 x 4 x 4 cell nodes (corners of a node in slot order), a
 * softmax per node giving its weights.  FP32 parameters, flat in the order
 * W1 [64][27], b1 [64], W2 [64][64], b2 [64], W3 [208][64], b3 [208]. */
#define RMG_MLP_NIN 27
#define RMG_MLP_NHIDDEN 64
#define RMG_MLP_NOUT 208
#define RMG_MLP_NPARAM 19472

/* Use the MLP with parameters theta (host FP32 [RMG_MLP_NPARAM], copied) for
 * the next rmg_setup_hierarchy: the setup evaluates it on every coarse cell of
 * the finest level, averages the predictions of all cells containing a fine
 * node, injects coarse points and drops Dirichlet weights as the geometric
 * interpolation does.  Weights that fail the validity rules (e.g. NaN
 * parameters) fall back to the geometric interpolation, as does a learned
 * hierarchy that the judge (rmg_options.judge_cycles) finds slower to
 * converge.  Features come from the element coefficients given to
 * rmg_assemble_q1 (zero for RMG_PDE_LAPLACE).  NULL restores geometric. */
rmg_status rmg_set_learned_prolongator(rmg_handle* h, const float* theta);

/* Interpolation of the current hierarchy: kind (RMG_P_*), the validity flags
 * and judge verdict that caused a fallback (0 if none), and the convergence
 * factors measured by the judge (-1 when not measured).  Any output may be NULL. */
rmg_status rmg_prolongator_info(rmg_handle* h, int* kind, int* flags, double* rho_learned, double* rho_geometric);

/* Stored weights of the current hierarchy's finest level (host FP64
 * [n_regional][8]); RMG_ERR_ARG when it interpolates geometrically. */
rmg_status rmg_get_prolongator_weights(rmg_handle* h, double* host_out);

/* Convergence factor of the preconditioner used as a stationary iteration on
 * A x = 0: x0 from the counter-based generator (stream 63 of the hierarchy's
 * seed, zero on Dirichlet dofs), x <- x + V(-A x) for `cycles` cycles,
 * rho = (||r_cycles|| / ||r_0||)^(1/cycles) in the composite 2-norm.  Synchronises. */
rmg_status rmg_convergence_factor(rmg_handle* h, int cycles, double* rho);

/* rmg_convergence_factor for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same computation and
 * result, with its four work vectors (the zero right-hand side, iterate, residual and correction)
 * in a fixed 32 MiB array per GPU instead of memory allocated per call, so it calls neither
 * hipMalloc nor the handle's allocator.  The hierarchy's own buffers, made by
 * rmg_setup_hierarchy, are used as by rmg_convergence_factor.  RMG_ERR_ARG when the finest level
 * has more than 1,048,576 regional dofs (4 x 8 bytes each must fit in the array).  Every call on
 * a GPU shares that GPU's array and leaves its contents behind (each call rewrites all it
 * reads), so calls that overlap on one GPU (several threads, or handles on different streams)
 * race.  Synchronises. */
rmg_status rmg_convergence_factor_noalloc(rmg_handle* h, int cycles, double* rho);

/* ---- MLP training on the device ----
 * Training data are pairs (X, E) per coarse cell: X the 27 features above and
 * E the values of a smooth error on the cell's 4 x 4 x 4 fine nodes (x
 * fastest).  Loss per pair: sum over the cell's nodes of (e_f - sum_c w_fc
 * e_c)^2 / sum_f e_f^2, with e_c the corner values; the training loss is the
 * mean over pairs.  Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8). */
typedef struct rmg_mlp rmg_mlp;

/* Create a trainer on HIP device `device`, work ordered on `hip_stream`.
 * Parameters start at zero; set them with rmg_mlp_set_params. */
rmg_status rmg_mlp_create(rmg_mlp** out, int device, void* hip_stream);
rmg_status rmg_mlp_destroy(rmg_mlp* m);
/* Initial parameters: hidden weights uniform in +-sqrt(6 / fan_in) and output
 * weights in +-out_scale sqrt(6 / 64), drawn from the SplitMix64 counter
 * generator (stream 96 of `seed`, seed < 2^16); zero hidden biases; output
 * biases log(w) of the trilinear weights w, so that small output weights start
 * every node at the geometric interpolation.  Resets Adam's state; theta_out
 * (host [RMG_MLP_NPARAM] or NULL) receives the parameters. */
rmg_status rmg_mlp_init_params(rmg_mlp* m, uint64_t seed, double out_scale, float* theta_out);
/* Training loss (default RMG_MLP_LOSS_L2, as above).  RMG_MLP_LOSS_ENERGY
 * measures the interpolation error delta (zero at the cell corners) in the
 * energy norm of the cell's local operator: delta^T A_cell delta / (cbar
 * sum_f e_f^2) with A_cell = sum over the 27 elements of exp(X_e) K_Q1 (unit
 * cube Laplacian) and cbar the mean of exp(X_e). */
#define RMG_MLP_LOSS_L2 0
#define RMG_MLP_LOSS_ENERGY 1
rmg_status rmg_mlp_set_loss(rmg_mlp* m, int kind);
/* Parameters (host FP32 [RMG_MLP_NPARAM]); setting them resets Adam's state. */
rmg_status rmg_mlp_set_params(rmg_mlp* m, const float* theta);
rmg_status rmg_mlp_get_params(rmg_mlp* m, float* theta);
/* Append n pairs: X [n][27], E [n][64] FP32 (host or device per on_device). */
rmg_status rmg_mlp_add_data(rmg_mlp* m, int64_t n, const float* X, const float* E, int on_device);
/* Append nsamples x (coarse cells of the finest level) pairs generated from a
 * set-up scalar 3D hierarchy: for each sample s the error starts from the
 * counter-based generator (stream 32 + s of `seed`, zero on Dirichlet nodes)
 * and is smoothed by `sweeps` degree-K Chebyshev applications to A e = 0;
 * cells are taken region by region, x fastest.  Synchronises h's stream. */
rmg_status rmg_mlp_add_samples(rmg_mlp* m, rmg_handle* h, int nsamples, uint64_t seed, int sweeps);
rmg_status rmg_mlp_clear_data(rmg_mlp* m);
rmg_status rmg_mlp_num_data(rmg_mlp* m, int64_t* n);
/* Copy pairs [first, first + count) to host arrays (either may be NULL). */
rmg_status rmg_mlp_get_data(rmg_mlp* m, int64_t first, int64_t count, float* X, float* E);
/* Logits Z [n][208] of inputs X [n][27] (host or device per on_device, both alike). */
rmg_status rmg_mlp_forward(rmg_mlp* m, int64_t n, const float* X, float* Z, int on_device);
/* Loss over all pairs and its gradient (grad: host FP32 [RMG_MLP_NPARAM] or
 * NULL; the gradient also stays on the device for rmg_mlp_adam_step). */
rmg_status rmg_mlp_loss_grad(rmg_mlp* m, double* loss, float* grad);
/* One Adam step with learning rate lr, using `grad` (host FP32) or, if NULL,
 * the gradient of the last rmg_mlp_loss_grad / training step. */
rmg_status rmg_mlp_adam_step(rmg_mlp* m, const float* grad, double lr);
/* `steps` full-batch steps (loss and gradient, then Adam) on the device;
 * loss_history (host [steps] or NULL) receives the loss before each step. */
rmg_status rmg_mlp_train(rmg_mlp* m, int steps, double lr, double* loss_history);

#ifdef __cplusplus
}
#endif
#endif /* REGMG_H */
