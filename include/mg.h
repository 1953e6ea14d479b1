/*
 * mg.h -- C ABI of the MI355X multigrid library for quadtree/octree block grids.
 *
 * Solves div(eps grad phi) - lambda phi = f (the paper's eq. poisson, and its Helmholtz
 * form with lambda >= 0) on one or more independent
 * domains, each a quadtree (2D) or octree (3D) of bs^d-cell blocks, with the
 * second-order cell-centred operators of Sec. 2.2 (eq. poisson-2d, poisson-2d-vcoeff),
 * red-black Gauss-Seidel smoothing, the transfer operators of Sec. 2.3, and FAS
 * V-cycles / FMG cycles of Sec. 2.4.  Grid construction (added coarse levels, 2:1
 * balance) follows Sec. 2.5; ghost cells and boundary conditions Sec. 2.6.
 *
 * Conventions
 *  - Every call returns an mg_status; nothing throws across the ABI.  The text of
 *    the last error of a tree is available from mg_last_error().
 *  - Ownership: the caller owns every array it passes and the device store it binds
 *    (one allocation of mg_tree_storage_bytes() bytes, 256-byte aligned); the library
 *    owns the tree's host metadata, never allocates device memory for data, and at
 *    bind creates one non-blocking stream (to capture HIP graphs) and a small pinned
 *    host buffer (residual norms).
 *  - Leaf order: domain, then refinement level (coarse to fine), then Morton order of
 *    the block coordinates on that level, then cells with x fastest (then y, then z).
 *  - Device work is asynchronous on the stream given to mg_tree_bind().  Calls that
 *    return host values (mg_residual_norm, mg_domain_residual_norms, mg_solve, and
 *    mg_get_phi / mg_face_gradient with host pointers) synchronise that stream.
 *  - A tree is not thread safe; calls on one tree must not overlap.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_tree mg_tree;

typedef enum {
    MG_OK = 0,
    MG_ERR_ARG = -1,            /* invalid argument (sizes, kinds, null pointers) */
    MG_ERR_NOT_BALANCED = -2,   /* reserved: trees built here are balanced by construction */
    MG_ERR_DEVICE = -3,         /* a HIP call failed; mg_last_error() names it */
    MG_ERR_NOT_CONVERGED = -4,  /* mg_solve reached max_cycles above the tolerance */
    MG_ERR_OOM = -5,            /* the bound store is smaller than mg_tree_storage_bytes() */
    MG_ERR_STATE = -6,          /* call out of order (e.g. cycles before mg_tree_bind) */
    MG_ERR_NAN = -7             /* the residual norm is not finite */
} mg_status;

/* Boundary kinds (Sec. 2.6).  Dirichlet: phi = value on the face, ghost 2a - phi_i.
 * Neumann: d phi / d x_d = value (derivative along +x_d), ghost phi_i +/- h value on
 * the upper/lower face.  Periodic: copy across the domain (both faces of an axis). */
typedef enum { MG_BC_DIRICHLET = 0, MG_BC_NEUMANN = 1, MG_BC_PERIODIC = 2 } mg_bc_kind;

/* Faces in the order -x, +x, -y, +y, -z, +z. */
typedef struct {
    int32_t kind[6];
    double value[6];
} mg_bc;

/* One independent domain: a box [lo, hi] of base_cells cells (the unrefined grid,
 * Sec. 2.5); base_cells[d] must be a multiple of the block size. */
typedef struct {
    int32_t dim;            /* 2 or 3; every domain of a tree has the same dim */
    int32_t base_cells[3];
    double lo[3], hi[3];
    mg_bc bc;
} mg_domain;

/* Refinement predicate, called while the tree is built for every candidate leaf
 * block below the top level: level = refinement depth above the base grid
 * (0 = base), origin = global index of the block's first cell on that level,
 * bs = block size.  Non-zero refines the block.  The tree is the least 2:1 balanced
 * tree (across faces, edges and corners) that refines every block for which the
 * predicate holds, so the result does not depend on the calling order. */
typedef int (*mg_refine_fn)(void *user_data, int domain, int level, const int32_t *origin,
                            int bs);

enum { MG_FP64 = 0, MG_MIXED = 1 };
enum { MG_SMOOTH_GSRB = 0, MG_SMOOTH_JACOBI = 1 };

typedef struct {
    int32_t n_down;           /* smoothing steps before restriction (paper default 2) */
    int32_t n_up;             /* smoothing steps after the correction (default 2) */
    int32_t n_max_coarse;     /* max smoothing steps on the coarsest grid (1000) */
    double coarse_abs_tol;    /* absolute max-norm target on the coarsest grid (0) */
    double coarse_rel_tol;    /* relative reduction on the coarsest grid (1e-8) */
    int32_t precision;        /* MG_FP64, or MG_MIXED: FP32 cycles in FP64 refinement */
    int32_t variable_eps;     /* 0: eps = 1, constant-coefficient stencil; 1: eps field */
    int32_t ir_first_fmg;     /* mixed: the first refinement step runs an FP32 FMG cycle */
    int32_t ir_vcycles;       /* mixed: FP32 V-cycles per plain refinement step (>= 1;
                                 default 4: with a contraction of ~0.1 per cycle four
                                 cycles (~1e-4) stay above the FP32 accuracy of the
                                 correction, and each step costs one FP64 residual and one
                                 host check).
                                 mg_solve runs fewer in a step (at least one) when the
                                 largest per-cycle reduction of the steps before says that
                                 fewer reach rel_tol with a quarter cycle to spare.
                                 The FGMRES preconditioner is always one V-cycle. */
    int32_t graphs;           /* 1 (default): each cycle sequence (V-cycle, FMG cycle,
                                 refinement step, residual norm) is captured once as a
                                 HIP graph and replayed; 0: kernels launched one by one */
    int32_t krylov;           /* mixed only.  0 (default): the refinement steps are plain
                                 (phi += e, e from FP32 cycles).  m >= 1: mg_solve runs
                                 FGMRES(m) in FP64 on the correction equation with the FP32
                                 cycles as the (flexible) preconditioner, one FP64 residual
                                 and update per restart; needs (2m + 1) FP64 leaf vectors in
                                 the store.  For coefficients with large jumps, where the
                                 plain cycles stall.  At most 64. */
    int32_t smoother;         /* MG_SMOOTH_GSRB (default; Sec. 2.2 red-black Gauss-Seidel)
                                 or MG_SMOOTH_JACOBI (weighted Jacobi, the smoother of the
                                 paper's timing runs, Sec. 3.3); one Jacobi step counts as
                                 one smoothing step */
    double jacobi_weight;     /* Jacobi weight in (0, 1]; default 2/3 (not given in the
                                 paper) */
    double helmholtz_lambda;  /* lambda >= 0 of the Helmholtz form div(eps grad phi) -
                                 lambda phi = f (Sec. 2.1 equation list); default 0 */
    int32_t axisymmetric;     /* 1: 2D cylindrical form of Sec. 2.1, x is the radius r >= 0
                                 and y the axis z: (1/r) d/dr (eps r dphi/dr) + d/dz (eps
                                 dphi/dz) in finite-volume form, i.e. the two r-face
                                 weights of a cell are scaled by (face radius) / (cell-centre
                                 radius).  Needs dim 2, lo[0] >= 0 and non-periodic x faces
                                 in every domain (the face at r = 0 gets weight 0, so its
                                 boundary condition has no effect there).  Restriction stays
                                 the plain mean and norms keep Cartesian cell volumes.
                                 mg_face_gradient is not available.  Default 0. */
} mg_params;

/* Fills p with the paper's defaults (Sec. 2.4) and FP64 precision. */
int mg_default_params(mg_params *p);

/* Builds the tree(s) on the host.  block_size must be 4, 8 or 16; every domain's
 * base_cells must be multiples of it.  max_refine_levels >= 0 limits refinement
 * above the base grid.  Returns MG_ERR_ARG for invalid input (also for a domain that
 * does not meet the requirements of params->axisymmetric when that is set).
 * Singular problems: with helmholtz_lambda = 0 a domain without a Dirichlet face has
 * constants in the operator's null space.  A fully periodic domain is accepted (its
 * coarsest grid subtracts the mean of f, so the solution is defined up to a constant);
 * a domain whose faces are all Neumann, or Neumann and periodic, is rejected with
 * MG_ERR_ARG (balancing the boundary fluxes against f is not part of the method of
 * Sec. 2.6).  With helmholtz_lambda > 0 every combination of kinds is regular. */
int mg_tree_create(const mg_domain *domains, int n_domains, int block_size,
                   int max_refine_levels, mg_refine_fn refine, void *user_data,
                   const mg_params *params, mg_tree **out);
void mg_tree_destroy(mg_tree *t);

/* Bytes of device memory the tree needs (fields of every level, index tables,
 * staging and reduction scratch). */
int mg_tree_storage_bytes(const mg_tree *t, size_t *bytes);

/* Binds a caller-allocated device buffer of at least mg_tree_storage_bytes() bytes
 * (256-byte aligned) and the HIP stream (hipStream_t, may be NULL for the null
 * stream) all later work is queued on.  Uploads the tables and sets phi = 0, f = 0,
 * eps = 1.  May be called again to move the tree to another buffer (state is reset). */
int mg_tree_bind(mg_tree *t, void *device_store, size_t bytes, void *hip_stream);

/* Structure: number of leaf cells (all domains), per-domain counts, levels. */
int mg_num_leaf_cells(const mg_tree *t, int64_t *n);
int mg_domain_leaf_cells(const mg_tree *t, int64_t *n_per_domain);
int mg_num_levels(const mg_tree *t, int *n_levels);
/* n_leaf rows of (domain, level above base, I, J, K) in leaf order. */
int mg_leaf_layout(const mg_tree *t, int32_t *out);
/* Blocks per level (levels with block size bs, coarsest first) and per-level cell
 * counts; arrays of mg_num_levels() entries (tail levels of reduced block size are
 * reported with 0 blocks). */
int mg_level_blocks(const mg_tree *t, int32_t *n_blocks, int64_t *n_cells);

/* Leaf data in leaf order, FP64.  on_device != 0: pointer to device memory.  The
 * right-hand side and eps are inputs of later cycles; eps is restricted to every
 * coarser level by the mean of the children (mg_set_eps requires variable_eps).
 * mg_set_phi sets the initial guess (default 0) and makes parents the restriction
 * of their children. */
int mg_set_rhs(mg_tree *t, const double *leaf_f, int on_device);
int mg_set_eps(mg_tree *t, const double *leaf_eps, int on_device);
int mg_set_phi(mg_tree *t, const double *leaf_phi, int on_device);
int mg_get_phi(mg_tree *t, double *leaf_phi, int on_device);

/* The composite operator of Sec. 2.2 applied to a leaf array: leaf_out = L phi
 * (div(eps grad phi) - lambda phi with the tree's eps and boundary values, or zero
 * boundary values after mg_set_homogeneous_bc), evaluated as the residual is: parents
 * take the mean of their children, ghosts are filled coarse to fine, then the stencil
 * runs on the leaves.  leaf_phi and leaf_out are leaf arrays (host, or device with
 * on_device = 1; they must not overlap).  The tree's phi and f are unchanged; the
 * v_old field, which only carries values within a cycle, is used as scratch.
 * Asynchronous for device pointers; synchronises for host pointers. */
int mg_apply_operator(mg_tree *t, const double *leaf_phi, double *leaf_out, int on_device);

/* Dirichlet values that vary along a face (Sec. 2.6; e.g. the boundary values of the
 * analytic solution in the convergence test of Sec. 3.1).
 *
 * mg_boundary_faces lists the leaf-cell faces that lie on a physical Dirichlet face:
 * face direction by direction (-x, +x, -y, +y, -z, +z), within a direction the leaf
 * blocks in leaf order, within a block the bs^(d-1) cells of that face with the lower
 * in-plane axis fastest.  n_faces receives the count; leaf_cell (the leaf index of the
 * cell, may be NULL) and face (its face, 0..5, may be NULL) receive n_faces entries.
 *
 * mg_fold_dirichlet takes one value a per listed face, in that order (host, or device
 * with on_device = 1), and folds them into the current right-hand side: the leaf
 * equations with these Dirichlet ghosts (2a - phi_b at a boundary face) differ from
 * the equations with the tree's own ghosts by a constant per cell, f is shifted by it,
 * and the solve keeps the tree's own ghosts (value from mg_domain, normally 0) on every
 * level.  The shift is the composite operator applied to phi = 0 with the values in
 * the physical ghosts of the leaf blocks: eps_b 2a/h^2 for a boundary cell (h its
 * spacing across the face) and, where a coarse-fine face meets the boundary, the
 * change of the interpolated ghost through the coarse cell's boundary ghost.  The
 * solution then solves the leaf problem with the given face values exactly (they add
 * to the face's mg_domain value).  Call after mg_set_rhs (and mg_set_eps); folding
 * twice adds twice; mg_set_rhs restores a plain right-hand side.  Uses the staging
 * buffers and the v_old field as scratch (MG_ERR_ARG if 6 x blocks, plus the values
 * when they are on the host, exceed the leaf cells) and synchronises the stream. */
int mg_boundary_faces(const mg_tree *t, int64_t *n_faces, int64_t *leaf_cell, int32_t *face);
int mg_fold_dirichlet(mg_tree *t, const double *values, int on_device);

/* Treat every Dirichlet/Neumann value as 0 (on != 0) -- used for adjoint solves. */
int mg_set_homogeneous_bc(mg_tree *t, int on);

/* n V-cycles (Sec. 2.4) with the tree's precision: FP64 cycles, or in MG_MIXED one
 * FP64 refinement step of FP32 cycles per call unit.  Asynchronous. */
int mg_vcycle(mg_tree *t, int n_cycles);
/* n FMG cycles (Sec. 2.4, fig. mg-cycles).  Asynchronous. */
int mg_fmg(mg_tree *t, int n_cycles);

/* Composite residual over leaf cells, FP64: max|f - L phi| / max|f| and the
 * volume-weighted L2 ratio (eq. l2-norm-example); the worst domain is returned.
 * Side effect: parents hold the mean of their children.  Synchronises.
 * Returns MG_ERR_NAN if the residual is not finite. */
int mg_residual_norm(mg_tree *t, double *max_rel, double *l2_rel);
int mg_domain_residual_norms(mg_tree *t, double *max_rel, double *l2_rel);

/* For callers that cannot allocate or synchronise (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the composite residual of
 * mg_residual_norm, asynchronous on the bound stream, with no allocation of any kind.
 * d_norms (device memory, 4 x n_domains doubles) receives per domain max|r|,
 * sum vol r^2, max|f|, sum vol f^2 (the relative norms are max|r|/max|f| and
 * sqrt(sum vol r^2 / sum vol f^2)).  The per-block reduction partials live in a fixed
 * device array of the library (one per GPU, 2 MiB, held until the process ends),
 * which limits the tree to 65536 leaf blocks (MG_ERR_ARG beyond).  Every call on a GPU
 * shares that array: calls that overlap on one GPU (several streams, threads or
 * trees at once) race and must be ordered by the caller.  Same side effect as
 * mg_residual_norm on refined trees (parents take the mean of their children). */
int mg_residual_norms_static(mg_tree *t, double *d_norms);

/* Solve to max-norm relative residual <= rel_tol: optional FMG first, then V-cycles
 * (FP64), or FP64 iterative refinement around FP32 cycles (MG_MIXED), checking the
 * norm after every cycle / refinement step.  (FP64: cycles that could not reach rel_tol
 * even at twice the fastest reduction per cycle seen so far, in log terms, run without
 * a check; the cycles run and the result are the same, and mg_solve_stats lists the
 * checked cycles only.)  With MG_MIXED and params.krylov = m > 0
 * the refinement is FGMRES(m) (flexible GMRES, restarted every m steps or when its
 * residual estimate falls by 1e-6; the true FP64 residual is checked at each restart);
 * one FP32 preconditioning solve counts as a cycle.  cycles_done may be NULL.
 * The FP64 form with use_fmg_first runs its FMG cycle before the first norm check
 * (the solve is meant to start from a guess that is not yet converged; this saves a
 * residual evaluation); the mixed forms check first, since their first step needs the
 * residual anyway.  Without FMG the norm is checked before any cycle, so a solve whose
 * guess already meets rel_tol returns at once with 0 cycles.
 * Returns MG_ERR_NOT_CONVERGED if max_cycles is reached first. */
int mg_solve(mg_tree *t, double rel_tol, int max_cycles, int use_fmg_first, int *cycles_done);
/* Per-check record of the last mg_solve: relative residual and seconds since start. */
int mg_solve_stats(const mg_tree *t, int max_records, double *rel_residual, double *seconds,
                   int *n_records);

/* Gradient of a loss J with respect to eps, given the state phi (L phi = f) and the
 * adjoint lambda (L^T lambda = dJ/dphi), per leaf cell: interior faces contribute
 * h^-2 (2 eps_j^2 / (eps_i + eps_j)^2) (lambda_j - lambda_i)(phi_j - phi_i), boundary
 * faces -h^-2 lambda_i (phi_g - phi_i).  Trees without refinement only
 * (MG_ERR_ARG otherwise).  Overwrites the tree's phi with leaf_phi. */
int mg_face_gradient(mg_tree *t, const double *leaf_phi, const double *leaf_lambda,
                     double *leaf_dJ_deps, int on_device);

/* Elliptic divergence cleaning (Sec. 4.1, eq. poisson-divb and poisson-divb-cleaning):
 * a cell-centred field B is projected with B <- B - grad phi, where lap phi = div B.
 * leaf_B holds dim components, each a leaf array ([dim][n_leaf], component-major).
 * Trees without refinement, with eps = 1, lambda = 0 and the Cartesian form only
 * (MG_ERR_ARG otherwise).  The call sequence is mg_divb_rhs, a solve (mg_solve,
 * mg_fmg, mg_vcycle; phi from mg_set_phi or zero), mg_divb_project.
 *
 * mg_divb_rhs sets f = div B, each derivative by second-order (order 2, eq.
 * divb-central-diff) or fourth-order (order 4, eq. divb-4th-order) central
 * differences; across a same-level (or periodic) face the neighbour block's cells are
 * used, outside a physical face B repeats the boundary cell (both layers).  With a
 * fully periodic domain the solve subtracts the mean of f on the coarsest grid.
 *
 * mg_divb_project sets B_d -= d phi / d x_d by second-order central differences of
 * the current phi and its boundary ghosts, in place; with leaf_e (may be NULL) the
 * energy density is updated as e += (|B_new|^2 - |B_old|^2) / 2 (eq.
 * divb-pressure-fix), which keeps e - |B|^2 / 2 fixed.  Host arrays are staged one
 * component at a time and both calls then synchronise the stream. */
int mg_divb_rhs(mg_tree *t, const double *leaf_B, int order, int on_device);
int mg_divb_project(mg_tree *t, double *leaf_B, double *leaf_e, int on_device);

/* Free-space boundary conditions (Sec. 2.8; test problem of Sec. 3.2): phi -> 0 at
 * infinity for the Laplacian.  The current right-hand side (mg_set_rhs) is restricted
 * to the uniform level 2^coarsen leaf cells coarser (the mean of each coarse cell's
 * leaf cells); the free-space potential of that grid, each coarse cell a point charge
 * q = mean(f) h_c^3 at its centre, phi(x) = -(1/4 pi) sum q / |x - x_c|, is summed at
 * the coarse face centres of the six boundary planes (plus one ghost position beyond
 * each edge); the planes are interpolated linearly to the centres of the leaf faces.
 * These Dirichlet values a enter the right-hand side in place, f -= 2 a / h^2 for each
 * boundary face of a cell (the Dirichlet ghost 2a - phi_b of Sec. 2.6), so that a solve
 * with the tree's homogeneous Dirichlet faces solves the free-space problem.  Calling
 * it twice folds the values twice; mg_set_rhs restores a plain right-hand side.
 *
 * Requirements (MG_ERR_ARG otherwise): 3D, no refinement, eps = 1, lambda = 0,
 * every face of every domain Dirichlet with value 0, 1 <= coarsen with 2^coarsen <=
 * block size, at most 2048 coarse cells along x.  Domains are independent problems.
 * bvals (may be NULL; host memory, or device memory with on_device = 1) receives the
 * boundary values: domain by domain, face by face (-x, +x, -y, +y, -z, +z), each face
 * over its leaf cells with the lower in-plane axis fastest; mg_freespace_values gives
 * the count.  Uses the library's staging buffers as scratch and synchronises the
 * stream. */
int mg_freespace_bc(mg_tree *t, int coarsen, double *bvals, int on_device);
int mg_freespace_values(const mg_tree *t, int64_t *n_values);

/* Initial guess for a free-space solve (same requirements and coarsen as
 * mg_freespace_bc; call it before mg_freespace_bc, while f is the plain right-hand
 * side): sets phi on the leaves to the far-field potential -Q / (4 pi r) of the
 * coarse charges' total Q placed at their centroid, r at least one coarse spacing, or
 * to zero for a neutral source.  The paper starts the cycles from the uniform-grid
 * free-space solution; this cheaper guess serves the same purpose: near the boundary
 * it already matches the folded values, so FMG's coarse problems are consistent there
 * (from phi = 0 they see a boundary forcing that doubles per level).  Uses the staging
 * buffers and synchronises the stream.  Returns MG_ERR_STATE if boundary values were
 * folded into f (mg_freespace_bc, mg_fold_dirichlet) since the last mg_set_rhs. */
int mg_freespace_guess(mg_tree *t, int coarsen);

/* Kernel timing: when enabled, HIP events bracket every launch of the smoothing
 * kernel on the finest level (on the bound stream); mg_profile_read returns the
 * number of such launches and their total milliseconds since enabling. */
int mg_profile_enable(mg_tree *t, int on);
int mg_profile_read(mg_tree *t, int64_t *launches, double *total_ms, double *bytes_per_launch);

const char *mg_strerror(int status);
const char *mg_last_error(const mg_tree *t);

#ifdef __cplusplus
}
#endif
#endif
