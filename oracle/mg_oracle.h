/*
 * mg_oracle.h -- reference FP64 CPU multigrid for quadtree/octree block grids.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain checker that the GPU
 * library is compared against.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load it; the product path never does.  It shares no
 * code, header or table with the GPU library.
 *
 * Method: Teunissen & Keppens, "A geometric multigrid library for quadtree/octree AMR
 * grids coupled to MPI-AMRVAC" -- operators (Sec. 2.2, eq. poisson-2d and
 * poisson-2d-vcoeff), red-black Gauss-Seidel (Sec. 2.2), prolongation and
 * restriction (Sec. 2.3, eq. interp_2d / interp_3d), V-cycle and FMG with the FAS
 * coarse right-hand side (Sec. 2.4, eq. coarse-rhs and coarse-corr), grid
 * construction with added coarse levels (Sec. 2.5, table coarse-grid-example),
 * ghost cells and boundary conditions (Sec. 2.6).
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct og_tree og_tree;

/* Boundary kinds per face (-x,+x,-y,+y,-z,+z). */
enum { OG_DIRICHLET = 0, OG_NEUMANN = 1, OG_PERIODIC = 2 };

/* Refinement predicate.  level = refinement depth of the candidate block relative
 * to the base grid (0 = base), origin = global cell index of the block's first cell
 * on its level, bs = block size.  Non-zero = refine. */
typedef int (*og_refine_fn)(void *ud, int domain, int level, const int32_t *origin, int bs);

/* Create one tree (one domain).  Returns NULL on invalid arguments.  base_cells[d]
 * must be a multiple of bs; bs must be a power of two. */
og_tree *og_create(int dim, const int32_t *base_cells, const double *lo, const double *hi,
                   const int32_t *bc_kind, const double *bc_value, int bs, int max_refine,
                   og_refine_fn refine, void *ud, int domain_id, int variable_eps);
void og_destroy(og_tree *t);

void og_set_params(og_tree *t, int n_down, int n_up, int n_max, double abs_tol, double rel_tol);
/* Smoother: red-black Gauss-Seidel (default) or weighted Jacobi with weight omega. */
enum { OG_SMOOTH_GSRB = 0, OG_SMOOTH_JACOBI = 1 };
void og_set_smoother(og_tree *t, int kind, double omega);
/* Helmholtz term (Sec. 2.1 equation list): L phi = div(eps grad phi) - lambda phi. */
void og_set_lambda(og_tree *t, double lambda);
/* 2D axisymmetric operator (x = r >= 0, y = z): (1/r) d/dr (r dphi/dr) + d2phi/dz2
 * (with eps and lambda as above).  Returns -1 unless dim = 2 and lo[0] >= 0. */
int og_set_axisymmetric(og_tree *t, int on);

/* Structure queries. */
int og_num_levels(const og_tree *t);
int og_base_level(const og_tree *t);
/* Per level (coarsest = 0): bs, ncell[3], number of blocks. */
void og_level_info(const og_tree *t, int l, int32_t *bs, int32_t *ncell, int32_t *nblocks);
int64_t og_num_leaf_cells(const og_tree *t);
int og_num_leaf_blocks(const og_tree *t);
/* Leaf layout: n_leaf_cells rows of (level - base, I, J, K). */
void og_leaf_layout(const og_tree *t, int32_t *out);

/* Data on leaf cells in leaf order. */
void og_set_rhs(og_tree *t, const double *leaf_f);
void og_set_eps(og_tree *t, const double *leaf_eps);
void og_set_phi(og_tree *t, const double *leaf_phi);
void og_get_phi(const og_tree *t, double *leaf_phi);

/* Cycles. */
void og_vcycle(og_tree *t);
void og_fmg(og_tree *t);
/* Composite residual on leaves: max|r|/max|f| and ||r||_2/||f||_2 (volume weighted).
 * Side effect: parents hold the restriction of their children, ghosts refreshed. */
void og_residual_norm(og_tree *t, double *max_rel, double *l2_rel);
/* Composite residual r = f - L(phi) into leaf_r (same side effect). */
void og_leaf_residual(og_tree *t, double *leaf_r);
/* Composite operator L(phi) on leaves for the given leaf phi (overwrites phi state). */
void og_apply(og_tree *t, const double *leaf_phi, double *leaf_out);
/* Steps taken by the last coarsest-grid solve, and why it stopped: the tolerance was
 * met, n_max steps were taken, or the stall window ended it. */
int og_last_coarse_steps(const og_tree *t);
enum { OG_EXIT_TARGET = 0, OG_EXIT_NMAX = 1, OG_EXIT_STALL = 2 };
int og_last_coarse_exit(const og_tree *t);
/* Length of the coarsest solve's stall window (default 8 steps); 0 removes it, which
 * leaves the paper's rule alone (tolerance or n_max). */
void og_set_coarse_stall(og_tree *t, int steps);
/* Threads for the loops over the blocks of a level (OpenMP builds); returns the count
 * in use.  Results are identical for every thread count. */
int og_set_threads(int n);
/* The coarsest-grid solve alone, on the current v and f of level 0. */
void og_coarse_solve(og_tree *t);

/* Face-varying Dirichlet values (Sec. 2.6): the physical Dirichlet faces of every
 * block of every level, with their centres (3 doubles each, may be NULL) and face
 * indices (may be NULL); returns the count.  og_set_boundary_values takes one value
 * per listed face, used by the ghost 2a - phi_i in place of the face's constant. */
int64_t og_boundary_faces(const og_tree *t, double *centres, int32_t *faces);
void og_set_boundary_values(og_tree *t, const double *vals);

/* Adjoint pieces: dJ/deps per leaf cell given the state phi and the adjoint lambda.
 * Uniform trees only (all leaves on one level); returns -1 otherwise. */
int og_face_gradient(og_tree *t, const double *leaf_phi, const double *leaf_lambda,
                     double *leaf_dJ_deps);

/* Inspection for tests: padded (bs+2)^d copy of a field of block b on level l
 * (index within the level's creation order).  field: 0 v, 1 f, 2 vold, 3 r, 4 eps. */
int og_level_nblocks(const og_tree *t, int l);
void og_block_meta(const og_tree *t, int l, int ib, int32_t *origin, int32_t *has_children);
void og_block_field(const og_tree *t, int l, int ib, int field, double *out);
void og_set_block_field(og_tree *t, int l, int ib, int field, const double *in);
/* Operations on one level, exposed for the invariant tests. */
void og_fill_ghosts_level(og_tree *t, int l);
void og_restrict_all(og_tree *t);
/* v^h += P(v^H - v_old^H) on level l, then ghosts of level l. */
void og_correct_level(og_tree *t, int l);
/* n smoothing steps on level l (ghosts of the level must be current). */
void og_smooth_level(og_tree *t, int l, int n);

#ifdef __cplusplus
}
#endif
#endif
