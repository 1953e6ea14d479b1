/*
 * mg_oracle.c -- reference FP64 CPU multigrid for quadtree/octree block grids.
 *
 * TEST INFRASTRUCTURE ONLY (see mg_oracle.h).  Plain, slow and written to be checked
 * against the paper by eye: every routine names the passage it follows.  It is built
 * with -O2 -ffp-contract=off so that no fused multiply-add changes its rounding.
 * With OpenMP the loops over the blocks of one level run in parallel; each block writes
 * only its own cells (and ghosts), and cells of one colour do not read each other, so
 * the results do not depend on the thread count.  Sums over cells stay serial.
 *
 * Data layout: every block of every level stores each field as a (bs+2)^d array with
 * one layer of face ghost cells (Sec. 2.6: a single ghost layer, no diagonal ghosts).
 * Global cell indices on a level are counted from the domain's lower corner.
 */
#include "mg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_MAXLEV 40
#define STALL 0.999     /* coarsest solve: progress means a residual below STALL x the lowest so far */
#define STALL_STEPS 8   /* coarsest solve: steps in a row without progress before it stops */
#define NFIELD 5
enum { F_V = 0, F_F = 1, F_VOLD = 2, F_R = 3, F_EPS = 4 };

typedef struct {
    int lev;
    int org[3];      /* global index of local cell (0,0,0) on this level */
    int parent;      /* block index on level lev-1, or -1 */
    int child[8];    /* block indices on level lev+1, -1 if absent */
    int has_children;
    int tested;      /* refinement predicate already evaluated */
    double *fld[NFIELD];
    double *bval;    /* per-ghost Dirichlet values [face][a2][a1], or NULL: the face's constant */
} OBlock;

typedef struct {
    int bs;
    int ncell[3];
    int nblk[3];
    double h[3];
    int *map;        /* block index by block coordinates, -1 if absent */
    int *list;
    int n, cap;
} OLevel;

struct og_tree {
    int dim, domain_id, var_eps;
    int bc_kind[6];
    double bc_val[6];
    double lo[3], hi[3];
    int nlev, lbase, lmax_allowed;
    OLevel lev[OG_MAXLEV];
    OBlock *blk;
    int nblk, cap;
    int n_down, n_up, n_max;
    double abs_tol, rel_tol;
    int smoother;    /* OG_SMOOTH_GSRB or OG_SMOOTH_JACOBI */
    double omega;    /* Jacobi weight */
    double lambda;   /* Helmholtz term: L phi = div(eps grad phi) - lambda phi, lambda >= 0 */
    int axisym;      /* 2D axisymmetric: x is the radius r, y the axis z */
    int *leaf;       /* leaf blocks in canonical order */
    int nleaf;
    int last_coarse_steps;
    int last_coarse_exit;   /* OG_EXIT_TARGET, OG_EXIT_NMAX or OG_EXIT_STALL */
    int stall_steps;        /* coarsest solve: stall window length, 0 = none */
    og_refine_fn refine;
    void *ud;
};

/* ------------------------------------------------------------------ helpers */

static int ext(const og_tree *t, int l, int d) { return d < t->dim ? t->lev[l].bs : 1; }

static int npad(const og_tree *t, int l) {
    int n = t->lev[l].bs + 2;
    return t->dim == 3 ? n * n * n : n * n;
}

/* Index of local cell (i,j,k), each in [-1, bs], in a padded block array. */
static int pidx(const og_tree *t, int l, int i, int j, int k) {
    int n = t->lev[l].bs + 2;
    if (t->dim == 2) return (j + 1) * n + (i + 1);
    return ((k + 1) * n + (j + 1)) * n + (i + 1);
}

static int pidx3(const og_tree *t, int l, const int *c) { return pidx(t, l, c[0], c[1], c[2]); }

static int map_index(const OLevel *L, const int *b) {
    return (b[2] * L->nblk[1] + b[1]) * L->nblk[0] + b[0];
}

/* Block on level l with block coordinates b, or -1. */
static int block_at(const og_tree *t, int l, const int *b) {
    const OLevel *L = &t->lev[l];
    for (int d = 0; d < 3; d++)
        if (b[d] < 0 || b[d] >= L->nblk[d]) return -1;
    return L->map[map_index(L, b)];
}

/* Wraps global cell g on level l across periodic faces.  Returns 0 if g lies inside
 * the domain afterwards, otherwise the face index + 1 of the physical boundary. */
static int wrap_cell(const og_tree *t, int l, int *g) {
    for (int d = 0; d < t->dim; d++) {
        int n = t->lev[l].ncell[d];
        if (g[d] < 0 || g[d] >= n) {
            int face = 2 * d + (g[d] >= n);
            if (t->bc_kind[face] != OG_PERIODIC) return face + 1;
            g[d] = ((g[d] % n) + n) % n;
        }
    }
    return 0;
}

/* Block on level l containing global cell g (g already inside the domain). */
static int block_of_cell(const og_tree *t, int l, const int *g) {
    int b[3];
    for (int d = 0; d < 3; d++) b[d] = g[d] / ext(t, l, d);
    return block_at(t, l, b);
}

static int new_block(og_tree *t, int l, const int *b) {
    if (t->nblk == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 256;
        t->blk = (OBlock *)realloc(t->blk, (size_t)t->cap * sizeof(OBlock));
    }
    int id = t->nblk++;
    OBlock *B = &t->blk[id];
    memset(B, 0, sizeof(*B));
    B->lev = l;
    for (int d = 0; d < 3; d++) B->org[d] = b[d] * ext(t, l, d);
    B->parent = -1;
    for (int c = 0; c < 8; c++) B->child[c] = -1;
    for (int f = 0; f < NFIELD; f++) B->fld[f] = (double *)calloc((size_t)npad(t, l), sizeof(double));
    int np = npad(t, l);
    for (int i = 0; i < np; i++) B->fld[F_EPS][i] = 1.0;
    OLevel *L = &t->lev[l];
    L->map[map_index(L, b)] = id;
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->list = (int *)realloc(L->list, (size_t)L->cap * sizeof(int));
    }
    L->list[L->n++] = id;
    return id;
}

/* ------------------------------------------------------------- tree build */
/* Sec. 2.5 (added coarse grids, table coarse-grid-example) and the 2:1 balance
 * requirement stated there. */

static void refine_block(og_tree *t, int id);

/* Make sure a block exists on level l at block coordinates b (b inside the domain),
 * refining coarser blocks as needed. */
static void ensure_block(og_tree *t, int l, const int *b) {
    if (block_at(t, l, b) >= 0) return;
    int pb[3] = {b[0] / 2, b[1] / 2, t->dim == 3 ? b[2] / 2 : 0};
    ensure_block(t, l - 1, pb);
    refine_block(t, block_at(t, l - 1, pb));
}

/* Split block id into 2^d children.  First the 3^d - 1 same-level neighbours of the
 * block must exist, so that no child touches a block two levels coarser (2:1
 * balance across faces, edges and corners). */
static void refine_block(og_tree *t, int id) {
    if (t->blk[id].has_children) return;
    int l = t->blk[id].lev;
    int b[3];
    for (int d = 0; d < 3; d++) b[d] = t->blk[id].org[d] / ext(t, l, d);
    int kz = t->dim == 3 ? 1 : 0;
    for (int dz = -kz; dz <= kz; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                int g[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
                int outside = 0;
                for (int d = 0; d < t->dim; d++) {
                    int n = t->lev[l].nblk[d];
                    if (g[d] < 0 || g[d] >= n) {
                        int face = 2 * d + (g[d] >= n);
                        if (t->bc_kind[face] == OG_PERIODIC) g[d] = (g[d] + n) % n;
                        else outside = 1;
                    }
                }
                if (!outside) ensure_block(t, l, g);
            }
    /* ensure_block may have moved t->blk; use the index again. */
    int nc = 1 << t->dim;
    for (int c = 0; c < nc; c++) {
        int cb[3] = {2 * b[0] + (c & 1), 2 * b[1] + ((c >> 1) & 1), t->dim == 3 ? 2 * b[2] + ((c >> 2) & 1) : 0};
        int cid = new_block(t, l + 1, cb);
        t->blk[cid].parent = id;
        t->blk[id].child[c] = cid;
    }
    t->blk[id].has_children = 1;
}

static uint64_t morton(const int *b, int dim) {
    uint64_t code = 0;
    for (int bit = 0; bit < 21; bit++)
        for (int d = 0; d < dim; d++)
            code |= (uint64_t)((b[d] >> bit) & 1) << (bit * dim + d);
    return code;
}

static const og_tree *sort_tree;
static int cmp_leaf(const void *a, const void *b) {
    const OBlock *A = &sort_tree->blk[*(const int *)a], *B = &sort_tree->blk[*(const int *)b];
    if (A->lev != B->lev) return A->lev < B->lev ? -1 : 1;
    int ba[3], bb[3];
    for (int d = 0; d < 3; d++) {
        ba[d] = A->org[d] / ext(sort_tree, A->lev, d);
        bb[d] = B->org[d] / ext(sort_tree, B->lev, d);
    }
    uint64_t ma = morton(ba, sort_tree->dim), mb = morton(bb, sort_tree->dim);
    return ma < mb ? -1 : (ma > mb ? 1 : 0);
}

og_tree *og_create(int dim, const int32_t *base_cells, const double *lo, const double *hi,
                   const int32_t *bc_kind, const double *bc_value, int bs, int max_refine,
                   og_refine_fn refine, void *ud, int domain_id, int variable_eps) {
    if (dim != 2 && dim != 3) return NULL;
    if (bs < 1 || (bs & (bs - 1)) || max_refine < 0) return NULL;
    if (max_refine > 0 && bs < 2) return NULL;
    for (int d = 0; d < dim; d++)
        if (base_cells[d] <= 0 || base_cells[d] % bs) return NULL;
    for (int f = 0; f < 2 * dim; f++) {
        if (bc_kind[f] < OG_DIRICHLET || bc_kind[f] > OG_PERIODIC) return NULL;
        if ((bc_kind[f] == OG_PERIODIC) != (bc_kind[f ^ 1] == OG_PERIODIC)) return NULL;
    }
    og_tree *t = (og_tree *)calloc(1, sizeof(og_tree));
    t->dim = dim;
    t->domain_id = domain_id;
    t->var_eps = variable_eps ? 1 : 0;
    for (int f = 0; f < 6; f++) {
        t->bc_kind[f] = f < 2 * dim ? bc_kind[f] : OG_PERIODIC;
        t->bc_val[f] = f < 2 * dim ? bc_value[f] : 0.0;
    }
    for (int d = 0; d < 3; d++) {
        t->lo[d] = d < dim ? lo[d] : 0.0;
        t->hi[d] = d < dim ? hi[d] : 1.0;
    }
    t->n_down = 2; t->n_up = 2; t->n_max = 1000; t->abs_tol = 0.0; t->rel_tol = 1e-8;
    t->smoother = OG_SMOOTH_GSRB; t->omega = 2.0 / 3.0; t->lambda = 0.0; t->axisym = 0;
    t->stall_steps = STALL_STEPS;
    t->refine = refine; t->ud = ud;

    /* Added coarse grids (Sec. 2.5): halve the grid while every halved size still
     * tiles by bs; then keep the block layout and halve the block size down to 1. */
    int nc[3] = {1, 1, 1}, sizes[OG_MAXLEV][4];
    for (int d = 0; d < dim; d++) nc[d] = base_cells[d];
    int ncoarse = 0;
    sizes[0][0] = nc[0]; sizes[0][1] = nc[1]; sizes[0][2] = nc[2]; sizes[0][3] = bs;
    for (;;) {
        int ok = 1;
        for (int d = 0; d < dim; d++)
            if (nc[d] % 2 || (nc[d] / 2) % bs) ok = 0;
        if (!ok) break;
        for (int d = 0; d < dim; d++) nc[d] /= 2;
        ncoarse++;
        sizes[ncoarse][0] = nc[0]; sizes[ncoarse][1] = nc[1]; sizes[ncoarse][2] = nc[2];
        sizes[ncoarse][3] = bs;
        if (ncoarse + 8 >= OG_MAXLEV) { free(t); return NULL; }
    }
    int b = bs;
    while (b > 1) {
        b /= 2;
        for (int d = 0; d < dim; d++) nc[d] /= 2;
        ncoarse++;
        sizes[ncoarse][0] = nc[0]; sizes[ncoarse][1] = nc[1]; sizes[ncoarse][2] = nc[2];
        sizes[ncoarse][3] = b;
    }
    t->lbase = ncoarse;
    t->nlev = ncoarse + 1 + max_refine;
    if (t->nlev > OG_MAXLEV) { free(t); return NULL; }
    for (int l = 0; l < t->nlev; l++) {
        OLevel *L = &t->lev[l];
        if (l <= ncoarse) {
            int *s = sizes[ncoarse - l];
            L->ncell[0] = s[0]; L->ncell[1] = s[1]; L->ncell[2] = s[2]; L->bs = s[3];
        } else {
            L->bs = bs;
            for (int d = 0; d < 3; d++)
                L->ncell[d] = d < dim ? t->lev[l - 1].ncell[d] * 2 : 1;
        }
        size_t nmap = 1;
        for (int d = 0; d < 3; d++) {
            L->nblk[d] = L->ncell[d] / ext(t, l, d);
            L->h[d] = (t->hi[d] - t->lo[d]) / L->ncell[d];
            nmap *= (size_t)L->nblk[d];
        }
        L->map = (int *)malloc(nmap * sizeof(int));
        for (size_t i = 0; i < nmap; i++) L->map[i] = -1;
    }
    /* All blocks of the coarse levels and the base level exist. */
    for (int l = 0; l <= t->lbase; l++) {
        OLevel *L = &t->lev[l];
        int bb[3];
        for (bb[2] = 0; bb[2] < L->nblk[2]; bb[2]++)
            for (bb[1] = 0; bb[1] < L->nblk[1]; bb[1]++)
                for (bb[0] = 0; bb[0] < L->nblk[0]; bb[0]++) {
                    int id = new_block(t, l, bb);
                    if (l == 0) continue;
                    const OLevel *P = &t->lev[l - 1];
                    int frozen = P->nblk[0] == L->nblk[0] && P->nblk[1] == L->nblk[1] && P->nblk[2] == L->nblk[2];
                    int pb[3], c = 0;
                    for (int d = 0; d < 3; d++) pb[d] = frozen ? bb[d] : bb[d] / 2;
                    if (!frozen) c = (bb[0] & 1) | ((bb[1] & 1) << 1) | ((bb[2] & 1) << 2);
                    int pid = block_at(t, l - 1, pb);
                    t->blk[id].parent = pid;
                    t->blk[pid].child[c] = id;
                    t->blk[pid].has_children = 1;
                }
    }
    /* Refinement: the least tree that refines every block (below the top level) on
     * which the predicate holds and is 2:1 balanced.  Passes repeat until nothing
     * changes, so the result does not depend on the visiting order. */
    if (max_refine > 0 && refine) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int l = t->lbase; l < t->nlev - 1; l++) {
                for (int i = 0; i < t->lev[l].n; i++) {
                    int id = t->lev[l].list[i];
                    if (t->blk[id].has_children || t->blk[id].tested) continue;
                    t->blk[id].tested = 1;
                    int32_t org[3] = {t->blk[id].org[0], t->blk[id].org[1], t->blk[id].org[2]};
                    if (refine(ud, domain_id, l - t->lbase, org, bs)) {
                        refine_block(t, id);
                        changed = 1;
                    }
                }
            }
        }
    }
    /* Drop empty top levels. */
    while (t->nlev - 1 > t->lbase && t->lev[t->nlev - 1].n == 0) {
        free(t->lev[t->nlev - 1].map);
        t->nlev--;
    }
    /* Canonical leaf order: level, then Morton order of the block coordinates. */
    t->leaf = (int *)malloc((size_t)t->nblk * sizeof(int));
    t->nleaf = 0;
    for (int id = 0; id < t->nblk; id++)
        if (!t->blk[id].has_children && t->blk[id].lev >= t->lbase) t->leaf[t->nleaf++] = id;
    sort_tree = t;
    qsort(t->leaf, (size_t)t->nleaf, sizeof(int), cmp_leaf);
    /* Initial state: phi = 0, ghosts filled on every level. */
    for (int l = 0; l < t->nlev; l++) og_fill_ghosts_level(t, l);
    return t;
}

void og_destroy(og_tree *t) {
    if (!t) return;
    for (int i = 0; i < t->nblk; i++) {
        for (int f = 0; f < NFIELD; f++) free(t->blk[i].fld[f]);
        free(t->blk[i].bval);
    }
    for (int l = 0; l < t->nlev; l++) {
        free(t->lev[l].map);
        free(t->lev[l].list);
    }
    free(t->blk);
    free(t->leaf);
    free(t);
}

void og_set_params(og_tree *t, int n_down, int n_up, int n_max, double abs_tol, double rel_tol) {
    t->n_down = n_down; t->n_up = n_up; t->n_max = n_max;
    t->abs_tol = abs_tol; t->rel_tol = rel_tol;
}

void og_set_lambda(og_tree *t, double lambda) { t->lambda = lambda; }

int og_set_axisymmetric(og_tree *t, int on) {
    if (on && (t->dim != 2 || t->lo[0] < 0.0)) return -1;
    t->axisym = on != 0;
    return 0;
}

void og_set_smoother(og_tree *t, int kind, double omega) {
    t->smoother = kind;
    t->omega = omega;
}

int og_num_levels(const og_tree *t) { return t->nlev; }
int og_base_level(const og_tree *t) { return t->lbase; }
void og_level_info(const og_tree *t, int l, int32_t *bs, int32_t *ncell, int32_t *nblocks) {
    *bs = t->lev[l].bs;
    for (int d = 0; d < 3; d++) ncell[d] = t->lev[l].ncell[d];
    *nblocks = t->lev[l].n;
}

static int cells_per_block(const og_tree *t, int l) {
    return ext(t, l, 0) * ext(t, l, 1) * ext(t, l, 2);
}

int64_t og_num_leaf_cells(const og_tree *t) {
    int64_t n = 0;
    for (int i = 0; i < t->nleaf; i++) n += cells_per_block(t, t->blk[t->leaf[i]].lev);
    return n;
}
int og_num_leaf_blocks(const og_tree *t) { return t->nleaf; }

#define FOR_CELLS(t, l, i, j, k)                                 \
    for (int k = 0; k < ext(t, l, 2); k++)                       \
        for (int j = 0; j < ext(t, l, 1); j++)                   \
            for (int i = 0; i < ext(t, l, 0); i++)

void og_leaf_layout(const og_tree *t, int32_t *out) {
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        const OBlock *B = &t->blk[t->leaf[q]];
        FOR_CELLS(t, B->lev, i, j, k) {
            out[4 * n + 0] = B->lev - t->lbase;
            out[4 * n + 1] = B->org[0] + i;
            out[4 * n + 2] = B->org[1] + j;
            out[4 * n + 3] = B->org[2] + k;
            n++;
        }
    }
}

static void scatter_leaf(og_tree *t, int field, const double *src) {
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        OBlock *B = &t->blk[t->leaf[q]];
        FOR_CELLS(t, B->lev, i, j, k) B->fld[field][pidx(t, B->lev, i, j, k)] = src[n++];
    }
}

static void gather_leaf(const og_tree *t, int field, double *dst) {
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        const OBlock *B = &t->blk[t->leaf[q]];
        FOR_CELLS(t, B->lev, i, j, k) dst[n++] = B->fld[field][pidx(t, B->lev, i, j, k)];
    }
}

/* ------------------------------------------------------------- ghost cells */
/* Sec. 2.6.  One layer of face ghosts.  Three cases:
 *  - a block on the same level covers the ghost (also across periodic faces): copy;
 *  - physical boundary: Dirichlet phi_g = 2a - phi_i, Neumann phi_g = phi_i +/- h b,
 *    with b the derivative along +x_d (upper face +, lower face -);
 *  - refinement boundary: g = (B' + c')/2 where B' is the coarse value B moved to the
 *    ghost's tangential position with the central-difference slope(s) of the coarse
 *    cell, and c' = (3c - c2)/2 is the two-point extrapolation of the fine cells c
 *    (next to the ghost) and c2 (next inward) to the face.
 * The coefficient eps is copied at same-level faces, copied from the interior cell at
 * physical faces, and taken from the coarse cell at refinement faces (piecewise
 * constant). */
static void fill_ghosts_field(og_tree *t, int l, int field, int homogeneous) {
    const OLevel *L = &t->lev[l];
    int bs = L->bs;
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        double *u = B->fld[field];
        for (int d = 0; d < t->dim; d++) {
            int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            int n1 = ext(t, l, t1), n2 = ext(t, l, t2);
            for (int side = 0; side < 2; side++) {
                int face = 2 * d + side;
                for (int a2 = 0; a2 < n2; a2++)
                    for (int a1 = 0; a1 < n1; a1++) {
                        int gl[3], in1[3], in2[3];
                        gl[t1] = a1; gl[t2] = a2; gl[d] = side ? bs : -1;
                        in1[t1] = a1; in1[t2] = a2; in1[d] = side ? bs - 1 : 0;
                        in2[t1] = a1; in2[t2] = a2; in2[d] = side ? bs - 2 : 1;
                        int g[3] = {B->org[0] + gl[0], B->org[1] + gl[1], B->org[2] + gl[2]};
                        int gp = pidx3(t, l, gl);
                        double ci = u[pidx3(t, l, in1)];
                        int phys = wrap_cell(t, l, g);
                        if (phys) {
                            if (field == F_EPS) {
                                u[gp] = ci;
                            } else {
                                double a = homogeneous ? 0.0 : t->bc_val[face];
                                if (!homogeneous && B->bval && t->bc_kind[face] == OG_DIRICHLET)
                                    a = B->bval[(face * n2 + a2) * n1 + a1];
                                if (t->bc_kind[face] == OG_DIRICHLET) u[gp] = 2.0 * a - ci;
                                else u[gp] = ci + (side ? 1.0 : -1.0) * L->h[d] * a;
                            }
                            continue;
                        }
                        int nb = block_of_cell(t, l, g);
                        if (nb >= 0) {
                            const OBlock *N = &t->blk[nb];
                            int loc[3] = {g[0] - N->org[0], g[1] - N->org[1], g[2] - N->org[2]};
                            u[gp] = N->fld[field][pidx3(t, l, loc)];
                            continue;
                        }
                        /* Refinement boundary: coarse cell containing the ghost centre. */
                        int gc[3] = {g[0] / 2, g[1] / 2, g[2] / 2};
                        if (t->dim == 2) gc[2] = 0;
                        int qb = block_of_cell(t, l - 1, gc);
                        const OBlock *Q = &t->blk[qb];
                        int cl[3] = {gc[0] - Q->org[0], gc[1] - Q->org[1], gc[2] - Q->org[2]};
                        const double *w = Q->fld[field];
                        double Bv = w[pidx3(t, l - 1, cl)];
                        if (field == F_EPS) {
                            u[gp] = Bv;
                            continue;
                        }
                        double Bp = Bv;
                        int tang[2] = {t1, t2};
                        for (int m = 0; m < t->dim - 1; m++) {
                            int td = tang[m];
                            double sigma = (g[td] & 1) ? 1.0 : -1.0;
                            int cp[3] = {cl[0], cl[1], cl[2]}, cm[3] = {cl[0], cl[1], cl[2]};
                            cp[td] += 1;
                            cm[td] -= 1;
                            Bp += sigma * (w[pidx3(t, l - 1, cp)] - w[pidx3(t, l - 1, cm)]) / 8.0;
                        }
                        double c = ci, c2 = u[pidx3(t, l, in2)];
                        double cprime = 1.5 * c - 0.5 * c2;
                        u[gp] = 0.5 * (Bp + cprime);
                    }
            }
        }
    }
}

/* Dirichlet values that vary along a face (Sec. 2.6: the ghost of a boundary cell is
 * 2a - phi_i with a the value at the centre of the cell's boundary face), on every
 * level.  The faces are enumerated level by level (coarsest first), then blocks in
 * creation order, then faces -x..+z, then the face's cells (lower in-plane axis
 * fastest); only faces on a physical Dirichlet boundary are listed.  With centres
 * (3 per face) and faces non-NULL the positions and face indices are written. */
int64_t og_boundary_faces(const og_tree *t, double *centres, int32_t *faces) {
    int64_t n = 0;
    for (int l = 0; l < t->nlev; l++) {
        const OLevel *L = &t->lev[l];
        for (int q = 0; q < L->n; q++) {
            const OBlock *B = &t->blk[L->list[q]];
            for (int d = 0; d < t->dim; d++) {
                int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                int n1 = ext(t, l, t1), n2 = ext(t, l, t2);
                for (int side = 0; side < 2; side++) {
                    int face = 2 * d + side;
                    if (t->bc_kind[face] != OG_DIRICHLET) continue;
                    int gd = side ? B->org[d] + L->bs : B->org[d] - 1;
                    if (gd >= 0 && gd < L->ncell[d]) continue;   /* not on the boundary */
                    for (int a2 = 0; a2 < n2; a2++)
                        for (int a1 = 0; a1 < n1; a1++) {
                            if (centres) {
                                double *x = centres + 3 * n;
                                x[d] = side ? t->hi[d] : t->lo[d];
                                x[t1] = t->lo[t1] + (B->org[t1] + a1 + 0.5) * L->h[t1];
                                x[t2] = t->dim == 3 ? t->lo[t2] + (B->org[t2] + a2 + 0.5) * L->h[t2] : 0.0;
                            }
                            if (faces) faces[n] = face;
                            n++;
                        }
                }
            }
        }
    }
    return n;
}

/* Values for the faces listed by og_boundary_faces, in that order; they replace the
 * face's constant value on every level. */
void og_set_boundary_values(og_tree *t, const double *vals) {
    int64_t n = 0;
    for (int l = 0; l < t->nlev; l++) {
        const OLevel *L = &t->lev[l];
        for (int q = 0; q < L->n; q++) {
            OBlock *B = &t->blk[L->list[q]];
            for (int d = 0; d < t->dim; d++) {
                int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                int n1 = ext(t, l, t1), n2 = ext(t, l, t2);
                for (int side = 0; side < 2; side++) {
                    int face = 2 * d + side;
                    if (t->bc_kind[face] != OG_DIRICHLET) continue;
                    int gd = side ? B->org[d] + L->bs : B->org[d] - 1;
                    if (gd >= 0 && gd < L->ncell[d]) continue;
                    if (!B->bval) {
                        B->bval = (double *)malloc((size_t)2 * t->dim * n1 * n2 * sizeof(double));
                        for (int f = 0; f < 2 * t->dim * n1 * n2; f++) B->bval[f] = 0.0;
                    }
                    for (int a2 = 0; a2 < n2; a2++)
                        for (int a1 = 0; a1 < n1; a1++) B->bval[(face * n2 + a2) * n1 + a1] = vals[n++];
                }
            }
        }
    }
    for (int l = 0; l < t->nlev; l++) og_fill_ghosts_level(t, l);
}

void og_fill_ghosts_level(og_tree *t, int l) {
    fill_ghosts_field(t, l, F_V, 0);
}

/* ---------------------------------------------------------------- operator */
/* eq. poisson-2d (constant coefficient) and eq. poisson-2d-vcoeff (harmonic mean of
 * the coefficient in the two cells sharing a face), with an extra z term in 3D. */

static double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

/* Face weights of axis d at cell (i,j,k) of block B: h_d^-2 times, in the 2D
 * axisymmetric form (Sec. 2.1: (1/r) d/dr (r dphi/dr) + d2phi/dz2, finite volumes), the
 * ratio of the face radius to the cell-centre radius on the r axis. */
static void face_weights(const og_tree *t, int l, const OBlock *B, int d, int i, double *wm, double *wp) {
    double ih2 = 1.0 / (t->lev[l].h[d] * t->lev[l].h[d]);
    *wm = ih2;
    *wp = ih2;
    if (t->axisym && d == 0) {
        double h = t->lev[l].h[0];
        double r = t->lo[0] + (B->org[0] + i + 0.5) * h;
        *wm = ih2 * (r - 0.5 * h) / r;
        *wp = ih2 * (r + 0.5 * h) / r;
    }
}

static double apply_L(const og_tree *t, int l, const OBlock *B, int i, int j, int k) {
    const double *v = B->fld[F_V];
    int c[3] = {i, j, k};
    int p = pidx3(t, l, c);
    double sum = 0.0;
    for (int d = 0; d < t->dim; d++) {
        int cm[3] = {i, j, k}, cp[3] = {i, j, k};
        cm[d] -= 1;
        cp[d] += 1;
        int pm = pidx3(t, l, cm), pp = pidx3(t, l, cp);
        double wm, wp;
        face_weights(t, l, B, d, i, &wm, &wp);
        if (!t->var_eps) {
            sum += wm * (v[pm] - v[p]) + wp * (v[pp] - v[p]);
        } else {
            const double *e = B->fld[F_EPS];
            sum += wm * harmonic(e[p], e[pm]) * (v[pm] - v[p]) + wp * harmonic(e[p], e[pp]) * (v[pp] - v[p]);
        }
    }
    return sum - t->lambda * v[p];
}

/* Gauss-Seidel local solve (Sec. 2.2): the cell's equation solved for phi_i with its
 * neighbours fixed, phi_i = (sum_f w_f phi_nb - f_i) / sum_f w_f, w_f = eps_f / h_d^2.
 * The denominator is the operator's diagonal (2 h_x^-2 + 2 h_y^-2 [+ 2 h_z^-2] for
 * constant eps). */
static double gs_value(const og_tree *t, int l, const OBlock *B, int i, int j, int k) {
    const double *v = B->fld[F_V];
    int c[3] = {i, j, k};
    int p = pidx3(t, l, c);
    double num = 0.0, den = 0.0;
    for (int d = 0; d < t->dim; d++) {
        int cm[3] = {i, j, k}, cp[3] = {i, j, k};
        cm[d] -= 1;
        cp[d] += 1;
        int pm = pidx3(t, l, cm), pp = pidx3(t, l, cp);
        double wm, wp;
        face_weights(t, l, B, d, i, &wm, &wp);
        if (t->var_eps) {
            const double *e = B->fld[F_EPS];
            wm *= harmonic(e[p], e[pm]);
            wp *= harmonic(e[p], e[pp]);
        }
        num += wm * v[pm] + wp * v[pp];
        den += wm + wp;
    }
    return (num - B->fld[F_F][p]) / (den + t->lambda);
}

/* ---------------------------------------------------------------- smoother */
/* Red-black Gauss-Seidel (Sec. 2.2): first all cells with an even sum of global
 * indices, then the odd ones.  Ghost cells are refreshed after each colour, so a
 * blocked sweep equals a sweep over the whole level (Sec. 2.6 states that ghosts are
 * updated after, not during, a smoothing step). */
/* Weighted Jacobi (the smoother of the paper's timing runs, Sec. 3.3; the weight is not
 * given there): every cell moves the fraction omega of the way from its value to its
 * Gauss-Seidel local solution, all computed from the values before the step (held in
 * the residual field meanwhile); then ghosts are refreshed. */
static void jacobi_step(og_tree *t, int l) {
    const OLevel *L = &t->lev[l];
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        FOR_CELLS(t, l, i, j, k) {
            int p = pidx(t, l, i, j, k);
            double v = B->fld[F_V][p];
            B->fld[F_R][p] = v + t->omega * (gs_value(t, l, B, i, j, k) - v);
        }
    }
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        FOR_CELLS(t, l, i, j, k) {
            int p = pidx(t, l, i, j, k);
            B->fld[F_V][p] = B->fld[F_R][p];
        }
    }
    og_fill_ghosts_level(t, l);
}

static void smooth_step(og_tree *t, int l) {
    const OLevel *L = &t->lev[l];
    if (t->smoother == OG_SMOOTH_JACOBI) {
        jacobi_step(t, l);
        return;
    }
    for (int colour = 0; colour < 2; colour++) {
        #pragma omp parallel for schedule(static)
        for (int q = 0; q < L->n; q++) {
            OBlock *B = &t->blk[L->list[q]];
            FOR_CELLS(t, l, i, j, k) {
                if (((B->org[0] + i + B->org[1] + j + B->org[2] + k) & 1) != colour) continue;
                B->fld[F_V][pidx(t, l, i, j, k)] = gs_value(t, l, B, i, j, k);
            }
        }
        og_fill_ghosts_level(t, l);
    }
}

/* r = f - L v on every block of level l (Sec. 2.4). */
static void residual_level(og_tree *t, int l) {
    const OLevel *L = &t->lev[l];
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        FOR_CELLS(t, l, i, j, k) {
            int p = pidx(t, l, i, j, k);
            B->fld[F_R][p] = B->fld[F_F][p] - apply_L(t, l, B, i, j, k);
        }
    }
}

/* ------------------------------------------------------ transfer operators */
/* Restriction (Sec. 2.3): a coarse value is the mean of the 2^d fine values it covers.
 * Applied to the given field for every block of level l-1 that has children. */
static void restrict_field(og_tree *t, int l, int src, int dst) {
    const OLevel *C = &t->lev[l - 1];
    int nsub = 1 << t->dim;
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < C->n; q++) {
        OBlock *P = &t->blk[C->list[q]];
        if (!P->has_children) continue;
        FOR_CELLS(t, l - 1, i, j, k) {
            int gc[3] = {P->org[0] + i, P->org[1] + j, P->org[2] + k};
            double s = 0.0;
            for (int a = 0; a < nsub; a++) {
                int g[3] = {2 * gc[0] + (a & 1), 2 * gc[1] + ((a >> 1) & 1), t->dim == 3 ? 2 * gc[2] + ((a >> 2) & 1) : 0};
                const OBlock *F = &t->blk[block_of_cell(t, l, g)];
                int loc[3] = {g[0] - F->org[0], g[1] - F->org[1], g[2] - F->org[2]};
                s += F->fld[src][pidx3(t, l, loc)];
            }
            P->fld[dst][pidx(t, l - 1, i, j, k)] = s / nsub;
        }
    }
}

/* Downward transfer of the FAS V-cycle (Sec. 2.4): v^H = R(v^h), then the ghosts of
 * level H, then v_old^H = v^H (ghost layer included, so that the correction can be
 * prolongated near block boundaries), then f^H = R(r^h) + L^H v^H (eq. coarse-rhs).
 * Blocks of level H without children keep their own v and f. */
static void restrict_fas(og_tree *t, int l) {
    residual_level(t, l);
    restrict_field(t, l, F_V, F_V);
    restrict_field(t, l, F_R, F_R);
    og_fill_ghosts_level(t, l - 1);
    const OLevel *C = &t->lev[l - 1];
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < C->n; q++) {
        OBlock *P = &t->blk[C->list[q]];
        if (!P->has_children) continue;
        memcpy(P->fld[F_VOLD], P->fld[F_V], (size_t)npad(t, l - 1) * sizeof(double));
        FOR_CELLS(t, l - 1, i, j, k) {
            int p = pidx(t, l - 1, i, j, k);
            P->fld[F_F][p] = P->fld[F_R][p] + apply_L(t, l - 1, P, i, j, k);
        }
    }
}

/* Correction (eq. coarse-corr): v^h += P(v^H - v_old^H) with the prolongation of
 * eq. interp_2d / interp_3d, which uses the coarse cell and its face neighbours on the
 * side of the fine cell (coarse ghost cells near block boundaries, no diagonal ones).
 * Then the ghosts of level h. */
static void correct_level(og_tree *t, int l) {
    const OLevel *L = &t->lev[l];
    #pragma omp parallel for schedule(static)
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        const OBlock *P = &t->blk[B->parent];
        const double *vc = P->fld[F_V], *vo = P->fld[F_VOLD];
        FOR_CELLS(t, l, i, j, k) {
            int g[3] = {B->org[0] + i, B->org[1] + j, B->org[2] + k};
            int pc[3], s[3];
            for (int d = 0; d < 3; d++) {
                pc[d] = g[d] / 2 - P->org[d];
                s[d] = (g[d] & 1) ? 1 : -1;
            }
            if (t->dim == 2) pc[2] = 0;
            int p0 = pidx3(t, l - 1, pc);
            double d0 = vc[p0] - vo[p0];
            double dn[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < t->dim; d++) {
                int cn[3] = {pc[0], pc[1], pc[2]};
                cn[d] += s[d];
                int pn = pidx3(t, l - 1, cn);
                dn[d] = vc[pn] - vo[pn];
            }
            double corr;
            if (t->dim == 2) corr = 0.25 * (2.0 * d0 + dn[0] + dn[1]);
            else corr = 0.25 * (d0 + dn[0] + dn[1] + dn[2]);
            B->fld[F_V][pidx(t, l, i, j, k)] += corr;
        }
    }
    og_fill_ghosts_level(t, l);
}

void og_smooth_level(og_tree *t, int l, int n) {
    for (int s = 0; s < n; s++) smooth_step(t, l);
}

void og_correct_level(og_tree *t, int l) { correct_level(t, l); }

/* ----------------------------------------------------------- coarsest grid */
static double level_residual_max(og_tree *t, int l) {
    const OLevel *L = &t->lev[l];
    double m = 0.0;
    for (int q = 0; q < L->n; q++) {
        OBlock *B = &t->blk[L->list[q]];
        FOR_CELLS(t, l, i, j, k) {
            double r = fabs(B->fld[F_F][pidx(t, l, i, j, k)] - apply_L(t, l, B, i, j, k));
            if (r > m || r != r) m = r;
        }
    }
    return m;
}

static int all_periodic(const og_tree *t) {
    for (int f = 0; f < 2 * t->dim; f++)
        if (t->bc_kind[f] != OG_PERIODIC) return 0;
    return 1;
}

/* Coarsest grid (Sec. 2.4): smoothing steps until the max-norm residual is below the
 * absolute threshold or reduced by the relative factor, at most n_max steps, at least
 * one.  It also stops once STALL_STEPS steps in a row have not brought the residual
 * 0.1% below the lowest value reached so far: at the rounding floor, and on a one-cell
 * grid with Dirichlet faces, where Gauss-Seidel with the ghost held fixed only
 * alternates between two values (the margin keeps that decision clear of rounding).
 * Several steps are allowed because the max-norm residual of a slowly converging grid
 * can rise for a few steps before it falls.  On a fully periodic domain the mean of f
 * is first removed on this level so that the singular system is consistent. */
static void coarse_solve(og_tree *t) {
    const OLevel *L = &t->lev[0];
    if (all_periodic(t) && t->lambda == 0.0) {
        double s = 0.0;
        long cnt = 0;
        for (int q = 0; q < L->n; q++) {
            OBlock *B = &t->blk[L->list[q]];
            FOR_CELLS(t, 0, i, j, k) { s += B->fld[F_F][pidx(t, 0, i, j, k)]; cnt++; }
        }
        double mean = s / cnt;
        for (int q = 0; q < L->n; q++) {
            OBlock *B = &t->blk[L->list[q]];
            FOR_CELLS(t, 0, i, j, k) B->fld[F_F][pidx(t, 0, i, j, k)] -= mean;
        }
    }
    double r0 = level_residual_max(t, 0), best = r0;
    double target = t->abs_tol > t->rel_tol * r0 ? t->abs_tol : t->rel_tol * r0;
    int k, since = 0;
    t->last_coarse_exit = OG_EXIT_NMAX;
    for (k = 1; k <= t->n_max; k++) {
        smooth_step(t, 0);
        double r = level_residual_max(t, 0);
        if (r <= target) {
            t->last_coarse_exit = OG_EXIT_TARGET;
            break;
        }
        if (r < STALL * best) {
            best = r;
            since = 0;
        } else if (t->stall_steps > 0 && ++since >= t->stall_steps) {
            t->last_coarse_exit = OG_EXIT_STALL;
            break;
        }
    }
    t->last_coarse_steps = k > t->n_max ? t->n_max : k;
}

int og_last_coarse_exit(const og_tree *t) { return t->last_coarse_exit; }

void og_coarse_solve(og_tree *t) { coarse_solve(t); }

void og_set_coarse_stall(og_tree *t, int steps) { t->stall_steps = steps > 0 ? steps : 0; }

int og_last_coarse_steps(const og_tree *t) { return t->last_coarse_steps; }

/* ------------------------------------------------------------------ cycles */
/* V-cycle with its top on level lt (Sec. 2.4). */
static void vcycle_from(og_tree *t, int lt) {
    for (int l = lt; l >= 1; l--) {
        for (int s = 0; s < t->n_down; s++) smooth_step(t, l);
        restrict_fas(t, l);
    }
    coarse_solve(t);
    for (int l = 1; l <= lt; l++) {
        correct_level(t, l);
        for (int s = 0; s < t->n_up; s++) smooth_step(t, l);
    }
}

void og_vcycle(og_tree *t) { vcycle_from(t, t->nlev - 1); }

/* FMG cycle (Sec. 2.4, fig. mg-cycles): the solution and the right-hand side are
 * restricted down to the coarsest grid, which is solved; then each finer level gets
 * the coarse correction and a V-cycle with its top on that level. */
void og_fmg(og_tree *t) {
    for (int l = t->nlev - 1; l >= 1; l--) restrict_fas(t, l);
    coarse_solve(t);
    for (int l = 1; l < t->nlev; l++) {
        correct_level(t, l);
        vcycle_from(t, l);
    }
}

/* ------------------------------------------------------ composite residual */
void og_restrict_all(og_tree *t) {
    for (int l = t->nlev - 1; l >= 1; l--) restrict_field(t, l, F_V, F_V);
}

/* Parents take the mean of their children on every level, then ghosts are refreshed
 * from the coarsest level up, so each leaf's stencil sees the composite grid. */
static void sync_levels(og_tree *t) {
    og_restrict_all(t);
    for (int l = 0; l < t->nlev; l++) og_fill_ghosts_level(t, l);
}

void og_leaf_residual(og_tree *t, double *leaf_r) {
    sync_levels(t);
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        OBlock *B = &t->blk[t->leaf[q]];
        FOR_CELLS(t, B->lev, i, j, k)
            leaf_r[n++] = B->fld[F_F][pidx(t, B->lev, i, j, k)] - apply_L(t, B->lev, B, i, j, k);
    }
}

/* Relative residual norms over leaf cells: max-norm ratio, and the volume-weighted
 * L2 ratio sqrt(sum vol r^2 / sum vol f^2) (eq. l2-norm-example). */
void og_residual_norm(og_tree *t, double *max_rel, double *l2_rel) {
    sync_levels(t);
    double rmax = 0.0, fmax = 0.0, r2 = 0.0, f2 = 0.0;
    for (int q = 0; q < t->nleaf; q++) {
        OBlock *B = &t->blk[t->leaf[q]];
        const double *h = t->lev[B->lev].h;
        double vol = h[0] * h[1] * (t->dim == 3 ? h[2] : 1.0);
        FOR_CELLS(t, B->lev, i, j, k) {
            double f = B->fld[F_F][pidx(t, B->lev, i, j, k)];
            double r = f - apply_L(t, B->lev, B, i, j, k);
            if (fabs(r) > rmax || r != r) rmax = fabs(r);
            if (fabs(f) > fmax) fmax = fabs(f);
            r2 += vol * r * r;
            f2 += vol * f * f;
        }
    }
    *max_rel = fmax > 0.0 ? rmax / fmax : rmax;
    *l2_rel = f2 > 0.0 ? sqrt(r2 / f2) : sqrt(r2);
}

void og_apply(og_tree *t, const double *leaf_phi, double *leaf_out) {
    scatter_leaf(t, F_V, leaf_phi);
    sync_levels(t);
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        OBlock *B = &t->blk[t->leaf[q]];
        FOR_CELLS(t, B->lev, i, j, k) leaf_out[n++] = apply_L(t, B->lev, B, i, j, k);
    }
}

/* ------------------------------------------------------------------- data */
void og_set_rhs(og_tree *t, const double *leaf_f) { scatter_leaf(t, F_F, leaf_f); }

void og_set_phi(og_tree *t, const double *leaf_phi) {
    scatter_leaf(t, F_V, leaf_phi);
    sync_levels(t);
}

void og_get_phi(const og_tree *t, double *leaf_phi) { gather_leaf(t, F_V, leaf_phi); }

/* The coefficient on coarse blocks is the mean of the children (the paper does not
 * say how eps is coarsened); ghosts as described at fill_ghosts_field. */
void og_set_eps(og_tree *t, const double *leaf_eps) {
    scatter_leaf(t, F_EPS, leaf_eps);
    for (int l = t->nlev - 1; l >= 1; l--) restrict_field(t, l, F_EPS, F_EPS);
    for (int l = 0; l < t->nlev; l++) fill_ghosts_field(t, l, F_EPS, 0);
    for (int l = 0; l < t->nlev; l++) og_fill_ghosts_level(t, l);
}

/* ---------------------------------------------------------------- adjoint */
/* For the discrete operator (L phi)_i = sum_f w_f (phi_nb - phi_i), w_f = ebar_f/h^2,
 * and J depending on phi with L phi = f: dJ/deps_i = -lambda^T (dL/deps_i) phi with
 * L^T lambda = dJ/dphi.  Interior face (i,j): d ebar/d eps_i = 2 eps_j^2/(eps_i+eps_j)^2,
 * giving + h^-2 d ebar/d eps_i (lambda_j - lambda_i)(phi_j - phi_i).  Physical face:
 * the ghost carries eps_i, so ebar = eps_i and the term is -h^-2 lambda_i (phi_g - phi_i). */
int og_face_gradient(og_tree *t, const double *leaf_phi, const double *leaf_lambda,
                     double *leaf_dJ_deps) {
    int top = t->nlev - 1;
    for (int q = 0; q < t->nleaf; q++)
        if (t->blk[t->leaf[q]].lev != top) return -1;
    scatter_leaf(t, F_V, leaf_phi);
    scatter_leaf(t, F_R, leaf_lambda);
    fill_ghosts_field(t, top, F_V, 0);
    fill_ghosts_field(t, top, F_R, 1);
    int64_t n = 0;
    for (int q = 0; q < t->nleaf; q++) {
        OBlock *B = &t->blk[t->leaf[q]];
        const double *v = B->fld[F_V], *lam = B->fld[F_R], *e = B->fld[F_EPS];
        FOR_CELLS(t, top, i, j, k) {
            int p = pidx(t, top, i, j, k);
            double g = 0.0;
            for (int d = 0; d < t->dim; d++) {
                double ih2 = 1.0 / (t->lev[top].h[d] * t->lev[top].h[d]);
                for (int side = 0; side < 2; side++) {
                    int c[3] = {i, j, k};
                    c[d] += side ? 1 : -1;
                    int pn = pidx3(t, top, c);
                    int gidx = B->org[d] + c[d];
                    int boundary = (gidx < 0 || gidx >= t->lev[top].ncell[d]) &&
                                   t->bc_kind[2 * d + side] != OG_PERIODIC;
                    if (boundary) {
                        g += -ih2 * lam[p] * (v[pn] - v[p]);
                    } else {
                        double s = e[p] + e[pn];
                        double debar = 2.0 * e[pn] * e[pn] / (s * s);
                        g += ih2 * debar * (lam[pn] - lam[p]) * (v[pn] - v[p]);
                    }
                }
            }
            leaf_dJ_deps[n++] = g;
        }
    }
    return 0;
}

/* ------------------------------------------------------------- inspection */
int og_level_nblocks(const og_tree *t, int l) { return t->lev[l].n; }

void og_block_meta(const og_tree *t, int l, int ib, int32_t *origin, int32_t *has_children) {
    const OBlock *B = &t->blk[t->lev[l].list[ib]];
    for (int d = 0; d < 3; d++) origin[d] = B->org[d];
    *has_children = B->has_children;
}

void og_block_field(const og_tree *t, int l, int ib, int field, double *out) {
    const OBlock *B = &t->blk[t->lev[l].list[ib]];
    memcpy(out, B->fld[field], (size_t)npad(t, l) * sizeof(double));
}

void og_set_block_field(og_tree *t, int l, int ib, int field, const double *in) {
    OBlock *B = &t->blk[t->lev[l].list[ib]];
    memcpy(B->fld[field], in, (size_t)npad(t, l) * sizeof(double));
}

/* Threads of the block loops (OpenMP builds; 1 otherwise). */
int og_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
