// Internal declarations shared by the host driver and the HIP kernels of the
// multigrid library.  Not part of the public ABI (that is include/mg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "mg.h"

namespace mgx {

constexpr int MAXLEV = 32;    // global levels (tail + block levels)
constexpr int MAXDOM = 64;    // domains per tree (a 64-bit mask selects them)

// ------------------------------------------------------------------ device view
// Index tables of the block levels, uploaded once per bind.  Blocks are numbered
// level-major (coarse to fine), then by domain, then in Morton order.
struct DevTables {
    const int32_t *org;       // [nb][3] global index of the block's first cell on its level
    const int32_t *nbr;       // [nb][6] same-level neighbour, -1 physical face, -2 coarse-fine
    const int32_t *cf;        // [nb][6] coarse block across a coarse-fine face, else -1
    const int32_t *parent;    // [nb] parent block, -1: the domain's top tail grid
    const int32_t *dom;       // [nb] domain of the block
    const int32_t *lev;       // [nb] global level of the block
    const int32_t *leaf_blk;  // [nleaf_blocks] blocks in leaf order
    const int32_t *leaf_first;// [ndom+1] first leaf rank of every domain
    const int32_t *leaf_rank; // [nb] position of a leaf block in leaf order, -1 for parents
    const double *h;          // [ndom][MAXLEV][3] grid spacing
    const double *ih2;        // [ndom][MAXLEV][3] 1 / h^2 (computed on the host, correctly rounded)
    const int32_t *ncell;     // [ndom][MAXLEV][3] cells per dimension of the full level grid
    const int32_t *bck;       // [ndom][6] boundary kinds
    const double *bcv;        // [ndom][6] boundary values (or zeros: homogeneous)
    const int64_t *tail_off;  // [ndom][MAXLEV] offset of a tail level's padded array (cells)
    const int32_t *tail_top;  // [ndom] highest tail level run by the one-workgroup kernel
    double lambda;            // Helmholtz term: L phi = div(eps grad phi) - lambda phi
    int axi;                  // 2D axisymmetric form (x = r): r-face factors on the x faces
    const double *lox;        // [ndom] lower x bound (the radius of the domain's inner face)
    // Per-cell Dirichlet values of physical faces (only while boundary values are folded
    // into f; null otherwise): fv_off[6 b + f] is the offset in fv of block b's face f
    // (bs^(d-1) values, lower in-plane axis fastest), or -1 for the domain's constant.
    const int64_t *fv_off;
    const double *fv;
};

// Tail levels with more cells than this (per domain) run as multi-workgroup launches;
// the levels below run inside one workgroup.
constexpr int kTailBig = 4096;

// One uniform tail grid of one domain, passed by value.
struct UGrid {
    int dm, lev;
    int n[3];
    int64_t off;
    double h[3];
};

// Fields of one precision.  Block levels store the interior of each block split by
// colour (the bs^d/2 cells with even global index sum first, then the odd ones, each
// in row order, x fastest) followed by nothing else; the 2d face ghost layers are a
// separate array ([block][face][bs^(d-1)], tangential axes in increasing order).
// The reduced-block-size levels below the lowest block level (the "tail") are whole
// uniform grids per domain with one ghost layer around them.
template <typename T>
struct Plane {
    T *v, *vg, *vold, *voldg, *f, *eps, *epsg;
    T *tv, *tvold, *tf, *teps;
    T *v2, *vg2, *tv2;   // second copies of v for the Jacobi smoother (else null)
    const T *vc, *vcg;   // if set: v of the coarser level for coarse-fine ghosts (else v)
};

struct TailParams {
    int n_down, n_up, n_max;
    double abs_tol, rel_tol;
    int jacobi;          // 0: red-black Gauss-Seidel, 1: weighted Jacobi
    double omega;        // Jacobi weight
};

// Launch context.
struct Launch {
    int dim, bs, nt;            // dimension, block size, number of tail levels
    int ndom;
    DevTables tb;
    hipStream_t stream;
    int32_t *coarse_steps;      // [ndom] device: steps taken by the last coarsest solve
    double *partials;           // [nleaf_blocks][4] device scratch
    double *dom_norms;          // [ndom][4] device: max|r|, sum vol r^2, max|f|, sum vol f^2
    double *host_norms;         // if set: device address of pinned host memory that receives
                                // dom_norms as well (no separate copy)
    uint64_t tail_lds[2];       // domains whose coarse grids fit in the coarse solver's LDS:
                                // [0] FP64 fields, [1] FP32 fields
};

// Kernel launchers (mg_kernels.hip).  `b0, nb` is a contiguous block range of one
// level; `mask` selects domains.
template <typename T>
struct K {
    // zero: the other colour is known to be zero and is not read.
    static void gsrb(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, int colour,
                     uint64_t mask, bool var, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool zero = false);
    static void ghost(const Launch &L, const Plane<T> &P, int b0, int nb, const int32_t *list,
                      int nlist, uint64_t mask, bool eps_field, bool cf_only);
    static void cf_ghost(const Launch &L, const Plane<T> &P, const int32_t *faces, int nfaces, uint64_t mask);
    static void restrict_down(const Launch &L, const Plane<T> &P, int lev, int b0, int nb,
                              uint64_t mask, int mode, bool var);
    static void fas(const Launch &L, const Plane<T> &P, int lev, const int32_t *list, int nlist,
                    uint64_t mask, bool var);
    // half: only colour 1 (and blocks with a physical face whole): a colour-0 half-sweep
    // follows on a level without coarse-fine faces
    static void correct(const Launch &L, const Plane<T> &P, int lev, int b0, int nb,
                        uint64_t mask, bool half = false);
    static void tail(const Launch &L, const Plane<T> &P, int mode, uint64_t mask,
                     const TailParams &tp, bool var);
    static void tail_eps(const Launch &L, const Plane<T> &P);
    static void zero(const Launch &L, T *p, size_t n);
    static void fill(const Launch &L, T *p, size_t n, T value);
    static void scatter(const Launch &L, T *dst, const double *src, int nleafblk);
    // uniform tail grids run as ordinary launches (large tail levels)
    static void ugsrb(const Launch &L, const Plane<T> &P, const UGrid &g, int colour, bool var);
    static void ughost(const Launch &L, const Plane<T> &P, const UGrid &g);
    static void ufas(const Launch &L, const Plane<T> &P, const UGrid &g, bool var);
    static void urestrict(const Launch &L, const Plane<T> &P, const UGrid &g, const UGrid &gc, bool var);
    static void ucorrect(const Launch &L, const Plane<T> &P, const UGrid &g, const UGrid &gc);
    // Weighted Jacobi step on one level's blocks: reads v (P.v, P.vg), writes dst, dstg.
    static void jacobi(const Launch &L, const Plane<T> &P, T *dst, T *dstg, int lev, int b0, int nb, uint64_t mask,
                       bool var, double omega);
    // Weighted Jacobi step on a large coarse grid: src -> dst (tail arrays).
    static void ujacobi(const Launch &L, const Plane<T> &P, const T *src, T *dst, const UGrid &g, bool var,
                        double omega);
    static void copy(const Launch &L, T *dst, const T *src, size_t n);
    static void gather(const Launch &L, const T *src, double *dst, int nleafblk);
};

enum { RESTRICT_FAS = 0, RESTRICT_V = 1, RESTRICT_EPS = 2 };
enum { TAIL_VCYCLE = 0, TAIL_FMG = 1 };

// Kernel attributes set once per process before any launch (large dynamic LDS of the
// coarse-grid kernel).
void prepare_kernels();
// LDS bytes the single-workgroup coarse solver has for a domain's grids.
int tail_lds_bytes();
// Device address, on the current device, of the fixed per-block reduction partials
// (looked up on first use per device); 0 on success.  Capacity in leaf blocks.
int static_partials(double **out);
int static_partial_blocks();

// FP64 composite residual over the leaf blocks; optionally writes r (cast) into rout.
void launch_norm64(const Launch &L, const Plane<double> &P, int nleafblk, bool var, float *rout32,
                   double *rout64);
// v += e on the leaf blocks, then the residual as launch_norm64 (trees without refinement).
void launch_add_norm64(const Launch &L, const Plane<double> &P, const float *e, const float *eg, int nleafblk,
                       bool var, float *rout32);
void launch_reduce_norms(const Launch &L);
void launch_add_leaf(const Launch &L, double *v64, double *vg64, const float *v32, int nleafblk);
// Krylov support on leaf vectors (rank-major: x[rank * cells_per_block + t]).
void launch_add_vec(const Launch &L, double *v64, double *vg64, const double *vec, int nleafblk);
template <typename S>
void launch_vec_blocks(const Launch &L, S *blk, double *vec, int nleafblk, bool to_blocks);
// blk -= vec on the leaf blocks (FP64; vec rank-major as above).
void launch_sub_vec_blocks(const Launch &L, double *blk, const double *vec, int nleafblk);
int dots_chunks(int64_t n);
// out[i] = <V_i, w> for i < k (V_i = V + i * stride); partial holds k * dots_chunks(n).
void launch_dots(const Launch &L, const double *V, int64_t stride, int k, const double *w, int64_t n,
                 double *partial, double *out);
// y = (overwrite ? 0 : y) + sign * sum_i coef[i] V_i (coef in device memory).
void launch_combo(const Launch &L, double *y, const double *V, int64_t stride, const double *coef, int k, double sign,
                  bool overwrite, int64_t n);
void launch_scale(const Launch &L, double *x, double a, int64_t n);
// Elliptic divergence cleaning on trees without refinement (leaf-ordered arrays, one
// component of B at a time): out (+)= dB_d/dx_d, central differences of order 2 or 4.
void launch_divb(const Launch &L, const double *Bd, double *out, int d, bool accumulate, int order,
                 int64_t nleaf_cells);
// B_d -= dphi/dx_d (second-order central differences of P.v with its ghosts); if e is
// set, e += (B_new^2 - B_old^2) / 2.
void launch_divb_project(const Launch &L, const Plane<double> &P, double *Bd, double *e, int d, int64_t nleaf_cells);
// Free-space boundaries (Sec. 2.8) on a 3D tree without refinement: per-domain geometry
// of the coarse charge grid, its boundary planes and the leaf boundary values.
struct FsDom {
    double lo[3], hi[3], h[3], hc[3];   // box, leaf and coarse spacing
    int32_t n[3], nc[3];                // leaf and coarse cells per axis
    int64_t qoff, poff, boff;           // this domain's charges, plane points, boundary values
    int64_t pofs[6], bofs[6];           // face offsets within the domain's planes / values
    int32_t npts;                       // plane points of the domain
    int32_t pad;
};
// Charges -> plane potentials (S slices of the charge rows, summed in a fixed order)
// -> boundary values folded into f (leaf blocks, in place); bv (may be null) receives
// the values.  partial holds S * total plane points.
void launch_freespace(const Launch &L, double *f, const FsDom *fd, int ndom, int max_pts, int64_t tot_pts,
                      int c, int slices, double *q, double *partial, double *pl, double *bv, int nleafblk);
// Far-field (monopole) potential of the coarse charges of f on the leaf cells, leaf
// order; q and mom (5 values per domain) are scratch.
void launch_freespace_guess(const Launch &L, const double *f, const FsDom *fd, int ndom, int c, double *q,
                            double *mom, double *out, int nleafblk, int64_t nleaf_cells);
void launch_face_gradient(const Launch &L, const Plane<double> &P, const double *lam_blocks,
                          const double *lam_g, double *out_leaf, int nleafblk);

// ------------------------------------------------------------------- host tree
struct HDomain {
    mg_domain d;
    int nblev;              // block levels of this domain (bs = block size), incl. refined
    int top;                // global level of the finest block level
    int base;               // global level of the unrefined grid
    int nblk_low[3];        // blocks per dim on the lowest block level
};

struct HBlock {
    int dom, lev;
    int bc[3];              // block coordinates on its level
    int parent;             // index into the builder's block vector, -1 for the lowest level
    int child[8];
    bool has_children;
    bool tested;
};

struct HostTree {
    int dim = 0, bs = 0, nt = 0, ndom = 0, nlev = 0;   // nlev: global levels
    std::vector<HDomain> doms;
    // final numbering
    std::vector<int32_t> org, nbr, cf, parent, dom, lev;
    std::vector<int32_t> leaf_blk, leaf_first;
    std::vector<int> lev_first;                 // [nlev+1] first block of every global level
    std::vector<std::vector<int32_t>> parents_of_level, cf_of_level;
    std::vector<double> h;                      // [ndom][MAXLEV][3]
    std::vector<int32_t> ncell;                 // [ndom][MAXLEV][3]
    std::vector<int64_t> tail_off;              // [ndom][MAXLEV]
    int64_t tail_cells = 0;                     // padded cells of every tail grid
    std::vector<int32_t> tail_top;              // [ndom] top level of the one-workgroup tail part
    int64_t nleaf_cells = 0;
    std::vector<int64_t> dom_leaf_cells;
    bool refined = false;                       // any block above a base level
};

// Builds the host tree; returns an empty string on success, else the error text.
std::string build_tree(HostTree &T, const mg_domain *doms, int ndom, int bs, int max_refine,
                       mg_refine_fn refine, void *ud);

}  // namespace mgx
