// HIP kernels (gfx950) of the multigrid library: red-black Gauss-Seidel with ghost
// push, ghost fill (same level, physical boundary, coarse-fine interpolation),
// residual + restriction, FAS right-hand side, prolongation + correction, the
// single-workgroup tail (reduced block sizes and the coarsest solve), norms,
// scatter/gather and the adjoint face gradient.
//
// All kernels are bandwidth-bound stencils (about one flop per byte), so they use no
// matrix cores.  Blocks store their interior split by colour so that a half-sweep
// reads only the other colour and writes only its own, with unit-stride access.
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdio>

#include <mutex>

#include "mg_internal.hpp"

namespace mgx {

// The coarsest solve stops once kStallSteps steps in a row have not lowered the
// max-norm residual below kStall times the lowest value reached so far (the rounding
// floor, or the two-value alternation of a one-cell Dirichlet grid; the residual of a
// slowly converging grid may rise for a few steps before it falls).
constexpr double kStall = 0.999;
constexpr int kStallSteps = 8;
// Coarsest grids of at most this many cells (one per lane) are iterated by one wave.
constexpr int kWaveCoarse = 64;
// FP32 levels with at least this many parent blocks take the LDS-staged FAS kernel
// (13.4 us against 17.5 at 512 blocks of 16^3; slower with 64: one workgroup per block
// leaves too few to hide the memory latency, and for FP64 its 45 KB per workgroup
// allow too few at once).
constexpr int kFasLdsMin = 256;

// Workgroups are dealt round-robin over the chip's 8 XCDs, each with its own L2.
// Workgroup w of a launch over n blocks takes block xcd_block(w, n): XCD x gets a
// contiguous run of the (Morton-ordered) blocks, so siblings that write halves of the
// same cache lines of their parent block (the restriction), or read them (the
// correction), run under one L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_block(int w, int n) {
    const int q = n >> 3, r = n & 7, x = w & 7;
    return x * q + (x < r ? x : r) + (w >> 3);
}

// ---------------------------------------------------------------- geometry
template <int D, int BS>
struct G {
    static constexpr int NC = D == 3 ? BS * BS * BS : BS * BS;   // cells per block
    static constexpr int NH = NC / 2;                            // cells per colour
    static constexpr int NF = D == 3 ? BS * BS : BS;             // ghosts per face
    static constexpr int NG = 2 * D * NF;                        // ghosts per block
    static constexpr int RH = BS / 2;                            // row length per colour
    // Interior offset of local cell (i,j,k): block origins are multiples of BS (even),
    // so the local index sum has the parity of the global one.
    __device__ __forceinline__ static int in(int i, int j, int k) {
        return ((i + j + k) & 1) * NH + (k * BS + j) * RH + (i >> 1);
    }
    // Ghost faces are split by colour too: on face f the cells whose global index sum
    // is even come first.  A ghost next to the lower face (f even) sits at local index
    // -1, next to the upper face at BS (even), so its parity is that of a1 + a2 (+1).
    __device__ __forceinline__ static int gpar(int f, int a1, int a2) { return (a1 + a2 + ((f & 1) ^ 1)) & 1; }
    __device__ __forceinline__ static int gh(int f, int a1, int a2) {
        return f * NF + gpar(f, a1, a2) * (NF / 2) + a2 * RH + (a1 >> 1);
    }
    // Decodes the colour-storage index t (0 <= t < NC) to local coordinates.
    __device__ __forceinline__ static void decode(int t, int &i, int &j, int &k) {
        int c = t >= NH;
        int q = t - c * NH;
        int row = q / RH;
        j = row % BS;
        k = row / BS;
        i = 2 * (q % RH) + ((j + k + c) & 1);
    }
};

// Value of local cell (i,j,k) of block b, at most one coordinate outside [0,BS).
template <int D, int BS, typename T>
__device__ __forceinline__ T ld(const T *__restrict__ v, const T *__restrict__ vg, int64_t b, int i,
                                int j, int k) {
    using g = G<D, BS>;
    if (i < 0) return vg[b * g::NG + g::gh(0, j, k)];
    if (i >= BS) return vg[b * g::NG + g::gh(1, j, k)];
    if (j < 0) return vg[b * g::NG + g::gh(2, i, k)];
    if (j >= BS) return vg[b * g::NG + g::gh(3, i, k)];
    if (D == 3) {
        if (k < 0) return vg[b * g::NG + g::gh(4, i, j)];
        if (k >= BS) return vg[b * g::NG + g::gh(5, i, j)];
    }
    return v[b * g::NC + g::in(i, j, k)];
}

// Address of local cell (i,j,k) of block b, at most one coordinate outside [0,BS).
template <int D, int BS, typename T>
__device__ __forceinline__ const T *ldp(const T *v, const T *vg, int64_t b, int i, int j, int k) {
    using g = G<D, BS>;
    if (i < 0) return vg + b * g::NG + g::gh(0, j, k);
    if (i >= BS) return vg + b * g::NG + g::gh(1, j, k);
    if (j < 0) return vg + b * g::NG + g::gh(2, i, k);
    if (j >= BS) return vg + b * g::NG + g::gh(3, i, k);
    if (D == 3) {
        if (k < 0) return vg + b * g::NG + g::gh(4, i, j);
        if (k >= BS) return vg + b * g::NG + g::gh(5, i, j);
    }
    return v + b * g::NC + g::in(i, j, k);
}

template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
    return T(2) * a * b / (a + b);
}

// Factors of the two x-face weights in the 2D axisymmetric form (x = r, finite volumes
// of (1/r) d/dr (r dphi/dr)): face radius over cell-centre radius, for the cell with
// global x index gi on a level of x spacing h (1 and 1 otherwise).
template <int D>
__device__ __forceinline__ void axi_factors(const DevTables &tb, int dm, double h, int gi, double &fm, double &fp) {
    fm = 1.0;
    fp = 1.0;
    if (D == 2 && tb.axi) {
        const double r = tb.lox[dm] + (gi + 0.5) * h;
        fm = (r - 0.5 * h) / r;
        fp = (r + 0.5 * h) / r;
    }
}

// ------------------------------------------------------- LDS staging helper
// Copies NRUN runs of LEN elements (run r at src + r * STRIDE) to dst + r * LEN with
// the widest aligned vector loads, all of a thread's loads issued before any store,
// so one workgroup's staging costs one memory latency instead of one per element.
template <int B> struct VecOf;
template <> struct VecOf<16> { using type = uint4; };
template <> struct VecOf<8> { using type = uint2; };
template <> struct VecOf<4> { using type = unsigned; };

template <typename T, int NRUN, int LEN, int STRIDE, int TPB>
struct Stager {
    static constexpr int BYTES = LEN * (int)sizeof(T);
    static constexpr int VB = BYTES % 16 == 0 ? 16 : (BYTES % 8 == 0 ? 8 : 4);
    using V = typename VecOf<VB>::type;
    static constexpr int CR = BYTES / VB;          // vectors per run
    static constexpr int NCH = NRUN * CR;
    static constexpr int IT = (NCH + TPB - 1) / TPB;
    V r[IT];
    // Loads are unconditional (a thread past the end re-reads the last vector) so
    // that none of them waits behind a branch.
    __device__ __forceinline__ void load(const T *src) {
#pragma unroll
        for (int m = 0; m < IT; m++) {
            int q = (int)threadIdx.x + m * TPB;
            if (NCH % TPB != 0) q = q < NCH ? q : NCH - 1;
            r[m] = reinterpret_cast<const V *>(src + (size_t)(q / CR) * STRIDE)[q % CR];
        }
    }
    __device__ __forceinline__ void store(T *dst) const {
#pragma unroll
        for (int m = 0; m < IT; m++) {
            const int q = (int)threadIdx.x + m * TPB;
            if (NCH % TPB == 0 || q < NCH) reinterpret_cast<V *>(dst + (q / CR) * LEN)[q % CR] = r[m];
        }
    }
};

// A thread's run of N consecutive values, moved with the widest aligned vectors (the
// run starts at a multiple of N values, and every array starts 256-byte aligned).
template <typename T, int N>
__device__ __forceinline__ void ld_run(const T *__restrict__ src, T (&dst)[N]) {
    constexpr int B = N * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; c++) reinterpret_cast<uint4 *>(dst)[c] = reinterpret_cast<const uint4 *>(src)[c];
    } else if constexpr (B % 8 == 0) {
#pragma unroll
        for (int c = 0; c < B / 8; c++) reinterpret_cast<uint2 *>(dst)[c] = reinterpret_cast<const uint2 *>(src)[c];
    } else {
#pragma unroll
        for (int m = 0; m < N; m++) dst[m] = src[m];
    }
}
template <typename T, int N>
__device__ __forceinline__ void st_run(T *__restrict__ dst, const T (&src)[N]) {
    constexpr int B = N * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; c++) reinterpret_cast<uint4 *>(dst)[c] = reinterpret_cast<const uint4 *>(src)[c];
    } else if constexpr (B % 8 == 0) {
#pragma unroll
        for (int c = 0; c < B / 8; c++) reinterpret_cast<uint2 *>(dst)[c] = reinterpret_cast<const uint2 *>(src)[c];
    } else {
#pragma unroll
        for (int m = 0; m < N; m++) dst[m] = src[m];
    }
}

struct Spacing {
    double ih2[3];
    double lam;   // Helmholtz term
    double hx;    // x spacing (axisymmetric factors, see axi_factors)
    int axi;
};

__device__ __forceinline__ Spacing spacing(const DevTables &tb, int dm, int lev) {
    const size_t o = ((size_t)dm * MAXLEV + lev) * 3;
    Spacing s;
    for (int a = 0; a < 3; a++) s.ih2[a] = tb.ih2[o + a];   // 1 / h^2, from the host
    s.lam = tb.lambda;
    s.axi = tb.axi;
    s.hx = tb.h[o];
    return s;
}

// (L v) and the Gauss-Seidel numerator/denominator at one cell of a block.
template <typename T, int D, int BS, bool VAR>
struct Stencil {
    T nb[6], w[6], vc, lam;
    __device__ __forceinline__ void load(const Plane<T> &P, int64_t b, int i, int j, int k,
                                         const Spacing &s, bool need_center, double rx = 0.0) {
        nb[0] = ld<D, BS>(P.v, P.vg, b, i - 1, j, k);
        nb[1] = ld<D, BS>(P.v, P.vg, b, i + 1, j, k);
        nb[2] = ld<D, BS>(P.v, P.vg, b, i, j - 1, k);
        nb[3] = ld<D, BS>(P.v, P.vg, b, i, j + 1, k);
        if (D == 3) {
            nb[4] = ld<D, BS>(P.v, P.vg, b, i, j, k - 1);
            nb[5] = ld<D, BS>(P.v, P.vg, b, i, j, k + 1);
        }
        vc = need_center ? P.v[b * G<D, BS>::NC + G<D, BS>::in(i, j, k)] : T(0);
        lam = T(s.lam);
        if (!VAR) {
            for (int f = 0; f < 2 * D; f++) w[f] = T(s.ih2[f / 2]);
        } else {
            T e0 = P.eps[b * G<D, BS>::NC + G<D, BS>::in(i, j, k)];
            T en[6];
            en[0] = ld<D, BS>(P.eps, P.epsg, b, i - 1, j, k);
            en[1] = ld<D, BS>(P.eps, P.epsg, b, i + 1, j, k);
            en[2] = ld<D, BS>(P.eps, P.epsg, b, i, j - 1, k);
            en[3] = ld<D, BS>(P.eps, P.epsg, b, i, j + 1, k);
            if (D == 3) {
                en[4] = ld<D, BS>(P.eps, P.epsg, b, i, j, k - 1);
                en[5] = ld<D, BS>(P.eps, P.epsg, b, i, j, k + 1);
            }
            for (int f = 0; f < 2 * D; f++) w[f] = harm(e0, en[f]) * T(s.ih2[f / 2]);
        }
        if (D == 2 && s.axi) {   // rx: radius of this cell's centre
            w[0] *= T((rx - 0.5 * s.hx) / rx);
            w[1] *= T((rx + 0.5 * s.hx) / rx);
        }
    }
    __device__ __forceinline__ T Lv() const {
        T s = T(0);
        for (int f = 0; f < 2 * D; f++) s += w[f] * (nb[f] - vc);
        return s - lam * vc;
    }
    __device__ __forceinline__ T gs(T fval) const {
        T num = T(0), den = lam;
        for (int f = 0; f < 2 * D; f++) {
            num += w[f] * nb[f];
            den += w[f];
        }
        return (num - fval) / den;
    }
};

// Physical boundary ghost from the adjacent interior value (Sec. 2.6).
template <typename T>
__device__ __forceinline__ T bc_ghost(int kind, double a, double h, int side, T inner) {
    if (kind == MG_BC_DIRICHLET) return T(2.0 * a) - inner;
    return inner + T((side ? 1.0 : -1.0) * h * a);
}

// ------------------------------------------------------------ ghost push
// After a cell of block b changes, the ghost that mirrors it is written: the
// neighbour block's ghost on a same-level face, the block's own ghost (boundary
// condition applied) on a physical face.  Coarse-fine ghosts depend on several fine
// cells and coarse data; a separate launch refreshes them.
template <typename T, int D, int BS>
__device__ __forceinline__ void push_ghosts(T *__restrict__ vg, const DevTables &tb, int64_t b, int dm,
                                            const double *hh, int i, int j, int k, T nv) {
    using g = G<D, BS>;
    const int coord[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < D; a++) {
        int side;
        if (coord[a] == 0) side = 0;
        else if (coord[a] == BS - 1) side = 1;
        else continue;
        const int f = 2 * a + side;
        const int a1 = a == 0 ? j : i, a2 = a == 2 ? j : k;
        const int n = tb.nbr[6 * b + f];
        if (n >= 0) vg[(int64_t)n * g::NG + g::gh(f ^ 1, a1, a2)] = nv;
        else if (n == -1) vg[b * g::NG + g::gh(f, a1, a2)] = bc_ghost<T>(tb.bck[6 * dm + f], tb.bcv[6 * dm + f], hh[a], side, nv);
    }
}

// Per-block data every block kernel needs (domain, neighbours, spacing, boundary
// conditions), read with scalar loads at kernel start so that they travel together
// with the first data loads instead of forming a chain of dependent round trips.
template <int D>
struct BlockCtx {
    int dm, orgx;
    int nbr[6];
    double h[3];
    int bck[6];
    double bcv[6];
    __device__ __forceinline__ void load(const DevTables &tb, int64_t b, int lev) {
        dm = tb.dom[b];
        orgx = tb.org[3 * b];
#pragma unroll
        for (int f = 0; f < 2 * D; f++) nbr[f] = tb.nbr[6 * b + f];
        const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
#pragma unroll
        for (int a = 0; a < D; a++) h[a] = hh[a];
#pragma unroll
        for (int f = 0; f < 2 * D; f++) {
            bck[f] = tb.bck[6 * dm + f];
            bcv[f] = tb.bcv[6 * dm + f];
        }
    }
};

// push_ghosts with the block's data preloaded.
template <typename T, int D, int BS>
__device__ __forceinline__ void push_ghosts(T *__restrict__ vg, const BlockCtx<D> &c, int64_t b, int i, int j,
                                            int k, T nv) {
    using g = G<D, BS>;
    const int coord[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < D; a++) {
        int side;
        if (coord[a] == 0) side = 0;
        else if (coord[a] == BS - 1) side = 1;
        else continue;
        const int f = 2 * a + side;
        const int a1 = a == 0 ? j : i, a2 = a == 2 ? j : k;
        // selects, not a run-time array index (which would live in scratch memory)
        const int n = side ? c.nbr[2 * a + 1] : c.nbr[2 * a];
        if (n >= 0) {
            vg[(int64_t)n * g::NG + g::gh(f ^ 1, a1, a2)] = nv;
        } else if (n == -1) {
            const int kind = side ? c.bck[2 * a + 1] : c.bck[2 * a];
            const double val = side ? c.bcv[2 * a + 1] : c.bcv[2 * a];
            vg[b * g::NG + g::gh(f, a1, a2)] = bc_ghost<T>(kind, val, c.h[a], side, nv);
        }
    }
}

// push_ghosts for a run of IT cells of one colour in one row (cells i0, i0 + 2, ...):
// on a y or z face the run's mirroring ghosts are consecutive slots of the face, written
// as one vector; only the run's first or last cell can lie on an x face.
template <typename T, int D, int BS, int IT>
__device__ __forceinline__ void push_run(T *__restrict__ vg, const BlockCtx<D> &c, int64_t b, int i0, int j, int k,
                                         const T (&nv)[IT]) {
    using g = G<D, BS>;
    // x faces
    if (i0 == 0 || i0 + 2 * (IT - 1) == BS - 1) {
        const int side = i0 == 0 ? 0 : 1;
        const T x = side ? nv[IT - 1] : nv[0];   // selects, not a run-time index (scratch)
        const int n = side ? c.nbr[1] : c.nbr[0];
        if (n >= 0) {
            vg[(int64_t)n * g::NG + g::gh(side ^ 1, j, k)] = x;
        } else if (n == -1) {
            const int kind = side ? c.bck[1] : c.bck[0];
            const double val = side ? c.bcv[1] : c.bcv[0];
            vg[b * g::NG + g::gh(side, j, k)] = bc_ghost<T>(kind, val, c.h[0], side, x);
        }
    }
    // y and z faces: the tangential coordinates are (i, k) and (i, j)
#pragma unroll
    for (int a = 1; a < D; a++) {
        const int coord = a == 1 ? j : k;
        int side;
        if (coord == 0) side = 0;
        else if (coord == BS - 1) side = 1;
        else continue;
        const int f = 2 * a + side, a2 = a == 2 ? j : k;
        const int n = side ? c.nbr[2 * a + 1] : c.nbr[2 * a];
        if (n >= 0) {
            st_run<T, IT>(vg + (int64_t)n * g::NG + g::gh(f ^ 1, i0, a2), nv);
        } else if (n == -1) {
            const int kind = side ? c.bck[2 * a + 1] : c.bck[2 * a];
            const double val = side ? c.bcv[2 * a + 1] : c.bcv[2 * a];
            T gv[IT];
#pragma unroll
            for (int m = 0; m < IT; m++) gv[m] = bc_ghost<T>(kind, val, c.h[a], side, nv[m]);
            st_run<T, IT>(vg + b * g::NG + g::gh(f, i0, a2), gv);
        }
    }
}

// ------------------------------------------------------------ GS-RB sweep
// One colour of red-black Gauss-Seidel (Sec. 2.2) for the blocks of one level, one
// workgroup per block.  The other colour of the block and the other-colour halves of
// its ghost faces are staged in LDS (each value read once from HBM, unit stride);
// each thread then updates cells of this colour, reading f and writing v with unit
// stride, and pushes boundary values into the mirroring ghosts.  A ghost position has
// the colour of the cell it mirrors, so the sweep never reads what it writes.
// SPLIT > 1 (levels with few blocks): SPLIT workgroups share a block, each stages the
// whole other colour and updates 1/SPLIT of the cells, which shortens every workgroup's
// serial part.  The parts of a block are nb workgroups apart: with nb a multiple of 8
// they run on the same XCD (workgroups go round-robin over the 8 XCDs), so the repeated
// staging reads hit that XCD's L2.
// ZERO: the other colour and its ghosts are known to be zero (the first half-sweep of a
// correction solve from e = 0, homogeneous boundary values), so they are not read, and
// this colour's ghosts on physical faces are set to zero for the next half-sweep.
// WIDE = 2 (levels of a few hundred blocks): 512-thread workgroups, twice the waves per
// CU for the same block count.
template <typename T, int D, int BS, bool VAR, int SPLIT, bool ZERO, int WIDE = 1>
__global__ void __launch_bounds__(256 * WIDE) k_gsrb(Plane<T> P, DevTables tb, int lev, int b0, int colour,
                                                     uint64_t mask) {
    using g = G<D, BS>;
    constexpr int TPB = (g::NH < 256 ? g::NH : 256) * WIDE;
    constexpr int HF = g::NF / 2;               // ghosts of one colour per face
    constexpr int NGH = 2 * D * HF;
    constexpr int IT = g::NH / TPB / SPLIT;
    static_assert(IT >= 1, "SPLIT too large for this block size");
    __shared__ __align__(16) T s_o[g::NH];
    __shared__ __align__(16) T s_g[NGH];
    __shared__ __align__(16) T s_eo[VAR ? g::NH : 1];
    __shared__ __align__(16) T s_eg[VAR ? NGH : 1];
    const int nbl = gridDim.x / SPLIT;
    const int64_t b = b0 + (SPLIT == 1 ? (int)blockIdx.x : (int)blockIdx.x % nbl);
    const int q0 = SPLIT == 1 ? 0 : (blockIdx.x / nbl) * IT * TPB;   // first cell of this part
    const int oc = colour ^ 1;
    const int tid = threadIdx.x;
    // issue every load of this thread first: other colour, its ghosts, own f (and eps),
    // the block's tables; a block of a domain outside the mask leaves after staging
    Stager<T, 1, g::NH, 0, TPB> st_o;
    Stager<T, 2 * D, HF, g::NF, TPB> st_g;
    if (!ZERO) {
        st_o.load(P.v + b * g::NC + oc * g::NH);
        st_g.load(P.vg + b * g::NG + oc * HF);
    }
    // each thread updates IT consecutive cells of this colour: f (and eps) are read and
    // v written as vectors
    const int qt = q0 + tid * IT;
    T fr[IT], er[VAR ? IT : 1];
    ld_run<T, IT>(P.f + b * g::NC + colour * g::NH + qt, fr);
    Stager<T, 1, VAR ? g::NH : 8, 0, TPB> st_eo;
    Stager<T, 2 * D, VAR ? HF : 8, g::NF, TPB> st_eg;
    if (VAR) {
        st_eo.load(P.eps + b * g::NC + oc * g::NH);
        st_eg.load(P.epsg + b * g::NG + oc * HF);
        if constexpr (VAR) ld_run<T, IT>(P.eps + b * g::NC + colour * g::NH + qt, er);
    }
    BlockCtx<D> cx;
    cx.load(tb, b, lev);
    if (!ZERO) {
        st_o.store(s_o);
        st_g.store(s_g);
    } else {
        // (the other colour is zero: it is neither staged nor read below)
        // On a physical face the ghosts of this colour mirror cells of the other colour
        // (zero), so with the homogeneous boundary values of a correction solve they are
        // zero as well; the next half-sweep reads them.
        unsigned phys = 0;
#pragma unroll
        for (int f = 0; f < 2 * D; f++) phys |= (cx.nbr[f] == -1 ? 1u : 0u) << f;
        if (phys && q0 == 0)
            for (int q = tid; q < NGH; q += TPB) {
                const int f = q / HF;
                if ((phys >> f) & 1) P.vg[b * g::NG + f * g::NF + colour * HF + (q - f * HF)] = T(0);
            }
    }
    if (VAR) {
        st_eo.store(s_eo);
        st_eg.store(s_eg);
    }
    if (!ZERO || VAR) __syncthreads();   // nothing is staged in the zero form without eps
    if (!((mask >> cx.dm) & 1)) return;
    T ih2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) ih2[a] = a < D ? T(1.0 / (cx.h[a] * cx.h[a])) : T(0);
    // constant coefficient (Cartesian): one diagonal for the whole block, so one
    // reciprocal in place of a division per cell
    T dconst = T(tb.lambda);
#pragma unroll
    for (int a = 0; a < D; a++) dconst += T(2) * ih2[a];
    const T inv_d = T(1) / dconst;
    const bool recip = !VAR && !(D == 2 && tb.axi);
    T nvs[IT];
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int q = qt + m;
        const int row = q / g::RH, pos = q % g::RH;
        const int j = row % BS, k = D == 3 ? row / BS : 0;
        const int i = 2 * pos + ((j + k + colour) & 1);
        // neighbour offsets in the other-colour arrays (interior or ghost half)
        int off[6];
        bool gho[6];
        gho[0] = i == 0;      off[0] = gho[0] ? 0 * HF + k * g::RH + (j >> 1) : row * g::RH + ((i - 1) >> 1);
        gho[1] = i == BS - 1; off[1] = gho[1] ? 1 * HF + k * g::RH + (j >> 1) : row * g::RH + ((i + 1) >> 1);
        gho[2] = j == 0;      off[2] = gho[2] ? 2 * HF + k * g::RH + (i >> 1) : (row - 1) * g::RH + (i >> 1);
        gho[3] = j == BS - 1; off[3] = gho[3] ? 3 * HF + k * g::RH + (i >> 1) : (row + 1) * g::RH + (i >> 1);
        if (D == 3) {
            gho[4] = k == 0;      off[4] = gho[4] ? 4 * HF + j * g::RH + (i >> 1) : (row - BS) * g::RH + (i >> 1);
            gho[5] = k == BS - 1; off[5] = gho[5] ? 5 * HF + j * g::RH + (i >> 1) : (row + BS) * g::RH + (i >> 1);
        }
        T num = T(0), den = T(tb.lambda);
        const T fval = fr[m];
        double fm, fp;
        axi_factors<D>(tb, cx.dm, cx.h[0], cx.orgx + i, fm, fp);
        // the other colour's value across face f (zero in the zero form)
        auto nbv = [&](int f) -> T { return ZERO ? T(0) : (gho[f] ? s_g[off[f]] : s_o[off[f]]); };
        if (!VAR) {
            if (D == 2 && tb.axi) {
                num += ih2[0] * (T(fm) * nbv(0) + T(fp) * nbv(1));
#pragma unroll
                for (int f = 2; f < 2 * D; f++) num += ih2[f >> 1] * nbv(f);
            } else {
#pragma unroll
                for (int f = 0; f < 2 * D; f++) num += ih2[f >> 1] * nbv(f);
            }
#pragma unroll
            for (int a = 0; a < D; a++) den += T(2) * ih2[a];
        } else {
            const T e0 = er[VAR ? m : 0];
#pragma unroll
            for (int f = 0; f < 2 * D; f++) {
                const T en = gho[f] ? s_eg[off[f]] : s_eo[off[f]];
                T w = harm(e0, en) * ih2[f >> 1];
                if (f == 0) w *= T(fm);
                if (f == 1) w *= T(fp);
                num += w * nbv(f);
                den += w;
            }
        }
        nvs[m] = recip ? (num - fval) * inv_d : (num - fval) / den;
    }
    st_run<T, IT>(P.v + b * g::NC + colour * g::NH + qt, nvs);
    static_assert(g::RH % IT == 0, "a run lies in one row");
    {
        const int row = qt / g::RH, pos = qt % g::RH;
        const int j = row % BS, k = D == 3 ? row / BS : 0;
        push_run<T, D, BS, IT>(P.vg, cx, b, 2 * pos + ((j + k + colour) & 1), j, k, nvs);
    }
}

// ------------------------------------------------------ weighted Jacobi step
// Every cell of the level's blocks moves the fraction omega of the way to its
// Gauss-Seidel local solution computed from the values before the step (the smoother of
// the paper's timing runs, Sec. 3.3).  Reads v (P.v, P.vg), writes dst and pushes the
// mirroring ghosts into dstg; one workgroup per block, the block and its ghosts staged
// in LDS.
template <typename T, int D, int BS, bool VAR>
__global__ void __launch_bounds__(256) k_jacobi(Plane<T> P, T *__restrict__ dst, T *__restrict__ dstg, DevTables tb,
                                                int lev, int b0, uint64_t mask, double omega) {
    using g = G<D, BS>;
    constexpr int TPB = g::NC < 256 ? g::NC : 256;
    constexpr int IT = g::NC / TPB;
    __shared__ __align__(16) T s_v[g::NC + g::NG];
    const int64_t b = b0 + blockIdx.x;
    const int tid = threadIdx.x;
    Stager<T, 1, g::NC, 0, TPB> st_v;
    Stager<T, 1, g::NG, 0, TPB> st_g;
    st_v.load(P.v + b * g::NC);
    st_g.load(P.vg + b * g::NG);
    T fr[IT];
#pragma unroll
    for (int m = 0; m < IT; m++) fr[m] = P.f[b * g::NC + tid + m * TPB];
    BlockCtx<D> cx;
    cx.load(tb, b, lev);
    st_v.store(s_v);
    st_g.store(s_v + g::NC);
    __syncthreads();
    if (!((mask >> cx.dm) & 1)) return;
    T ih2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) ih2[a] = a < D ? T(1.0 / (cx.h[a] * cx.h[a])) : T(0);
    const T om = T(omega);
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int t = tid + m * TPB;
        int i, j, k;
        g::decode(t, i, j, k);
        const T vc = s_v[t];
        T nb[6];
        nb[0] = i > 0 ? s_v[g::in(i - 1, j, k)] : s_v[g::NC + g::gh(0, j, k)];
        nb[1] = i < BS - 1 ? s_v[g::in(i + 1, j, k)] : s_v[g::NC + g::gh(1, j, k)];
        nb[2] = j > 0 ? s_v[g::in(i, j - 1, k)] : s_v[g::NC + g::gh(2, i, k)];
        nb[3] = j < BS - 1 ? s_v[g::in(i, j + 1, k)] : s_v[g::NC + g::gh(3, i, k)];
        if (D == 3) {
            nb[4] = k > 0 ? s_v[g::in(i, j, k - 1)] : s_v[g::NC + g::gh(4, i, j)];
            nb[5] = k < BS - 1 ? s_v[g::in(i, j, k + 1)] : s_v[g::NC + g::gh(5, i, j)];
        }
        T num = T(0), den = T(tb.lambda);
        double fm, fp;
        axi_factors<D>(tb, cx.dm, cx.h[0], cx.orgx + i, fm, fp);
        if (!VAR) {
            // the axisymmetric x-face factors sum to 2: the diagonal is unchanged
            const T nx0 = D == 2 && tb.axi ? T(fm) * nb[0] : nb[0], nx1 = D == 2 && tb.axi ? T(fp) * nb[1] : nb[1];
            num += ih2[0] * nx0;
            num += ih2[0] * nx1;
            den += ih2[0];
            den += ih2[0];
#pragma unroll
            for (int f = 2; f < 2 * D; f++) {
                num += ih2[f >> 1] * nb[f];
                den += ih2[f >> 1];
            }
        } else {
            const T e0 = P.eps[b * g::NC + t];
            T en[6];
            en[0] = ld<D, BS>(P.eps, P.epsg, b, i - 1, j, k);
            en[1] = ld<D, BS>(P.eps, P.epsg, b, i + 1, j, k);
            en[2] = ld<D, BS>(P.eps, P.epsg, b, i, j - 1, k);
            en[3] = ld<D, BS>(P.eps, P.epsg, b, i, j + 1, k);
            if (D == 3) {
                en[4] = ld<D, BS>(P.eps, P.epsg, b, i, j, k - 1);
                en[5] = ld<D, BS>(P.eps, P.epsg, b, i, j, k + 1);
            }
#pragma unroll
            for (int f = 0; f < 2 * D; f++) {
                T w = harm(e0, en[f]) * ih2[f >> 1];
                if (f == 0) w *= T(fm);
                if (f == 1) w *= T(fp);
                num += w * nb[f];
                den += w;
            }
        }
        const T gs = (num - fr[m]) / den;
        const T nv = vc + om * (gs - vc);
        dst[b * g::NC + t] = nv;
        push_ghosts<T, D, BS>(dstg, cx, b, i, j, k, nv);
    }
}

// -------------------------------------------------------------- ghost fill
// Fills the face ghosts of a block (Sec. 2.6).  Same-level faces copy the
// neighbour's boundary cell; physical faces apply the boundary condition; coarse-fine
// faces take g = (B' + c')/2 with B' the coarse cell value moved to the ghost's
// tangential position by the central-difference slope(s) of the coarse cell and
// c' = (3c - c2)/2 the two-point extrapolation of the fine cells to the face.  For the
// eps field: copy, copy of the interior cell, and the coarse cell's value.
// Coarse-fine ghost (face f of block b at level lv of domain dm, tangential position
// a1, a2; qb the coarse block across the face, org the block's origin): the coarse cell
// B moved to the ghost's tangential position by the central differences of the coarse
// values, averaged with the two-point extrapolation (3c - c2)/2 of the fine cells c, c2
// next to the face (Sec. 2.6, refinement boundaries).  For eps: the coarse cell.
template <typename T, int D, int BS, bool EPS>
__device__ __forceinline__ T cf_ghost_value(const Plane<T> &P, const DevTables &tb, int64_t b, int f, int a1,
                                            int a2, int dm, int lv, int64_t qb, const int org[3]) {
    using g = G<D, BS>;
    const T *v = EPS ? P.eps : P.v;
    const int a = f >> 1, side = f & 1;
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    int in1[3], in2[3];
    in1[t1] = a1; in1[t2] = a2; in1[a] = side ? BS - 1 : 0;
    in2[t1] = a1; in2[t2] = a2; in2[a] = side ? BS - 2 : 1;
    if (D == 2) { in1[2] = 0; in2[2] = 0; }
    T out;
    int gi[3];
    for (int c = 0; c < 3; c++) gi[c] = org[c] + in1[c];
    gi[a] += side ? 1 : -1;
    // wrap across a periodic face (the coarse region may lie beyond it)
    const int32_t *nc = tb.ncell + ((size_t)dm * MAXLEV + lv) * 3;
    if (gi[a] < 0) gi[a] += nc[a];
    if (gi[a] >= nc[a]) gi[a] -= nc[a];
    int cl[3];
    for (int c = 0; c < 3; c++) cl[c] = (gi[c] >> 1) - tb.org[3 * qb + c];
    if (D == 2) cl[2] = 0;
    const T *w = EPS ? P.eps : (P.vc ? P.vc : P.v);
    const T *wg = EPS ? P.epsg : (P.vcg ? P.vcg : P.vg);
    T B = w[qb * g::NC + g::in(cl[0], cl[1], cl[2])];
    if (EPS) {
        out = B;
    } else {
        T Bp = B;
        int tang[2] = {t1, t2};
#pragma unroll
        for (int m = 0; m < D - 1; m++) {
            int td = tang[m];
            T sigma = (gi[td] & 1) ? T(1) : T(-1);
            int cp[3] = {cl[0], cl[1], cl[2]}, cm[3] = {cl[0], cl[1], cl[2]};
            cp[td] += 1;
            cm[td] -= 1;
            T up = ld<D, BS>(w, wg, qb, cp[0], cp[1], cp[2]);
            T dn = ld<D, BS>(w, wg, qb, cm[0], cm[1], cm[2]);
            Bp += sigma * (up - dn) / T(8);
        }
        T c = v[b * g::NC + g::in(in1[0], in1[1], in1[2])];
        T c2 = v[b * g::NC + g::in(in2[0], in2[1], in2[2])];
        out = T(0.5) * (Bp + (T(1.5) * c - T(0.5) * c2));
    }
    return out;
}

template <typename T, int D, int BS, bool EPS>
__device__ void ghost_cell(const Plane<T> &P, const DevTables &tb, int64_t b, int f, int a1, int a2,
                           bool cf_only) {
    using g = G<D, BS>;
    T *v = EPS ? P.eps : P.v;
    T *vg = EPS ? P.epsg : P.vg;
    const int a = f >> 1, side = f & 1;
    const int n = tb.nbr[6 * b + f];
    if (cf_only && n != -2) return;
    int in1[3];
    // tangential axes in increasing order
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    in1[t1] = a1; in1[t2] = a2; in1[a] = side ? BS - 1 : 0;
    if (D == 2) in1[2] = 0;
    T out;
    if (n >= 0) {
        int q[3] = {in1[0], in1[1], in1[2]};
        q[a] = side ? 0 : BS - 1;
        out = v[(int64_t)n * g::NC + g::in(q[0], q[1], q[2])];
    } else if (n == -1) {
        const int dm = tb.dom[b];
        T ci = v[b * g::NC + g::in(in1[0], in1[1], in1[2])];
        if (EPS) {
            out = ci;
        } else {
            const double *hh = tb.h + ((size_t)dm * MAXLEV + tb.lev[b]) * 3;
            double bv = tb.bcv[6 * dm + f];
            if (tb.fv_off) {
                const int64_t o = tb.fv_off[6 * b + f];
                if (o >= 0) bv = tb.fv[o + (D == 3 ? a2 * BS : 0) + a1];
            }
            out = bc_ghost<T>(tb.bck[6 * dm + f], bv, hh[a], side, ci);
        }
    } else {
        const int org[3] = {tb.org[3 * b], tb.org[3 * b + 1], tb.org[3 * b + 2]};
        out = cf_ghost_value<T, D, BS, EPS>(P, tb, b, f, a1, a2, tb.dom[b], tb.lev[b], tb.cf[6 * b + f], org);
    }
    vg[b * g::NG + g::gh(f, a1, a2)] = out;
}

template <typename T, int D, int BS, bool EPS>
__global__ void __launch_bounds__(256) k_ghost(Plane<T> P, DevTables tb, int b0, const int32_t *list,
                                               uint64_t mask, int cf_only) {
    using g = G<D, BS>;
    const int64_t b = list ? list[blockIdx.x] : b0 + blockIdx.x;
    if (!((mask >> tb.dom[b]) & 1)) return;
    for (int t = threadIdx.x; t < g::NG; t += (g::NG < 256 ? g::NG : 256)) {
        int f = t / g::NF, r = t % g::NF;
        ghost_cell<T, D, BS, EPS>(P, tb, b, f, r % BS, r / BS, cf_only != 0);
    }
}

// Coarse-fine ghosts of a list of (block, face) pairs (entry 8 b + f), one ghost cell
// per thread: every thread issues its table loads at once and no thread idles on a
// face without a coarse neighbour.
template <typename T, int D, int BS>
__global__ void __launch_bounds__(256) k_cf_ghost(Plane<T> P, DevTables tb, const int32_t *faces, int nfaces,
                                                  uint64_t mask) {
    using g = G<D, BS>;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nfaces * g::NF) return;
    const int32_t e = faces[t / g::NF];
    const int64_t b = e >> 3;
    const int f = e & 7;
    const int r = (int)(t % g::NF);
    const int dm = tb.dom[b], lv = tb.lev[b];
    const int64_t qb = tb.cf[6 * b + f];
    const int org[3] = {tb.org[3 * b], tb.org[3 * b + 1], tb.org[3 * b + 2]};
    const T out = cf_ghost_value<T, D, BS, false>(P, tb, b, f, r % BS, r / BS, dm, lv, qb, org);
    if ((mask >> dm) & 1) P.vg[b * g::NG + g::gh(f, r % BS, r / BS)] = out;
}

// ------------------------------------------------------ tail grid indexing
struct TailGeo {
    int n[3];
    int64_t off;
    __device__ __forceinline__ int64_t idx(int i, int j, int k, int dim) const {
        if (dim == 2) return off + (int64_t)(j + 1) * (n[0] + 2) + (i + 1);
        return off + ((int64_t)(k + 1) * (n[1] + 2) + (j + 1)) * (n[0] + 2) + (i + 1);
    }
};

__device__ __forceinline__ TailGeo tail_geo(const DevTables &tb, int dm, int lev, int dim) {
    TailGeo t;
    const int32_t *nc = tb.ncell + ((size_t)dm * MAXLEV + lev) * 3;
    t.n[0] = nc[0]; t.n[1] = nc[1]; t.n[2] = dim == 3 ? nc[2] : 1;
    t.off = tb.tail_off[(size_t)dm * MAXLEV + lev];
    return t;
}

// ----------------------------------------------- residual + restriction
// For every coarse cell under a block of level `lev`: the mean of its 2^d fine values
// (restriction, Sec. 2.3) of v, and in the FAS mode also of r = f - L v, written to
// the parent block (v, and R(r) into f) or to the domain's top tail grid.  One
// workgroup per fine block; for the FAS mode the block's v with its ghosts is staged
// in LDS.  Parent boundary values are pushed into the mirroring ghosts of the parent
// level, so no separate ghost fill is needed before the FAS right-hand side.  Mode
// RESTRICT_EPS restricts the coefficient instead (no push).
template <typename T, int D, int BS, bool VAR, int MODE>
__global__ void __launch_bounds__(256) k_restrict(Plane<T> P, DevTables tb, int lev, int b0,
                                                  uint64_t mask, int nt) {
    using g = G<D, BS>;
    constexpr int HB = BS / 2;
    constexpr int NQ = D == 3 ? HB * HB * HB : HB * HB;
    constexpr int TPB = NQ < 256 ? NQ : 256;
    constexpr bool FAS = MODE == RESTRICT_FAS;
    constexpr int IT = (NQ + TPB - 1) / TPB;
    __shared__ __align__(16) T s_v[FAS ? g::NC + g::NG : 4];
    const int64_t b = b0 + xcd_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    // tables first (independent loads): domain, parent, origin; the parent's
    // neighbours follow once the parent is known
    const int dm = tb.dom[b];
    const int64_t p = tb.parent[b];
    const int ob[3] = {tb.org[3 * b], tb.org[3 * b + 1], tb.org[3 * b + 2]};
    BlockCtx<D> px;
    if (MODE != RESTRICT_EPS && p >= 0) px.load(tb, p, lev - 1);
    // fine values of this thread's coarse cells (the field itself, or f for FAS)
    const T *src = MODE == RESTRICT_EPS ? P.eps : (FAS ? P.f : P.v);
    T pre[IT][1 << D];
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int t = (NQ % TPB == 0 || tid + m * TPB < NQ) ? tid + m * TPB : 0;
        const int ci = t % HB, cj = (t / HB) % HB, ck = D == 3 ? t / (HB * HB) : 0;
#pragma unroll
        for (int q = 0; q < (1 << D); q++)
            pre[m][q] = src[b * g::NC + g::in(2 * ci + (q & 1), 2 * cj + ((q >> 1) & 1), D == 3 ? 2 * ck + (q >> 2) : 0)];
    }
    if (FAS) {
        Stager<T, 1, g::NC, 0, TPB> st_v;
        Stager<T, 1, g::NG, 0, TPB> st_g;
        st_v.load(P.v + b * g::NC);
        st_g.load(P.vg + b * g::NG);
        st_v.store(s_v);
        st_g.store(s_v + g::NC);
        __syncthreads();
    }
    if (!((mask >> dm) & 1)) return;
    const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
    T ih2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) ih2[a] = T(1.0 / (hh[a] * hh[a]));
    // offset of this block's octant in its parent
    int po[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) po[a] = ((ob[a] / BS) & 1) * HB;
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int t = tid + m * TPB;
        if (NQ % TPB != 0 && t >= NQ) break;
        const int ci = t % HB, cj = (t / HB) % HB, ck = D == 3 ? t / (HB * HB) : 0;
        T sv = T(0), sr = T(0);
#pragma unroll
        for (int q = 0; q < (1 << D); q++) {
            const int i = 2 * ci + (q & 1), j = 2 * cj + ((q >> 1) & 1), k = D == 3 ? 2 * ck + (q >> 2) : 0;
            const int c = g::in(i, j, k);
            if (!FAS) {
                sv += pre[m][q];
            } else {
                const T vc = s_v[c];
                sv += vc;
                T nb[6];
                nb[0] = i > 0 ? s_v[g::in(i - 1, j, k)] : s_v[g::NC + g::gh(0, j, k)];
                nb[1] = i < BS - 1 ? s_v[g::in(i + 1, j, k)] : s_v[g::NC + g::gh(1, j, k)];
                nb[2] = j > 0 ? s_v[g::in(i, j - 1, k)] : s_v[g::NC + g::gh(2, i, k)];
                nb[3] = j < BS - 1 ? s_v[g::in(i, j + 1, k)] : s_v[g::NC + g::gh(3, i, k)];
                if (D == 3) {
                    nb[4] = k > 0 ? s_v[g::in(i, j, k - 1)] : s_v[g::NC + g::gh(4, i, j)];
                    nb[5] = k < BS - 1 ? s_v[g::in(i, j, k + 1)] : s_v[g::NC + g::gh(5, i, j)];
                }
                T lv = T(0);
                if (D == 2 && tb.axi) {   // axisymmetric x-face factors (see axi_factors)
                    double fm, fp;
                    axi_factors<D>(tb, dm, hh[0], ob[0] + i, fm, fp);
                    nb[0] = vc + T(fm) * (nb[0] - vc);
                    nb[1] = vc + T(fp) * (nb[1] - vc);
                }
                if (!VAR) {
#pragma unroll
                    for (int f = 0; f < 2 * D; f++) lv += ih2[f >> 1] * (nb[f] - vc);
                } else {
                    const T e0 = P.eps[b * g::NC + c];
                    T en[6];
                    en[0] = ld<D, BS>(P.eps, P.epsg, b, i - 1, j, k);
                    en[1] = ld<D, BS>(P.eps, P.epsg, b, i + 1, j, k);
                    en[2] = ld<D, BS>(P.eps, P.epsg, b, i, j - 1, k);
                    en[3] = ld<D, BS>(P.eps, P.epsg, b, i, j + 1, k);
                    if (D == 3) {
                        en[4] = ld<D, BS>(P.eps, P.epsg, b, i, j, k - 1);
                        en[5] = ld<D, BS>(P.eps, P.epsg, b, i, j, k + 1);
                    }
#pragma unroll
                    for (int f = 0; f < 2 * D; f++) lv += harm(e0, en[f]) * ih2[f >> 1] * (nb[f] - vc);
                }
                lv -= T(tb.lambda) * vc;
                sr += pre[m][q] - lv;
            }
        }
        const T inv = T(1) / T(1 << D);
        sv *= inv;
        sr *= inv;
        const int gc[3] = {(ob[0] >> 1) + ci, (ob[1] >> 1) + cj, D == 3 ? (ob[2] >> 1) + ck : 0};
        if (p >= 0) {
            const int l0 = po[0] + ci, l1 = po[1] + cj, l2 = D == 3 ? po[2] + ck : 0;
            const int64_t o = p * g::NC + g::in(l0, l1, l2);
            if (MODE == RESTRICT_EPS) {
                P.eps[o] = sv;
            } else {
                P.v[o] = sv;
                if (FAS) P.f[o] = sr;
                push_ghosts<T, D, BS>(P.vg, px, p, l0, l1, l2, sv);
            }
        } else {
            const TailGeo tg = tail_geo(tb, dm, nt - 1, D);
            const int64_t o = tg.idx(gc[0], gc[1], gc[2], D);
            if (MODE == RESTRICT_EPS) P.teps[o] = sv;
            else P.tv[o] = sv;
            if (FAS) P.tf[o] = sr;
        }
    }
}

// --------------------------------------------------------- FAS right side
// On parent blocks, after the restriction (which also refreshed their ghosts):
// v_old = v (ghosts included) and f = R(r) + L v (eq. coarse-rhs).  Several
// workgroups per block, one cell or ghost per thread.
template <typename T, int D, int BS, bool VAR>
__global__ void __launch_bounds__(256) k_fas(Plane<T> P, DevTables tb, int lev, const int32_t *list,
                                             uint64_t mask, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t b = list[blockIdx.x / wg_per_block];
    const int t = (blockIdx.x % wg_per_block) * 256 + threadIdx.x;
    // the domain test comes last so that the data loads need not wait for it
    const int dm = tb.dom[b];
    if (t < g::NC) {
        const Spacing s = spacing(tb, dm, lev);
        int i, j, k;
        g::decode(t, i, j, k);
        const double rx = D == 2 && tb.axi ? tb.lox[dm] + (tb.org[3 * b] + i + 0.5) * s.hx : 0.0;
        Stencil<T, D, BS, VAR> st;
        st.load(P, b, i, j, k, s, true, rx);
        const T fv = P.f[b * g::NC + t];
        if (!((mask >> dm) & 1)) return;
        P.vold[b * g::NC + t] = st.vc;
        P.f[b * g::NC + t] = fv + st.Lv();
    } else if (t < g::NC + g::NG) {
        const T gv = P.vg[b * g::NG + t - g::NC];
        if (!((mask >> dm) & 1)) return;
        P.voldg[b * g::NG + t - g::NC] = gv;
    }
}

// The same for 3D constant coefficients in FP32 on levels with many parent blocks
// (kFasLdsMin or more): one workgroup per block stages v and its ghosts in LDS with
// 16-byte loads, writes v_old from there and takes every neighbour of L v from LDS.
// The arithmetic is that of k_fas (Stencil::Lv with constant weights).
template <typename T, int D, int BS>
__global__ void __launch_bounds__(256) k_fas_lds(Plane<T> P, DevTables tb, int lev, const int32_t *list,
                                                 uint64_t mask) {
    using g = G<D, BS>;
    static_assert(D == 3 && g::NC % 256 == 0 && (g::NC * sizeof(T)) % 16 == 0 && (g::NG * sizeof(T)) % 16 == 0,
                  "block shape");
    constexpr int NF = g::NC / 256;                 // cells per thread
    __shared__ uint4 s_raw[(g::NC + g::NG) * sizeof(T) / 16];
    T *s_v = reinterpret_cast<T *>(s_raw);
    T *s_g = s_v + g::NC;
    const int64_t b = list[blockIdx.x];
    const int tid = threadIdx.x;
    // every load first: v and its ghosts as vectors, then this thread's f values
    Stager<T, 1, g::NC, g::NC, 256> cv;
    Stager<T, 1, g::NG, g::NG, 256> cg;
    cv.load(P.v + b * g::NC);
    cg.load(P.vg + b * g::NG);
    T fv[NF];
#pragma unroll
    for (int m = 0; m < NF; m++) fv[m] = P.f[b * g::NC + tid + m * 256];
    // the domain test comes last so that the data loads need not wait for it (the
    // whole workgroup leaves together, before its barrier)
    const int dm = tb.dom[b];
    if (!((mask >> dm) & 1)) return;
    cv.store(s_v);
    cg.store(s_g);
    __syncthreads();
    // v_old = v, ghosts included, as vectors from LDS (stored straight from the
    // loaded registers, those would be kept in scratch memory)
    {
        constexpr int NVC = g::NC * sizeof(T) / 16, NVT = (g::NC + g::NG) * sizeof(T) / 16;
        uint4 *ov = reinterpret_cast<uint4 *>(P.vold + b * g::NC);
        uint4 *og = reinterpret_cast<uint4 *>(P.voldg + b * g::NG);
#pragma unroll
        for (int m = 0; m < (NVT + 255) / 256; m++) {
            const int q = tid + m * 256;
            if (q >= NVT) break;
            const uint4 x = s_raw[q];
            if (q < NVC) ov[q] = x;
            else og[q - NVC] = x;
        }
    }
    const Spacing sp = spacing(tb, dm, lev);
#pragma unroll
    for (int m = 0; m < NF; m++) {
        const int t = tid + m * 256;
        int i, j, k;
        g::decode(t, i, j, k);
        T nb[6];
        nb[0] = ld<D, BS>(s_v, s_g, 0, i - 1, j, k);
        nb[1] = ld<D, BS>(s_v, s_g, 0, i + 1, j, k);
        nb[2] = ld<D, BS>(s_v, s_g, 0, i, j - 1, k);
        nb[3] = ld<D, BS>(s_v, s_g, 0, i, j + 1, k);
        nb[4] = ld<D, BS>(s_v, s_g, 0, i, j, k - 1);
        nb[5] = ld<D, BS>(s_v, s_g, 0, i, j, k + 1);
        const T vc = s_v[t];
        // Stencil::Lv's operations in its order (written out: its loops would not
        // unroll inside this one)
        T acc = T(0);
#pragma unroll
        for (int f = 0; f < 2 * D; f++) acc += T(sp.ih2[f / 2]) * (nb[f] - vc);
        P.f[b * g::NC + t] = fv[m] + (acc - T(sp.lam) * vc);
    }
}

// ------------------------------------------------- prolongation + correction
// v^h += P(v^H - v_old^H) (eq. coarse-corr) with the nearest-neighbour interpolation
// of eq. interp_2d / interp_3d: 2D (2 d_p + d_x + d_y)/4, 3D (d_p + d_x + d_y + d_z)/4,
// the neighbours taken on the side of the fine cell (coarse ghosts near block faces).
// One workgroup per fine block: d = v - v_old on the parent's octant and its face
// halo is staged in LDS; the fine block is updated with unit stride and its boundary
// values pushed into the mirroring ghosts.
// (SPLIT workgroups per block on levels with few blocks, as for the smoothing.)
// HALF: a red-black half-sweep of colour 0 follows.  It reads only colour 1 and the
// colour-1 ghost halves and rewrites every colour-0 cell (pushing its same-level
// ghosts), so only colour 1 is corrected -- except in blocks with a physical face,
// whose colour-0 boundary cells are read through the ghosts that mirror them
// (Dirichlet, Neumann), or with a coarse-fine face, whose ghosts are extrapolated from
// cells of both colours: those blocks correct both colours.
template <typename T, int D, int BS, int SPLIT, bool HALF>
__global__ void __launch_bounds__(256) k_correct(Plane<T> P, DevTables tb, int lev, int b0, uint64_t mask,
                                                 int nt) {
    using g = G<D, BS>;
    constexpr int HB = BS / 2, HP = HB + 2;
    constexpr int NBOX = D == 3 ? HP * HP * HP : HP * HP;
    constexpr int TPB = g::NC < 256 ? g::NC : 256;
    static_assert(SPLIT == 1 || g::NC % (TPB * SPLIT) == 0, "SPLIT must divide the block");
    // cells of one pass: the whole block, or (HALF) one colour, split over SPLIT parts
    constexpr int NPASS = (HALF ? g::NH : g::NC) / SPLIT;
    __shared__ T s_d[NBOX];
    const int nbl = gridDim.x / SPLIT;   // parts of a block nb workgroups apart (same XCD)
    // (one workgroup per block: the Morton-ordered blocks in one contiguous run per XCD,
    // so siblings, whose octants and halos share cache lines of the parent, share an L2)
    const int64_t b = b0 + (SPLIT == 1 ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x % nbl);
    const int part = SPLIT == 1 ? 0 : (int)blockIdx.x / nbl;
    const int t0 = (HALF ? g::NH : 0) + part * NPASS;   // first storage index of this part
    const int tid = threadIdx.x;
    // the block's tables, all independent loads; the octant of the block in its parent
    // follows from its own origin (block coordinates' parity)
    BlockCtx<D> cx;
    cx.load(tb, b, lev);
    const int dm = cx.dm;
    const int64_t p = tb.parent[b];
    const int gc0[3] = {tb.org[3 * b] >> 1, tb.org[3 * b + 1] >> 1, D == 3 ? tb.org[3 * b + 2] >> 1 : 0};
    int po[3] = {0, 0, 0};
    for (int a = 0; a < D; a++) po[a] = ((gc0[a] / HB) & 1) * HB;
    constexpr int ITB = (NBOX + TPB - 1) / TPB;
    constexpr int IT = (NPASS + TPB - 1) / TPB;
    const TailGeo tg = tail_geo(tb, dm, nt - 1, D);
    // issue all loads first: the fine values this thread updates (a run of IT
    // consecutive cells, read as vectors, when the pass divides evenly and the values
    // are FP32), then the box
    // (FP32 only: for FP64 the strided form, one 512-byte span per wave and load, is
    // faster)
    constexpr bool RUN = NPASS % TPB == 0 && sizeof(T) == 4;
    T vr[IT];
    if constexpr (RUN) {
        ld_run<T, IT>(P.v + b * g::NC + t0 + tid * IT, vr);
    } else {
#pragma unroll
        for (int m = 0; m < IT; m++) {
            const int u = tid + m * TPB;
            vr[m] = P.v[b * g::NC + t0 + (u < NPASS ? u : 0)];
        }
    }
    // box cell -> addresses of v and v_old (edges and corners of the halo, never
    // used, read the box centre instead)
    T av[ITB], ao[ITB];
#pragma unroll
    for (int m = 0; m < ITB; m++) {
        int q = tid + m * TPB;
        if (NBOX % TPB != 0 && q >= NBOX) q = 0;
        int x = q % HP, y = (q / HP) % HP, z = D == 3 ? q / (HP * HP) : 1;
        const int out = (x == 0 || x == HP - 1) + (y == 0 || y == HP - 1) + (D == 3 && (z == 0 || z == HP - 1));
        if (out > 1) { x = 1; y = 1; z = 1; }
        const int c[3] = {x - 1, y - 1, D == 3 ? z - 1 : 0};
        const T *pv, *pvo;
        if (p >= 0) {
            const int l0 = po[0] + c[0], l1 = po[1] + c[1], l2 = po[2] + c[2];
            pv = ldp<D, BS>(P.v, P.vg, p, l0, l1, l2);
            pvo = ldp<D, BS>(P.vold, P.voldg, p, l0, l1, l2);
        } else {
            const int64_t o = tg.idx(gc0[0] + c[0], gc0[1] + c[1], gc0[2] + c[2], D);
            pv = P.tv + o;
            pvo = P.tvold + o;
        }
        av[m] = *pv;
        ao[m] = *pvo;
    }
    T dv[ITB];
#pragma unroll
    for (int m = 0; m < ITB; m++) dv[m] = av[m] - ao[m];
#pragma unroll
    for (int m = 0; m < ITB; m++) {
        const int q = tid + m * TPB;
        if (q < NBOX) s_d[q] = dv[m];
    }
    __syncthreads();
    if (!((mask >> dm) & 1)) return;
    auto corrected = [&](int t, T vold) -> T {
        int i, j, k;
        g::decode(t, i, j, k);
        const int x = (i >> 1) + 1, y = (j >> 1) + 1, z = D == 3 ? (k >> 1) + 1 : 0;
        const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        const int c0 = (z * HP + y) * HP + x;
        const T d0 = s_d[c0], dx = s_d[c0 + sx], dy = s_d[c0 + sy * HP];
        T corr;
        if (D == 2) corr = T(0.25) * (T(2) * d0 + dx + dy);
        else corr = T(0.25) * (d0 + dx + dy + s_d[c0 + sz * HP * HP]);
        return vold + corr;
    };
    auto push = [&](int t, T nv) {
        int i, j, k;
        g::decode(t, i, j, k);
        push_ghosts<T, D, BS>(P.vg, cx, b, i, j, k, nv);
    };
    auto update = [&](int t, T vold) {
        const T nv = corrected(t, vold);
        P.v[b * g::NC + t] = nv;
        push(t, nv);
    };
    if constexpr (RUN) {
        T nvs[IT];
#pragma unroll
        for (int m = 0; m < IT; m++) nvs[m] = corrected(t0 + tid * IT + m, vr[m]);
        st_run<T, IT>(P.v + b * g::NC + t0 + tid * IT, nvs);
        if constexpr (IT % g::RH == 0) {
            // the run is whole rows of one colour: each row's pushes as vector stores
#pragma unroll
            for (int r = 0; r < IT / g::RH; r++) {
                const int tq = t0 + tid * IT + r * g::RH;
                const int col = tq >= g::NH, row = (tq - col * g::NH) / g::RH;
                const int j = row % BS, k = D == 3 ? row / BS : 0;
                T seg[g::RH];
#pragma unroll
                for (int m = 0; m < g::RH; m++) seg[m] = nvs[r * g::RH + m];
                push_run<T, D, BS, g::RH>(P.vg, cx, b, (j + k + col) & 1, j, k, seg);
            }
        } else {
#pragma unroll
            for (int m = 0; m < IT; m++) push(t0 + tid * IT + m, nvs[m]);
        }
    } else {
#pragma unroll
        for (int m = 0; m < IT; m++) {
            const int u = tid + m * TPB;
            if (u >= NPASS) break;
            update(t0 + u, vr[m]);
        }
    }
    if (HALF) {
        // blocks with a physical face (whose ghosts mirror colour-0 cells) or a
        // coarse-fine face (whose ghosts extrapolate from both colours) are corrected whole
        bool whole = false;
#pragma unroll
        for (int f = 0; f < 2 * D; f++) whole = whole || cx.nbr[f] < 0;
        if (whole) {
#pragma unroll
            for (int m = 0; m < IT; m++) {
                const int u = tid + m * TPB;
                if (NPASS % TPB != 0 && u >= NPASS) break;
                const int t = part * NPASS + u;   // colour 0
                update(t, P.v[b * g::NC + t]);
            }
        }
    }
}

// --------------------------------------------------------------- the tail
// One workgroup per domain runs the coarse grids below the lowest block level: the
// levels whose block size was halved down to one cell (Sec. 2.5; the paper keeps
// them on a single process), except the large ones that the grid-wide launches
// handle.  They are uniform grids, stored whole with one ghost layer.  Red-black
// Gauss-Seidel over the whole grid: a cell that changes writes the ghosts that mirror
// it (a ghost then holds the other colour's value, so a sweep never reads what it
// writes), except on grids with an odd cell count along a periodic axis, where the
// two ends of a row share a colour and the ghost layer is refilled after each colour.
// When a domain's grids fit in LDS they are copied in, cycled there and copied back.

// Operations of a tail cycle.
enum { TOP_ENTER = 0, TOP_DOWN, TOP_UP, TOP_RESTRICT, TOP_CORRECT, TOP_COARSE };
constexpr int kTailOps = 512;

// Geometry of one tail grid (offsets relative to the domain's first tail array).
struct TailLev {
    int n[3];          // cells per axis (1 on unused axes)
    int sy, sz;        // padded strides of j and k
    int off;           // offset of the padded grid
    int ncell, npad;   // cells, padded cells
    int rh;            // colour slots per row, (n[0] + 1) / 2
    int ghost_pass;    // periodic axis with an odd cell count
    float inv_rh, inv_n0, inv_n1;
    int lg[3], lrh;    // log2 of n[a] and of rh where they are powers of two, else -1
    double h[3], ih2[3];
    double inv_den;    // 1 / (2 sum ih2 + lambda): the constant-coefficient diagonal
    double lam;        // Helmholtz term
    double rlo;        // axisymmetric form: radius of the domain's inner x face
    int axi;
};
struct TailBC {
    int kind[6];
    double value[6];
};

// q = x / d, r = x % d for 0 <= x < 2^22 (a float reciprocal, then one correction).
__device__ __forceinline__ void divmod(int x, int d, float inv, int &q, int &r) {
    q = (int)((float)x * inv);
    r = x - q * d;
    if (r < 0) {
        q--;
        r += d;
    } else if (r >= d) {
        q++;
        r -= d;
    }
}

// divmod by d = 2^lg with a shift and a mask (lg is the same in every lane).
__device__ __forceinline__ void divmod2(int x, int d, float inv, int lg, int &q, int &r) {
    if (lg >= 0) {
        q = x >> lg;
        r = x & (d - 1);
    } else {
        divmod(x, d, inv, q, r);
    }
}

template <int D>
__device__ __forceinline__ int tix(const TailLev &g, int i, int j, int k) {
    return g.off + (D == 3 ? (k + 1) * g.sz : 0) + (j + 1) * g.sy + (i + 1);
}

// Threads of the single-workgroup coarse solver (the variable-coefficient and 2D
// forms need more registers; 2D tail grids are small).  Kernels use this constant
// rather than the block size at run time, which the device library reads from memory
// at every use.
template <bool VAR, int D = 3>
constexpr int tail_threads() { return VAR || D == 2 ? 512 : 1024; }

template <typename T, int D, bool VAR>
struct Tail {
    static constexpr int NT = tail_threads<VAR, D>();
    const TailLev *lv;         // [levels] in LDS
    TailBC bc;                 // boundary data (registers)
    double *red;               // reduction scratch in LDS, one slot per wave
    T *tv, *tvold, *tf, *teps; // this domain's tail arrays (LDS or global memory)
    T *tvold_top;              // with the arrays in LDS: v_old of the top grid, in global
    int top;                   // memory (only the block level above reads it)
    T *ttmp;                   // Jacobi: global scratch grids (same offsets) for large grids
    int jac;                   // smoother: 0 red-black Gauss-Seidel, 1 weighted Jacobi
    double omega;              // Jacobi weight

    __device__ __forceinline__ void cell(const TailLev &g, int c, int &i, int &j, int &k) const {
        int r;
        divmod2(c, g.n[0], g.inv_n0, g.lg[0], r, i);
        if (D == 3) divmod2(r, g.n[1], g.inv_n1, g.lg[1], k, j);
        else { j = r; k = 0; }
    }
    // Colour slot s of grid g -> cell of that colour; false past the end of a row.
    __device__ __forceinline__ bool slot(const TailLev &g, int s, int colour, int &i, int &j, int &k) const {
        int row, pos;
        divmod2(s, g.rh, g.inv_rh, g.lrh, row, pos);
        if (D == 3) divmod2(row, g.n[1], g.inv_n1, g.lg[1], k, j);
        else { j = row; k = 0; }
        i = 2 * pos + ((j + k + colour) & 1);
        return i < g.n[0];
    }
    __device__ __forceinline__ int nslot(const TailLev &g) const { return g.rh * g.n[1] * (D == 3 ? g.n[2] : 1); }

    // Writes the ghosts mirroring cell (i,j,k) after it changed to nv (physical faces
    // always, periodic faces if `periodic`).
    __device__ __forceinline__ void push(T *u, const TailLev &g, int i, int j, int k, T nv, bool periodic) const {
        const int c[3] = {i, j, k};
#pragma unroll
        for (int a = 0; a < D; a++) {
#pragma unroll
            for (int side = 0; side < 2; side++) {
                if (c[a] != (side ? g.n[a] - 1 : 0)) continue;
                const int f = 2 * a + side;
                const int kind = bc.kind[f];
                int q[3] = {i, j, k};
                T val;
                if (kind == MG_BC_PERIODIC) {
                    if (!periodic) continue;
                    q[a] = side ? -1 : g.n[a];
                    val = nv;
                } else {
                    q[a] = side ? g.n[a] : -1;
                    val = bc_ghost<T>(kind, bc.value[f], g.h[a], side, nv);
                }
                u[tix<D>(g, q[0], q[1], q[2])] = val;
            }
        }
    }
    // The whole ghost layer of one grid (faces only): periodic copy or boundary
    // condition (for eps, a copy of the interior cell).
    __device__ __forceinline__ void fill_ghosts(int lev, T *u, bool eps, int stride = NT) const {
        const TailLev g = lv[lev];
#pragma unroll
        for (int a = 0; a < D; a++) {
            const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            const int n1 = g.n[t1], n2 = D == 3 ? g.n[t2] : 1;
            const int tot = 2 * n1 * n2;
            for (int q = threadIdx.x; q < tot; q += stride) {
                const int side = q >= n1 * n2;
                const int r = q - side * n1 * n2;
                int c[3], in[3], op[3];
                const int l1 = g.lg[t1];
                c[t1] = l1 >= 0 ? r & (n1 - 1) : r % n1;
                c[t2] = D == 3 ? (l1 >= 0 ? r >> l1 : r / n1) : 0;
                in[t1] = op[t1] = c[t1];
                in[t2] = op[t2] = c[t2];
                c[a] = side ? g.n[a] : -1;
                in[a] = side ? g.n[a] - 1 : 0;
                op[a] = side ? 0 : g.n[a] - 1;
                if (D == 2) c[2] = in[2] = op[2] = 0;
                // selects, not a run-time index into bc (which would live in scratch)
                const int kind = side ? bc.kind[2 * a + 1] : bc.kind[2 * a];
                const double bval = side ? bc.value[2 * a + 1] : bc.value[2 * a];
                T val;
                if (kind == MG_BC_PERIODIC) val = u[tix<D>(g, op[0], op[1], op[2])];
                else if (eps) val = u[tix<D>(g, in[0], in[1], in[2])];
                else val = bc_ghost<T>(kind, bval, g.h[a], side, u[tix<D>(g, in[0], in[1], in[2])]);
                u[tix<D>(g, c[0], c[1], c[2])] = val;
            }
        }
    }

    __device__ __forceinline__ void stencil(const TailLev &g, int i, int j, int k, T *w, T *nb) const {
        const int o = tix<D>(g, i, j, k);
        const int st[3] = {1, g.sy, g.sz};
#pragma unroll
        for (int f = 0; f < 2 * D; f++) {
            const int d = (f & 1) ? st[f >> 1] : -st[f >> 1];
            nb[f] = tv[o + d];
            w[f] = T(g.ih2[f >> 1]);
            if (VAR) w[f] *= harm(teps[o], teps[o + d]);
        }
        if (D == 2 && g.axi) {   // axisymmetric x-face factors (see axi_factors)
            const double r = g.rlo + (i + 0.5) * g.h[0];
            w[0] *= T((r - 0.5 * g.h[0]) / r);
            w[1] *= T((r + 0.5 * g.h[0]) / r);
        }
    }
    __device__ __forceinline__ T Lv(const TailLev &g, int i, int j, int k) const {
        T w[6], nb[6];
        stencil(g, i, j, k, w, nb);
        const T vc = tv[tix<D>(g, i, j, k)];
        T s = T(0);
#pragma unroll
        for (int f = 0; f < 2 * D; f++) s += w[f] * (nb[f] - vc);
        return s - T(g.lam) * vc;
    }

    // Orders the accesses of one wave (LDS and memory) where only that wave runs.
    __device__ __forceinline__ void wave_fence() const { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }
    // One colour of Gauss-Seidel on grid lev, then a barrier (wave: run by wave 0
    // alone, a fence in place of the barrier).
    __device__ __forceinline__ void sweep(int lev, int colour, bool wave = false) const {
        const TailLev g = lv[lev];
        const bool gp = g.ghost_pass;
        const int ns = nslot(g);
        const int nt = wave ? 64 : NT;
        // Two slots per pass, every load of both issued before either store: a
        // half-sweep reads only the other colour, and a physical ghost it writes is
        // read only by the cell it mirrors, before that cell's update.
        for (int s0 = threadIdx.x; s0 < ns; s0 += 2 * nt) {
            int ii[2] = {0, 0}, jj[2] = {0, 0}, kk[2] = {0, 0}, oo[2] = {0, 0};
            bool ok[2];
            T fo[2], w[2][6], nb[2][6];
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int s = s0 + u * nt;
                ok[u] = s < ns && slot(g, s, colour, ii[u], jj[u], kk[u]);
                if (ok[u]) {
                    oo[u] = tix<D>(g, ii[u], jj[u], kk[u]);
                    fo[u] = tf[oo[u]];
                    stencil(g, ii[u], jj[u], kk[u], w[u], nb[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
                if (!ok[u]) continue;
                T num = T(0), den = T(g.lam);
#pragma unroll
                for (int f = 0; f < 2 * D; f++) {
                    num += w[u][f] * nb[u][f];
                    den += w[u][f];
                }
                const T nv = VAR ? (num - fo[u]) / den : (num - fo[u]) * T(g.inv_den);
                tv[oo[u]] = nv;
                if (!gp) push(tv, g, ii[u], jj[u], kk[u], nv, true);
            }
        }
        if (wave) wave_fence();
        else __syncthreads();
        if (gp) {
            fill_ghosts(lev, tv, false, nt);
            if (wave) wave_fence();
            else __syncthreads();
        }
    }
    // Weighted Jacobi value of cell (i,j,k) from the current (old) values.
    __device__ __forceinline__ T jacobi_value(const TailLev &g, int i, int j, int k) const {
        T w[6], nb[6];
        stencil(g, i, j, k, w, nb);
        T num = T(0), den = T(g.lam);
#pragma unroll
        for (int f = 0; f < 2 * D; f++) {
            num += w[f] * nb[f];
            den += w[f];
        }
        const int o = tix<D>(g, i, j, k);
        const T gs = VAR ? (num - tf[o]) / den : (num - tf[o]) * T(g.inv_den);
        return tv[o] + T(omega) * (gs - tv[o]);
    }
    // One weighted Jacobi step: all new values first (registers, or the scratch grid
    // for large grids), then they replace the old ones and push their ghosts.
    __device__ __forceinline__ void jacobi_step(int lev) const {
        constexpr int R = 8;
        const TailLev g = lv[lev];
        const bool regs = g.ncell <= R * NT;
        T nv[R];
        if (regs) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int c = threadIdx.x + r * NT;
                if (c < g.ncell) {
                    int i, j, k;
                    cell(g, c, i, j, k);
                    nv[r] = jacobi_value(g, i, j, k);
                }
            }
        } else {
            for (int c = threadIdx.x; c < g.ncell; c += NT) {
                int i, j, k;
                cell(g, c, i, j, k);
                ttmp[tix<D>(g, i, j, k)] = jacobi_value(g, i, j, k);
            }
        }
        __syncthreads();
        if (regs) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int c = threadIdx.x + r * NT;
                if (c < g.ncell) {
                    int i, j, k;
                    cell(g, c, i, j, k);
                    tv[tix<D>(g, i, j, k)] = nv[r];
                    push(tv, g, i, j, k, nv[r], true);
                }
            }
        } else {
            for (int c = threadIdx.x; c < g.ncell; c += NT) {
                int i, j, k;
                cell(g, c, i, j, k);
                const T x = ttmp[tix<D>(g, i, j, k)];
                tv[tix<D>(g, i, j, k)] = x;
                push(tv, g, i, j, k, x, true);
            }
        }
        __syncthreads();
    }
    __device__ __forceinline__ void smooth(int lev) const {
        if (jac) {
            jacobi_step(lev);
            return;
        }
        sweep(lev, 0);
        sweep(lev, 1);
    }

    // Block-wide reductions (all threads get the result): wave shuffles, then one
    // exchange through LDS.
    __device__ __forceinline__ double reduce_max(double x, bool wave = false) const {
        for (int o = 32; o > 0; o >>= 1) {
            double y = __shfl_xor(x, o);
            if (y > x || y != y) x = y;
        }
        if (wave) return x;   // one wave only
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        x = red[0];
        for (int w = 1; w < (int)(NT >> 6); w++)
            if (red[w] > x || red[w] != red[w]) x = red[w];
        __syncthreads();
        return x;
    }
    __device__ __forceinline__ double reduce_sum(double x) const {
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        x = 0.0;
        for (int w = 0; w < (int)(NT >> 6); w++) x += red[w];
        __syncthreads();
        return x;
    }

    __device__ __forceinline__ double resmax(int lev, bool wave = false) const {
        const TailLev g = lv[lev];
        double m = 0.0;
        for (int c = threadIdx.x; c < g.ncell; c += wave ? 64 : NT) {
            int i, j, k;
            cell(g, c, i, j, k);
            const double r = fabs((double)(tf[tix<D>(g, i, j, k)] - Lv(g, i, j, k)));
            if (r > m || r != r) m = r;
        }
        return reduce_max(m, wave);
    }

    // dst = v on the padded grid g, two elements per pass (loads before stores; the
    // arrays are distinct).  Separate call sites keep LDS and global stores apart.
    __device__ __forceinline__ void copy_pad(T *dst, const TailLev &g) const {
        for (int q = threadIdx.x; q < g.npad; q += 2 * NT) {
            const bool two = q + NT < g.npad;
            const T a = tv[g.off + q], b = two ? tv[g.off + q + NT] : T(0);
            dst[g.off + q] = a;
            if (two) dst[g.off + q + NT] = b;
        }
    }
    // v_old = v (ghosts included) and f += L v on grid lev (ghosts already valid).
    __device__ __forceinline__ void fas(int lev) const {
        const TailLev g = lv[lev];
        if (tvold_top && lev == top) copy_pad(tvold_top, g);
        else copy_pad(tvold, g);
        for (int c0 = threadIdx.x; c0 < g.ncell; c0 += 2 * NT) {
            int ii[2] = {0, 0}, jj[2] = {0, 0}, kk[2] = {0, 0};
            const bool two = c0 + NT < g.ncell;
            cell(g, c0, ii[0], jj[0], kk[0]);
            if (two) cell(g, c0 + NT, ii[1], jj[1], kk[1]);
            const int o0 = tix<D>(g, ii[0], jj[0], kk[0]), o1 = tix<D>(g, ii[1], jj[1], kk[1]);
            const T f0 = tf[o0], l0 = Lv(g, ii[0], jj[0], kk[0]);
            const T f1 = two ? tf[o1] : T(0), l1 = two ? Lv(g, ii[1], jj[1], kk[1]) : T(0);
            tf[o0] = f0 + l0;
            if (two) tf[o1] = f1 + l1;
        }
        __syncthreads();
    }
    // Entry to the top grid, which a restriction from above filled without ghosts.
    __device__ __forceinline__ void enter(int lev) const {
        fill_ghosts(lev, tv, false);
        __syncthreads();
        fas(lev);
    }
    // Restriction lev -> lev-1 of v and of the residual (pushing the coarse ghosts),
    // then the FAS right-hand side there.
    __device__ __forceinline__ void restrict_fas(int lev) const {
        const TailLev gf = lv[lev], gc = lv[lev - 1];
        for (int c = threadIdx.x; c < gc.ncell; c += NT) {
            int I, J, K;
            cell(gc, c, I, J, K);
            T sv = T(0), sr = T(0);
#pragma unroll
            for (int q = 0; q < (1 << D); q++) {
                const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = D == 3 ? 2 * K + (q >> 2) : 0;
                const int o = tix<D>(gf, i, j, k);
                sv += tv[o];
                sr += tf[o] - Lv(gf, i, j, k);
            }
            const T inv = T(1) / T(1 << D);
            const int oc = tix<D>(gc, I, J, K);
            tv[oc] = sv * inv;
            tf[oc] = sr * inv;
            push(tv, gc, I, J, K, sv * inv, true);
        }
        __syncthreads();
        fas(lev - 1);
    }
    // Prolongation of v - v_old from lev-1 (eq. interp_2d / interp_3d) added to lev,
    // with the ghosts of lev pushed.
    __device__ __forceinline__ void correct(int lev) const {
        const TailLev gf = lv[lev], gc = lv[lev - 1];
        // two fine cells per pass, every load of both before either store (the stores
        // touch fine cells and their ghosts, the loads coarse cells and the cell itself)
        for (int c0 = threadIdx.x; c0 < gf.ncell; c0 += 2 * NT) {
            int ii[2] = {0, 0}, jj[2] = {0, 0}, kk[2] = {0, 0}, of[2];
            T nv[2];
            const bool two = c0 + NT < gf.ncell;
#pragma unroll
            for (int u = 0; u < 2; u++) {
                if (u == 1 && !two) break;
                cell(gf, c0 + u * NT, ii[u], jj[u], kk[u]);
                const int i = ii[u], j = jj[u], k = kk[u];
                const int p[3] = {i >> 1, j >> 1, k >> 1};
                const int sg[3] = {(i & 1) ? 1 : -1, (j & 1) ? 1 : -1, (k & 1) ? 1 : -1};
                const int o = tix<D>(gc, p[0], p[1], p[2]);
                const T d0 = tv[o] - tvold[o];
                const int st[3] = {1, gc.sy, gc.sz};
                T dn[3];
#pragma unroll
                for (int a = 0; a < D; a++) dn[a] = tv[o + sg[a] * st[a]] - tvold[o + sg[a] * st[a]];
                const T corr = D == 2 ? T(0.25) * (T(2) * d0 + dn[0] + dn[1]) : T(0.25) * (d0 + dn[0] + dn[1] + dn[2]);
                of[u] = tix<D>(gf, i, j, k);
                nv[u] = tv[of[u]] + corr;
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
                if (u == 1 && !two) break;
                tv[of[u]] = nv[u];
                push(tv, gf, ii[u], jj[u], kk[u], nv[u], true);
            }
        }
        __syncthreads();
    }

    // Coarsest grid: smoothing steps until the max-norm residual is <= max(abs,
    // rel * initial), at most n_max, at least one; stop early once 8 steps in a row have
    // not lowered it 0.1% below the lowest value so far (see kStall).  Fully periodic:
    // remove the mean of f first.
    __device__ __forceinline__ int coarse_solve(const TailParams &tp) const {
        const TailLev g = lv[0];
        bool per = g.lam == 0.0;   // the regular Helmholtz operator needs no mean removal
        for (int f = 0; f < 2 * D; f++) per = per && bc.kind[f] == MG_BC_PERIODIC;
        if (per && g.ncell == 1) {
            // one cell, periodic on every axis: the operator is zero, the mean removal
            // leaves f = 0 and so a zero residual, and the rule stops after its one step,
            // which leaves v unchanged (its value is the free constant of the problem)
            if (threadIdx.x == 0) tf[tix<D>(g, 0, 0, 0)] = T(0);
            __syncthreads();
            return 1;
        }
        if (per) {
            double s = 0.0;
            for (int c = threadIdx.x; c < g.ncell; c += NT) {
                int i, j, k;
                cell(g, c, i, j, k);
                s += (double)tf[tix<D>(g, i, j, k)];
            }
            const double mean = reduce_sum(s) / (double)g.ncell;
            for (int c = threadIdx.x; c < g.ncell; c += NT) {
                int i, j, k;
                cell(g, c, i, j, k);
                tf[tix<D>(g, i, j, k)] -= T(mean);
            }
            __syncthreads();
        }
        // A small grid (Gauss-Seidel) is iterated by wave 0 alone, its phases ordered
        // by fences: cells of one colour read only the other colour, and a ghost a cell
        // pushes is read in that half-sweep only by the cell itself (periodic axes of
        // odd length are refilled after it), so the updates are those of the whole
        // workgroup.  The other waves wait at the closing barrier; the step count is
        // wave 0's, the one reported.
        const bool wave = !jac && g.ncell <= kWaveCoarse;
        int k = 0;
        if (!wave || threadIdx.x < 64) {
            const double r0 = resmax(0, wave);
            double best = r0;
            const double target = fmax(tp.abs_tol, tp.rel_tol * r0);
            int since = 0;
            for (k = 1; k <= tp.n_max; k++) {
                if (wave) {
                    sweep(0, 0, true);
                    sweep(0, 1, true);
                } else {
                    smooth(0);
                }
                const double r = resmax(0, wave);
                if (r <= target) break;
                if (r < kStall * best) {
                    best = r;
                    since = 0;
                } else if (++since >= kStallSteps) {
                    break;
                }
            }
        }
        if (wave) __syncthreads();
        return k > tp.n_max ? tp.n_max : k;
    }

    // Runs a cycle given as a list of operations (each operation's code appears once
    // in the kernel, which keeps the instruction footprint small).
    __device__ __forceinline__ int run(const int *ops, int nops, const TailParams &tp) const {
        int steps = 0;
        for (int q = 0; q < nops; q++) {
            // the same word for every lane: kept in scalar registers (the level index
            // would otherwise occupy a vector register across the whole operation)
            const int op = __builtin_amdgcn_readfirstlane(ops[q]);
            const int kind = op >> 8, l = op & 255;
            switch (kind) {
            case TOP_ENTER: enter(l); break;
            case TOP_DOWN:
            case TOP_UP: {
                const int reps = kind == TOP_DOWN ? tp.n_down : tp.n_up;
                for (int s = 0; s < reps; s++) smooth(l);
                break;
            }
            case TOP_RESTRICT: restrict_fas(l); break;
            case TOP_CORRECT: correct(l); break;
            default: steps = coarse_solve(tp); break;
            }
        }
        return steps;
    }
};

// Operation list of a tail V-cycle (mode TAIL_VCYCLE) or FMG cycle (TAIL_FMG) from
// grid top; at most 2 top^2 + 5 top + 2 entries.
__device__ __forceinline__ int tail_ops(int *ops, int mode, int top) {
    int n = 0;
    ops[n++] = TOP_ENTER << 8 | top;
    auto vcycle = [&](int t) {
        for (int l = t; l >= 1; l--) {
            ops[n++] = TOP_DOWN << 8 | l;
            ops[n++] = TOP_RESTRICT << 8 | l;
        }
        ops[n++] = TOP_COARSE << 8;
        for (int l = 1; l <= t; l++) {
            ops[n++] = TOP_CORRECT << 8 | l;
            ops[n++] = TOP_UP << 8 | l;
        }
    };
    if (mode == TAIL_VCYCLE) {
        vcycle(top);
    } else {
        for (int l = top; l >= 1; l--) ops[n++] = TOP_RESTRICT << 8 | l;
        ops[n++] = TOP_COARSE << 8;
        for (int t = 1; t <= top; t++) {
            ops[n++] = TOP_CORRECT << 8 | t;
            vcycle(t);
        }
    }
    return n;
}

// Padded cells of the tail grids 0..top of domain dm (stored in level order).
__device__ __forceinline__ int64_t tail_span(const DevTables &tb, int dm, int top, int dim, int64_t *first) {
    *first = tb.tail_off[(size_t)dm * MAXLEV];
    const int32_t *nc = tb.ncell + ((size_t)dm * MAXLEV + top) * 3;
    int64_t last = (int64_t)(nc[0] + 2) * (nc[1] + 2) * (dim == 3 ? nc[2] + 2 : 1);
    return tb.tail_off[(size_t)dm * MAXLEV + top] + last - *first;
}

// Offset of the padded tail grid `top` of domain dm.
__device__ __forceinline__ int64_t tail_last_off(const DevTables &tb, int dm, int top) {
    return tb.tail_off[(size_t)dm * MAXLEV + top];
}

// Caches the geometry of tail grids 0..nlev-1 of domain dm and its boundary data in
// LDS.
__device__ __forceinline__ void tail_setup(const DevTables &tb, int dm, int nlev, int dim, int64_t first, TailLev *lv,
                           TailBC *bc) {
    if (threadIdx.x < nlev) {
        const int l = threadIdx.x;
        const int32_t *nc = tb.ncell + ((size_t)dm * MAXLEV + l) * 3;
        const double *h = tb.h + ((size_t)dm * MAXLEV + l) * 3;
        TailLev g;
        g.n[0] = nc[0];
        g.n[1] = nc[1];
        g.n[2] = dim == 3 ? nc[2] : 1;
        g.sy = g.n[0] + 2;
        g.sz = (g.n[0] + 2) * (g.n[1] + 2);
        g.off = (int)(tb.tail_off[(size_t)dm * MAXLEV + l] - first);
        g.ncell = g.n[0] * g.n[1] * g.n[2];
        g.npad = g.sz * (dim == 3 ? g.n[2] + 2 : 1);
        g.rh = (g.n[0] + 1) / 2;
        g.inv_rh = 1.0f / (float)g.rh;
        g.inv_n0 = 1.0f / (float)g.n[0];
        g.inv_n1 = 1.0f / (float)g.n[1];
        for (int a = 0; a < 3; a++) g.lg[a] = (g.n[a] & (g.n[a] - 1)) == 0 ? __builtin_ctz(g.n[a]) : -1;
        g.lrh = (g.rh & (g.rh - 1)) == 0 ? __builtin_ctz(g.rh) : -1;
        g.ghost_pass = 0;
        for (int a = 0; a < dim; a++) {
            if (tb.bck[6 * dm + 2 * a] == MG_BC_PERIODIC && (g.n[a] & 1)) g.ghost_pass = 1;
            g.h[a] = h[a];
            g.ih2[a] = 1.0 / (h[a] * h[a]);
        }
        for (int a = dim; a < 3; a++) {
            g.h[a] = 1.0;
            g.ih2[a] = 0.0;
        }
        g.lam = tb.lambda;
        g.axi = tb.axi;
        g.rlo = tb.axi ? tb.lox[dm] : 0.0;
        g.inv_den = 1.0 / (2.0 * (g.ih2[0] + g.ih2[1] + g.ih2[2]) + g.lam);
        lv[l] = g;
    }
    if (threadIdx.x < 6) {
        bc->kind[threadIdx.x] = tb.bck[6 * dm + threadIdx.x];
        bc->value[threadIdx.x] = tb.bcv[6 * dm + threadIdx.x];
    }
}

// One workgroup per domain in the mask: the grids 0..tail_top of the domain run a
// V-cycle or an FMG cycle.
// LDS: the domain's grids are copied into LDS and cycled there (the host launches
// this form only for domains whose grids fit); else they are cycled in global memory.
// The two forms are separate kernels: each holds one copy of the cycle code, which
// keeps the instruction footprint within the instruction cache.
template <typename T, int D, bool VAR, bool LDS>
__global__ void __launch_bounds__((tail_threads<VAR, D>())) k_tail(Plane<T> P, DevTables tb, int mode, uint64_t mask,
                                                              TailParams tp, int32_t *steps_out, int lds_bytes) {
    constexpr int NT = tail_threads<VAR, D>();
    extern __shared__ double smem[];
    __shared__ double red[16];
    __shared__ TailLev lvs[MAXLEV];
    __shared__ TailBC bcs;
    __shared__ int ops[kTailOps];
    __shared__ int nops;
    const int dm = blockIdx.x;
    if (!((mask >> dm) & 1)) return;
    const int top = tb.tail_top[dm];
    int64_t first;
    const int n = (int)tail_span(tb, dm, top, D, &first);
    // LDS holds v and f of every grid, v_old below the top grid (v_old of the top grid
    // is written to global memory, where the block level above reads it) and eps.  The
    // cycle reads only v and f of the top grid (and eps) from outside and leaves only v
    // and v_old of the top grid to the outside, so only those are copied.
    const int nold = (int)(tail_last_off(tb, dm, top) - first);    // v_old cells below the top grid
    const int64_t lds_need = (2 * (int64_t)n + nold + (VAR ? n : 0)) * (int64_t)sizeof(T);
    int steps;
    if (LDS) {
        if (lds_need > lds_bytes) {   // the host's fit test disagrees: leave the grids untouched
            if (threadIdx.x == 0) steps_out[dm] = -1;
            return;
        }
        T *sv = reinterpret_cast<T *>(smem);
        T *sf = sv + n, *so = sf + n, *se = so + nold;
        // The top grid (padded) is the last one: offset nold, n - nold cells.  Its copy
        // needs no set-up data, so its loads and the set-up's table loads are in flight
        // together; all loads of a batch come before its first LDS store.
        const int toff = nold, tnp = n - nold;
        constexpr int CB = 8;
        tail_setup(tb, dm, top + 1, D, first, lvs, &bcs);
        if (threadIdx.x == 0) nops = tail_ops(ops, mode, top);
        for (int q0 = 0; q0 < tnp; q0 += CB * NT) {
            T a[CB], c[CB];
#pragma unroll
            for (int r = 0; r < CB; r++) {
                const int q = q0 + threadIdx.x + r * NT;
                if (q < tnp) {
                    a[r] = P.tv[first + toff + q];
                    c[r] = P.tf[first + toff + q];
                }
            }
#pragma unroll
            for (int r = 0; r < CB; r++) {
                const int q = q0 + threadIdx.x + r * NT;
                if (q < tnp) {
                    sv[toff + q] = a[r];
                    sf[toff + q] = c[r];
                }
            }
        }
        if (VAR)
            for (int q0 = 0; q0 < n; q0 += CB * NT) {
                T a[CB];
#pragma unroll
                for (int r = 0; r < CB; r++) {
                    const int q = q0 + threadIdx.x + r * NT;
                    if (q < n) a[r] = P.teps[first + q];
                }
#pragma unroll
                for (int r = 0; r < CB; r++) {
                    const int q = q0 + threadIdx.x + r * NT;
                    if (q < n) se[q] = a[r];
                }
            }
        __syncthreads();
        const Tail<T, D, VAR> tl{lvs, bcs, red, sv, so, sf, VAR ? se : nullptr, P.tvold + first, top,
                                 P.tv2 ? P.tv2 + first : nullptr, tp.jacobi, tp.omega};
        steps = tl.run(ops, __builtin_amdgcn_readfirstlane(nops), tp);
        for (int q = threadIdx.x; q < tnp; q += NT) P.tv[first + toff + q] = sv[toff + q];
    } else {
        tail_setup(tb, dm, top + 1, D, first, lvs, &bcs);
        if (threadIdx.x == 0) nops = tail_ops(ops, mode, top);
        __syncthreads();
        const Tail<T, D, VAR> tl{lvs, bcs, red, P.tv + first, P.tvold + first, P.tf + first,
                                 VAR ? P.teps + first : nullptr, nullptr, top,
                                 P.tv2 ? P.tv2 + first : nullptr, tp.jacobi, tp.omega};
        steps = tl.run(ops, __builtin_amdgcn_readfirstlane(nops), tp);
    }
    if (threadIdx.x == 0) steps_out[dm] = steps;
}

// eps on the tail grids: restrict down from the top tail grid, then ghost layers.
template <typename T, int D>
__global__ void __launch_bounds__(tail_threads<true>()) k_tail_eps(Plane<T> P, DevTables tb, int nt) {
    constexpr int NT = tail_threads<true>();
    static_assert(NT == Tail<T, D, true>::NT, "the Tail methods called here stride by Tail::NT");
    __shared__ double red[16];
    __shared__ TailLev lvs[MAXLEV];
    __shared__ TailBC bcs;
    const int dm = blockIdx.x;
    int64_t first;
    tail_span(tb, dm, nt - 1, D, &first);
    tail_setup(tb, dm, nt, D, first, lvs, &bcs);
    __syncthreads();
    const Tail<T, D, true> tl{lvs, bcs, red, P.tv + first, P.tvold + first, P.tf + first, P.teps + first,
                              nullptr, nt - 1, nullptr, 0, 0.0};
    for (int l = nt - 1; l >= 1; l--) {
        const TailLev &gf = lvs[l], &gc = lvs[l - 1];
        for (int c = threadIdx.x; c < gc.ncell; c += NT) {
            int I, J, K;
            tl.cell(gc, c, I, J, K);
            T s = T(0);
            for (int q = 0; q < (1 << D); q++)
                s += tl.teps[tix<D>(gf, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), D == 3 ? 2 * K + (q >> 2) : 0)];
            tl.teps[tix<D>(gc, I, J, K)] = s / T(1 << D);
        }
        __syncthreads();
    }
    for (int l = 0; l < nt; l++) {
        tl.fill_ghosts(l, tl.teps, true);
        __syncthreads();
    }
}

// ------------------------------------------------- large tail grids (uniform)
// Tail levels with many cells run as ordinary multi-workgroup launches over one
// domain's uniform grid (one ghost layer).  The operations are those of the block
// levels: a colour of Gauss-Seidel that pushes the mirroring ghosts (every axis has
// an even cell count, so a ghost has the colour of the cell it mirrors), the
// restriction with the residual, the FAS right-hand side and the correction.
__device__ __forceinline__ int64_t uidx(const UGrid &g, int i, int j, int k, int dim) {
    if (dim == 2) return g.off + (int64_t)(j + 1) * (g.n[0] + 2) + (i + 1);
    return g.off + ((int64_t)(k + 1) * (g.n[1] + 2) + (j + 1)) * (g.n[0] + 2) + (i + 1);
}

template <typename T, int D, bool VAR>
__device__ __forceinline__ void ustencil(const Plane<T> &P, const DevTables &tb, const UGrid &g, int i, int j, int k,
                                         T *w, T *nb) {
    nb[0] = P.tv[uidx(g, i - 1, j, k, D)];
    nb[1] = P.tv[uidx(g, i + 1, j, k, D)];
    nb[2] = P.tv[uidx(g, i, j - 1, k, D)];
    nb[3] = P.tv[uidx(g, i, j + 1, k, D)];
    if (D == 3) {
        nb[4] = P.tv[uidx(g, i, j, k - 1, D)];
        nb[5] = P.tv[uidx(g, i, j, k + 1, D)];
    }
    for (int f = 0; f < 2 * D; f++) w[f] = T(1.0 / (g.h[f >> 1] * g.h[f >> 1]));
    if (VAR) {
        const T e0 = P.teps[uidx(g, i, j, k, D)];
        const int o[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
        for (int f = 0; f < 2 * D; f++) w[f] *= harm(e0, P.teps[uidx(g, o[f][0], o[f][1], o[f][2], D)]);
    }
    if (D == 2 && tb.axi) {
        double fm, fp;
        axi_factors<D>(tb, g.dm, g.h[0], i, fm, fp);
        w[0] *= T(fm);
        w[1] *= T(fp);
    }
}

// Writes the ghosts that mirror cell (i,j,k) of a uniform grid after it changed.
template <typename T, int D>
__device__ __forceinline__ void upush(const Plane<T> &P, const DevTables &tb, const UGrid &g, int i, int j, int k,
                                      T nv) {
    const int c[3] = {i, j, k};
    for (int a = 0; a < D; a++) {
        int side;
        if (c[a] == 0) side = 0;
        else if (c[a] == g.n[a] - 1) side = 1;
        else continue;
        const int f = 2 * a + side;
        int q[3] = {i, j, k};
        const int kind = tb.bck[6 * g.dm + f];
        T val;
        if (kind == MG_BC_PERIODIC) {
            q[a] = side ? -1 : g.n[a];      // the opposite face's ghost
            val = nv;
        } else {
            q[a] = side ? g.n[a] : -1;
            val = bc_ghost<T>(kind, tb.bcv[6 * g.dm + f], g.h[a], side, nv);
        }
        P.tv[uidx(g, q[0], q[1], q[2], D)] = val;
    }
}

template <typename T, int D, bool VAR>
__global__ void __launch_bounds__(256) k_ugsrb(Plane<T> P, DevTables tb, UGrid g, int colour) {
    const int half = g.n[0] / 2;
    const int64_t nh = (int64_t)half * g.n[1] * (D == 3 ? g.n[2] : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nh) return;
    const int row = (int)(q / half), pos = (int)(q % half);
    const int j = row % g.n[1], k = D == 3 ? row / g.n[1] : 0;
    const int i = 2 * pos + ((j + k + colour) & 1);
    T w[6], nb[6];
    ustencil<T, D, VAR>(P, tb, g, i, j, k, w, nb);
    T num = T(0), den = T(tb.lambda);
    for (int f = 0; f < 2 * D; f++) {
        num += w[f] * nb[f];
        den += w[f];
    }
    const int64_t o = uidx(g, i, j, k, D);
    const T nv = (num - P.tf[o]) / den;
    P.tv[o] = nv;
    upush<T, D>(P, tb, g, i, j, k, nv);
}

// Weighted Jacobi step on a large coarse grid: src -> dst (padded tail arrays).
template <typename T, int D, bool VAR>
__global__ void __launch_bounds__(256) k_ujacobi(Plane<T> P, const T *src, T *dst, DevTables tb, UGrid g,
                                                 double omega) {
    const int64_t n = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % g.n[0]);
    const int r = (int)(q / g.n[0]);
    const int j = r % g.n[1], k = D == 3 ? r / g.n[1] : 0;
    Plane<T> S = P, Q = P;
    S.tv = const_cast<T *>(src);
    Q.tv = dst;
    T w[6], nb[6];
    ustencil<T, D, VAR>(S, tb, g, i, j, k, w, nb);
    T num = T(0), den = T(tb.lambda);
    for (int f = 0; f < 2 * D; f++) {
        num += w[f] * nb[f];
        den += w[f];
    }
    const int64_t o = uidx(g, i, j, k, D);
    const T vc = src[o];
    const T nv = vc + T(omega) * ((num - P.tf[o]) / den - vc);
    dst[o] = nv;
    upush<T, D>(Q, tb, g, i, j, k, nv);
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_ughost(Plane<T> P, DevTables tb, UGrid g) {
    const int64_t n = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % g.n[0]);
    const int r = (int)(q / g.n[0]);
    const int j = r % g.n[1], k = D == 3 ? r / g.n[1] : 0;
    const bool edge = i == 0 || i == g.n[0] - 1 || j == 0 || j == g.n[1] - 1 ||
                      (D == 3 && (k == 0 || k == g.n[2] - 1));
    if (edge) upush<T, D>(P, tb, g, i, j, k, P.tv[uidx(g, i, j, k, D)]);
}

template <typename T, int D, bool VAR>
__global__ void __launch_bounds__(256) k_ufas(Plane<T> P, DevTables tb, UGrid g) {
    const int64_t npad = (int64_t)(g.n[0] + 2) * (g.n[1] + 2) * (D == 3 ? g.n[2] + 2 : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= npad) return;
    P.tvold[g.off + q] = P.tv[g.off + q];
    const int i = (int)(q % (g.n[0] + 2)) - 1;
    const int r = (int)(q / (g.n[0] + 2));
    const int j = r % (g.n[1] + 2) - 1, k = D == 3 ? r / (g.n[1] + 2) - 1 : 0;
    if (i < 0 || i >= g.n[0] || j < 0 || j >= g.n[1] || (D == 3 && (k < 0 || k >= g.n[2]))) return;
    T w[6], nb[6];
    ustencil<T, D, VAR>(P, tb, g, i, j, k, w, nb);
    const T vc = P.tv[g.off + q];
    T lv = -T(tb.lambda) * vc;
    for (int f = 0; f < 2 * D; f++) lv += w[f] * (nb[f] - vc);
    P.tf[g.off + q] += lv;
}

template <typename T, int D, bool VAR>
__global__ void __launch_bounds__(256) k_urestrict(Plane<T> P, DevTables tb, UGrid g, UGrid gc) {
    const int64_t n = (int64_t)gc.n[0] * gc.n[1] * (D == 3 ? gc.n[2] : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int I = (int)(q % gc.n[0]);
    const int r = (int)(q / gc.n[0]);
    const int J = r % gc.n[1], K = D == 3 ? r / gc.n[1] : 0;
    T sv = T(0), sr = T(0);
    for (int c = 0; c < (1 << D); c++) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = D == 3 ? 2 * K + (c >> 2) : 0;
        T w[6], nb[6];
        ustencil<T, D, VAR>(P, tb, g, i, j, k, w, nb);
        const int64_t o = uidx(g, i, j, k, D);
        const T vc = P.tv[o];
        T lv = -T(tb.lambda) * vc;
        for (int f = 0; f < 2 * D; f++) lv += w[f] * (nb[f] - vc);
        sv += vc;
        sr += P.tf[o] - lv;
    }
    const T inv = T(1) / T(1 << D);
    const int64_t oc = uidx(gc, I, J, K, D);
    P.tv[oc] = sv * inv;
    P.tf[oc] = sr * inv;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_ucorrect(Plane<T> P, DevTables tb, UGrid g, UGrid gc) {
    const int64_t n = (int64_t)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % g.n[0]);
    const int r = (int)(q / g.n[0]);
    const int j = r % g.n[1], k = D == 3 ? r / g.n[1] : 0;
    const int p[3] = {i >> 1, j >> 1, k >> 1};
    const int sg[3] = {(i & 1) ? 1 : -1, (j & 1) ? 1 : -1, (k & 1) ? 1 : -1};
    const int64_t o = uidx(gc, p[0], p[1], p[2], D);
    const T d0 = P.tv[o] - P.tvold[o];
    T dn[3];
    for (int a = 0; a < D; a++) {
        int c[3] = {p[0], p[1], p[2]};
        c[a] += sg[a];
        const int64_t oq = uidx(gc, c[0], c[1], c[2], D);
        dn[a] = P.tv[oq] - P.tvold[oq];
    }
    const T corr = D == 2 ? T(0.25) * (T(2) * d0 + dn[0] + dn[1]) : T(0.25) * (d0 + dn[0] + dn[1] + dn[2]);
    const int64_t of = uidx(g, i, j, k, D);
    const T nv = P.tv[of] + corr;
    P.tv[of] = nv;
    upush<T, D>(P, tb, g, i, j, k, nv);
}

// ------------------------------------------------------------ small utilities
template <typename T>
__global__ void k_fill(T *p, size_t n, T value) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < n; i += stride) p[i] = value;
}

template <typename T>
__global__ void k_copy(T *dst, const T *src, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < n; i += stride) dst[i] = src[i];
}

// Leaf-ordered user array (x fastest within a block) <-> colour-split block storage.
template <typename T, int D, int BS, bool TO_BLOCKS>
__global__ void __launch_bounds__(256) k_scatter(T *blk, double *user, DevTables tb, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t rank = blockIdx.x / wg_per_block;
    const int64_t b = tb.leaf_blk[rank];
    const int t = (blockIdx.x % wg_per_block) * (g::NC < 256 ? g::NC : 256) + threadIdx.x;
    if (t >= g::NC) return;
    int i = t % BS, j = (t / BS) % BS, k = D == 3 ? t / (BS * BS) : 0;
    int64_t o = b * g::NC + g::in(i, j, k);
    if (TO_BLOCKS) blk[o] = T(user[rank * g::NC + t]);
    else user[rank * g::NC + t] = (double)blk[o];
}

// ------------------------------------------------------------------ norms
// Workgroup-wide sum and max (wave shuffles, then one LDS exchange).
template <int TPB>
__device__ __forceinline__ void block_reduce4(double &mr, double &sr, double &mf, double &sf) {
    __shared__ double red[4][TPB / 64];
    for (int o = 32; o > 0; o >>= 1) {
        double a = __shfl_xor(mr, o), b = __shfl_xor(sr, o), c = __shfl_xor(mf, o), d = __shfl_xor(sf, o);
        if (a > mr || a != a) mr = a;
        sr += b;
        mf = fmax(mf, c);
        sf += d;
    }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = mr; red[1][w] = sr; red[2][w] = mf; red[3][w] = sf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < TPB / 64; q++) {
            if (red[0][q] > mr || red[0][q] != red[0][q]) mr = red[0][q];
            sr += red[1][q];
            mf = fmax(mf, red[2][q]);
            sf += red[3][q];
        }
    }
}

// Composite residual r = f - L v on every leaf block (FP64), with per-block partial
// max |r|, sum vol r^2, max |f|, sum vol f^2; optionally writes r into the leaf
// blocks of an output field (the right-hand side of an FP32 correction solve) or into
// a leaf vector (rank-major, see the Krylov section).  Without f (P.f null) the
// vector receives L v instead: the operator applied to v.
// One workgroup per leaf block, v with its ghosts staged in LDS (16-byte loads, all
// issued before the first LDS store).
// ADD: the block first takes the FP32 correction, v += e, and the residual is that of
// the corrected v.  Same-level ghosts become ghost(v) + ghost(e) (both hold the
// neighbour's values, so the sum is the neighbour's new value, rounded the same way),
// physical-boundary ghosts are recomputed from the new boundary cells, and v and the
// block's own ghosts are written back.  Only for trees without refinement: there are
// no coarse-fine ghosts, and no block writes another block's memory.
template <int D, int BS, bool VAR, bool ADD, int TPB>
__global__ void __launch_bounds__(TPB) k_resid(Plane<double> P, DevTables tb, const float *__restrict__ e,
                                               const float *__restrict__ eg, double *partials, float *rout32,
                                               double *rout64) {
    using g = G<D, BS>;
    constexpr int NP = g::NC / 2, NGP = g::NG / 2;   // 16-byte pairs
    constexpr int IP = (NP + TPB - 1) / TPB, IG = (NGP + TPB - 1) / TPB;
    constexpr int IT = (g::NC + TPB - 1) / TPB;
    __shared__ __align__(16) double s_v[g::NC + g::NG];
    const int rank = blockIdx.x;
    const int64_t b = tb.leaf_blk[rank];
    const int tid = threadIdx.x;
    double2 vr[IP], gr[IG];
    float2 er[ADD ? IP : 1], egr[ADD ? IG : 1];
#pragma unroll
    for (int m = 0; m < IP; m++) {
        int p = tid + m * TPB;
        if (NP % TPB != 0) p = p < NP ? p : NP - 1;
        vr[m] = reinterpret_cast<const double2 *>(P.v + b * g::NC)[p];
        if (ADD) er[m] = reinterpret_cast<const float2 *>(e + b * g::NC)[p];
    }
#pragma unroll
    for (int m = 0; m < IG; m++) {
        int p = tid + m * TPB;
        if (NGP % TPB != 0) p = p < NGP ? p : NGP - 1;
        gr[m] = reinterpret_cast<const double2 *>(P.vg + b * g::NG)[p];
        if (ADD) egr[m] = reinterpret_cast<const float2 *>(eg + b * g::NG)[p];
    }
    double fr[IT];
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int t = tid + m * TPB;
        fr[m] = P.f ? P.f[b * g::NC + (g::NC % TPB == 0 || t < g::NC ? t : 0)] : 0.0;
    }
    BlockCtx<D> cx;
    cx.load(tb, b, tb.lev[b]);
    const int dm = cx.dm;
    const double h0 = cx.h[0], h1 = cx.h[1], h2 = D == 3 ? cx.h[2] : 1.0;
    unsigned same = 0;   // faces with a same-level neighbour (bit f); constant indices only
#pragma unroll
    for (int f = 0; f < 2 * D; f++) same |= (cx.nbr[f] >= 0 ? 1u : 0u) << f;
#pragma unroll
    for (int m = 0; m < IP; m++) {
        const int p = tid + m * TPB;
        if (NP % TPB != 0 && p >= NP) break;
        double2 nv = vr[m];
        if (ADD) {
            nv.x += (double)er[m].x;
            nv.y += (double)er[m].y;
            reinterpret_cast<double2 *>(P.v + b * g::NC)[p] = nv;
        }
        reinterpret_cast<double2 *>(s_v)[p] = nv;
    }
#pragma unroll
    for (int m = 0; m < IG; m++) {
        const int p = tid + m * TPB;
        if (NGP % TPB != 0 && p >= NGP) break;
        double2 ng = gr[m];
        if (ADD) {
            if (!((same >> (2 * p / g::NF)) & 1u)) continue;   // physical face: below
            ng.x += (double)egr[m].x;
            ng.y += (double)egr[m].y;
            reinterpret_cast<double2 *>(P.vg + b * g::NG)[p] = ng;
        }
        reinterpret_cast<double2 *>(s_v + g::NC)[p] = ng;
    }
    if (ADD) {
        // physical-boundary ghosts from the corrected boundary cells
        __syncthreads();
#pragma unroll
        for (int f = 0; f < 2 * D; f++) {
            if (cx.nbr[f] != -1) continue;
            const int a = f >> 1, side = f & 1, c = side ? BS - 1 : 0;
            for (int r = tid; r < g::NF; r += TPB) {
                // invert g::gh: colour half, then tangential coordinates (a1, a2)
                const int par = r / (g::NF / 2), rr = r % (g::NF / 2);
                const int a2 = D == 3 ? rr / g::RH : 0;
                const int a1 = 2 * (rr % g::RH) + ((par + a2 + (side ^ 1)) & 1);
                const int i = a == 0 ? c : a1, j = a == 1 ? c : (a == 0 ? a1 : a2), k = a == 2 ? c : a2;
                const double gv = bc_ghost<double>(cx.bck[f], cx.bcv[f], cx.h[a], side, s_v[g::in(i, j, k)]);
                s_v[g::NC + f * g::NF + r] = gv;
                P.vg[b * g::NG + f * g::NF + r] = gv;
            }
        }
    }
    __syncthreads();
    double ih2[3];
    ih2[0] = 1.0 / (h0 * h0);
    ih2[1] = 1.0 / (h1 * h1);
    ih2[2] = 1.0 / (h2 * h2);
    const double vol = h0 * h1 * (D == 3 ? h2 : 1.0);
    double mr = 0, sr = 0, mf = 0, sf = 0;
#pragma unroll
    for (int m = 0; m < IT; m++) {
        const int t = tid + m * TPB;
        if (g::NC % TPB != 0 && t >= g::NC) break;
        int i, j, k;
        g::decode(t, i, j, k);
        const double vc = s_v[t];
        double nb[6];
        nb[0] = i > 0 ? s_v[g::in(i - 1, j, k)] : s_v[g::NC + g::gh(0, j, k)];
        nb[1] = i < BS - 1 ? s_v[g::in(i + 1, j, k)] : s_v[g::NC + g::gh(1, j, k)];
        nb[2] = j > 0 ? s_v[g::in(i, j - 1, k)] : s_v[g::NC + g::gh(2, i, k)];
        nb[3] = j < BS - 1 ? s_v[g::in(i, j + 1, k)] : s_v[g::NC + g::gh(3, i, k)];
        if (D == 3) {
            nb[4] = k > 0 ? s_v[g::in(i, j, k - 1)] : s_v[g::NC + g::gh(4, i, j)];
            nb[5] = k < BS - 1 ? s_v[g::in(i, j, k + 1)] : s_v[g::NC + g::gh(5, i, j)];
        }
        if (D == 2 && tb.axi) {   // axisymmetric x-face factors (see axi_factors)
            double fm, fp;
            axi_factors<D>(tb, dm, h0, cx.orgx + i, fm, fp);
            nb[0] = vc + fm * (nb[0] - vc);
            nb[1] = vc + fp * (nb[1] - vc);
        }
        double lv = 0.0;
        if (!VAR) {
            for (int f = 0; f < 2 * D; f++) lv += ih2[f >> 1] * (nb[f] - vc);
        } else {
            const double e0 = P.eps[b * g::NC + t];
            double en[6];
            en[0] = ld<D, BS>(P.eps, P.epsg, b, i - 1, j, k);
            en[1] = ld<D, BS>(P.eps, P.epsg, b, i + 1, j, k);
            en[2] = ld<D, BS>(P.eps, P.epsg, b, i, j - 1, k);
            en[3] = ld<D, BS>(P.eps, P.epsg, b, i, j + 1, k);
            if (D == 3) {
                en[4] = ld<D, BS>(P.eps, P.epsg, b, i, j, k - 1);
                en[5] = ld<D, BS>(P.eps, P.epsg, b, i, j, k + 1);
            }
            for (int f = 0; f < 2 * D; f++) lv += harm(e0, en[f]) * ih2[f >> 1] * (nb[f] - vc);
        }
        lv -= tb.lambda * vc;
        const double fv = fr[m];
        const double r = fv - lv;
        if (fabs(r) > mr || r != r) mr = fabs(r);
        if (fabs(fv) > mf) mf = fabs(fv);
        sr += vol * r * r;
        sf += vol * fv * fv;
        if (rout32) rout32[b * g::NC + t] = (float)r;
        if (rout64) rout64[rank * g::NC + t] = P.f ? r : lv;
    }
    block_reduce4<TPB>(mr, sr, mf, sf);
    if (tid == 0) {
        double *o = partials + 4 * (int64_t)rank;
        o[0] = mr; o[1] = sr; o[2] = mf; o[3] = sf;
    }
}

// Per-domain combination of the per-block partials (fixed order: deterministic).
__global__ void __launch_bounds__(256) k_reduce_norms(DevTables tb, const double *partials, double *out,
                                                      double *host_out) {
    __shared__ double sm[4][256];
    const int dm = blockIdx.x;
    const int r0 = tb.leaf_first[dm], r1 = tb.leaf_first[dm + 1];
    double mr = 0, sr = 0, mf = 0, sf = 0;
    for (int r = r0 + threadIdx.x; r < r1; r += 256) {
        const double *p = partials + 4 * (int64_t)r;
        if (p[0] > mr || p[0] != p[0]) mr = p[0];
        sr += p[1];
        mf = fmax(mf, p[2]);
        sf += p[3];
    }
    sm[0][threadIdx.x] = mr; sm[1][threadIdx.x] = sr; sm[2][threadIdx.x] = mf; sm[3][threadIdx.x] = sf;
    __syncthreads();
    for (int st = 256 / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            double o = sm[0][threadIdx.x + st];
            if (o > sm[0][threadIdx.x] || o != o) sm[0][threadIdx.x] = o;
            sm[1][threadIdx.x] += sm[1][threadIdx.x + st];
            sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + st]);
            sm[3][threadIdx.x] += sm[3][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        out[4 * dm + threadIdx.x] = sm[threadIdx.x][0];
        if (host_out) host_out[4 * dm + threadIdx.x] = sm[threadIdx.x][0];
    }
}

// v64 += v32 on every leaf block (the FP64 update of iterative refinement), with the
// same-level and boundary ghosts of the FP64 field pushed.
// (The source is FP32 block storage, or an FP64 leaf vector when VEC.)  Each thread
// takes one row of one colour (RH consecutive storage cells), read and written as
// vectors, and pushes the row's ghosts with push_run.
template <int D, int BS>
constexpr int add_leaf_threads() { return G<D, BS>::NC / G<D, BS>::RH < 256 ? G<D, BS>::NC / G<D, BS>::RH : 256; }
template <int D, int BS, typename S, bool VEC>
__global__ void __launch_bounds__(256) k_add_leaf(double *v64, double *vg64, const S *src, DevTables tb,
                                                  int wg_per_block) {
    using g = G<D, BS>;
    constexpr int R = g::RH;
    const int64_t rank = blockIdx.x / wg_per_block;
    const int64_t b = tb.leaf_blk[rank];
    const int t0 = ((blockIdx.x % wg_per_block) * add_leaf_threads<D, BS>() + threadIdx.x) * R;
    if (t0 >= g::NC) return;
    BlockCtx<D> cx;
    cx.load(tb, b, tb.lev[b]);
    double v[R];
    S e[R];
    ld_run<double, R>(v64 + b * g::NC + t0, v);
    ld_run<S, R>(src + (VEC ? rank : b) * g::NC + t0, e);
#pragma unroll
    for (int m = 0; m < R; m++) v[m] += (double)e[m];
    st_run<double, R>(v64 + b * g::NC + t0, v);
    const int col = t0 >= g::NH, row = (t0 - col * g::NH) / R;
    const int j = row % BS, k = D == 3 ? row / BS : 0;
    push_run<double, D, BS, R>(vg64, cx, b, (j + k + col) & 1, j, k, v);
}

// dJ/deps per leaf cell from phi (v plane, ghosts filled) and lambda (blocks + ghosts).
template <int D, int BS>
__global__ void __launch_bounds__(256) k_face_grad(Plane<double> P, DevTables tb, const double *lam,
                                                   const double *lamg, double *out, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t rank = blockIdx.x / wg_per_block;
    const int64_t b = tb.leaf_blk[rank];
    const int dm = tb.dom[b], lev = tb.lev[b];
    const Spacing s = spacing(tb, dm, lev);
    {
        const int t = (blockIdx.x % wg_per_block) * (g::NC < 256 ? g::NC : 256) + threadIdx.x;
        if (t >= g::NC) return;
        int i = t % BS, j = (t / BS) % BS, k = D == 3 ? t / (BS * BS) : 0;
        int c = g::in(i, j, k);
        double p0 = P.v[b * g::NC + c], l0 = lam[b * g::NC + c], e0 = P.eps[b * g::NC + c];
        double acc = 0.0;
        int co[3] = {i, j, k};
        for (int f = 0; f < 2 * D; f++) {
            int a = f >> 1, side = f & 1;
            int q[3] = {i, j, k};
            q[a] += side ? 1 : -1;
            double pn = ld<D, BS>(P.v, P.vg, b, q[0], q[1], q[2]);
            bool outside = (co[a] == (side ? BS - 1 : 0)) && tb.nbr[6 * b + f] == -1;
            if (outside) {
                acc += -s.ih2[a] * l0 * (pn - p0);
            } else {
                double en = ld<D, BS>(P.eps, P.epsg, b, q[0], q[1], q[2]);
                double ln = ld<D, BS>(lam, lamg, b, q[0], q[1], q[2]);
                double sum = e0 + en;
                acc += s.ih2[a] * (2.0 * en * en / (sum * sum)) * (ln - l0) * (pn - p0);
            }
        }
        out[rank * g::NC + t] = acc;
    }
}

// ----------------------------------------------- elliptic divergence cleaning
// Sec. 4.1 on trees without refinement.  B is given per component as a leaf array
// (leaf block by leaf block, cells x fastest), one thread per leaf cell.
// The value of component B_d o cells along x_d from local cell (i,j,k) of leaf block
// b (rank r): a same-level neighbour's cell across the face, or (physical face) the
// block's boundary cell repeated.  |o| <= 2 <= BS.
template <int D, int BS>
__device__ __forceinline__ double divb_at(const double *__restrict__ Bd, const DevTables &tb, int64_t b, int64_t r,
                                          int t, int cd, int sd, int d, int o) {
    using g = G<D, BS>;
    const int q = cd + o;
    if (q >= 0 && q < BS) return Bd[r * g::NC + t + o * sd];
    const int side = q >= BS;
    const int n = tb.nbr[6 * b + 2 * d + side];
    if (n >= 0) return Bd[(int64_t)tb.leaf_rank[n] * g::NC + t + (side ? o - BS : o + BS) * sd];
    return Bd[r * g::NC + t + ((side ? BS - 1 : 0) - cd) * sd];
}

// out (+)= dB_d/dx_d: eq. divb-central-diff (ORDER 2) or eq. divb-4th-order (ORDER 4).
template <int D, int BS, int ORDER>
__global__ void __launch_bounds__(256) k_divb(const double *__restrict__ Bd, double *__restrict__ out, DevTables tb,
                                              int d, int accumulate, int64_t ncells) {
    using g = G<D, BS>;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= ncells) return;
    const int64_t r = id / g::NC;
    const int t = (int)(id % g::NC);
    const int64_t b = tb.leaf_blk[r];
    const int i = t % BS, j = (t / BS) % BS, k = D == 3 ? t / (BS * BS) : 0;
    const int cd = d == 0 ? i : (d == 1 ? j : k);
    const int sd = d == 0 ? 1 : (d == 1 ? BS : BS * BS);
    const double h = tb.h[((size_t)tb.dom[b] * MAXLEV + tb.lev[b]) * 3 + d];
    double der;
    if (ORDER == 2) {
        der = (divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, 1) - divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, -1)) /
              (2.0 * h);
    } else {
        const double p2 = divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, 2), p1 = divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, 1);
        const double m1 = divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, -1), m2 = divb_at<D, BS>(Bd, tb, b, r, t, cd, sd, d, -2);
        der = (-p2 + 8.0 * p1 - 8.0 * m1 + m2) / (12.0 * h);
    }
    out[id] = accumulate ? out[id] + der : der;
}

// B_d -= dphi/dx_d (eq. poisson-divb-cleaning, second-order central differences of
// phi with its ghost cells); e += (B_new^2 - B_old^2) / 2 (eq. divb-pressure-fix).
template <int D, int BS>
__global__ void __launch_bounds__(256) k_divb_project(Plane<double> P, double *__restrict__ Bd, double *__restrict__ e,
                                                      DevTables tb, int d, int64_t ncells) {
    using g = G<D, BS>;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= ncells) return;
    const int64_t r = id / g::NC;
    const int t = (int)(id % g::NC);
    const int64_t b = tb.leaf_blk[r];
    const int i = t % BS, j = (t / BS) % BS, k = D == 3 ? t / (BS * BS) : 0;
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const double h = tb.h[((size_t)tb.dom[b] * MAXLEV + tb.lev[b]) * 3 + d];
    const double gp = (ld<D, BS>(P.v, P.vg, b, i + di, j + dj, k + dk) - ld<D, BS>(P.v, P.vg, b, i - di, j - dj, k - dk)) /
                      (2.0 * h);
    const double bo = Bd[id], bn = bo - gp;
    Bd[id] = bn;
    if (e) e[id] += 0.5 * (bn * bn - bo * bo);
}

// ------------------------------------------------------ free-space boundaries
// Sec. 2.8: the right-hand side restricted to a uniform level c = 2^k leaf cells
// coarser, the free-space potential of that grid on the six boundary planes (coarse
// face centres plus one ghost position on each side of a row), linear interpolation of
// the planes to the leaf faces, and those Dirichlet values folded into the right-hand
// side of a solve with homogeneous faces: f -= 2 a / h^2 per boundary face (the
// Dirichlet ghost 2a - phi_b of Sec. 2.6).  The potential of the coarse grid is summed
// directly, each coarse cell a point charge q = mean(f) h_c^3 at its centre.

// One workgroup per leaf block: the charges of the coarse cells inside it (c <= BS).
template <int BS>
__global__ void __launch_bounds__(256) k_fs_charge(const double *__restrict__ f, DevTables tb,
                                                   const FsDom *__restrict__ fd, int c, double *__restrict__ q) {
    using g = G<3, BS>;
    const int64_t b = tb.leaf_blk[blockIdx.x];
    const FsDom d = fd[tb.dom[b]];
    const int m = BS / c;
    const int ox = tb.org[3 * b] / c, oy = tb.org[3 * b + 1] / c, oz = tb.org[3 * b + 2] / c;
    const double vol = d.hc[0] * d.hc[1] * d.hc[2];
    const double inv = 1.0 / (double)(c * c * c);
    for (int t = threadIdx.x; t < m * m * m; t += 256) {
        const int I = t % m, J = (t / m) % m, K = t / (m * m);
        double s = 0.0;
        for (int kk = 0; kk < c; kk++)
            for (int jj = 0; jj < c; jj++)
                for (int ii = 0; ii < c; ii++) s += f[b * g::NC + g::in(I * c + ii, J * c + jj, K * c + kk)];
        q[d.qoff + ((int64_t)(oz + K) * d.nc[1] + (oy + J)) * d.nc[0] + (ox + I)] = s * inv * vol;
    }
}

// Partial sums sum_c q_c / |x - x_c| at the plane points of domain blockIdx.y over the
// charge rows of slice blockIdx.z; the rows pass through LDS in chunks and every thread
// adds them in index order.
constexpr int kFsChunk = 2048;
__global__ void __launch_bounds__(256) k_fs_plane(const double *__restrict__ q, const FsDom *__restrict__ fd,
                                                  double *__restrict__ partial, int64_t tot_pts, int slices) {
    __shared__ double sq[kFsChunk];
    const FsDom *dp = fd + blockIdx.y;
    const int npts = dp->npts;
    if ((int)blockIdx.x * 256 >= npts) return;   // the whole workgroup is past this domain's points
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool live = p < npts;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (live) {
        int r = p, face = 0;
        while (face < 5 && r >= (int)(dp->pofs[face + 1] - dp->pofs[face])) {
            r -= (int)(dp->pofs[face + 1] - dp->pofs[face]);
            face++;
        }
        const int a = face >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;   // in-plane axes t1 < t2
        const int m1 = dp->nc[t1] + 2;
        const int i1 = r % m1 - 1, i2 = r / m1 - 1;
        const double c1 = dp->lo[t1] + (i1 + 0.5) * dp->hc[t1];
        const double c2 = dp->lo[t2] + (i2 + 0.5) * dp->hc[t2];
        const double ca = (face & 1) ? dp->hi[a] : dp->lo[a];
        px = a == 0 ? ca : c1;
        py = a == 1 ? ca : (a == 0 ? c1 : c2);
        pz = a == 2 ? ca : c2;
    }
    const int nx = dp->nc[0], ny = dp->nc[1], rows = dp->nc[1] * dp->nc[2];
    const double lo0 = dp->lo[0], lo1 = dp->lo[1], lo2 = dp->lo[2];
    const double hc0 = dp->hc[0], hc1 = dp->hc[1], hc2 = dp->hc[2];
    const int64_t qoff = dp->qoff, poff = dp->poff;
    const int r0 = (int)((int64_t)rows * blockIdx.z / slices), r1 = (int)((int64_t)rows * (blockIdx.z + 1) / slices);
    const int rc = kFsChunk / nx;                   // rows per chunk (nx <= kFsChunk)
    double s = 0.0;
    for (int c0 = r0; c0 < r1; c0 += rc) {
        const int nr = min(rc, r1 - c0);
        __syncthreads();
        for (int u = threadIdx.x; u < nr * nx; u += 256) sq[u] = q[qoff + (int64_t)c0 * nx + u];
        __syncthreads();
        if (live) {
            for (int rr = 0; rr < nr; rr++) {
                const int row = c0 + rr, J = row % ny, K = row / ny;
                const double dy = py - (lo1 + (J + 0.5) * hc1);
                const double dz = pz - (lo2 + (K + 0.5) * hc2);
                const double dyz = dy * dy + dz * dz;
                for (int I = 0; I < nx; I++) {
                    const double dx = px - (lo0 + (I + 0.5) * hc0);
                    s += sq[rr * nx + I] * rsqrt(dx * dx + dyz);
                }
            }
        }
    }
    if (live) partial[blockIdx.z * tot_pts + poff + p] = s;
}

// The slices' partial sums in slice order, times -1 / (4 pi).
__global__ void __launch_bounds__(256) k_fs_sum(const double *__restrict__ partial, double *__restrict__ pl,
                                                int64_t tot_pts, int slices) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= tot_pts) return;
    double s = 0.0;
    for (int z = 0; z < slices; z++) s += partial[z * tot_pts + i];
    pl[i] = -s / (4.0 * M_PI);
}

// One workgroup per leaf block on a domain face: the boundary values of its face cells
// by linear interpolation of the plane, folded into f face by face (x-, x+, ..., z+);
// bv (may be null) receives them in the face-by-face order of the public interface.
template <int BS>
__global__ void __launch_bounds__(256) k_fs_fold(double *__restrict__ f, DevTables tb, const FsDom *__restrict__ fd,
                                                 int c, const double *__restrict__ pl, double *__restrict__ bv) {
    using g = G<3, BS>;
    const int64_t b = tb.leaf_blk[blockIdx.x];
    unsigned phys = 0;
#pragma unroll
    for (int face = 0; face < 6; face++) phys |= (tb.nbr[6 * b + face] == -1 ? 1u : 0u) << face;
    if (!phys) return;
    const FsDom d = fd[tb.dom[b]];
    const int o[3] = {tb.org[3 * b], tb.org[3 * b + 1], tb.org[3 * b + 2]};
    for (int t = threadIdx.x; t < g::NC; t += 256) {
        const int cc[3] = {t % BS, (t / BS) % BS, t / (BS * BS)};
        const int64_t at = b * g::NC + g::in(cc[0], cc[1], cc[2]);
        double fv = 0.0;
        bool any = false;
#pragma unroll
        for (int face = 0; face < 6; face++) {
            const int a = face >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            if (!((phys >> face) & 1) || cc[a] != ((face & 1) ? BS - 1 : 0)) continue;
            if (!any) fv = f[at];
            any = true;
            const int j1 = o[t1] + cc[t1], j2 = o[t2] + cc[t2];
            const double u1 = (j1 + 0.5) * d.h[t1] / d.hc[t1] - 0.5, u2 = (j2 + 0.5) * d.h[t2] / d.hc[t2] - 0.5;
            const int i1 = (int)floor(u1), i2 = (int)floor(u2);
            const double w1 = u1 - i1, w2 = u2 - i2;
            const int m1 = d.nc[t1] + 2;
            const double *P = pl + d.poff + d.pofs[face];
            const double p00 = P[(i2 + 1) * m1 + i1 + 1], p01 = P[(i2 + 1) * m1 + i1 + 2];
            const double p10 = P[(i2 + 2) * m1 + i1 + 1], p11 = P[(i2 + 2) * m1 + i1 + 2];
            const double av = (1 - w2) * ((1 - w1) * p00 + w1 * p01) + w2 * ((1 - w1) * p10 + w1 * p11);
            if (bv) bv[d.boff + d.bofs[face] + (int64_t)j2 * d.n[t1] + j1] = av;
            fv -= 2.0 * av / (d.h[a] * d.h[a]);
        }
        if (any) f[at] = fv;
    }
}

// Far-field initial guess for a free-space solve: per domain the total charge Q, its
// first moments and sum |q| of the coarse charges (one workgroup per domain, fixed
// summation order), then on every leaf cell the potential -Q / (4 pi r) of Q at the
// charge centroid, r at least one coarse spacing (zero for a neutral source).
__global__ void __launch_bounds__(256) k_fs_moments(const double *__restrict__ q, const FsDom *__restrict__ fd,
                                                    double *__restrict__ mom) {
    __shared__ double red[5][256];
    const FsDom *dp = fd + blockIdx.x;
    const int nx = dp->nc[0], ny = dp->nc[1], nq = dp->nc[0] * dp->nc[1] * dp->nc[2];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < nq; c += 256) {
        const double v = q[dp->qoff + c];
        const int I = c % nx, J = (c / nx) % ny, K = c / (nx * ny);
        a[0] += v;
        a[1] += v * (dp->lo[0] + (I + 0.5) * dp->hc[0]);
        a[2] += v * (dp->lo[1] + (J + 0.5) * dp->hc[1]);
        a[3] += v * (dp->lo[2] + (K + 0.5) * dp->hc[2]);
        a[4] += fabs(v);
    }
#pragma unroll
    for (int m = 0; m < 5; m++) red[m][threadIdx.x] = a[m];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int m = 0; m < 5; m++) red[m][threadIdx.x] += red[m][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) mom[5 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

template <int BS>
__global__ void __launch_bounds__(256) k_fs_guess(const FsDom *__restrict__ fd, const double *__restrict__ mom,
                                                  DevTables tb, double *__restrict__ out, int64_t ncells) {
    using g = G<3, BS>;
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= ncells) return;
    const int64_t r = id / g::NC;
    const int t = (int)(id % g::NC);
    const int64_t b = tb.leaf_blk[r];
    const int dm = tb.dom[b];
    const FsDom *dp = fd + dm;
    const double *m = mom + 5 * dm;
    const double Q = m[0];
    if (!(fabs(Q) > 1e-12 * m[4])) {
        out[id] = 0.0;
        return;
    }
    const int ii[3] = {t % BS, (t / BS) % BS, t / (BS * BS)};
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double x = dp->lo[a] + (tb.org[3 * b + a] + ii[a] + 0.5) * dp->h[a];
        const double dx = x - m[1 + a] / Q;
        d2 += dx * dx;
    }
    const double rmin = fmin(dp->hc[0], fmin(dp->hc[1], dp->hc[2]));
    out[id] = -Q / (4.0 * M_PI * fmax(sqrt(d2), rmin));
}

// ================================================================ launchers
#define HIPCHK(x) (x)

static inline int cells(int dim, int bs) { return dim == 3 ? bs * bs * bs : bs * bs; }

// ------------------------------------------------------- Krylov vector kernels
// Vectors over the leaf cells are stored rank-major: x[rank * NC + t], rank the leaf
// block's position in leaf order and t the cell's position in the block's
// colour-split storage (a fixed permutation of the leaf order, which inner products
// and linear combinations do not see).
template <typename S, int D, int BS, bool TO_BLOCKS>
__global__ void __launch_bounds__(256) k_vec_blocks(S *blk, double *vec, DevTables tb, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t rank = blockIdx.x / wg_per_block;
    const int t = (blockIdx.x % wg_per_block) * (g::NC < 256 ? g::NC : 256) + threadIdx.x;
    if (t >= g::NC) return;
    const int64_t b = tb.leaf_blk[rank];
    if (TO_BLOCKS) blk[b * g::NC + t] = (S)vec[rank * g::NC + t];
    else vec[rank * g::NC + t] = (double)blk[b * g::NC + t];
}

__global__ void __launch_bounds__(256) k_sub_vec_blocks(double *blk, const double *vec, DevTables tb, int nc,
                                                        int wg_per_block) {
    const int64_t rank = blockIdx.x / wg_per_block;
    const int t = (blockIdx.x % wg_per_block) * (nc < 256 ? nc : 256) + threadIdx.x;
    if (t >= nc) return;
    const int64_t b = tb.leaf_blk[rank];
    blk[b * nc + t] -= vec[rank * nc + t];
}

constexpr int kChunk = 4096;   // vector elements per workgroup of the inner products

// partial[i * nchunk + c] = sum over chunk c of V_i[x] w[x] for i < k (V_i = V + i stride).
__global__ void __launch_bounds__(256) k_dots(const double *V, int64_t stride, int k, const double *w, int64_t n,
                                              double *partial, int nchunk) {
    constexpr int PER = kChunk / 256;
    __shared__ double red[4];
    const int64_t x0 = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    double wr[PER];
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int64_t x = x0 + 256 * m;
        wr[m] = x < n ? w[x] : 0.0;
    }
    for (int i = 0; i < k; i++) {
        const double *vi = V + i * stride;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int64_t x = x0 + 256 * m;
            if (x < n) s += vi[x] * wr[m];
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[(int64_t)i * nchunk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// out[i] = sum over chunks of partial[i * nchunk + c], in a fixed order.
__global__ void __launch_bounds__(256) k_dots_reduce(const double *partial, int nchunk, double *out) {
    __shared__ double sm[256];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += 256) s += partial[(int64_t)i * nchunk + c];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sm[0];
}

// y = (overwrite ? 0 : y) + sign * sum_i coef[i] V_i, coefficients in device memory.
__global__ void __launch_bounds__(256) k_combo(double *y, const double *V, int64_t stride, const double *coef, int k,
                                               double sign, int overwrite, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n) return;
    double s = 0.0;
    for (int i = 0; i < k; i++) s += coef[i] * V[i * stride + x];
    y[x] = (overwrite ? 0.0 : y[x]) + sign * s;
}

__global__ void __launch_bounds__(256) k_scale(double *x, double a, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < n) x[q] *= a;
}

#define DISPATCH_DB(L, ...)                                                   \
    do {                                                                      \
        if ((L).dim == 3) {                                                   \
            if ((L).bs == 16) { constexpr int D = 3, BS = 16; __VA_ARGS__; }  \
            else if ((L).bs == 8) { constexpr int D = 3, BS = 8; __VA_ARGS__; } \
            else { constexpr int D = 3, BS = 4; __VA_ARGS__; }                \
        } else {                                                              \
            if ((L).bs == 16) { constexpr int D = 2, BS = 16; __VA_ARGS__; }  \
            else if ((L).bs == 8) { constexpr int D = 2, BS = 8; __VA_ARGS__; } \
            else { constexpr int D = 2, BS = 4; __VA_ARGS__; }                \
        }                                                                     \
    } while (0)

// With events, the launch records the kernel's own start and end (no extra packets).
template <typename T>
void K<T>::gsrb(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, int colour, uint64_t mask,
                bool var, hipEvent_t ev0, hipEvent_t ev1, bool zero) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NH = G<D, BS>::NH;
        constexpr int TPB = NH < 256 ? NH : 256;
        constexpr int SP = NH / TPB >= 4 ? 4 : 1;
        constexpr int WF = SP > 1 ? 2 : 1;   // large levels: 512-thread workgroups
        if (zero) {
            // only the FP32 correction solves start from zero
            if constexpr (sizeof(T) == 4) {
                if (SP > 1 && nb <= 256) {
                    if (var) k_gsrb<T, D, BS, true, SP, true><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
                    else k_gsrb<T, D, BS, false, SP, true><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
                } else {
                    if (var) k_gsrb<T, D, BS, true, 1, true, WF><<<nb, TPB * WF, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
                    else k_gsrb<T, D, BS, false, 1, true, WF><<<nb, TPB * WF, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
                }
            }
        } else if (ev0) {
            if (var)
                hipExtLaunchKernelGGL((k_gsrb<T, D, BS, true, 1, false, WF>), dim3(nb), dim3(TPB * WF), 0, L.stream, ev0, ev1, 0,
                                      P, L.tb, lev, b0, colour, mask);
            else
                hipExtLaunchKernelGGL((k_gsrb<T, D, BS, false, 1, false, WF>), dim3(nb), dim3(TPB * WF), 0, L.stream, ev0, ev1,
                                      0, P, L.tb, lev, b0, colour, mask);
        } else if (SP > 1 && nb <= 256) {
            if (var) k_gsrb<T, D, BS, true, SP, false><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
            else k_gsrb<T, D, BS, false, SP, false><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
        } else if (SP > 1 && nb <= 1024) {
            constexpr int WD = SP > 1 ? 2 : 1;
            if (var) k_gsrb<T, D, BS, true, 1, false, WD><<<nb, TPB * WD, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
            else k_gsrb<T, D, BS, false, 1, false, WD><<<nb, TPB * WD, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
        } else {
            if (var) k_gsrb<T, D, BS, true, 1, false, WF><<<nb, TPB * WF, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
            else k_gsrb<T, D, BS, false, 1, false, WF><<<nb, TPB * WF, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask);
        }
    });
}

template <typename T>
void K<T>::ghost(const Launch &L, const Plane<T> &P, int b0, int nb, const int32_t *list, int nlist,
                 uint64_t mask, bool eps_field, bool cf_only) {
    int n = list ? nlist : nb;
    if (n <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NG = G<D, BS>::NG;
        constexpr int TPB = NG < 256 ? NG : 256;
        if (eps_field) k_ghost<T, D, BS, true><<<n, TPB, 0, L.stream>>>(P, L.tb, b0, list, mask, cf_only);
        else k_ghost<T, D, BS, false><<<n, TPB, 0, L.stream>>>(P, L.tb, b0, list, mask, cf_only);
    });
}

template <typename T>
void K<T>::cf_ghost(const Launch &L, const Plane<T> &P, const int32_t *faces, int nfaces, uint64_t mask) {
    if (nfaces <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NF = G<D, BS>::NF;
        const int64_t n = (int64_t)nfaces * NF;
        k_cf_ghost<T, D, BS><<<(unsigned)((n + 255) / 256), 256, 0, L.stream>>>(P, L.tb, faces, nfaces, mask);
    });
}

template <typename T>
void K<T>::restrict_down(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, uint64_t mask,
                         int mode, bool var) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int HB = BS / 2;
        constexpr int NQ = D == 3 ? HB * HB * HB : HB * HB;
        constexpr int TPB = NQ < 256 ? NQ : 256;
        if (mode == RESTRICT_FAS) {
            if (var) k_restrict<T, D, BS, true, RESTRICT_FAS><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
            else k_restrict<T, D, BS, false, RESTRICT_FAS><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
        } else if (mode == RESTRICT_V) {
            k_restrict<T, D, BS, false, RESTRICT_V><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
        } else {
            k_restrict<T, D, BS, false, RESTRICT_EPS><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
        }
    });
}

// The LDS-staged FAS kernel where it is the faster one (FP32, 16^3 blocks in 3D, many
// parents); false where the per-cell kernel is to run.
template <typename T, int D, int BS>
static bool launch_fas_lds(const Launch &L, const Plane<T> &P, int lev, const int32_t *list, int nlist,
                           uint64_t mask) {
    if constexpr (sizeof(T) == 4 && D == 3 && BS == 16) {
        if (nlist < kFasLdsMin) return false;
        k_fas_lds<T, 3, 16><<<nlist, 256, 0, L.stream>>>(P, L.tb, lev, list, mask);
        return true;
    }
    return false;
}

template <typename T>
void K<T>::fas(const Launch &L, const Plane<T> &P, int lev, const int32_t *list, int nlist, uint64_t mask,
               bool var) {
    if (nlist <= 0) return;
    DISPATCH_DB(L, {
        constexpr int N = G<D, BS>::NC + G<D, BS>::NG;
        constexpr int WPB = (N + 255) / 256;
        if (var) k_fas<T, D, BS, true><<<nlist * WPB, 256, 0, L.stream>>>(P, L.tb, lev, list, mask, WPB);
        else if (!launch_fas_lds<T, D, BS>(L, P, lev, list, nlist, mask))
            k_fas<T, D, BS, false><<<nlist * WPB, 256, 0, L.stream>>>(P, L.tb, lev, list, mask, WPB);
    });
}

template <typename T>
void K<T>::correct(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, uint64_t mask, bool half) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        constexpr int SP = NC / TPB >= 4 ? 4 : 1;
        if (half) {
            if (SP > 1 && nb <= 256) k_correct<T, D, BS, SP, true><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
            else k_correct<T, D, BS, 1, true><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
        } else {
            if (SP > 1 && nb <= 256) k_correct<T, D, BS, SP, false><<<nb * SP, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
            else k_correct<T, D, BS, 1, false><<<nb, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, L.nt);
        }
    });
}

// The single-workgroup coarse solver keeps a domain's grids in up to this much LDS
// (gfx950: 160 KB per workgroup; the rest holds the kernel's static arrays).
constexpr int kTailLds = 150 * 1024;

template <typename K>
static void allow_lds(K kernel) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, kTailLds);
}

// ------------------------------------------------ fixed reduction scratch
// Per-block partials of the allocation-free residual norm live in this file-scope
// device array: one copy per GPU, held until the process ends.  Its name is a
// host-side stand-in in host code, so it is never passed to a kernel; the device
// address of each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) and that address is used instead.
constexpr int kStaticPartialBlocks = 1 << 16;   // leaf blocks, 4 doubles each: 2 MiB
static __device__ __align__(256) double scratch[4 * kStaticPartialBlocks];

namespace {
constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

int static_partials(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return 0;
}

int static_partial_blocks() { return kStaticPartialBlocks; }

void prepare_kernels() {
    allow_lds(k_tail<double, 3, true, true>);
    allow_lds(k_tail<double, 3, false, true>);
    allow_lds(k_tail<double, 2, true, true>);
    allow_lds(k_tail<double, 2, false, true>);
    allow_lds(k_tail<float, 3, true, true>);
    allow_lds(k_tail<float, 3, false, true>);
    allow_lds(k_tail<float, 2, true, true>);
    allow_lds(k_tail<float, 2, false, true>);
}

template <typename T, int D, bool VAR>
static void launch_tail(const Launch &L, const Plane<T> &P, int mode, uint64_t mask, const TailParams &tp) {
    constexpr int TPB = tail_threads<VAR, D>();
    const uint64_t fit = L.tail_lds[sizeof(T) == 4 ? 1 : 0];
    if (mask & fit)
        k_tail<T, D, VAR, true><<<L.ndom, TPB, kTailLds, L.stream>>>(P, L.tb, mode, mask & fit, tp, L.coarse_steps,
                                                                     kTailLds);
    if (mask & ~fit)
        k_tail<T, D, VAR, false><<<L.ndom, TPB, 0, L.stream>>>(P, L.tb, mode, mask & ~fit, tp, L.coarse_steps, 0);
}

template <typename T>
void K<T>::tail(const Launch &L, const Plane<T> &P, int mode, uint64_t mask, const TailParams &tp, bool var) {
    if (L.dim == 3) {
        if (var) launch_tail<T, 3, true>(L, P, mode, mask, tp);
        else launch_tail<T, 3, false>(L, P, mode, mask, tp);
    } else {
        if (var) launch_tail<T, 2, true>(L, P, mode, mask, tp);
        else launch_tail<T, 2, false>(L, P, mode, mask, tp);
    }
}

int tail_lds_bytes() { return kTailLds; }

template <typename T>
void K<T>::tail_eps(const Launch &L, const Plane<T> &P) {
    if (L.dim == 3) k_tail_eps<T, 3><<<L.ndom, tail_threads<true>(), 0, L.stream>>>(P, L.tb, L.nt);
    else k_tail_eps<T, 2><<<L.ndom, tail_threads<true>(), 0, L.stream>>>(P, L.tb, L.nt);
}

static inline unsigned ublocks(int64_t n) { return (unsigned)((n + 255) / 256); }
static inline int64_t ucells(const UGrid &g, int dim) { return (int64_t)g.n[0] * g.n[1] * (dim == 3 ? g.n[2] : 1); }

template <typename T>
void K<T>::ugsrb(const Launch &L, const Plane<T> &P, const UGrid &g, int colour, bool var) {
    const unsigned nb = ublocks(ucells(g, L.dim) / 2);
    if (L.dim == 3) {
        if (var) k_ugsrb<T, 3, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g, colour);
        else k_ugsrb<T, 3, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g, colour);
    } else {
        if (var) k_ugsrb<T, 2, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g, colour);
        else k_ugsrb<T, 2, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g, colour);
    }
}

template <typename T>
void K<T>::ughost(const Launch &L, const Plane<T> &P, const UGrid &g) {
    const unsigned nb = ublocks(ucells(g, L.dim));
    if (L.dim == 3) k_ughost<T, 3><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
    else k_ughost<T, 2><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
}

template <typename T>
void K<T>::ufas(const Launch &L, const Plane<T> &P, const UGrid &g, bool var) {
    const int64_t npad = (int64_t)(g.n[0] + 2) * (g.n[1] + 2) * (L.dim == 3 ? g.n[2] + 2 : 1);
    const unsigned nb = ublocks(npad);
    if (L.dim == 3) {
        if (var) k_ufas<T, 3, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
        else k_ufas<T, 3, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
    } else {
        if (var) k_ufas<T, 2, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
        else k_ufas<T, 2, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g);
    }
}

template <typename T>
void K<T>::urestrict(const Launch &L, const Plane<T> &P, const UGrid &g, const UGrid &gc, bool var) {
    const unsigned nb = ublocks(ucells(gc, L.dim));
    if (L.dim == 3) {
        if (var) k_urestrict<T, 3, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
        else k_urestrict<T, 3, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
    } else {
        if (var) k_urestrict<T, 2, true><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
        else k_urestrict<T, 2, false><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
    }
}

template <typename T>
void K<T>::ucorrect(const Launch &L, const Plane<T> &P, const UGrid &g, const UGrid &gc) {
    const unsigned nb = ublocks(ucells(g, L.dim));
    if (L.dim == 3) k_ucorrect<T, 3><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
    else k_ucorrect<T, 2><<<nb, 256, 0, L.stream>>>(P, L.tb, g, gc);
}

template <typename T>
void K<T>::copy(const Launch &L, T *dst, const T *src, size_t n) {
    if (!n) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_copy<T><<<(unsigned)blocks, 256, 0, L.stream>>>(dst, src, n);
}

template <typename T>
void K<T>::jacobi(const Launch &L, const Plane<T> &P, T *dst, T *dstg, int lev, int b0, int nb, uint64_t mask,
                  bool var, double omega) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        if (var) k_jacobi<T, D, BS, true><<<nb, TPB, 0, L.stream>>>(P, dst, dstg, L.tb, lev, b0, mask, omega);
        else k_jacobi<T, D, BS, false><<<nb, TPB, 0, L.stream>>>(P, dst, dstg, L.tb, lev, b0, mask, omega);
    });
}

template <typename T>
void K<T>::ujacobi(const Launch &L, const Plane<T> &P, const T *src, T *dst, const UGrid &g, bool var, double omega) {
    const unsigned nb = ublocks(ucells(g, L.dim));
    if (L.dim == 3) {
        if (var) k_ujacobi<T, 3, true><<<nb, 256, 0, L.stream>>>(P, src, dst, L.tb, g, omega);
        else k_ujacobi<T, 3, false><<<nb, 256, 0, L.stream>>>(P, src, dst, L.tb, g, omega);
    } else {
        if (var) k_ujacobi<T, 2, true><<<nb, 256, 0, L.stream>>>(P, src, dst, L.tb, g, omega);
        else k_ujacobi<T, 2, false><<<nb, 256, 0, L.stream>>>(P, src, dst, L.tb, g, omega);
    }
}

template <typename T>
void K<T>::fill(const Launch &L, T *p, size_t n, T value) {
    if (!n) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_fill<T><<<(unsigned)blocks, 256, 0, L.stream>>>(p, n, value);
}

template <typename T>
void K<T>::zero(const Launch &L, T *p, size_t n) {
    fill(L, p, n, T(0));
}

template <typename T>
void K<T>::scatter(const Launch &L, T *dst, const double *src, int nleafblk) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        k_scatter<T, D, BS, true><<<(unsigned)(nleafblk * (NC / TPB)), TPB, 0, L.stream>>>(dst, const_cast<double *>(src), L.tb, NC / TPB);
    });
}

template <typename T>
void K<T>::gather(const Launch &L, const T *src, double *dst, int nleafblk) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        k_scatter<T, D, BS, false><<<(unsigned)(nleafblk * (NC / TPB)), TPB, 0, L.stream>>>(const_cast<T *>(src), dst, L.tb, NC / TPB);
    });
}

template struct K<double>;
template struct K<float>;

// Threads per workgroup of the residual kernels.
template <int D, int BS>
constexpr int resid_tpb() { return 256; }

void launch_norm64(const Launch &L, const Plane<double> &P, int nleafblk, bool var, float *rout32,
                   double *rout64) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int TPB = resid_tpb<D, BS>();
        if (var)
            k_resid<D, BS, true, false, TPB><<<nleafblk, TPB, 0, L.stream>>>(P, L.tb, nullptr, nullptr, L.partials,
                                                                             rout32, rout64);
        else
            k_resid<D, BS, false, false, TPB><<<nleafblk, TPB, 0, L.stream>>>(P, L.tb, nullptr, nullptr, L.partials,
                                                                              rout32, rout64);
    });
}

void launch_add_norm64(const Launch &L, const Plane<double> &P, const float *e, const float *eg, int nleafblk,
                       bool var, float *rout32) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int TPB = resid_tpb<D, BS>();
        if (var)
            k_resid<D, BS, true, true, TPB><<<nleafblk, TPB, 0, L.stream>>>(P, L.tb, e, eg, L.partials, rout32,
                                                                            nullptr);
        else
            k_resid<D, BS, false, true, TPB><<<nleafblk, TPB, 0, L.stream>>>(P, L.tb, e, eg, L.partials, rout32,
                                                                             nullptr);
    });
}

void launch_divb(const Launch &L, const double *Bd, double *out, int d, bool accumulate, int order,
                 int64_t nleaf_cells) {
    if (nleaf_cells <= 0) return;
    const unsigned grid = (unsigned)((nleaf_cells + 255) / 256);
    DISPATCH_DB(L, {
        if (order == 4) k_divb<D, BS, 4><<<grid, 256, 0, L.stream>>>(Bd, out, L.tb, d, accumulate ? 1 : 0, nleaf_cells);
        else k_divb<D, BS, 2><<<grid, 256, 0, L.stream>>>(Bd, out, L.tb, d, accumulate ? 1 : 0, nleaf_cells);
    });
}

void launch_divb_project(const Launch &L, const Plane<double> &P, double *Bd, double *e, int d, int64_t nleaf_cells) {
    if (nleaf_cells <= 0) return;
    const unsigned grid = (unsigned)((nleaf_cells + 255) / 256);
    DISPATCH_DB(L, { k_divb_project<D, BS><<<grid, 256, 0, L.stream>>>(P, Bd, e, L.tb, d, nleaf_cells); });
}

void launch_freespace(const Launch &L, double *f, const FsDom *fd, int ndom, int max_pts, int64_t tot_pts,
                      int c, int slices, double *q, double *partial, double *pl, double *bv, int nleafblk) {
    if (nleafblk <= 0 || tot_pts <= 0) return;
    switch (L.bs) {
    case 16: k_fs_charge<16><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    case 8: k_fs_charge<8><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    default: k_fs_charge<4><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    }
    k_fs_plane<<<dim3((unsigned)((max_pts + 255) / 256), (unsigned)ndom, (unsigned)slices), 256, 0, L.stream>>>(
        q, fd, partial, tot_pts, slices);
    k_fs_sum<<<(unsigned)((tot_pts + 255) / 256), 256, 0, L.stream>>>(partial, pl, tot_pts, slices);
    switch (L.bs) {
    case 16: k_fs_fold<16><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, pl, bv); break;
    case 8: k_fs_fold<8><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, pl, bv); break;
    default: k_fs_fold<4><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, pl, bv); break;
    }
}

void launch_freespace_guess(const Launch &L, const double *f, const FsDom *fd, int ndom, int c, double *q,
                            double *mom, double *out, int nleafblk, int64_t nleaf_cells) {
    if (nleaf_cells <= 0) return;
    switch (L.bs) {
    case 16: k_fs_charge<16><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    case 8: k_fs_charge<8><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    default: k_fs_charge<4><<<nleafblk, 256, 0, L.stream>>>(f, L.tb, fd, c, q); break;
    }
    k_fs_moments<<<ndom, 256, 0, L.stream>>>(q, fd, mom);
    const unsigned grid = (unsigned)((nleaf_cells + 255) / 256);
    switch (L.bs) {
    case 16: k_fs_guess<16><<<grid, 256, 0, L.stream>>>(fd, mom, L.tb, out, nleaf_cells); break;
    case 8: k_fs_guess<8><<<grid, 256, 0, L.stream>>>(fd, mom, L.tb, out, nleaf_cells); break;
    default: k_fs_guess<4><<<grid, 256, 0, L.stream>>>(fd, mom, L.tb, out, nleaf_cells); break;
    }
}

void launch_reduce_norms(const Launch &L) {
    k_reduce_norms<<<L.ndom, 256, 0, L.stream>>>(L.tb, L.partials, L.dom_norms, L.host_norms);
}

void launch_add_leaf(const Launch &L, double *v64, double *vg64, const float *v32, int nleafblk) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NT = G<D, BS>::NC / G<D, BS>::RH;   // one thread per row of one colour
        constexpr int TPB = add_leaf_threads<D, BS>();
        k_add_leaf<D, BS, float, false><<<(unsigned)(nleafblk * (NT / TPB)), TPB, 0, L.stream>>>(v64, vg64, v32,
                                                                                               L.tb, NT / TPB);
    });
}

void launch_add_vec(const Launch &L, double *v64, double *vg64, const double *vec, int nleafblk) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NT = G<D, BS>::NC / G<D, BS>::RH;
        constexpr int TPB = add_leaf_threads<D, BS>();
        k_add_leaf<D, BS, double, true><<<(unsigned)(nleafblk * (NT / TPB)), TPB, 0, L.stream>>>(v64, vg64, vec,
                                                                                               L.tb, NT / TPB);
    });
}

template <typename S>
void launch_vec_blocks(const Launch &L, S *blk, double *vec, int nleafblk, bool to_blocks) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        const unsigned nb = (unsigned)(nleafblk * (NC / TPB));
        if (to_blocks) k_vec_blocks<S, D, BS, true><<<nb, TPB, 0, L.stream>>>(blk, vec, L.tb, NC / TPB);
        else k_vec_blocks<S, D, BS, false><<<nb, TPB, 0, L.stream>>>(blk, vec, L.tb, NC / TPB);
    });
}
void launch_sub_vec_blocks(const Launch &L, double *blk, const double *vec, int nleafblk) {
    if (nleafblk <= 0) return;
    const int nc = cells(L.dim, L.bs);
    const int tpb = nc < 256 ? nc : 256;
    k_sub_vec_blocks<<<(unsigned)(nleafblk * (nc / tpb)), tpb, 0, L.stream>>>(blk, vec, L.tb, nc, nc / tpb);
}
template void launch_vec_blocks<float>(const Launch &, float *, double *, int, bool);
template void launch_vec_blocks<double>(const Launch &, double *, double *, int, bool);

int dots_chunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

void launch_dots(const Launch &L, const double *V, int64_t stride, int k, const double *w, int64_t n,
                 double *partial, double *out) {
    if (k <= 0 || n <= 0) return;
    const int nchunk = dots_chunks(n);
    k_dots<<<nchunk, 256, 0, L.stream>>>(V, stride, k, w, n, partial, nchunk);
    k_dots_reduce<<<k, 256, 0, L.stream>>>(partial, nchunk, out);
}

void launch_combo(const Launch &L, double *y, const double *V, int64_t stride, const double *coef, int k, double sign,
                  bool overwrite, int64_t n) {
    if (n <= 0) return;
    k_combo<<<(unsigned)((n + 255) / 256), 256, 0, L.stream>>>(y, V, stride, coef, k, sign, overwrite ? 1 : 0, n);
}

void launch_scale(const Launch &L, double *x, double a, int64_t n) {
    if (n <= 0) return;
    k_scale<<<(unsigned)((n + 255) / 256), 256, 0, L.stream>>>(x, a, n);
}

void launch_face_gradient(const Launch &L, const Plane<double> &P, const double *lam, const double *lamg,
                          double *out, int nleafblk) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        k_face_grad<D, BS><<<(unsigned)(nleafblk * (NC / TPB)), TPB, 0, L.stream>>>(P, L.tb, lam, lamg, out, NC / TPB);
    });
}

}  // namespace mgx
