// HIP kernels (gfx950) of the multigrid library: red-black Gauss-Seidel with ghost
// push, ghost fill (same level, physical boundary, coarse-fine interpolation),
// residual + restriction, FAS right-hand side, prolongation + correction, the
// single-workgroup tail (reduced block sizes and the coarsest solve), norms,
// scatter/gather and the adjoint face gradient.
//
// All kernels are bandwidth-bound stencils (about one flop per byte), so they use no
// matrix cores.  Blocks store their interior split by colour so that a half-sweep
// reads only the other colour and writes only its own, with unit-stride access.
#include <cmath>
#include <cstdio>

#include "mg_internal.hpp"

namespace mgx {

// A coarsest-grid smoothing step must lower the max-norm residual below this factor
// times the previous one, or the coarsest solve stops.
constexpr double kStall = 0.999;

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
    __device__ __forceinline__ static int gh(int f, int a1, int a2) { return f * NF + a2 * BS + a1; }
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

template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
    return T(2) * a * b / (a + b);
}

struct Spacing {
    double ih2[3];
};

__device__ __forceinline__ Spacing spacing(const DevTables &tb, int dm, int lev) {
    const double *h = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
    Spacing s;
    for (int a = 0; a < 3; a++) s.ih2[a] = 1.0 / (h[a] * h[a]);
    return s;
}

// (L v) and the Gauss-Seidel numerator/denominator at one cell of a block.
template <typename T, int D, int BS, bool VAR>
struct Stencil {
    T nb[6], w[6], vc;
    __device__ __forceinline__ void load(const Plane<T> &P, int64_t b, int i, int j, int k,
                                         const Spacing &s, bool need_center) {
        nb[0] = ld<D, BS>(P.v, P.vg, b, i - 1, j, k);
        nb[1] = ld<D, BS>(P.v, P.vg, b, i + 1, j, k);
        nb[2] = ld<D, BS>(P.v, P.vg, b, i, j - 1, k);
        nb[3] = ld<D, BS>(P.v, P.vg, b, i, j + 1, k);
        if (D == 3) {
            nb[4] = ld<D, BS>(P.v, P.vg, b, i, j, k - 1);
            nb[5] = ld<D, BS>(P.v, P.vg, b, i, j, k + 1);
        }
        vc = need_center ? P.v[b * G<D, BS>::NC + G<D, BS>::in(i, j, k)] : T(0);
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
    }
    __device__ __forceinline__ T Lv() const {
        T s = T(0);
        for (int f = 0; f < 2 * D; f++) s += w[f] * (nb[f] - vc);
        return s;
    }
    __device__ __forceinline__ T gs(T fval) const {
        T num = T(0), den = T(0);
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

// ------------------------------------------------------------ GS-RB sweep
// One colour of red-black Gauss-Seidel (Sec. 2.2) on a contiguous block range of one
// level.  Each thread updates one cell of the colour and pushes the new value into
// the ghost layer that mirrors it: the neighbour block's ghost on a same-level face,
// its own ghost on a physical face.  Ghost positions hold the colour of the cell they
// mirror, so a half-sweep never reads a ghost another thread writes.  Coarse-fine
// ghosts are refreshed by a separate launch.
template <typename T, int D, int BS, bool VAR>
__global__ void __launch_bounds__(256) k_gsrb(Plane<T> P, DevTables tb, int lev, int b0, int colour,
                                              uint64_t mask, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t b = b0 + blockIdx.x / wg_per_block;
    const int dm = tb.dom[b];
    if (!((mask >> dm) & 1)) return;
    const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
    if (t >= g::NH) return;
    int i, j, k;
    g::decode(colour * g::NH + t, i, j, k);
    const Spacing s = spacing(tb, dm, lev);
    Stencil<T, D, BS, VAR> st;
    st.load(P, b, i, j, k, s, false);
    const int64_t self = b * g::NC + colour * g::NH + t;
    const T nv = st.gs(P.f[self]);
    P.v[self] = nv;
    // ghost push
    const int32_t *nbr = tb.nbr + 6 * b;
    int coord[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < D; a++) {
        int side = -1;
        if (coord[a] == 0) side = 0;
        else if (coord[a] == BS - 1) side = 1;
        if (side < 0) continue;
        int f = 2 * a + side;
        int a1 = a == 0 ? j : i, a2 = a == 2 ? j : k;
        int n = nbr[f];
        if (n >= 0) {
            P.vg[(int64_t)n * g::NG + g::gh(f ^ 1, a1, a2)] = nv;
        } else if (n == -1) {
            const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
            P.vg[b * g::NG + g::gh(f, a1, a2)] = bc_ghost<T>(tb.bck[6 * dm + f], tb.bcv[6 * dm + f], hh[a], side, nv);
        }
    }
}

// -------------------------------------------------------------- ghost fill
// Fills the face ghosts of a block (Sec. 2.6).  Same-level faces copy the
// neighbour's boundary cell; physical faces apply the boundary condition; coarse-fine
// faces take g = (B' + c')/2 with B' the coarse cell value moved to the ghost's
// tangential position by the central-difference slope(s) of the coarse cell and
// c' = (3c - c2)/2 the two-point extrapolation of the fine cells to the face.  For the
// eps field: copy, copy of the interior cell, and the coarse cell's value.
template <typename T, int D, int BS, bool EPS>
__device__ void ghost_cell(const Plane<T> &P, const DevTables &tb, int64_t b, int f, int a1, int a2,
                           bool cf_only) {
    using g = G<D, BS>;
    T *v = EPS ? P.eps : P.v;
    T *vg = EPS ? P.epsg : P.vg;
    const int a = f >> 1, side = f & 1;
    const int n = tb.nbr[6 * b + f];
    if (cf_only && n != -2) return;
    int in1[3], in2[3];
    // tangential axes in increasing order
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    in1[t1] = a1; in1[t2] = a2; in1[a] = side ? BS - 1 : 0;
    in2[t1] = a1; in2[t2] = a2; in2[a] = side ? BS - 2 : 1;
    if (D == 2) { in1[2] = 0; in2[2] = 0; }
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
            out = bc_ghost<T>(tb.bck[6 * dm + f], tb.bcv[6 * dm + f], hh[a], side, ci);
        }
    } else {
        const int dm = tb.dom[b];
        const int lv = tb.lev[b];
        const int64_t qb = tb.cf[6 * b + f];
        int gi[3];
        for (int c = 0; c < 3; c++) gi[c] = tb.org[3 * b + c] + in1[c];
        gi[a] += side ? 1 : -1;
        // wrap across a periodic face (the coarse region may lie beyond it)
        const int32_t *nc = tb.ncell + ((size_t)dm * MAXLEV + lv) * 3;
        if (gi[a] < 0) gi[a] += nc[a];
        if (gi[a] >= nc[a]) gi[a] -= nc[a];
        int cl[3];
        for (int c = 0; c < 3; c++) cl[c] = (gi[c] >> 1) - tb.org[3 * qb + c];
        if (D == 2) cl[2] = 0;
        const T *w = EPS ? P.eps : P.v;
        const T *wg = EPS ? P.epsg : P.vg;
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
    }
    vg[b * g::NG + g::gh(f, a1, a2)] = out;
}

template <typename T, int D, int BS, bool EPS>
__global__ void __launch_bounds__(256) k_ghost(Plane<T> P, DevTables tb, int b0, const int32_t *list,
                                               uint64_t mask, int cf_only) {
    using g = G<D, BS>;
    const int64_t b = list ? list[blockIdx.x] : b0 + blockIdx.x;
    if (!((mask >> tb.dom[b]) & 1)) return;
    for (int t = threadIdx.x; t < g::NG; t += blockDim.x) {
        int f = t / g::NF, r = t % g::NF;
        ghost_cell<T, D, BS, EPS>(P, tb, b, f, r % BS, r / BS, cf_only != 0);
    }
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
// For each coarse cell under a block of level `lev`: the mean of the 2^d fine values
// (restriction, Sec. 2.3) of v, and for the FAS mode also of r = f - L v, written to
// the parent block (v and f) or to the domain's top tail grid.  Mode RESTRICT_EPS
// restricts the coefficient.
template <typename T, int D, int BS, bool VAR, int MODE>
__global__ void __launch_bounds__(256) k_restrict(Plane<T> P, DevTables tb, int lev, int b0,
                                                  uint64_t mask, int wg_per_block, int nt) {
    using g = G<D, BS>;
    constexpr int HB = BS / 2;
    constexpr int NQ = D == 3 ? HB * HB * HB : HB * HB;
    const int64_t b = b0 + blockIdx.x / wg_per_block;
    const int dm = tb.dom[b];
    if (!((mask >> dm) & 1)) return;
    const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
    if (t >= NQ) return;
    const int ci = t % HB, cj = (t / HB) % HB, ck = D == 3 ? t / (HB * HB) : 0;
    const Spacing s = spacing(tb, dm, lev);
    const T *src = MODE == RESTRICT_EPS ? P.eps : P.v;
    T sv = T(0), sr = T(0);
#pragma unroll
    for (int q = 0; q < (1 << D); q++) {
        int i = 2 * ci + (q & 1), j = 2 * cj + ((q >> 1) & 1), k = D == 3 ? 2 * ck + (q >> 2) : 0;
        sv += src[b * g::NC + g::in(i, j, k)];
        if (MODE == RESTRICT_FAS) {
            Stencil<T, D, BS, VAR> st;
            st.load(P, b, i, j, k, s, true);
            sr += P.f[b * g::NC + g::in(i, j, k)] - st.Lv();
        }
    }
    const T inv = T(1) / T(1 << D);
    sv *= inv;
    sr *= inv;
    int gc[3] = {(tb.org[3 * b] >> 1) + ci, (tb.org[3 * b + 1] >> 1) + cj, D == 3 ? (tb.org[3 * b + 2] >> 1) + ck : 0};
    const int64_t p = tb.parent[b];
    if (p >= 0) {
        int l0 = gc[0] - tb.org[3 * p], l1 = gc[1] - tb.org[3 * p + 1], l2 = D == 3 ? gc[2] - tb.org[3 * p + 2] : 0;
        int64_t o = p * g::NC + g::in(l0, l1, l2);
        if (MODE == RESTRICT_EPS) P.eps[o] = sv;
        else P.v[o] = sv;
        if (MODE == RESTRICT_FAS) P.f[o] = sr;
    } else {
        TailGeo tg = tail_geo(tb, dm, nt - 1, D);
        int64_t o = tg.idx(gc[0], gc[1], gc[2], D);
        if (MODE == RESTRICT_EPS) P.teps[o] = sv;
        else P.tv[o] = sv;
        if (MODE == RESTRICT_FAS) P.tf[o] = sr;
    }
}

// --------------------------------------------------------- FAS right side
// On parent blocks after the restriction and the ghost fill of their level:
// v_old = v (ghosts included) and f = R(r) + L v (eq. coarse-rhs).
template <typename T, int D, int BS, bool VAR>
__global__ void __launch_bounds__(256) k_fas(Plane<T> P, DevTables tb, int lev, const int32_t *list,
                                             uint64_t mask) {
    using g = G<D, BS>;
    const int64_t b = list[blockIdx.x];
    const int dm = tb.dom[b];
    if (!((mask >> dm) & 1)) return;
    const Spacing s = spacing(tb, dm, lev);
    for (int t = threadIdx.x; t < g::NC; t += blockDim.x) {
        int i, j, k;
        g::decode(t, i, j, k);
        Stencil<T, D, BS, VAR> st;
        st.load(P, b, i, j, k, s, true);
        P.vold[b * g::NC + t] = st.vc;
        P.f[b * g::NC + t] += st.Lv();
    }
    for (int t = threadIdx.x; t < g::NG; t += blockDim.x) P.voldg[b * g::NG + t] = P.vg[b * g::NG + t];
}

// ------------------------------------------------- prolongation + correction
// v^h += P(v^H - v_old^H) (eq. coarse-corr) with the nearest-neighbour interpolation
// of eq. interp_2d / interp_3d: 2D (2 d_p + d_x + d_y)/4, 3D (d_p + d_x + d_y + d_z)/4,
// the neighbours taken on the side of the fine cell (coarse ghosts near block faces).
template <typename T, int D, int BS>
__global__ void __launch_bounds__(256) k_correct(Plane<T> P, DevTables tb, int b0, uint64_t mask,
                                                 int wg_per_block, int nt) {
    using g = G<D, BS>;
    const int64_t b = b0 + blockIdx.x / wg_per_block;
    const int dm = tb.dom[b];
    if (!((mask >> dm) & 1)) return;
    const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
    if (t >= g::NC) return;
    int i, j, k;
    g::decode(t, i, j, k);
    int gl[3] = {tb.org[3 * b] + i, tb.org[3 * b + 1] + j, D == 3 ? tb.org[3 * b + 2] + k : 0};
    int pc[3], sg[3];
    for (int a = 0; a < 3; a++) {
        pc[a] = gl[a] >> 1;
        sg[a] = (gl[a] & 1) ? 1 : -1;
    }
    const int64_t p = tb.parent[b];
    T d[4];
    if (p >= 0) {
        int l[3] = {pc[0] - tb.org[3 * p], pc[1] - tb.org[3 * p + 1], D == 3 ? pc[2] - tb.org[3 * p + 2] : 0};
        d[0] = ld<D, BS>(P.v, P.vg, p, l[0], l[1], l[2]) - ld<D, BS>(P.vold, P.voldg, p, l[0], l[1], l[2]);
#pragma unroll
        for (int a = 0; a < D; a++) {
            int q[3] = {l[0], l[1], l[2]};
            q[a] += sg[a];
            d[1 + a] = ld<D, BS>(P.v, P.vg, p, q[0], q[1], q[2]) - ld<D, BS>(P.vold, P.voldg, p, q[0], q[1], q[2]);
        }
    } else {
        TailGeo tg = tail_geo(tb, dm, nt - 1, D);
        int64_t o = tg.idx(pc[0], pc[1], pc[2], D);
        d[0] = P.tv[o] - P.tvold[o];
#pragma unroll
        for (int a = 0; a < D; a++) {
            int q[3] = {pc[0], pc[1], pc[2]};
            q[a] += sg[a];
            int64_t oq = tg.idx(q[0], q[1], q[2], D);
            d[1 + a] = P.tv[oq] - P.tvold[oq];
        }
    }
    T corr;
    if (D == 2) corr = T(0.25) * (T(2) * d[0] + d[1] + d[2]);
    else corr = T(0.25) * (d[0] + d[1] + d[2] + d[3]);
    P.v[b * g::NC + t] += corr;
}

// --------------------------------------------------------------- the tail
// One workgroup per domain runs everything below the lowest block level: the levels
// whose block size was halved down to one cell (Sec. 2.5; the paper keeps them on a
// single process).  They are uniform grids, so each is stored whole with one ghost
// layer; blocked red-black Gauss-Seidel with ghost refresh after each colour equals a
// sweep over the whole grid.
template <typename T, int D, bool VAR>
struct Tail {
    const Plane<T> &P;
    const DevTables &tb;
    int dm;
    int nt;
    double *red;   // shared reduction scratch

    __device__ TailGeo geo(int lev) const { return tail_geo(tb, dm, lev, D); }
    __device__ int64_t count(const TailGeo &g) const { return (int64_t)g.n[0] * g.n[1] * g.n[2]; }
    __device__ void cell(const TailGeo &g, int64_t c, int &i, int &j, int &k) const {
        i = (int)(c % g.n[0]);
        j = (int)((c / g.n[0]) % g.n[1]);
        k = (int)(c / ((int64_t)g.n[0] * g.n[1]));
    }

    // Ghost layer of one tail grid (faces only): periodic copy or boundary condition.
    __device__ void ghosts(int lev, T *u, bool eps) const {
        TailGeo g = geo(lev);
        const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
        for (int a = 0; a < D; a++) {
            int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            int n1 = g.n[t1], n2 = D == 3 ? g.n[t2] : 1;
            int64_t tot = 2 * (int64_t)n1 * n2;
            for (int64_t q = threadIdx.x; q < tot; q += blockDim.x) {
                int side = (int)(q / ((int64_t)n1 * n2));
                int r = (int)(q % ((int64_t)n1 * n2));
                int c[3], in[3], op[3];
                c[t1] = r % n1; c[t2] = D == 3 ? r / n1 : 0;
                in[t1] = c[t1]; in[t2] = c[t2]; op[t1] = c[t1]; op[t2] = c[t2];
                c[a] = side ? g.n[a] : -1;
                in[a] = side ? g.n[a] - 1 : 0;
                op[a] = side ? 0 : g.n[a] - 1;
                if (D == 2) { c[2] = 0; in[2] = 0; op[2] = 0; }
                int f = 2 * a + side;
                int kind = tb.bck[6 * dm + f];
                T val;
                if (kind == MG_BC_PERIODIC) val = u[g.idx(op[0], op[1], op[2], D)];
                else if (eps) val = u[g.idx(in[0], in[1], in[2], D)];
                else val = bc_ghost<T>(kind, tb.bcv[6 * dm + f], hh[a], side, u[g.idx(in[0], in[1], in[2], D)]);
                u[g.idx(c[0], c[1], c[2], D)] = val;
            }
        }
    }

    __device__ void weights(int lev, const TailGeo &g, int i, int j, int k, T *w) const {
        const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
        if (!VAR) {
            for (int f = 0; f < 2 * D; f++) w[f] = T(1.0 / (hh[f / 2] * hh[f / 2]));
        } else {
            T e0 = P.teps[g.idx(i, j, k, D)];
            int o[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
            for (int f = 0; f < 2 * D; f++)
                w[f] = harm(e0, P.teps[g.idx(o[f][0], o[f][1], o[f][2], D)]) * T(1.0 / (hh[f / 2] * hh[f / 2]));
        }
    }
    __device__ void nbrs(const TailGeo &g, const T *u, int i, int j, int k, T *nb) const {
        nb[0] = u[g.idx(i - 1, j, k, D)];
        nb[1] = u[g.idx(i + 1, j, k, D)];
        nb[2] = u[g.idx(i, j - 1, k, D)];
        nb[3] = u[g.idx(i, j + 1, k, D)];
        if (D == 3) {
            nb[4] = u[g.idx(i, j, k - 1, D)];
            nb[5] = u[g.idx(i, j, k + 1, D)];
        }
    }
    __device__ T Lv(int lev, const TailGeo &g, int i, int j, int k) const {
        T w[6], nb[6];
        weights(lev, g, i, j, k, w);
        nbrs(g, P.tv, i, j, k, nb);
        T vc = P.tv[g.idx(i, j, k, D)], s = T(0);
        for (int f = 0; f < 2 * D; f++) s += w[f] * (nb[f] - vc);
        return s;
    }

    __device__ void smooth(int lev) const {
        TailGeo g = geo(lev);
        int64_t n = count(g);
        for (int colour = 0; colour < 2; colour++) {
            for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
                int i, j, k;
                cell(g, c, i, j, k);
                if (((i + j + k) & 1) != colour) continue;
                T w[6], nb[6];
                weights(lev, g, i, j, k, w);
                nbrs(g, P.tv, i, j, k, nb);
                T num = T(0), den = T(0);
                for (int f = 0; f < 2 * D; f++) {
                    num += w[f] * nb[f];
                    den += w[f];
                }
                int64_t o = g.idx(i, j, k, D);
                P.tv[o] = (num - P.tf[o]) / den;
            }
            __syncthreads();
            ghosts(lev, P.tv, false);
            __syncthreads();
        }
    }

    // Block-wide reductions (all threads get the result).
    __device__ double reduce_max(double x) const {
        red[threadIdx.x] = x;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                double o = red[threadIdx.x + s];
                if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
            }
            __syncthreads();
        }
        double r = red[0];
        __syncthreads();
        return r;
    }
    __device__ double reduce_sum(double x) const {
        red[threadIdx.x] = x;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        double r = red[0];
        __syncthreads();
        return r;
    }

    __device__ double resmax(int lev) const {
        TailGeo g = geo(lev);
        int64_t n = count(g);
        double m = 0.0;
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            int i, j, k;
            cell(g, c, i, j, k);
            double r = fabs((double)(P.tf[g.idx(i, j, k, D)] - Lv(lev, g, i, j, k)));
            if (r > m || r != r) m = r;
        }
        return reduce_max(m);
    }

    // Restriction lev -> lev-1 with the FAS right-hand side (as for block levels).
    __device__ void restrict_fas(int lev) const {
        TailGeo gf = geo(lev), gc = geo(lev - 1);
        int64_t n = count(gc);
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            int I, J, K;
            cell(gc, c, I, J, K);
            T sv = T(0), sr = T(0);
            for (int q = 0; q < (1 << D); q++) {
                int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = D == 3 ? 2 * K + (q >> 2) : 0;
                int64_t o = gf.idx(i, j, k, D);
                sv += P.tv[o];
                sr += P.tf[o] - Lv(lev, gf, i, j, k);
            }
            const T inv = T(1) / T(1 << D);
            int64_t oc = gc.idx(I, J, K, D);
            P.tv[oc] = sv * inv;
            P.tf[oc] = sr * inv;
        }
        __syncthreads();
        finish_fas(lev - 1);
    }
    // Ghosts, v_old = v (ghosts included), f = R(r) + L v on one tail grid.
    __device__ void finish_fas(int lev) const {
        ghosts(lev, P.tv, false);
        __syncthreads();
        TailGeo g = geo(lev);
        int64_t np = (int64_t)(g.n[0] + 2) * (g.n[1] + 2) * (D == 3 ? g.n[2] + 2 : 1);
        for (int64_t c = threadIdx.x; c < np; c += blockDim.x) P.tvold[g.off + c] = P.tv[g.off + c];
        int64_t n = count(g);
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            int i, j, k;
            cell(g, c, i, j, k);
            P.tf[g.idx(i, j, k, D)] += Lv(lev, g, i, j, k);
        }
        __syncthreads();
    }

    __device__ void correct(int lev) const {
        TailGeo gf = geo(lev), gc = geo(lev - 1);
        int64_t n = count(gf);
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            int i, j, k;
            cell(gf, c, i, j, k);
            int p[3] = {i >> 1, j >> 1, k >> 1};
            int sg[3] = {(i & 1) ? 1 : -1, (j & 1) ? 1 : -1, (k & 1) ? 1 : -1};
            int64_t o = gc.idx(p[0], p[1], p[2], D);
            T d0 = P.tv[o] - P.tvold[o], dn[3];
            for (int a = 0; a < D; a++) {
                int q[3] = {p[0], p[1], p[2]};
                q[a] += sg[a];
                int64_t oq = gc.idx(q[0], q[1], q[2], D);
                dn[a] = P.tv[oq] - P.tvold[oq];
            }
            T corr = D == 2 ? T(0.25) * (T(2) * d0 + dn[0] + dn[1]) : T(0.25) * (d0 + dn[0] + dn[1] + dn[2]);
            P.tv[gf.idx(i, j, k, D)] += corr;
        }
        __syncthreads();
        ghosts(lev, P.tv, false);
        __syncthreads();
    }

    // Coarsest grid: smoothing steps until the max-norm residual is <= max(abs,
    // rel * initial), at most n_max, at least one; stop early once a step (from the
    // second on) lowers it by less than 0.1% (rounding floor; the two-value
    // alternation of a one-cell Dirichlet grid).  Fully periodic: remove the mean of
    // f first.
    __device__ int coarse_solve(const TailParams &tp) const {
        TailGeo g = geo(0);
        int64_t n = count(g);
        bool per = true;
        for (int f = 0; f < 2 * D; f++) per = per && tb.bck[6 * dm + f] == MG_BC_PERIODIC;
        if (per) {
            double s = 0.0;
            for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
                int i, j, k;
                cell(g, c, i, j, k);
                s += (double)P.tf[g.idx(i, j, k, D)];
            }
            double mean = reduce_sum(s) / (double)n;
            for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
                int i, j, k;
                cell(g, c, i, j, k);
                P.tf[g.idx(i, j, k, D)] -= T(mean);
            }
            __syncthreads();
        }
        double r0 = resmax(0), rprev = r0;
        double target = fmax(tp.abs_tol, tp.rel_tol * r0);
        int k;
        for (k = 1; k <= tp.n_max; k++) {
            smooth(0);
            double r = resmax(0);
            if (r <= target) break;
            if (k >= 2 && r > kStall * rprev) break;
            rprev = r;
        }
        return k > tp.n_max ? tp.n_max : k;
    }

    __device__ int vcycle(int top, const TailParams &tp) const {
        for (int l = top; l >= 1; l--) {
            for (int s = 0; s < tp.n_down; s++) smooth(l);
            restrict_fas(l);
        }
        int steps = coarse_solve(tp);
        for (int l = 1; l <= top; l++) {
            correct(l);
            for (int s = 0; s < tp.n_up; s++) smooth(l);
        }
        return steps;
    }
};

template <typename T, int D, bool VAR>
__global__ void __launch_bounds__(1024) k_tail(Plane<T> P, DevTables tb, int nt, int mode, uint64_t mask,
                                               TailParams tp, int32_t *steps_out) {
    __shared__ double red[1024];
    const int dm = blockIdx.x;
    if (!((mask >> dm) & 1)) return;
    Tail<T, D, VAR> tl{P, tb, dm, nt, red};
    const int top = nt - 1;
    // The restriction from the lowest block level left R(v) in v and R(r) in f.
    tl.finish_fas(top);
    int steps;
    if (mode == TAIL_VCYCLE) {
        steps = tl.vcycle(top, tp);
    } else {
        for (int l = top; l >= 1; l--) tl.restrict_fas(l);
        steps = tl.coarse_solve(tp);
        for (int l = 1; l <= top; l++) {
            tl.correct(l);
            steps = tl.vcycle(l, tp);
        }
    }
    if (threadIdx.x == 0) steps_out[dm] = steps;
}

// eps on the tail grids: restrict down from the top tail grid, then ghost layers.
template <typename T, int D>
__global__ void __launch_bounds__(1024) k_tail_eps(Plane<T> P, DevTables tb, int nt) {
    __shared__ double red[1024];
    const int dm = blockIdx.x;
    Tail<T, D, true> tl{P, tb, dm, nt, red};
    for (int l = nt - 1; l >= 1; l--) {
        TailGeo gf = tl.geo(l), gc = tl.geo(l - 1);
        int64_t n = tl.count(gc);
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            int I, J, K;
            tl.cell(gc, c, I, J, K);
            T s = T(0);
            for (int q = 0; q < (1 << D); q++)
                s += P.teps[gf.idx(2 * I + (q & 1), 2 * J + ((q >> 1) & 1), D == 3 ? 2 * K + (q >> 2) : 0, D)];
            P.teps[gc.idx(I, J, K, D)] = s / T(1 << D);
        }
        __syncthreads();
    }
    for (int l = 0; l < nt; l++) {
        tl.ghosts(l, P.teps, true);
        __syncthreads();
    }
}

// ------------------------------------------------------------ small utilities
template <typename T>
__global__ void k_fill(T *p, size_t n, T value) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

// Leaf-ordered user array (x fastest within a block) <-> colour-split block storage.
template <typename T, int D, int BS, bool TO_BLOCKS>
__global__ void __launch_bounds__(256) k_scatter(T *blk, double *user, DevTables tb, int wg_per_block) {
    using g = G<D, BS>;
    const int64_t rank = blockIdx.x / wg_per_block;
    const int64_t b = tb.leaf_blk[rank];
    const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
    if (t >= g::NC) return;
    int i = t % BS, j = (t / BS) % BS, k = D == 3 ? t / (BS * BS) : 0;
    int64_t o = b * g::NC + g::in(i, j, k);
    if (TO_BLOCKS) blk[o] = T(user[rank * g::NC + t]);
    else user[rank * g::NC + t] = (double)blk[o];
}

// ------------------------------------------------------------------ norms
// Composite residual r = f - L v on every leaf block (FP64), with per-block partial
// max |r|, sum vol r^2, max |f|, sum vol f^2; optionally writes r into the leaf
// blocks of an output field (the right-hand side of an FP32 correction solve).
template <int D, int BS, bool VAR>
__global__ void __launch_bounds__(256) k_norm(Plane<double> P, DevTables tb, double *partials,
                                              float *rout32, double *rout64) {
    using g = G<D, BS>;
    __shared__ double sm[4][256];
    const int rank = blockIdx.x;
    const int64_t b = tb.leaf_blk[rank];
    const int dm = tb.dom[b], lev = tb.lev[b];
    const Spacing s = spacing(tb, dm, lev);
    const double *hh = tb.h + ((size_t)dm * MAXLEV + lev) * 3;
    const double vol = hh[0] * hh[1] * (D == 3 ? hh[2] : 1.0);
    double mr = 0, sr = 0, mf = 0, sf = 0;
    for (int t = threadIdx.x; t < g::NC; t += blockDim.x) {
        int i, j, k;
        g::decode(t, i, j, k);
        Stencil<double, D, BS, VAR> st;
        st.load(P, b, i, j, k, s, true);
        double f = P.f[b * g::NC + t];
        double r = f - st.Lv();
        if (fabs(r) > mr || r != r) mr = fabs(r);
        if (fabs(f) > mf) mf = fabs(f);
        sr += vol * r * r;
        sf += vol * f * f;
        if (rout32) rout32[b * g::NC + t] = (float)r;
        if (rout64) rout64[b * g::NC + t] = r;
    }
    sm[0][threadIdx.x] = mr; sm[1][threadIdx.x] = sr; sm[2][threadIdx.x] = mf; sm[3][threadIdx.x] = sf;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            double o = sm[0][threadIdx.x + st];
            if (o > sm[0][threadIdx.x] || o != o) sm[0][threadIdx.x] = o;
            sm[1][threadIdx.x] += sm[1][threadIdx.x + st];
            sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + st]);
            sm[3][threadIdx.x] += sm[3][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[4 * (int64_t)rank + threadIdx.x] = sm[threadIdx.x][0];
}

// Per-domain combination of the per-block partials (fixed order: deterministic).
__global__ void __launch_bounds__(256) k_reduce_norms(DevTables tb, const double *partials, double *out) {
    __shared__ double sm[4][256];
    const int dm = blockIdx.x;
    const int r0 = tb.leaf_first[dm], r1 = tb.leaf_first[dm + 1];
    double mr = 0, sr = 0, mf = 0, sf = 0;
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const double *p = partials + 4 * (int64_t)r;
        if (p[0] > mr || p[0] != p[0]) mr = p[0];
        sr += p[1];
        mf = fmax(mf, p[2]);
        sf += p[3];
    }
    sm[0][threadIdx.x] = mr; sm[1][threadIdx.x] = sr; sm[2][threadIdx.x] = mf; sm[3][threadIdx.x] = sf;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            double o = sm[0][threadIdx.x + st];
            if (o > sm[0][threadIdx.x] || o != o) sm[0][threadIdx.x] = o;
            sm[1][threadIdx.x] += sm[1][threadIdx.x + st];
            sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + st]);
            sm[3][threadIdx.x] += sm[3][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[4 * dm + threadIdx.x] = sm[threadIdx.x][0];
}

// v64 += v32 on every leaf block (the FP64 update of iterative refinement).
template <int NC>
__global__ void __launch_bounds__(256) k_add_leaf(double *v64, const float *v32, DevTables tb, int wg_per_block) {
    const int64_t b = tb.leaf_blk[blockIdx.x / wg_per_block];
    const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
    if (t < NC) v64[b * NC + t] += (double)v32[b * NC + t];
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
        const int t = (blockIdx.x % wg_per_block) * blockDim.x + threadIdx.x;
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

// ================================================================ launchers
#define HIPCHK(x) (x)

static inline int cells(int dim, int bs) { return dim == 3 ? bs * bs * bs : bs * bs; }

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

template <typename T>
void K<T>::gsrb(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, int colour, uint64_t mask,
                bool var) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NH = G<D, BS>::NH;
        constexpr int TPB = NH < 256 ? NH : 256;
        constexpr int WPB = NH / TPB;
        dim3 grid((unsigned)(nb * WPB));
        if (var) k_gsrb<T, D, BS, true><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask, WPB);
        else k_gsrb<T, D, BS, false><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, colour, mask, WPB);
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
void K<T>::restrict_down(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, uint64_t mask,
                         int mode, bool var) {
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int HB = BS / 2;
        constexpr int NQ = D == 3 ? HB * HB * HB : HB * HB;
        constexpr int TPB = NQ < 256 ? NQ : 256;
        constexpr int WPB = NQ / TPB;
        dim3 grid((unsigned)(nb * WPB));
        if (mode == RESTRICT_FAS) {
            if (var) k_restrict<T, D, BS, true, RESTRICT_FAS><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, WPB, L.nt);
            else k_restrict<T, D, BS, false, RESTRICT_FAS><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, WPB, L.nt);
        } else if (mode == RESTRICT_V) {
            k_restrict<T, D, BS, false, RESTRICT_V><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, WPB, L.nt);
        } else {
            k_restrict<T, D, BS, false, RESTRICT_EPS><<<grid, TPB, 0, L.stream>>>(P, L.tb, lev, b0, mask, WPB, L.nt);
        }
    });
}

template <typename T>
void K<T>::fas(const Launch &L, const Plane<T> &P, int lev, const int32_t *list, int nlist, uint64_t mask,
               bool var) {
    if (nlist <= 0) return;
    DISPATCH_DB(L, {
        if (var) k_fas<T, D, BS, true><<<nlist, 256, 0, L.stream>>>(P, L.tb, lev, list, mask);
        else k_fas<T, D, BS, false><<<nlist, 256, 0, L.stream>>>(P, L.tb, lev, list, mask);
    });
}

template <typename T>
void K<T>::correct(const Launch &L, const Plane<T> &P, int lev, int b0, int nb, uint64_t mask) {
    (void)lev;
    if (nb <= 0) return;
    DISPATCH_DB(L, {
        constexpr int NC = G<D, BS>::NC;
        constexpr int TPB = NC < 256 ? NC : 256;
        constexpr int WPB = NC / TPB;
        k_correct<T, D, BS><<<(unsigned)(nb * WPB), TPB, 0, L.stream>>>(P, L.tb, b0, mask, WPB, L.nt);
    });
}

template <typename T>
void K<T>::tail(const Launch &L, const Plane<T> &P, int mode, uint64_t mask, const TailParams &tp, bool var) {
    const int TPB = 512;
    if (L.dim == 3) {
        if (var) k_tail<T, 3, true><<<L.ndom, TPB, 0, L.stream>>>(P, L.tb, L.nt, mode, mask, tp, L.coarse_steps);
        else k_tail<T, 3, false><<<L.ndom, TPB, 0, L.stream>>>(P, L.tb, L.nt, mode, mask, tp, L.coarse_steps);
    } else {
        if (var) k_tail<T, 2, true><<<L.ndom, TPB, 0, L.stream>>>(P, L.tb, L.nt, mode, mask, tp, L.coarse_steps);
        else k_tail<T, 2, false><<<L.ndom, TPB, 0, L.stream>>>(P, L.tb, L.nt, mode, mask, tp, L.coarse_steps);
    }
}

template <typename T>
void K<T>::tail_eps(const Launch &L, const Plane<T> &P) {
    if (L.dim == 3) k_tail_eps<T, 3><<<L.ndom, 512, 0, L.stream>>>(P, L.tb, L.nt);
    else k_tail_eps<T, 2><<<L.ndom, 512, 0, L.stream>>>(P, L.tb, L.nt);
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

void launch_norm64(const Launch &L, const Plane<double> &P, int nleafblk, bool var, float *rout32,
                   double *rout64) {
    if (nleafblk <= 0) return;
    DISPATCH_DB(L, {
        if (var) k_norm<D, BS, true><<<nleafblk, 256, 0, L.stream>>>(P, L.tb, L.partials, rout32, rout64);
        else k_norm<D, BS, false><<<nleafblk, 256, 0, L.stream>>>(P, L.tb, L.partials, rout32, rout64);
    });
}

void launch_reduce_norms(const Launch &L) {
    k_reduce_norms<<<L.ndom, 256, 0, L.stream>>>(L.tb, L.partials, L.dom_norms);
}

void launch_add_leaf(const Launch &L, double *v64, const float *v32, int nleafblk) {
    if (nleafblk <= 0) return;
    const int nc = cells(L.dim, L.bs);
    const int tpb = nc < 256 ? nc : 256, wpb = nc / tpb;
    const unsigned grid = (unsigned)(nleafblk * wpb);
    switch (nc) {
        case 4096: k_add_leaf<4096><<<grid, tpb, 0, L.stream>>>(v64, v32, L.tb, wpb); break;
        case 512: k_add_leaf<512><<<grid, tpb, 0, L.stream>>>(v64, v32, L.tb, wpb); break;
        case 256: k_add_leaf<256><<<grid, tpb, 0, L.stream>>>(v64, v32, L.tb, wpb); break;
        case 64: k_add_leaf<64><<<grid, tpb, 0, L.stream>>>(v64, v32, L.tb, wpb); break;
        default: k_add_leaf<16><<<grid, tpb, 0, L.stream>>>(v64, v32, L.tb, wpb); break;
    }
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
