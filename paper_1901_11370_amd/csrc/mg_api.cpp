// C ABI (include/mg.h) and the host-side cycle driver of the multigrid library.
//
// The driver walks the global levels and queues kernels on the bound stream: the
// FAS V-cycle and FMG cycle of Sec. 2.4, the composite residual, and FP64 iterative
// refinement around FP32 cycles.  Several domains (independent problems) share one
// store; their levels are aligned at the bottom (every domain's reduced-block-size
// levels occupy global levels 0..nt-1), so each level's blocks of all domains are
// processed by one launch and every domain still sees its own cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mg_internal.hpp"

using namespace mgx;

struct mg_tree {
    HostTree T;
    mg_params prm{};
    std::string err;
    // binding
    char *store = nullptr;
    size_t need = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool homog = false;
    bool folded = false;            // boundary values folded into f since the last mg_set_rhs
    // device views
    DevTables tb{}, tb0{};          // real boundary values / homogeneous
    uint64_t tail_lds[2] = {0, 0};  // domains whose coarse grids fit in LDS (FP64, FP32)
    Plane<double> P64{};
    Plane<float> P32{};
    std::vector<int32_t *> d_parents, d_cff;
    std::vector<std::vector<int32_t>> cf_faces;   // per level: 8 b + f of each coarse-fine face
    double *d_stage = nullptr, *d_stage2 = nullptr;
    int32_t *d_steps = nullptr;
    double *d_partials = nullptr, *d_domnorms = nullptr;
    double *d_hnorms = nullptr;      // device address of h_norms
    // FGMRES (mixed mode with krylov = m): V[m+1], Z[m] leaf vectors, inner-product
    // partials, dot results (3 sets), combination coefficients; pinned host copies
    double *d_kv = nullptr, *d_kz = nullptr, *d_kpart = nullptr, *d_kdots = nullptr, *d_ky = nullptr;
    double *h_k = nullptr;
    size_t off_tables = 0, bytes_tables = 0;
    std::vector<char> host_tables;  // image of the table region
    // layout bookkeeping
    int64_t nb = 0, nleafblk = 0, nc = 0, ng = 0;
    // stats
    std::vector<double> stat_res, stat_sec;
    // captured cycle sequences (graph kind x homogeneous flag), replayed on `stream`
    hipStream_t cap = nullptr;       // capture stream (non-blocking, default priority)
    double *h_norms = nullptr;       // pinned host copy of the per-domain norms
    hipGraphExec_t gexec[64] = {};
    bool gfail[64] = {};
    // profiling: event pairs around the finest-level smoothing launches (kernels are
    // then launched one by one, not replayed from graphs)
    bool prof = false;
    std::vector<hipEvent_t> ev;      // pool
    size_t ev_used = 0;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
};

namespace {

int fail(mg_tree *t, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (t) t->err = buf;
    return code;
}

#define HIP_OR_FAIL(t, call)                                                                   \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(t, MG_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int check_launch(mg_tree *t) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(t, MG_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return MG_OK;
}

struct Layout {
    size_t off = 0;
    template <typename X>
    size_t take(size_t count) {
        off = (off + 255) & ~size_t(255);
        size_t o = off;
        off += count * sizeof(X);
        return o;
    }
};

bool mixed(const mg_tree *t) { return t->prm.precision == MG_MIXED; }
bool jacobi(const mg_tree *t) { return t->prm.smoother == MG_SMOOTH_JACOBI; }
bool var(const mg_tree *t) { return t->prm.variable_eps != 0; }

// Computes the byte offsets of every array of the store; with base != nullptr also
// sets the device pointers.
size_t plan(mg_tree *t, char *base) {
    HostTree &T = t->T;
    Layout L;
    const int64_t nb = T.lev_first[T.nlev];
    int64_t nc = 1;
    for (int a = 0; a < T.dim; a++) nc *= T.bs;
    int64_t nf = T.dim == 3 ? (int64_t)T.bs * T.bs : T.bs;
    int64_t ng = 2 * T.dim * nf;
    t->nb = nb; t->nc = nc; t->ng = ng;
    t->nleafblk = (int64_t)T.leaf_blk.size();
    auto P = [&](size_t o) { return base ? base + o : nullptr; };
    // tables
    size_t o_org = L.take<int32_t>(3 * nb), o_nbr = L.take<int32_t>(6 * nb), o_cf = L.take<int32_t>(6 * nb);
    size_t o_par = L.take<int32_t>(nb), o_dom = L.take<int32_t>(nb), o_lev = L.take<int32_t>(nb);
    size_t o_leaf = L.take<int32_t>(t->nleafblk), o_lf = L.take<int32_t>(T.ndom + 1);
    size_t o_lrank = L.take<int32_t>(nb);
    size_t o_h = L.take<double>((size_t)T.ndom * MAXLEV * 3), o_nc = L.take<int32_t>((size_t)T.ndom * MAXLEV * 3);
    size_t o_ih2 = L.take<double>((size_t)T.ndom * MAXLEV * 3);
    size_t o_bck = L.take<int32_t>(6 * T.ndom), o_bcv = L.take<double>(6 * T.ndom), o_bc0 = L.take<double>(6 * T.ndom);
    size_t o_toff = L.take<int64_t>((size_t)T.ndom * MAXLEV);
    size_t o_ttop = L.take<int32_t>(T.ndom);
    size_t o_lox = L.take<double>(T.ndom);
    // per level the (block, face) pairs with a coarse neighbour, as 8 b + f
    t->cf_faces.assign(T.nlev, {});
    for (int l = 0; l < T.nlev; l++)
        for (int32_t b : T.cf_of_level[l])
            for (int f = 0; f < 2 * T.dim; f++)
                if (T.nbr[6 * (size_t)b + f] == -2) t->cf_faces[l].push_back(8 * b + f);
    std::vector<size_t> o_parl(T.nlev), o_cff(T.nlev);
    for (int l = 0; l < T.nlev; l++) {
        o_parl[l] = L.take<int32_t>(T.parents_of_level[l].size());
        o_cff[l] = L.take<int32_t>(t->cf_faces[l].size());
    }
    t->off_tables = 0;
    t->bytes_tables = L.off;
    if (base) {
        // host image of the tables
        std::vector<char> &img = t->host_tables;
        img.assign(L.off, 0);
        auto put = [&](size_t o, const void *src, size_t n) { if (n) memcpy(img.data() + o, src, n); };
        put(o_org, T.org.data(), T.org.size() * 4);
        put(o_nbr, T.nbr.data(), T.nbr.size() * 4);
        put(o_cf, T.cf.data(), T.cf.size() * 4);
        put(o_par, T.parent.data(), T.parent.size() * 4);
        put(o_dom, T.dom.data(), T.dom.size() * 4);
        put(o_lev, T.lev.data(), T.lev.size() * 4);
        put(o_leaf, T.leaf_blk.data(), T.leaf_blk.size() * 4);
        put(o_lf, T.leaf_first.data(), T.leaf_first.size() * 4);
        std::vector<int32_t> lrank(nb, -1);
        for (size_t r = 0; r < T.leaf_blk.size(); r++) lrank[T.leaf_blk[r]] = (int32_t)r;
        put(o_lrank, lrank.data(), lrank.size() * 4);
        put(o_h, T.h.data(), T.h.size() * 8);
        std::vector<double> ih2(T.h.size());
        for (size_t q = 0; q < T.h.size(); q++) ih2[q] = T.h[q] > 0.0 ? 1.0 / (T.h[q] * T.h[q]) : 0.0;
        put(o_ih2, ih2.data(), ih2.size() * 8);
        put(o_nc, T.ncell.data(), T.ncell.size() * 4);
        std::vector<int32_t> bck(6 * T.ndom);
        std::vector<double> bcv(6 * T.ndom), bc0(6 * T.ndom, 0.0);
        for (int i = 0; i < T.ndom; i++)
            for (int f = 0; f < 6; f++) {
                bck[6 * i + f] = f < 2 * T.dim ? T.doms[i].d.bc.kind[f] : MG_BC_PERIODIC;
                bcv[6 * i + f] = f < 2 * T.dim ? T.doms[i].d.bc.value[f] : 0.0;
            }
        put(o_bck, bck.data(), bck.size() * 4);
        put(o_bcv, bcv.data(), bcv.size() * 8);
        put(o_bc0, bc0.data(), bc0.size() * 8);
        put(o_toff, T.tail_off.data(), T.tail_off.size() * 8);
        put(o_ttop, T.tail_top.data(), T.tail_top.size() * 4);
        std::vector<double> lox(T.ndom);
        for (int i = 0; i < T.ndom; i++) lox[i] = T.doms[i].d.lo[0];
        put(o_lox, lox.data(), lox.size() * 8);
        for (int l = 0; l < T.nlev; l++) {
            put(o_parl[l], T.parents_of_level[l].data(), T.parents_of_level[l].size() * 4);
            put(o_cff[l], t->cf_faces[l].data(), t->cf_faces[l].size() * 4);
        }
        DevTables &tb = t->tb;
        tb.org = (const int32_t *)P(o_org);
        tb.nbr = (const int32_t *)P(o_nbr);
        tb.cf = (const int32_t *)P(o_cf);
        tb.parent = (const int32_t *)P(o_par);
        tb.dom = (const int32_t *)P(o_dom);
        tb.lev = (const int32_t *)P(o_lev);
        tb.leaf_blk = (const int32_t *)P(o_leaf);
        tb.leaf_first = (const int32_t *)P(o_lf);
        tb.leaf_rank = (const int32_t *)P(o_lrank);
        tb.h = (const double *)P(o_h);
        tb.ih2 = (const double *)P(o_ih2);
        tb.ncell = (const int32_t *)P(o_nc);
        tb.bck = (const int32_t *)P(o_bck);
        tb.bcv = (const double *)P(o_bcv);
        tb.tail_off = (const int64_t *)P(o_toff);
        tb.tail_top = (const int32_t *)P(o_ttop);
        tb.lambda = t->prm.helmholtz_lambda;
        tb.axi = t->prm.axisymmetric;
        tb.lox = (const double *)P(o_lox);
        t->tb0 = tb;
        t->tb0.bcv = (const double *)P(o_bc0);
        t->d_parents.assign(T.nlev, nullptr);
        t->d_cff.assign(T.nlev, nullptr);
        for (int l = 0; l < T.nlev; l++) {
            t->d_parents[l] = (int32_t *)P(o_parl[l]);
            t->d_cff[l] = (int32_t *)P(o_cff[l]);
        }
    }
    // fields
    auto plane = [&](auto *pl, auto tag) {
        using TT = decltype(tag);
        size_t ov = L.take<TT>(nb * nc), ovg = L.take<TT>(nb * ng);
        size_t oo = L.take<TT>(nb * nc), oog = L.take<TT>(nb * ng);
        size_t of = L.take<TT>(nb * nc);
        size_t oe = 0, oeg = 0;
        if (var(t)) { oe = L.take<TT>(nb * nc); oeg = L.take<TT>(nb * ng); }
        size_t otv = L.take<TT>(T.tail_cells), oto = L.take<TT>(T.tail_cells), otf = L.take<TT>(T.tail_cells);
        size_t ote = var(t) ? L.take<TT>(T.tail_cells) : 0;
        size_t ov2 = 0, ovg2 = 0, otv2 = 0;
        if (jacobi(t)) { ov2 = L.take<TT>(nb * nc); ovg2 = L.take<TT>(nb * ng); otv2 = L.take<TT>(T.tail_cells); }
        if (base) {
            pl->v = (TT *)P(ov); pl->vg = (TT *)P(ovg);
            pl->vold = (TT *)P(oo); pl->voldg = (TT *)P(oog);
            pl->f = (TT *)P(of);
            pl->eps = var(t) ? (TT *)P(oe) : nullptr;
            pl->epsg = var(t) ? (TT *)P(oeg) : nullptr;
            pl->tv = (TT *)P(otv); pl->tvold = (TT *)P(oto); pl->tf = (TT *)P(otf);
            pl->teps = var(t) ? (TT *)P(ote) : nullptr;
            pl->v2 = jacobi(t) ? (TT *)P(ov2) : nullptr;
            pl->vg2 = jacobi(t) ? (TT *)P(ovg2) : nullptr;
            pl->tv2 = jacobi(t) ? (TT *)P(otv2) : nullptr;
        }
    };
    plane(&t->P64, double(0));
    if (mixed(t)) plane(&t->P32, float(0));
    size_t o_st = L.take<double>(T.nleaf_cells), o_st2 = L.take<double>(T.nleaf_cells);
    size_t o_steps = L.take<int32_t>(T.ndom), o_part = L.take<double>(4 * std::max<int64_t>(t->nleafblk, 1));
    size_t o_dn = L.take<double>(4 * T.ndom);
    const int km = mixed(t) ? t->prm.krylov : 0;
    size_t o_kv = 0, o_kz = 0, o_kp = 0, o_kd = 0, o_ky = 0;
    if (km > 0) {
        o_kv = L.take<double>((size_t)(km + 1) * T.nleaf_cells);
        o_kz = L.take<double>((size_t)km * T.nleaf_cells);
        o_kp = L.take<double>((size_t)(km + 1) * dots_chunks(T.nleaf_cells));
        o_kd = L.take<double>(3 * (size_t)(km + 1));
        o_ky = L.take<double>((size_t)(km + 1));
    }
    if (base) {
        if (km > 0) {
            t->d_kv = (double *)P(o_kv);
            t->d_kz = (double *)P(o_kz);
            t->d_kpart = (double *)P(o_kp);
            t->d_kdots = (double *)P(o_kd);
            t->d_ky = (double *)P(o_ky);
        }
        t->d_stage = (double *)P(o_st);
        t->d_stage2 = (double *)P(o_st2);
        t->d_steps = (int32_t *)P(o_steps);
        t->d_partials = (double *)P(o_part);
        t->d_domnorms = (double *)P(o_dn);
    }
    return (L.off + 255) & ~size_t(255);
}

Launch launch(mg_tree *t, bool homogeneous) {
    Launch L;
    L.dim = t->T.dim; L.bs = t->T.bs; L.nt = t->T.nt; L.ndom = t->T.ndom;
    L.tb = homogeneous ? t->tb0 : t->tb;
    L.stream = t->stream;
    L.coarse_steps = t->d_steps;
    L.partials = t->d_partials;
    L.dom_norms = t->d_domnorms;
    L.host_norms = nullptr;
    L.tail_lds[0] = t->tail_lds[0];
    L.tail_lds[1] = t->tail_lds[1];
    return L;
}

// Domains whose coarse grids (v and f of every grid, v_old below the top grid, eps)
// fit in the coarse solver's LDS for fields of `bytes` bytes; the solver kernel makes
// the same test.
uint64_t tail_fit_mask(const HostTree &T, int bytes, bool var) {
    uint64_t m = 0;
    for (int dm = 0; dm < T.ndom && dm < 64; dm++) {
        const int top = T.tail_top[dm];
        const int64_t first = T.tail_off[(size_t)dm * MAXLEV];
        const int32_t *nc = &T.ncell[((size_t)dm * MAXLEV + top) * 3];
        const int64_t last = (int64_t)(nc[0] + 2) * (nc[1] + 2) * (T.dim == 3 ? nc[2] + 2 : 1);
        const int64_t n = T.tail_off[(size_t)dm * MAXLEV + top] + last - first;
        const int64_t nold = T.tail_off[(size_t)dm * MAXLEV + top] - first;
        const int64_t need = (2 * n + nold + (var ? n : 0)) * bytes;
        if (need <= tail_lds_bytes()) m |= 1ull << dm;
    }
    return m;
}

uint64_t all_mask(const mg_tree *t) {
    return t->T.ndom >= 64 ? ~0ull : ((1ull << t->T.ndom) - 1);
}

uint64_t mask_top_at_least(const mg_tree *t, int lev) {
    uint64_t m = 0;
    for (int i = 0; i < t->T.ndom; i++)
        if (t->T.doms[i].top >= lev) m |= 1ull << i;
    return m;
}

TailParams tail_params(const mg_tree *t) {
    TailParams tp;
    tp.n_down = t->prm.n_down; tp.n_up = t->prm.n_up; tp.n_max = t->prm.n_max_coarse;
    tp.abs_tol = t->prm.coarse_abs_tol; tp.rel_tol = t->prm.coarse_rel_tol;
    tp.jacobi = jacobi(t) ? 1 : 0;
    tp.omega = t->prm.jacobi_weight;
    return tp;
}

int lvb0(const mg_tree *t, int l) { return t->T.lev_first[l]; }
int lvnb(const mg_tree *t, int l) { return t->T.lev_first[l + 1] - t->T.lev_first[l]; }

// ------------------------------------------------------------ cycle driver
template <typename T>
struct Driver {
    mg_tree *t;
    Launch L;
    Plane<T> P;
    bool v;   // variable eps
    // The first half-sweep of the next smoothing starts from v = 0 on its level: it
    // reads neither colour's old values (set for correction solves from e = 0).
    bool zero_first = false;

    void ghost_level(int l, uint64_t m) { K<T>::ghost(L, P, lvb0(t, l), lvnb(t, l), nullptr, 0, m, false, false); }

    // Weighted Jacobi: steps alternate between v and its second copy; after an odd
    // number the level's blocks are copied back.  Coarse-fine ghosts of the copy being
    // written take their coarse values from v of the coarser level.
    void jacobi_smooth(int l, uint64_t m, int steps) {
        const int ncf = (int)t->T.cf_of_level[l].size();
        const int b0 = lvb0(t, l), nb = lvnb(t, l);
        for (int s = 0; s < steps; s++) {
            const bool fwd = (s & 1) == 0;
            Plane<T> S = P;
            if (!fwd) { S.v = P.v2; S.vg = P.vg2; }
            T *dst = fwd ? P.v2 : P.v, *dstg = fwd ? P.vg2 : P.vg;
            K<T>::jacobi(L, S, dst, dstg, l, b0, nb, m, v, t->prm.jacobi_weight);
            if (ncf) {
                Plane<T> Dp = P;
                Dp.v = dst;
                Dp.vg = dstg;
                Dp.vc = P.v;
                Dp.vcg = P.vg;
                K<T>::cf_ghost(L, Dp, t->d_cff[l], (int)t->cf_faces[l].size(), m);
            }
        }
        if (steps & 1) {
            K<T>::copy(L, P.v + (size_t)b0 * t->nc, P.v2 + (size_t)b0 * t->nc, (size_t)nb * t->nc);
            K<T>::copy(L, P.vg + (size_t)b0 * t->ng, P.vg2 + (size_t)b0 * t->ng, (size_t)nb * t->ng);
        }
    }

    void smooth(int l, uint64_t m, int steps) {
        if (jacobi(t)) {
            jacobi_smooth(l, m, steps);
            return;
        }
        const bool timed = t->prof && l == t->T.nlev - 1;
        const int ncf = (int)t->T.cf_of_level[l].size();
        for (int s = 0; s < steps; s++)
            for (int c = 0; c < 2; c++) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                const bool z = zero_first && s == 0 && c == 0;
                // (the zero-start half-sweep moves other bytes and is not timed)
                if (timed && !z) {
                    if (t->ev_used + 2 > t->ev.size()) {
                        for (int q = 0; q < 64; q++) {
                            hipEvent_t e;
                            if (hipEventCreate(&e) == hipSuccess) t->ev.push_back(e);
                        }
                    }
                    if (t->ev_used + 2 <= t->ev.size()) {
                        e0 = t->ev[t->ev_used];
                        e1 = t->ev[t->ev_used + 1];
                        t->ev_used += 2;
                    }
                }
                K<T>::gsrb(L, P, l, lvb0(t, l), lvnb(t, l), c, m, v, e0, e1, z);
                zero_first = false;
                if (ncf) cf_refresh(l, m);
            }
    }
    // Coarse-fine ghosts of level l from the current fine and coarse values.
    void cf_refresh(int l, uint64_t m) {
        const int nf = (int)t->cf_faces[l].size();
        if (nf) K<T>::cf_ghost(L, P, t->d_cff[l], nf, m);
    }
    // The restriction pushes the parents' new boundary values into the ghosts of
    // level l-1; the other ghosts of that level are unchanged since its last update.
    void restrict_fas(int l, uint64_t m) {
        K<T>::restrict_down(L, P, l, lvb0(t, l), lvnb(t, l), m, RESTRICT_FAS, v);
        if (l > t->T.nt)
            K<T>::fas(L, P, l - 1, t->d_parents[l - 1], (int)t->T.parents_of_level[l - 1].size(), m, v);
    }
    // The correction pushes same-level and boundary ghosts; coarse-fine ghosts follow.
    // next_steps: smoothing steps that follow on level l; with red-black Gauss-Seidel the
    // first half-sweep rewrites colour 0 without reading it, so only colour 1 needs the
    // correction, except in blocks with a physical or coarse-fine face, whose ghosts
    // are computed from colour-0 cells before that half-sweep reads them.
    void correct(int l, uint64_t m, int next_steps) {
        const bool half = next_steps > 0 && !jacobi(t);
        K<T>::correct(L, P, l, lvb0(t, l), lvnb(t, l), m, half);
        cf_refresh(l, m);
    }
    // ---- tail levels: the large ones (per domain) as multi-workgroup launches, the
    // rest inside the one-workgroup kernel
    UGrid ugrid(int dm, int l) const {
        const HostTree &H = t->T;
        UGrid g;
        g.dm = dm;
        g.lev = l;
        for (int a = 0; a < 3; a++) {
            g.n[a] = H.ncell[((size_t)dm * MAXLEV + l) * 3 + a];
            g.h[a] = H.h[((size_t)dm * MAXLEV + l) * 3 + a];
        }
        g.off = H.tail_off[(size_t)dm * MAXLEV + l];
        return g;
    }
    bool big(int dm, int l) const { return l < t->T.nt && l > t->T.tail_top[dm]; }
    bool in(uint64_t m, int dm) const { return (m >> dm) & 1; }
    // Ghosts, then v_old and the FAS right-hand side, of a large tail grid whose
    // values a restriction just wrote.
    void uenter(int dm, int l) {
        const UGrid g = ugrid(dm, l);
        K<T>::ughost(L, P, g);
        K<T>::ufas(L, P, g, v);
    }
    void usmooth(int dm, int l, int steps) {
        const UGrid g = ugrid(dm, l);
        if (jacobi(t)) {
            for (int s = 0; s < steps; s++) {
                const bool fwd = (s & 1) == 0;
                K<T>::ujacobi(L, P, fwd ? P.tv : P.tv2, fwd ? P.tv2 : P.tv, g, v, t->prm.jacobi_weight);
            }
            if (steps & 1) {
                size_t npad = (size_t)(g.n[0] + 2) * (g.n[1] + 2) * (t->T.dim == 3 ? g.n[2] + 2 : 1);
                K<T>::copy(L, P.tv + g.off, P.tv2 + g.off, npad);
            }
            return;
        }
        for (int s = 0; s < steps; s++)
            for (int c = 0; c < 2; c++) K<T>::ugsrb(L, P, g, c, v);
    }
    // V-cycle over the tail levels <= top of the domains in m.
    void tail_vcycle(int top, uint64_t m) {
        for (int l = top; l >= 1; l--)
            for (int dm = 0; dm < t->T.ndom; dm++) {
                if (!in(m, dm) || !big(dm, l)) continue;
                usmooth(dm, l, t->prm.n_down);
                K<T>::urestrict(L, P, ugrid(dm, l), ugrid(dm, l - 1), v);
                if (big(dm, l - 1)) uenter(dm, l - 1);
            }
        K<T>::tail(L, P, TAIL_VCYCLE, m, tail_params(t), v);
        for (int l = 1; l <= top; l++)
            for (int dm = 0; dm < t->T.ndom; dm++) {
                if (!in(m, dm) || !big(dm, l)) continue;
                K<T>::ucorrect(L, P, ugrid(dm, l), ugrid(dm, l - 1));
                usmooth(dm, l, t->prm.n_up);
            }
    }
    // The restriction from the lowest block level wrote the top tail grid.
    void enter_tail(uint64_t m) {
        for (int dm = 0; dm < t->T.ndom; dm++)
            if (in(m, dm) && big(dm, t->T.nt - 1)) uenter(dm, t->T.nt - 1);
    }

    void vcycle(int top, uint64_t m) {
        const int nt = t->T.nt;
        for (int l = top; l >= nt; l--) {
            smooth(l, m, t->prm.n_down);
            restrict_fas(l, m);
        }
        enter_tail(m);
        tail_vcycle(nt - 1, m);
        for (int l = nt; l <= top; l++) {
            correct(l, m, t->prm.n_up);
            smooth(l, m, t->prm.n_up);
        }
    }
    void fmg() {
        const int nt = t->T.nt, top = t->T.nlev - 1;
        const uint64_t all = all_mask(t);
        for (int l = top; l >= nt; l--) restrict_fas(l, all);
        enter_tail(all);
        for (int l = nt - 1; l >= 1; l--)
            for (int dm = 0; dm < t->T.ndom; dm++) {
                if (!big(dm, l)) continue;
                K<T>::urestrict(L, P, ugrid(dm, l), ugrid(dm, l - 1), v);
                if (big(dm, l - 1)) uenter(dm, l - 1);
            }
        K<T>::tail(L, P, TAIL_FMG, all, tail_params(t), v);
        for (int l = 1; l < nt; l++) {
            uint64_t m = 0;
            for (int dm = 0; dm < t->T.ndom; dm++)
                if (big(dm, l)) {
                    m |= 1ull << dm;
                    K<T>::ucorrect(L, P, ugrid(dm, l), ugrid(dm, l - 1));
                }
            if (m) tail_vcycle(l, m);
        }
        for (int l = nt; l <= top; l++) {
            uint64_t m = mask_top_at_least(t, l);
            correct(l, m, t->prm.n_down);   // the V-cycle starts by smoothing level l
            vcycle(l, m);
        }
    }
    // Parents take the mean of their children, then ghosts from coarse to fine.  With
    // pushed set, every same-level and boundary ghost is already current (the last
    // kernel to change each cell pushed it: after a cycle, or after a leaf update that
    // pushes) and the restriction pushes the parents' new values, so only the
    // coarse-fine ghosts are recomputed; otherwise every ghost is.  Both give the same
    // values.
    void sync(bool pushed = false) {
        const int nt = t->T.nt, top = t->T.nlev - 1;
        const uint64_t all = all_mask(t);
        for (int l = top; l > nt; l--) K<T>::restrict_down(L, P, l, lvb0(t, l), lvnb(t, l), all, RESTRICT_V, false);
        for (int l = nt; l <= top; l++) {
            if (pushed) cf_refresh(l, all);
            else ghost_level(l, all);
        }
    }
};

Driver<double> d64(mg_tree *t) { return Driver<double>{t, launch(t, t->homog), t->P64, var(t)}; }
Driver<float> d32(mg_tree *t) { return Driver<float>{t, launch(t, true), t->P32, var(t)}; }

// FP64 composite residual (per-domain norms in d_domnorms); r may be written into the
// FP32 right-hand side; with copy_out the norms are copied to the pinned host buffer.
// after_cycle: the FP64 values were last changed by a cycle or by launch_add_leaf in
// the same sequence, so their same-level and boundary ghosts are current.
void enq_residual(mg_tree *t, bool write_r32, bool copy_out, bool after_cycle = false) {
    Driver<double> D = d64(t);
    // Without refinement the leaf residual uses only same-level and boundary ghosts,
    // which every kernel keeps current; parents enter only through coarse-fine ghosts.
    if (t->T.refined) D.sync(after_cycle);
    launch_norm64(D.L, t->P64, (int)t->nleafblk, var(t), write_r32 ? t->P32.f : nullptr, nullptr);
    if (copy_out) D.L.host_norms = t->d_hnorms;   // the reduction writes the pinned host buffer too
    launch_reduce_norms(D.L);
}

// Waits for the stream and returns the norms copied by the last enq_residual.
int read_norms(mg_tree *t, std::vector<double> *norms) {
    HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    norms->assign(t->h_norms, t->h_norms + 4 * t->T.ndom);
    return MG_OK;
}

// Kinds of captured sequences.
enum {
    G_V = 0, G_FMG, G_V_NORM, G_FMG_NORM, G_NORM, G_NORM_R32, G_IRV_NORM, G_IRFMG_NORM, G_IRV_FULL, G_IRFMG_FULL,
    G_V_SYNC,                          // a V-cycle and the state updates of the norm (refined trees)
    G_IRV_FEWER,                       // G_IRV_NORM with 1 ... kIrFewer V-cycles (kinds G_IRV_FEWER + n - 1)
    G_KINDS = G_IRV_FEWER + 8
};
constexpr int kIrFewer = G_KINDS - G_IRV_FEWER;
static_assert(2 * G_KINDS <= 64, "graph slots");

void drop_graphs(mg_tree *t) {
    for (auto &g : t->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (bool &f : t->gfail) f = false;
}

// Queues body()'s kernels on the bound stream: replays the captured graph of this
// kind (capturing it on first use), or launches directly when graphs are off, while
// profiling, or if capture failed.
template <typename F>
int run_seq(mg_tree *t, int kind, F &&body) {
    const int key = 2 * kind + (t->homog ? 1 : 0);
    if (t->prm.graphs && !t->prof && !t->gfail[key]) {
        if (!t->gexec[key]) {
            hipStream_t user = t->stream;
            bool ok = hipStreamBeginCapture(t->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
            hipGraph_t g = nullptr;
            if (ok) {
                t->stream = t->cap;
                body();
                t->stream = user;
                ok = hipStreamEndCapture(t->cap, &g) == hipSuccess && g;
                ok = ok && hipGetLastError() == hipSuccess;
            }
            if (ok) ok = hipGraphInstantiate(&t->gexec[key], g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                t->gexec[key] = nullptr;
                t->gfail[key] = true;
                (void)hipGetLastError();
            }
        }
        if (t->gexec[key]) {
            HIP_OR_FAIL(t, hipGraphLaunch(t->gexec[key], t->stream));
            return MG_OK;
        }
    }
    body();
    return check_launch(t);
}

void rel_norms(const mg_tree *t, const std::vector<double> &n, double *mx, double *l2) {
    for (int i = 0; i < t->T.ndom; i++) {
        const double *p = &n[4 * i];
        mx[i] = p[2] > 0 ? p[0] / p[2] : p[0];
        l2[i] = p[3] > 0 ? std::sqrt(p[1] / p[3]) : std::sqrt(p[1]);
    }
}

int worst(const mg_tree *t, const std::vector<double> &n, double *mx, double *l2) {
    std::vector<double> a(t->T.ndom), b(t->T.ndom);
    rel_norms(t, n, a.data(), b.data());
    double m = 0, q = 0;
    bool bad = false;
    for (int i = 0; i < t->T.ndom; i++) {
        if (!std::isfinite(a[i]) || !std::isfinite(b[i])) bad = true;
        m = std::max(m, a[i]);
        q = std::max(q, b[i]);
    }
    if (mx) *mx = bad ? NAN : m;
    if (l2) *l2 = bad ? NAN : q;
    return bad ? MG_ERR_NAN : MG_OK;
}

// One step of iterative refinement: r = f - L phi in FP64 (also the norm), then the
// FP32 correction solve L e = r with zero initial guess and homogeneous boundary
// values, then phi += e on the leaves.
// One refinement step's correction: FP32 cycle(s) on L e = r (r in the FP32 right-hand
// side, e from zero), then phi += e unless the caller fuses that with the next residual
// (enq_add_residual).
void ir_enqueue(mg_tree *t, bool use_fmg, bool defer_add = false, int n_v = 0) {
    Driver<float> D = d32(t);
    const Plane<float> &P = t->P32;
    // A V-cycle from e = 0 on a tree whose leaves are all on the top level (of every
    // domain) first smooths the top level, whose first half-sweep then needs no old
    // values; every other value it reads is written by the cycle before it is read
    // (restriction writes the parents and their ghosts, and the coarse grids).  Other
    // cases start from explicitly zeroed fields.
    bool same_top = true;
    for (const HDomain &d : t->T.doms) same_top = same_top && d.top == t->T.nlev - 1;
    const bool zs = !use_fmg && !t->T.refined && same_top && !jacobi(t) && t->prm.n_down > 0;
    if (!zs) {
        K<float>::zero(D.L, P.v, (size_t)(t->nb * t->nc));
        K<float>::zero(D.L, P.vg, (size_t)(t->nb * t->ng));
        K<float>::zero(D.L, P.tv, (size_t)t->T.tail_cells);
    }
    D.zero_first = zs;
    if (use_fmg) {
        D.fmg();
    } else {
        const int nv = n_v > 0 ? n_v : std::max(1, t->prm.ir_vcycles);
        for (int c = 0; c < nv; c++) D.vcycle(t->T.nlev - 1, all_mask(t));
    }
    if (defer_add) return;
    Launch L64 = launch(t, t->homog);
    launch_add_leaf(L64, t->P64.v, t->P64.vg, P.v, (int)t->nleafblk);
}

// phi += e (the FP32 correction left by ir_enqueue(..., true)), then the residual as
// enq_residual: one fused launch on trees without refinement.
void enq_add_residual(mg_tree *t, bool write_r32, bool copy_out) {
    if (t->T.refined) {
        launch_add_leaf(launch(t, t->homog), t->P64.v, t->P64.vg, t->P32.v, (int)t->nleafblk);
        enq_residual(t, write_r32, copy_out, true);
        return;
    }
    Driver<double> D = d64(t);
    launch_add_norm64(D.L, t->P64, t->P32.v, t->P32.vg, (int)t->nleafblk, var(t), write_r32 ? t->P32.f : nullptr);
    if (copy_out) D.L.host_norms = t->d_hnorms;
    launch_reduce_norms(D.L);
}

// ---- FGMRES refinement (mixed mode, krylov = m)
// r = f - L phi (FP64, actual boundary values) into the leaf vector out; norms copied
// to the host buffer.
void enq_residual_vec(mg_tree *t, double *out) {
    Driver<double> D = d64(t);
    if (t->T.refined) D.sync();
    launch_norm64(D.L, t->P64, (int)t->nleafblk, var(t), nullptr, out);
    D.L.host_norms = t->d_hnorms;
    launch_reduce_norms(D.L);
}

// w = A z, A the composite operator with homogeneous boundary values; z is placed in
// the v_old field of the FP64 plane (unused by mixed-mode solves).
void enq_apply(mg_tree *t, double *z, double *w) {
    Plane<double> Q = t->P64;
    Q.v = t->P64.vold;
    Q.vg = t->P64.voldg;
    Q.f = nullptr;
    Driver<double> D{t, launch(t, true), Q, var(t)};
    launch_vec_blocks<double>(D.L, Q.v, z, (int)t->nleafblk, true);
    if (t->T.refined) D.sync();
    else
        for (int l = t->T.nt; l < t->T.nlev; l++) D.ghost_level(l, all_mask(t));
    launch_norm64(D.L, Q, (int)t->nleafblk, var(t), nullptr, w);
}

// z = M^-1 v: one FP32 V-cycle from zero (homogeneous boundary values) on the
// correction equation with right-hand side v.
void enq_precond(mg_tree *t, double *v, double *z) {
    Driver<float> D = d32(t);
    const Plane<float> &P = t->P32;
    launch_vec_blocks<float>(D.L, P.f, v, (int)t->nleafblk, true);
    K<float>::zero(D.L, P.v, (size_t)(t->nb * t->nc));
    K<float>::zero(D.L, P.vg, (size_t)(t->nb * t->ng));
    K<float>::zero(D.L, P.tv, (size_t)t->T.tail_cells);
    D.vcycle(t->T.nlev - 1, all_mask(t));
    launch_vec_blocks<float>(D.L, P.v, z, (int)t->nleafblk, false);
}

// Restarted flexible GMRES on A e = r in FP64 (classical Gram-Schmidt with one
// re-orthogonalisation pass, Givens rotations), preconditioned by enq_precond; each
// restart starts from the true residual of the current phi and ends with phi += Z y.
template <typename Rec>
int solve_fgmres(mg_tree *t, double rel_tol, int max_cycles, bool fmg_first, int *cycles_io, double *rel_out,
                 Rec &&record) {
    const int m = t->prm.krylov;
    const int64_t n = t->T.nleaf_cells;
    const int nlb = (int)t->nleafblk;
    double *V = t->d_kv, *Z = t->d_kz, *part = t->d_kpart, *dd = t->d_kdots;
    auto Vi = [&](int i) { return V + (int64_t)i * n; };
    auto Zi = [&](int i) { return Z + (int64_t)i * n; };
    const Launch L = launch(t, true);
    const size_t stride3 = (size_t)(m + 1);
    std::vector<double> H((size_t)(m + 1) * m, 0.0), g(m + 1), cs(m), sn(m), y(m);
    auto h = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    std::vector<double> nrm;
    int &cycles = *cycles_io;
    int rc;
    for (;;) {
        enq_residual_vec(t, Vi(0));
        if ((rc = read_norms(t, &nrm))) return rc;
        rc = worst(t, nrm, rel_out, nullptr);
        record(*rel_out);
        if (rc) return rc;
        if (*rel_out <= rel_tol || cycles >= max_cycles) return MG_OK;
        if (cycles == 0 && fmg_first && t->prm.ir_first_fmg) {
            // first step: a plain refinement step with an FP32 FMG cycle
            launch_vec_blocks<float>(L, t->P32.f, Vi(0), nlb, true);
            ir_enqueue(t, true);
            cycles++;
            continue;
        }
        launch_dots(L, Vi(0), n, 1, Vi(0), n, part, dd);
        HIP_OR_FAIL(t, hipMemcpyAsync(t->h_k, dd, 8, hipMemcpyDeviceToHost, t->stream));
        HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
        const double beta = std::sqrt(t->h_k[0]);
        if (!std::isfinite(beta)) return fail(t, MG_ERR_NAN, "residual is not finite");
        if (beta == 0.0) return MG_OK;
        launch_scale(L, Vi(0), 1.0 / beta, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && cycles < max_cycles; j++) {
            enq_precond(t, Vi(j), Zi(j));
            cycles++;
            enq_apply(t, Zi(j), Vi(j + 1));
            launch_dots(L, V, n, j + 1, Vi(j + 1), n, part, dd);
            launch_combo(L, Vi(j + 1), V, n, dd, j + 1, -1.0, false, n);
            launch_dots(L, V, n, j + 1, Vi(j + 1), n, part, dd + stride3);
            launch_combo(L, Vi(j + 1), V, n, dd + stride3, j + 1, -1.0, false, n);
            launch_dots(L, Vi(j + 1), n, 1, Vi(j + 1), n, part, dd + 2 * stride3);
            if ((rc = check_launch(t))) return rc;
            HIP_OR_FAIL(t, hipMemcpyAsync(t->h_k, dd, 3 * stride3 * 8, hipMemcpyDeviceToHost, t->stream));
            HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
            for (int i = 0; i <= j; i++) h(i, j) = t->h_k[i] + t->h_k[stride3 + i];
            const double hn = std::sqrt(t->h_k[2 * stride3]);
            if (!std::isfinite(hn)) return fail(t, MG_ERR_NAN, "Krylov vector is not finite");
            h(j + 1, j) = hn;
            for (int i = 0; i < j; i++) {
                const double a = h(i, j), b = h(i + 1, j);
                h(i, j) = cs[i] * a + sn[i] * b;
                h(i + 1, j) = -sn[i] * a + cs[i] * b;
            }
            const double den = std::hypot(h(j, j), h(j + 1, j));
            cs[j] = den > 0 ? h(j, j) / den : 1.0;
            sn[j] = den > 0 ? h(j + 1, j) / den : 0.0;
            h(j, j) = den;
            h(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (hn == 0.0 || std::fabs(g[j + 1]) <= 1e-6 * beta) break;
            launch_scale(L, Vi(j + 1), 1.0 / hn, n);
        }
        if (k == 0) return MG_OK;
        for (int i = k - 1; i >= 0; i--) {
            double s = g[i];
            for (int q = i + 1; q < k; q++) s -= h(i, q) * y[q];
            y[i] = h(i, i) != 0.0 ? s / h(i, i) : 0.0;
        }
        double *hy = t->h_k + 3 * stride3;
        for (int i = 0; i < k; i++) hy[i] = y[i];
        HIP_OR_FAIL(t, hipMemcpyAsync(t->d_ky, hy, (size_t)k * 8, hipMemcpyHostToDevice, t->stream));
        launch_combo(L, Vi(0), Z, n, t->d_ky, k, 1.0, true, n);
        launch_add_vec(launch(t, t->homog), t->P64.v, t->P64.vg, Vi(0), nlb);
        if ((rc = check_launch(t))) return rc;
    }
}

int require_bound(mg_tree *t) {
    if (!t) return MG_ERR_ARG;
    if (!t->bound) return fail(t, MG_ERR_STATE, "tree is not bound to a device store");
    return MG_OK;
}

const double *stage_in(mg_tree *t, const double *src, int on_device, double *stage, int *rc) {
    *rc = MG_OK;
    if (on_device) return src;
    hipError_t e = hipMemcpyAsync(stage, src, (size_t)t->T.nleaf_cells * 8, hipMemcpyHostToDevice, t->stream);
    if (e != hipSuccess) *rc = fail(t, MG_ERR_DEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    return stage;
}

template <typename E>
void prep_eps(mg_tree *t, const Launch &L, const Plane<E> &P, const double *src) {
    K<E>::scatter(L, P.eps, src, (int)t->nleafblk);
    const int nt = t->T.nt, top = t->T.nlev - 1;
    for (int l = top; l >= nt; l--) K<E>::restrict_down(L, P, l, lvb0(t, l), lvnb(t, l), all_mask(t), RESTRICT_EPS, false);
    for (int l = nt; l <= top; l++) K<E>::ghost(L, P, lvb0(t, l), lvnb(t, l), nullptr, 0, all_mask(t), true, false);
    K<E>::tail_eps(L, P);
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int mg_default_params(mg_params *p) {
    if (!p) return MG_ERR_ARG;
    memset(p, 0, sizeof *p);
    p->n_down = 2;
    p->n_up = 2;
    p->n_max_coarse = 1000;
    p->coarse_abs_tol = 0.0;
    p->coarse_rel_tol = 1e-8;
    p->precision = MG_FP64;
    p->variable_eps = 0;
    p->ir_first_fmg = 1;
    p->ir_vcycles = 4;
    p->graphs = 1;
    p->krylov = 0;
    p->smoother = MG_SMOOTH_GSRB;
    p->jacobi_weight = 2.0 / 3.0;
    p->helmholtz_lambda = 0.0;
    p->axisymmetric = 0;
    return MG_OK;
}

int mg_tree_create(const mg_domain *domains, int n_domains, int block_size, int max_refine_levels,
                   mg_refine_fn refine, void *user_data, const mg_params *params, mg_tree **out) {
    if (!out) return MG_ERR_ARG;
    *out = nullptr;
    mg_tree *t = new mg_tree();
    if (params) t->prm = *params;
    else mg_default_params(&t->prm);
    const mg_params &p = t->prm;
    if (p.n_down < 0 || p.n_up < 0 || p.n_max_coarse < 1 || p.coarse_rel_tol < 0 || p.coarse_abs_tol < 0 ||
        (p.precision != MG_FP64 && p.precision != MG_MIXED) || p.ir_vcycles < 1 || (p.graphs != 0 && p.graphs != 1) ||
        p.krylov < 0 || p.krylov > 64 || (p.krylov > 0 && p.precision != MG_MIXED) ||
        (p.smoother != MG_SMOOTH_GSRB && p.smoother != MG_SMOOTH_JACOBI) ||
        !(p.jacobi_weight > 0.0 && p.jacobi_weight <= 1.0) || !(p.helmholtz_lambda >= 0.0) ||
        (p.axisymmetric != 0 && p.axisymmetric != 1)) {
        delete t;
        return MG_ERR_ARG;
    }
    if (p.axisymmetric && domains) {
        // the cylindrical form: x is a radius (>= 0) and has no periodic copy
        for (int i = 0; i < n_domains; i++)
            if (domains[i].dim != 2 || !(domains[i].lo[0] >= 0.0) || domains[i].bc.kind[0] == MG_BC_PERIODIC ||
                domains[i].bc.kind[1] == MG_BC_PERIODIC) {
                delete t;
                return MG_ERR_ARG;
            }
    }
    if (domains && p.helmholtz_lambda == 0.0) {
        // Without a Dirichlet face the operator annihilates constants.  A fully periodic
        // domain is made consistent on its coarsest grid (the mean of f is removed); a
        // domain whose faces are Neumann, or Neumann and periodic, would need its
        // boundary fluxes balanced against f, which the paper does not describe: rejected.
        for (int i = 0; i < n_domains; i++) {
            const int nf = domains[i].dim == 2 ? 4 : 6;
            bool dirichlet = false, periodic = true;
            for (int f = 0; f < nf && f < 6; f++) {
                dirichlet = dirichlet || domains[i].bc.kind[f] == MG_BC_DIRICHLET;
                periodic = periodic && domains[i].bc.kind[f] == MG_BC_PERIODIC;
            }
            if (!dirichlet && !periodic) {
                delete t;
                return MG_ERR_ARG;
            }
        }
    }
    std::string e = build_tree(t->T, domains, n_domains, block_size, max_refine_levels, refine, user_data);
    if (!e.empty()) {
        delete t;
        return MG_ERR_ARG;
    }
    t->need = plan(t, nullptr);
    t->tail_lds[0] = tail_fit_mask(t->T, 8, p.variable_eps != 0);
    t->tail_lds[1] = tail_fit_mask(t->T, 4, p.variable_eps != 0);
    *out = t;
    return MG_OK;
}

void mg_tree_destroy(mg_tree *t) {
    if (!t) return;
    for (hipEvent_t e : t->ev) (void)hipEventDestroy(e);
    drop_graphs(t);
    if (t->cap) (void)hipStreamDestroy(t->cap);
    if (t->h_norms) (void)hipHostFree(t->h_norms);
    if (t->h_k) (void)hipHostFree(t->h_k);
    delete t;
}

int mg_tree_storage_bytes(const mg_tree *t, size_t *bytes) {
    if (!t || !bytes) return MG_ERR_ARG;
    *bytes = t->need;
    return MG_OK;
}

int mg_tree_bind(mg_tree *t, void *device_store, size_t bytes, void *hip_stream) {
    if (!t || !device_store) return MG_ERR_ARG;
    if (((uintptr_t)device_store) & 255) return fail(t, MG_ERR_ARG, "store must be 256-byte aligned");
    if (bytes < t->need) return fail(t, MG_ERR_OOM, "store has %zu bytes, %zu needed", bytes, t->need);
    drop_graphs(t);
    if (!t->cap) {
        prepare_kernels();
        HIP_OR_FAIL(t, hipStreamCreateWithFlags(&t->cap, hipStreamNonBlocking));
    }
    {
        // device address of the fixed reduction scratch on this device (set-up of
        // mg_residual_norms_static)
        double *p = nullptr;
        if (static_partials(&p)) return fail(t, MG_ERR_DEVICE, "hipGetSymbolAddress of the reduction scratch failed");
    }
    if (!t->h_norms) {
        HIP_OR_FAIL(t, hipHostMalloc((void **)&t->h_norms, 4 * (size_t)t->T.ndom * 8, hipHostMallocDefault));
        HIP_OR_FAIL(t, hipHostGetDevicePointer((void **)&t->d_hnorms, t->h_norms, 0));
    }
    if (!t->h_k && mixed(t) && t->prm.krylov > 0)
        HIP_OR_FAIL(t, hipHostMalloc((void **)&t->h_k, 4 * (size_t)(t->prm.krylov + 1) * 8, hipHostMallocDefault));
    t->store = (char *)device_store;
    t->stream = (hipStream_t)hip_stream;
    plan(t, t->store);
    HIP_OR_FAIL(t, hipMemcpyAsync(t->store, t->host_tables.data(), t->host_tables.size(), hipMemcpyHostToDevice,
                                  t->stream));
    t->bound = true;
    t->homog = false;
    t->folded = false;
    // phi = 0, f = 0, eps = 1 everywhere; ghosts of the block levels filled.
    Launch L = launch(t, false);
    auto init = [&](auto &P, auto one) {
        using TT = decltype(one);
        K<TT>::zero(L, P.v, (size_t)(t->nb * t->nc));
        K<TT>::zero(L, P.vg, (size_t)(t->nb * t->ng));
        K<TT>::zero(L, P.vold, (size_t)(t->nb * t->nc));
        K<TT>::zero(L, P.voldg, (size_t)(t->nb * t->ng));
        K<TT>::zero(L, P.f, (size_t)(t->nb * t->nc));
        K<TT>::zero(L, P.tv, (size_t)t->T.tail_cells);
        K<TT>::zero(L, P.tvold, (size_t)t->T.tail_cells);
        K<TT>::zero(L, P.tf, (size_t)t->T.tail_cells);
        if (var(t)) {
            K<TT>::fill(L, P.eps, (size_t)(t->nb * t->nc), one);
            K<TT>::fill(L, P.epsg, (size_t)(t->nb * t->ng), one);
            K<TT>::fill(L, P.teps, (size_t)t->T.tail_cells, one);
        }
    };
    init(t->P64, double(1));
    if (mixed(t)) init(t->P32, float(1));
    Driver<double> D = d64(t);
    for (int l = t->T.nt; l < t->T.nlev; l++) D.ghost_level(l, all_mask(t));
    return check_launch(t);
}

int mg_num_leaf_cells(const mg_tree *t, int64_t *n) {
    if (!t || !n) return MG_ERR_ARG;
    *n = t->T.nleaf_cells;
    return MG_OK;
}

int mg_domain_leaf_cells(const mg_tree *t, int64_t *n) {
    if (!t || !n) return MG_ERR_ARG;
    for (int i = 0; i < t->T.ndom; i++) n[i] = t->T.dom_leaf_cells[i];
    return MG_OK;
}

int mg_num_levels(const mg_tree *t, int *n) {
    if (!t || !n) return MG_ERR_ARG;
    *n = t->T.nlev;
    return MG_OK;
}

int mg_level_blocks(const mg_tree *t, int32_t *n_blocks, int64_t *n_cells) {
    if (!t || !n_blocks || !n_cells) return MG_ERR_ARG;
    const HostTree &T = t->T;
    for (int l = 0; l < T.nlev; l++) {
        n_blocks[l] = T.lev_first[l + 1] - T.lev_first[l];
        int64_t c = 0;
        if (l >= T.nt) {
            c = (int64_t)n_blocks[l] * t->nc;
        } else {
            for (int i = 0; i < T.ndom; i++) {
                int64_t p = 1;
                for (int a = 0; a < T.dim; a++) p *= T.ncell[((size_t)i * MAXLEV + l) * 3 + a];
                c += p;
            }
        }
        n_cells[l] = c;
    }
    return MG_OK;
}

int mg_leaf_layout(const mg_tree *t, int32_t *out) {
    if (!t || !out) return MG_ERR_ARG;
    const HostTree &T = t->T;
    int64_t n = 0;
    const int bs = T.bs;
    for (size_t r = 0; r < T.leaf_blk.size(); r++) {
        int b = T.leaf_blk[r];
        int dm = T.dom[b];
        int rel = T.lev[b] - T.doms[dm].base;
        int kz = T.dim == 3 ? bs : 1;
        for (int k = 0; k < kz; k++)
            for (int j = 0; j < bs; j++)
                for (int i = 0; i < bs; i++) {
                    out[5 * n + 0] = dm;
                    out[5 * n + 1] = rel;
                    out[5 * n + 2] = T.org[3 * b] + i;
                    out[5 * n + 3] = T.org[3 * b + 1] + j;
                    out[5 * n + 4] = T.org[3 * b + 2] + k;
                    n++;
                }
    }
    return MG_OK;
}

int mg_set_rhs(mg_tree *t, const double *leaf_f, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_f) return MG_ERR_ARG;
    const double *src = stage_in(t, leaf_f, on_device, t->d_stage, &rc);
    if (rc) return rc;
    K<double>::scatter(launch(t, false), t->P64.f, src, (int)t->nleafblk);
    t->folded = false;
    return check_launch(t);
}

int mg_set_eps(mg_tree *t, const double *leaf_eps, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_eps) return MG_ERR_ARG;
    if (!var(t)) return fail(t, MG_ERR_STATE, "tree was created with variable_eps = 0");
    const double *src = stage_in(t, leaf_eps, on_device, t->d_stage, &rc);
    if (rc) return rc;
    prep_eps<double>(t, launch(t, false), t->P64, src);
    if (mixed(t)) prep_eps<float>(t, launch(t, true), t->P32, src);
    return check_launch(t);
}

int mg_set_phi(mg_tree *t, const double *leaf_phi, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_phi) return MG_ERR_ARG;
    const double *src = stage_in(t, leaf_phi, on_device, t->d_stage, &rc);
    if (rc) return rc;
    Driver<double> D = d64(t);
    K<double>::scatter(D.L, t->P64.v, src, (int)t->nleafblk);
    D.sync();
    return check_launch(t);
}

int mg_get_phi(mg_tree *t, double *leaf_phi, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_phi) return MG_ERR_ARG;
    double *dst = on_device ? leaf_phi : t->d_stage;
    K<double>::gather(launch(t, false), t->P64.v, dst, (int)t->nleafblk);
    if ((rc = check_launch(t))) return rc;
    if (!on_device) {
        HIP_OR_FAIL(t, hipMemcpyAsync(leaf_phi, dst, (size_t)t->T.nleaf_cells * 8, hipMemcpyDeviceToHost, t->stream));
        HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    }
    return MG_OK;
}

int mg_apply_operator(mg_tree *t, const double *leaf_phi, double *leaf_out, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_phi || !leaf_out) return MG_ERR_ARG;
    const double *src = stage_in(t, leaf_phi, on_device, t->d_stage, &rc);
    if (rc) return rc;
    // phi goes into the FP64 v_old field (scratch between cycles: every restriction
    // rewrites it before a correction reads it); the tree's phi is not touched
    Plane<double> Q = t->P64;
    Q.v = t->P64.vold;
    Q.vg = t->P64.voldg;
    Q.f = nullptr;
    Driver<double> D{t, launch(t, t->homog), Q, var(t)};
    K<double>::scatter(D.L, Q.v, src, (int)t->nleafblk);
    if (t->T.refined) D.sync();
    else
        for (int l = t->T.nt; l < t->T.nlev; l++) D.ghost_level(l, all_mask(t));
    // L phi as a rank-major leaf vector, back into the leaf blocks, then leaf order
    launch_norm64(D.L, Q, (int)t->nleafblk, var(t), nullptr, t->d_stage2);
    launch_vec_blocks<double>(D.L, Q.v, t->d_stage2, (int)t->nleafblk, true);
    double *dst = on_device ? leaf_out : t->d_stage;
    K<double>::gather(D.L, Q.v, dst, (int)t->nleafblk);
    if ((rc = check_launch(t))) return rc;
    if (!on_device) {
        HIP_OR_FAIL(t, hipMemcpyAsync(leaf_out, dst, (size_t)t->T.nleaf_cells * 8, hipMemcpyDeviceToHost, t->stream));
        HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    }
    return MG_OK;
}

// Leaf blocks (in leaf order, as leaf ranks) whose face `face` lies on a physical
// Dirichlet boundary.
static std::vector<int32_t> dirichlet_face_ranks(const mg_tree *t, int face) {
    const HostTree &T = t->T;
    std::vector<int32_t> out;
    for (size_t r = 0; r < T.leaf_blk.size(); r++) {
        const int b = T.leaf_blk[r];
        if (T.nbr[6 * (size_t)b + face] == -1 && T.doms[T.dom[b]].d.bc.kind[face] == MG_BC_DIRICHLET)
            out.push_back((int32_t)r);
    }
    return out;
}

int mg_boundary_faces(const mg_tree *t, int64_t *n_faces, int64_t *leaf_cell, int32_t *face) {
    if (!t || !n_faces) return MG_ERR_ARG;
    const HostTree &T = t->T;
    const int bs = T.bs, nf = T.dim == 3 ? bs * bs : bs;
    const int64_t nc = T.dim == 3 ? (int64_t)bs * bs * bs : (int64_t)bs * bs;
    int64_t n = 0;
    for (int f = 0; f < 2 * T.dim; f++) {
        const int a = f / 2, c = (f & 1) ? bs - 1 : 0;
        for (int32_t r : dirichlet_face_ranks(t, f)) {
            for (int q = 0; q < nf; q++, n++) {
                if (!leaf_cell && !face) continue;
                const int a1 = q % bs, a2 = T.dim == 3 ? q / bs : 0;
                const int i = a == 0 ? c : a1, j = a == 1 ? c : (a == 0 ? a1 : a2), k = a == 2 ? c : a2;
                if (leaf_cell) leaf_cell[n] = (int64_t)r * nc + ((int64_t)k * bs + j) * bs + i;
                if (face) face[n] = f;
            }
        }
    }
    *n_faces = n;
    return MG_OK;
}

int mg_fold_dirichlet(mg_tree *t, const double *values, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!values) return MG_ERR_ARG;
    const HostTree &T = t->T;
    const int nf = T.dim == 3 ? T.bs * T.bs : T.bs;
    // per block and face the offset of its values in the list (leaf blocks on a
    // Dirichlet face), -1 elsewhere
    std::vector<int64_t> off(6 * (size_t)t->nb, -1);
    int64_t nv = 0;
    for (int f = 0; f < 2 * T.dim; f++)
        for (int32_t r : dirichlet_face_ranks(t, f)) {
            off[6 * (size_t)T.leaf_blk[r] + f] = nv;
            nv += nf;
        }
    // scratch: the offset table (and host values) in the first staging buffer, L_a(0) in
    // the second, the zero field in v_old
    const int64_t words = 6 * t->nb + (on_device ? 0 : nv);
    if (words > T.nleaf_cells) return fail(t, MG_ERR_ARG, "grid too small for the boundary-value scratch");
    int64_t *d_off = reinterpret_cast<int64_t *>(t->d_stage);
    HIP_OR_FAIL(t, hipMemcpyAsync(d_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, t->stream));
    const double *d_val = values;
    if (!on_device) {
        double *dst = t->d_stage + 6 * t->nb;
        if (nv) HIP_OR_FAIL(t, hipMemcpyAsync(dst, values, (size_t)nv * 8, hipMemcpyHostToDevice, t->stream));
        d_val = dst;
    }
    // The shift of the leaf equations is the composite operator applied to phi = 0 with
    // these values in the physical ghosts (2a at a Dirichlet face) and zero elsewhere:
    // the boundary cells' 2a eps/h^2 terms and, where a coarse-fine face meets the
    // boundary, the change of the interpolated ghost through the coarse cell's
    // boundary ghost.  It is computed by the ghost and stencil kernels themselves.
    Plane<double> Q = t->P64;
    Q.v = t->P64.vold;
    Q.vg = t->P64.voldg;
    Q.f = nullptr;
    // (homogeneous tables: every face without listed values contributes nothing)
    Driver<double> D{t, launch(t, true), Q, var(t)};
    D.L.tb.fv_off = d_off;
    D.L.tb.fv = d_val;
    K<double>::zero(D.L, Q.v, (size_t)(t->nb * t->nc));
    K<double>::zero(D.L, Q.vg, (size_t)(t->nb * t->ng));
    for (int l = T.nt; l < T.nlev; l++) D.ghost_level(l, all_mask(t));
    launch_norm64(D.L, Q, (int)t->nleafblk, var(t), nullptr, t->d_stage2);
    launch_sub_vec_blocks(D.L, t->P64.f, t->d_stage2, (int)t->nleafblk);
    if ((rc = check_launch(t))) return rc;
    t->folded = true;
    // the host offset table (and host values) must outlive the copies
    HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    return MG_OK;
}

int mg_set_homogeneous_bc(mg_tree *t, int on) {
    if (!t) return MG_ERR_ARG;
    t->homog = on != 0;
    return MG_OK;
}

int mg_vcycle(mg_tree *t, int n) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (n < 0) return MG_ERR_ARG;
    for (int c = 0; c < n; c++) {
        if (mixed(t)) {
            rc = run_seq(t, G_IRV_FULL, [&] {
                enq_residual(t, true, false);
                ir_enqueue(t, false);
            });
        } else {
            rc = run_seq(t, G_V, [&] { d64(t).vcycle(t->T.nlev - 1, all_mask(t)); });
        }
        if (rc) return rc;
    }
    return check_launch(t);
}

int mg_fmg(mg_tree *t, int n) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (n < 0) return MG_ERR_ARG;
    for (int c = 0; c < n; c++) {
        if (mixed(t)) {
            rc = run_seq(t, G_IRFMG_FULL, [&] {
                enq_residual(t, true, false);
                ir_enqueue(t, true);
            });
        } else {
            rc = run_seq(t, G_FMG, [&] { d64(t).fmg(); });
        }
        if (rc) return rc;
    }
    return check_launch(t);
}

int mg_domain_residual_norms(mg_tree *t, double *max_rel, double *l2_rel) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!max_rel || !l2_rel) return MG_ERR_ARG;
    std::vector<double> n;
    if ((rc = run_seq(t, G_NORM, [&] { enq_residual(t, false, true); }))) return rc;
    if ((rc = read_norms(t, &n))) return rc;
    rel_norms(t, n, max_rel, l2_rel);
    return MG_OK;
}

int mg_residual_norms_static(mg_tree *t, double *d_norms) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!d_norms) return MG_ERR_ARG;
    if (t->nleafblk > static_partial_blocks())
        return fail(t, MG_ERR_ARG, "%lld leaf blocks exceed the %d of the fixed reduction scratch",
                    (long long)t->nleafblk, static_partial_blocks());
    double *part = nullptr;
    if (static_partials(&part)) return fail(t, MG_ERR_DEVICE, "hipGetSymbolAddress of the reduction scratch failed");
    // the kernels of mg_residual_norm; every partial is written before it is read
    Driver<double> D = d64(t);
    if (t->T.refined) D.sync();
    D.L.partials = part;
    D.L.dom_norms = d_norms;
    D.L.host_norms = nullptr;
    launch_norm64(D.L, t->P64, (int)t->nleafblk, var(t), nullptr, nullptr);
    launch_reduce_norms(D.L);
    return check_launch(t);
}

int mg_residual_norm(mg_tree *t, double *max_rel, double *l2_rel) {
    int rc = require_bound(t);
    if (rc) return rc;
    std::vector<double> n;
    if ((rc = run_seq(t, G_NORM, [&] { enq_residual(t, false, true); }))) return rc;
    if ((rc = read_norms(t, &n))) return rc;
    return worst(t, n, max_rel, l2_rel);
}

int mg_solve(mg_tree *t, double rel_tol, int max_cycles, int use_fmg_first, int *cycles_done) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (max_cycles < 0 || !(rel_tol >= 0)) return MG_ERR_ARG;
    t->stat_res.clear();
    t->stat_sec.clear();
    auto t0 = std::chrono::steady_clock::now();
    auto record = [&](double r) {
        t->stat_res.push_back(r);
        t->stat_sec.push_back(std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    };
    int cycles = 0;
    double rel = INFINITY;
    std::vector<double> n;
    // Each step queues one captured sequence: the cycle followed by the residual norms
    // (copied to the host), then the host reads the norms and decides.
    const uint64_t all = all_mask(t);
    const int top = t->T.nlev - 1;
    if (!mixed(t)) {
        if (use_fmg_first && max_cycles > 0) {
            rc = run_seq(t, G_FMG_NORM, [&] {
                d64(t).fmg();
                enq_residual(t, false, true, true);
            });
            cycles++;
        } else {
            rc = run_seq(t, G_NORM, [&] { enq_residual(t, false, true); });
        }
        if (rc) return rc;
        // Cycles whose residual cannot reach rel_tol run without the norm: before each
        // check, the cycles that could not reach it even at twice the fastest reduction
        // per cycle seen so far (in log terms) run unchecked.  The cycles run and the
        // iterate are those of a check after every cycle: on refined trees an unchecked
        // cycle still makes the norm's state updates (parents = mean of the children,
        // coarse-fine ghosts), only the residual and its reduction are left out.
        double prev_rel = 0.0, rho = 1.0;
        int prev_cycles = 0;
        for (;;) {
            if ((rc = read_norms(t, &n))) return rc;
            rc = worst(t, n, &rel, nullptr);
            record(rel);
            if (rc) break;
            if (cycles > prev_cycles && prev_rel > 0.0 && rel > 0.0)
                rho = std::min(rho, std::pow(rel / prev_rel, 1.0 / (cycles - prev_cycles)));
            if (rel <= rel_tol || cycles >= max_cycles) break;
            int skip = 0;
            if (rho > 0.0 && rho < 1.0 && rel_tol > 0.0) {
                const double need = std::log(rel_tol / rel) / std::log(rho * rho);
                if (need > 1.0 && need < 1e6) skip = std::min((int)std::ceil(need) - 1, max_cycles - cycles - 1);
            }
            prev_rel = rel;
            prev_cycles = cycles;
            for (int c = 0; c < skip; c++) {
                if (t->T.refined) {
                    rc = run_seq(t, G_V_SYNC, [&] {
                        Driver<double> D = d64(t);
                        D.vcycle(top, all);
                        D.sync(true);
                    });
                } else {
                    rc = run_seq(t, G_V, [&] { d64(t).vcycle(top, all); });
                }
                if (rc) return rc;
                cycles++;
            }
            if ((rc = run_seq(t, G_V_NORM, [&] {
                     d64(t).vcycle(top, all);
                     enq_residual(t, false, true, true);
                 })))
                return rc;
            cycles++;
        }
    } else if (t->prm.krylov > 0) {
        if ((rc = solve_fgmres(t, rel_tol, max_cycles, use_fmg_first != 0, &cycles, &rel, record))) {
            if (cycles_done) *cycles_done = cycles;
            return rc;
        }
    } else {
        if ((rc = run_seq(t, G_NORM_R32, [&] { enq_residual(t, true, true); }))) return rc;
        // rho: the largest residual reduction per V-cycle seen in the plain steps so far.
        // A step runs fewer than ir_vcycles V-cycles when, at that rate and with a margin
        // of a quarter cycle, fewer reach rel_tol (typically the last step).
        double prev = INFINITY, rho = 0.0;
        int prev_nv = 0;
        for (;;) {
            if ((rc = read_norms(t, &n))) return rc;
            rc = worst(t, n, &rel, nullptr);
            record(rel);
            if (rc) break;
            if (prev_nv > 0 && rel > 0.0 && prev > 0.0 && std::isfinite(prev))
                rho = std::max(rho, std::pow(rel / prev, 1.0 / prev_nv));
            if (rel <= rel_tol || cycles >= max_cycles) break;
            const bool f = cycles == 0 && use_fmg_first && t->prm.ir_first_fmg;
            int nv = std::max(1, t->prm.ir_vcycles);
            if (!f && rho > 0.0 && rho < 1.0 && rel_tol > 0.0) {
                const double need = std::log(rel_tol / rel) / std::log(rho);
                const int k = (int)std::ceil(need + 0.25);
                if (k >= 1 && k < nv && k <= kIrFewer) nv = k;
            }
            const int kind = f ? G_IRFMG_NORM : nv == std::max(1, t->prm.ir_vcycles) ? G_IRV_NORM : G_IRV_FEWER + nv - 1;
            if ((rc = run_seq(t, kind, [&] {
                     ir_enqueue(t, f, true, f ? 0 : nv);
                     enq_add_residual(t, true, true);
                 })))
                return rc;
            prev = rel;
            prev_nv = f ? 0 : nv;
            cycles++;
        }
    }
    if (cycles_done) *cycles_done = cycles;
    if (rc) return rc;
    if ((rc = check_launch(t))) return rc;
    return rel <= rel_tol ? MG_OK : MG_ERR_NOT_CONVERGED;
}

int mg_solve_stats(const mg_tree *t, int max_records, double *rel, double *sec, int *n) {
    if (!t || !n || max_records < 0) return MG_ERR_ARG;
    int m = std::min<int>(max_records, (int)t->stat_res.size());
    for (int i = 0; i < m; i++) {
        if (rel) rel[i] = t->stat_res[i];
        if (sec) sec[i] = t->stat_sec[i];
    }
    *n = (int)t->stat_res.size();
    return MG_OK;
}

int mg_face_gradient(mg_tree *t, const double *leaf_phi, const double *leaf_lambda, double *out, int on_device) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_phi || !leaf_lambda || !out) return MG_ERR_ARG;
    if (t->T.refined) return fail(t, MG_ERR_ARG, "face gradient needs a tree without refinement");
    if (t->prm.axisymmetric) return fail(t, MG_ERR_ARG, "face gradient is Cartesian only (axisymmetric tree)");
    if (!var(t)) return fail(t, MG_ERR_STATE, "tree was created with variable_eps = 0");
    const double *phi = stage_in(t, leaf_phi, on_device, t->d_stage, &rc);
    if (rc) return rc;
    Driver<double> D = d64(t);
    K<double>::scatter(D.L, t->P64.v, phi, (int)t->nleafblk);
    for (int l = t->T.nt; l < t->T.nlev; l++) D.ghost_level(l, all_mask(t));
    const double *lam = stage_in(t, leaf_lambda, on_device, t->d_stage2, &rc);
    if (rc) return rc;
    // lambda is held in the v_old field (with homogeneous ghost values)
    Plane<double> Q = t->P64;
    Q.v = t->P64.vold;
    Q.vg = t->P64.voldg;
    Launch L0 = launch(t, true);
    K<double>::scatter(L0, Q.v, lam, (int)t->nleafblk);
    for (int l = t->T.nt; l < t->T.nlev; l++)
        K<double>::ghost(L0, Q, lvb0(t, l), lvnb(t, l), nullptr, 0, all_mask(t), false, false);
    double *dst = on_device ? out : t->d_stage;
    launch_face_gradient(D.L, t->P64, Q.v, Q.vg, dst, (int)t->nleafblk);
    if ((rc = check_launch(t))) return rc;
    if (!on_device) {
        HIP_OR_FAIL(t, hipMemcpyAsync(out, dst, (size_t)t->T.nleaf_cells * 8, hipMemcpyDeviceToHost, t->stream));
        HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    }
    return MG_OK;
}

// Elliptic divergence cleaning (Sec. 4.1): shared argument checks.
static int divb_check(mg_tree *t, const double *leaf_B) {
    int rc = require_bound(t);
    if (rc) return rc;
    if (!leaf_B) return MG_ERR_ARG;
    if (t->T.refined) return fail(t, MG_ERR_ARG, "divergence cleaning needs a tree without refinement");
    if (var(t) || t->prm.helmholtz_lambda != 0.0 || t->prm.axisymmetric)
        return fail(t, MG_ERR_ARG, "divergence cleaning needs the plain Cartesian Laplacian (eps = 1, lambda = 0)");
    return MG_OK;
}

int mg_divb_rhs(mg_tree *t, const double *leaf_B, int order, int on_device) {
    int rc = divb_check(t, leaf_B);
    if (rc) return rc;
    if (order != 2 && order != 4) return fail(t, MG_ERR_ARG, "order must be 2 or 4");
    const int64_t n = t->T.nleaf_cells;
    const Launch L = launch(t, false);
    for (int d = 0; d < t->T.dim; d++) {
        // a host component goes through the staging buffer (stream order protects it)
        const double *src = stage_in(t, leaf_B + d * n, on_device, t->d_stage, &rc);
        if (rc) return rc;
        launch_divb(L, src, t->d_stage2, d, d > 0, order, n);
    }
    K<double>::scatter(L, t->P64.f, t->d_stage2, (int)t->nleafblk);
    t->folded = false;
    if ((rc = check_launch(t))) return rc;
    if (!on_device) HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));   // the host buffer may be reused
    return MG_OK;
}

int mg_divb_project(mg_tree *t, double *leaf_B, double *leaf_e, int on_device) {
    int rc = divb_check(t, leaf_B);
    if (rc) return rc;
    const int64_t n = t->T.nleaf_cells;
    const Launch L = launch(t, t->homog);
    double *e = nullptr;
    if (leaf_e) {
        e = on_device ? leaf_e : t->d_stage2;
        if (!on_device)
            HIP_OR_FAIL(t, hipMemcpyAsync(e, leaf_e, (size_t)n * 8, hipMemcpyHostToDevice, t->stream));
    }
    for (int d = 0; d < t->T.dim; d++) {
        double *Bd = on_device ? leaf_B + d * n : t->d_stage;
        if (!on_device)
            HIP_OR_FAIL(t, hipMemcpyAsync(Bd, leaf_B + d * n, (size_t)n * 8, hipMemcpyHostToDevice, t->stream));
        launch_divb_project(L, t->P64, Bd, e, d, n);
        if (!on_device)
            HIP_OR_FAIL(t, hipMemcpyAsync(leaf_B + d * n, Bd, (size_t)n * 8, hipMemcpyDeviceToHost, t->stream));
    }
    if (leaf_e && !on_device)
        HIP_OR_FAIL(t, hipMemcpyAsync(leaf_e, e, (size_t)n * 8, hipMemcpyDeviceToHost, t->stream));
    if ((rc = check_launch(t))) return rc;
    if (!on_device) HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    return MG_OK;
}

// Checks and per-domain geometry of the free-space boundaries (mg_freespace_bc,
// mg_freespace_guess).
static int fs_setup(mg_tree *t, int coarsen, std::vector<FsDom> &fd, int64_t &qtot, int64_t &ptot, int64_t &btot,
                    int &max_pts) {
    int rc = require_bound(t);
    if (rc) return rc;
    const HostTree &T = t->T;
    if (T.dim != 3) return fail(t, MG_ERR_ARG, "free-space boundaries are three-dimensional");
    if (T.refined) return fail(t, MG_ERR_ARG, "free-space boundaries need a tree without refinement");
    if (var(t) || t->prm.helmholtz_lambda != 0.0 || t->prm.axisymmetric)
        return fail(t, MG_ERR_ARG, "free-space boundaries need the plain Laplacian (eps = 1, lambda = 0)");
    if (coarsen < 1 || (1 << coarsen) > T.bs)
        return fail(t, MG_ERR_ARG, "coarsen must satisfy 1 <= coarsen and 2^coarsen <= block size");
    const int c = 1 << coarsen;
    fd.assign(T.ndom, FsDom{});
    qtot = ptot = btot = 0;
    max_pts = 0;
    for (int i = 0; i < T.ndom; i++) {
        const mg_domain &d = T.doms[i].d;
        for (int f = 0; f < 6; f++)
            if (d.bc.kind[f] != MG_BC_DIRICHLET || d.bc.value[f] != 0.0)
                return fail(t, MG_ERR_ARG, "free-space boundaries need homogeneous Dirichlet faces");
        FsDom &g = fd[i];
        std::memset(&g, 0, sizeof g);
        for (int a = 0; a < 3; a++) {
            g.lo[a] = d.lo[a];
            g.hi[a] = d.hi[a];
            g.n[a] = d.base_cells[a];
            g.nc[a] = d.base_cells[a] / c;
            g.h[a] = (d.hi[a] - d.lo[a]) / d.base_cells[a];
            g.hc[a] = g.h[a] * c;
        }
        if (g.nc[0] > 2048) return fail(t, MG_ERR_ARG, "more than 2048 coarse cells along x");
        g.qoff = qtot;
        g.poff = ptot;
        g.boff = btot;
        int64_t pp = 0, bb = 0;
        for (int f = 0; f < 6; f++) {
            const int a = f / 2, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
            g.pofs[f] = pp;
            g.bofs[f] = bb;
            pp += (int64_t)(g.nc[t1] + 2) * (g.nc[t2] + 2);
            bb += (int64_t)g.n[t1] * g.n[t2];
        }
        g.npts = (int32_t)pp;
        max_pts = std::max(max_pts, g.npts);
        qtot += (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
        ptot += pp;
        btot += bb;
    }
    return MG_OK;
}

int mg_freespace_bc(mg_tree *t, int coarsen, double *bvals, int on_device) {
    std::vector<FsDom> fd;
    int64_t qtot, ptot, btot;
    int max_pts;
    int rc = fs_setup(t, coarsen, fd, qtot, ptot, btot, max_pts);
    if (rc) return rc;
    const HostTree &T = t->T;
    const int c = 1 << coarsen;
    // scratch in the two leaf-sized staging buffers: charges and the domain table in the
    // first; planes, staged boundary values and the slices' partial sums in the second
    const int64_t n = T.nleaf_cells;
    const int64_t fd_words = ((int64_t)sizeof(FsDom) * T.ndom + 7) / 8;
    // (the staging room for host output is always set aside, so that the slice count,
    // and with it the summation order, does not depend on where the values go)
    const int64_t bstage = btot;
    const int64_t room = n - ptot - bstage;
    if (qtot + fd_words > n || room < ptot) return fail(t, MG_ERR_ARG, "grids too small for the free-space scratch");
    const int wgs = (int)((max_pts + 255) / 256) * T.ndom;
    int slices = std::max(1, (4096 + wgs - 1) / wgs);   // about 4096 workgroups in all
    slices = (int)std::min<int64_t>(std::min(slices, 64), room / ptot);
    double *q = t->d_stage;
    FsDom *dfd = reinterpret_cast<FsDom *>(t->d_stage + qtot);
    double *pl = t->d_stage2, *bst = t->d_stage2 + ptot, *partial = t->d_stage2 + ptot + bstage;
    HIP_OR_FAIL(t, hipMemcpyAsync(dfd, fd.data(), sizeof(FsDom) * T.ndom, hipMemcpyHostToDevice, t->stream));
    double *bv = bvals ? (on_device ? bvals : bst) : nullptr;
    launch_freespace(launch(t, false), t->P64.f, dfd, T.ndom, max_pts, ptot, c, slices, q, partial, pl, bv,
                     (int)t->nleafblk);
    if ((rc = check_launch(t))) return rc;
    t->folded = true;
    if (bvals && !on_device)
        HIP_OR_FAIL(t, hipMemcpyAsync(bvals, bst, (size_t)btot * 8, hipMemcpyDeviceToHost, t->stream));
    HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));   // the domain table lives on this stack
    return MG_OK;
}

int mg_freespace_guess(mg_tree *t, int coarsen) {
    std::vector<FsDom> fd;
    int64_t qtot, ptot, btot;
    int max_pts;
    int rc = fs_setup(t, coarsen, fd, qtot, ptot, btot, max_pts);
    if (rc) return rc;
    if (t->folded)
        return fail(t, MG_ERR_STATE, "the far-field guess needs the plain right-hand side: call it before the "
                                     "boundary values are folded into f (or set f again)");
    const HostTree &T = t->T;
    const int64_t n = T.nleaf_cells;
    const int64_t fd_words = ((int64_t)sizeof(FsDom) * T.ndom + 7) / 8;
    if (qtot + fd_words + 5 * T.ndom > n) return fail(t, MG_ERR_ARG, "grids too small for the free-space scratch");
    double *q = t->d_stage;
    FsDom *dfd = reinterpret_cast<FsDom *>(t->d_stage + qtot);
    double *mom = t->d_stage + qtot + fd_words;
    HIP_OR_FAIL(t, hipMemcpyAsync(dfd, fd.data(), sizeof(FsDom) * T.ndom, hipMemcpyHostToDevice, t->stream));
    launch_freespace_guess(launch(t, false), t->P64.f, dfd, T.ndom, 1 << coarsen, q, mom, t->d_stage2,
                           (int)t->nleafblk, n);
    if ((rc = check_launch(t))) return rc;
    if ((rc = mg_set_phi(t, t->d_stage2, 1))) return rc;
    HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));   // the domain table lives on this stack
    return MG_OK;
}

int mg_freespace_values(const mg_tree *t, int64_t *n_values) {
    if (!t || !n_values) return MG_ERR_ARG;
    int64_t b = 0;
    for (int i = 0; i < t->T.ndom; i++) {
        const int32_t *m = t->T.doms[i].d.base_cells;
        b += 2 * ((int64_t)m[0] * m[1] + (int64_t)m[1] * m[2] + (int64_t)m[0] * m[2]);
    }
    *n_values = t->T.dim == 3 ? b : 0;
    return MG_OK;
}

int mg_profile_enable(mg_tree *t, int on) {
    if (!t) return MG_ERR_ARG;
    t->prof = on != 0;
    t->ev_used = 0;
    t->prof_launches = 0;
    t->prof_ms = 0.0;
    return MG_OK;
}

int mg_profile_read(mg_tree *t, int64_t *launches, double *total_ms, double *bytes_per_launch) {
    int rc = require_bound(t);
    if (rc) return rc;
    HIP_OR_FAIL(t, hipStreamSynchronize(t->stream));
    for (size_t i = 0; i + 1 < t->ev_used; i += 2) {
        float ms = 0.f;
        HIP_OR_FAIL(t, hipEventElapsedTime(&ms, t->ev[i], t->ev[i + 1]));
        t->prof_ms += ms;
        t->prof_launches++;
    }
    t->ev_used = 0;
    if (launches) *launches = t->prof_launches;
    if (total_ms) *total_ms = t->prof_ms;
    if (bytes_per_launch) {
        // one colour of one sweep on the finest level: read the other colour of v and
        // this colour of f, write this colour of v (plus eps of both colours)
        const int top = t->T.nlev - 1;
        double cellsN = (double)lvnb(t, top) * (double)t->nc;
        double elem = mixed(t) ? 4.0 : 8.0;   // precision of the cycles
        *bytes_per_launch = cellsN * (1.5 * elem + (var(t) ? elem : 0.0));
    }
    return MG_OK;
}

const char *mg_strerror(int s) {
    switch (s) {
        case MG_OK: return "ok";
        case MG_ERR_ARG: return "invalid argument";
        case MG_ERR_NOT_BALANCED: return "tree not 2:1 balanced";
        case MG_ERR_DEVICE: return "device error";
        case MG_ERR_NOT_CONVERGED: return "not converged";
        case MG_ERR_OOM: return "device store too small";
        case MG_ERR_STATE: return "invalid state";
        case MG_ERR_NAN: return "residual is not finite";
        default: return "unknown status";
    }
}

const char *mg_last_error(const mg_tree *t) { return t ? t->err.c_str() : "null tree"; }

}  // extern "C"
