// Host-side construction of the block tree(s): the paper's added coarse levels
// (Sec. 2.5, table coarse-grid-example), refinement by a predicate closed under 2:1
// balance, Morton ordering, and the index tables the kernels use.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "mg_internal.hpp"

namespace mgx {
namespace {

uint64_t morton_code(const int *b, int dim) {
    uint64_t code = 0;
    for (int bit = 0; bit < 21; bit++)
        for (int a = 0; a < dim; a++) code |= (uint64_t)((b[a] >> bit) & 1) << (bit * dim + a);
    return code;
}

struct Builder {
    int dim = 0, bs = 0, nt = 0;
    std::vector<HDomain> *doms = nullptr;
    std::vector<HBlock> B;
    std::unordered_map<uint64_t, int> at;
    std::vector<std::vector<int>> by_level;

    static uint64_t key(int d, int l, const int *b) {
        return ((uint64_t)d << 58) | ((uint64_t)l << 52) | ((uint64_t)b[0] << 34) |
               ((uint64_t)b[1] << 17) | (uint64_t)b[2];
    }
    int nblk(int d, int l, int a) const {
        if (a >= dim) return 1;
        return (*doms)[d].nblk_low[a] << (l - nt);
    }
    int find(int d, int l, const int *b) const {
        auto it = at.find(key(d, l, b));
        return it == at.end() ? -1 : it->second;
    }
    int add(int d, int l, const int *b, int parent) {
        HBlock h{};
        h.dom = d; h.lev = l;
        for (int a = 0; a < 3; a++) h.bc[a] = b[a];
        h.parent = parent;
        for (int c = 0; c < 8; c++) h.child[c] = -1;
        int id = (int)B.size();
        B.push_back(h);
        at[key(d, l, b)] = id;
        if ((int)by_level.size() <= l) by_level.resize(l + 1);
        by_level[l].push_back(id);
        return id;
    }
    // Maps block coordinates across periodic faces; false if outside a physical face.
    bool wrap(int d, int l, int *b) const {
        for (int a = 0; a < dim; a++) {
            int n = nblk(d, l, a);
            if (b[a] < 0 || b[a] >= n) {
                int face = 2 * a + (b[a] >= n);
                if ((*doms)[d].d.bc.kind[face] != MG_BC_PERIODIC) return false;
                b[a] = (b[a] % n + n) % n;
            }
        }
        return true;
    }
    // Creates the block at (d, l, b) by splitting the finest existing ancestor until it
    // exists.
    void make_exist(int d, int l, const int *b) {
        while (find(d, l, b) < 0) {
            int m = l - 1, q[3] = {b[0] / 2, b[1] / 2, b[2] / 2};
            while (find(d, m, q) < 0) {
                m--;
                for (int a = 0; a < 3; a++) q[a] /= 2;
            }
            split(find(d, m, q));
        }
    }
    // Splits a block after all of its face/edge/corner neighbours on its own level
    // exist; then no child can touch a block more than one level coarser.
    void split(int id) {
        if (B[id].has_children) return;
        int d = B[id].dom, l = B[id].lev;
        int b[3] = {B[id].bc[0], B[id].bc[1], B[id].bc[2]};
        int r = dim == 3 ? 1 : 0;
        for (int oz = -r; oz <= r; oz++)
            for (int oy = -1; oy <= 1; oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    if (ox == 0 && oy == 0 && oz == 0) continue;
                    int q[3] = {b[0] + ox, b[1] + oy, b[2] + oz};
                    if (wrap(d, l, q)) make_exist(d, l, q);
                }
        for (int c = 0; c < (1 << dim); c++) {
            int q[3] = {2 * b[0] + (c & 1), 2 * b[1] + ((c >> 1) & 1), dim == 3 ? 2 * b[2] + (c >> 2) : 0};
            int cid = add(d, l + 1, q, id);
            B[id].child[c] = cid;
        }
        B[id].has_children = true;
    }
};

}  // namespace

std::string build_tree(HostTree &T, const mg_domain *doms, int ndom, int bs, int max_refine,
                       mg_refine_fn refine, void *ud) {
    if (!doms || ndom < 1 || ndom > MAXDOM) return "n_domains must be in [1, 64]";
    if (bs != 4 && bs != 8 && bs != 16) return "block_size must be 4, 8 or 16";
    if (max_refine < 0) return "max_refine_levels must be >= 0";
    int dim = doms[0].dim;
    if (dim != 2 && dim != 3) return "dim must be 2 or 3";
    T = HostTree();
    T.dim = dim; T.bs = bs; T.ndom = ndom;
    T.nt = 0;
    for (int b = bs; b > 1; b >>= 1) T.nt++;
    int nt = T.nt;
    for (int i = 0; i < ndom; i++) {
        const mg_domain &D = doms[i];
        if (D.dim != dim) return "all domains must have the same dim";
        for (int a = 0; a < dim; a++) {
            if (D.base_cells[a] <= 0 || D.base_cells[a] % bs) return "base_cells must be positive multiples of block_size";
            if (!(D.hi[a] > D.lo[a])) return "hi must exceed lo";
        }
        for (int f = 0; f < 2 * dim; f++) {
            int k = D.bc.kind[f];
            if (k < MG_BC_DIRICHLET || k > MG_BC_PERIODIC) return "invalid boundary kind";
            if ((k == MG_BC_PERIODIC) != (D.bc.kind[f ^ 1] == MG_BC_PERIODIC)) return "periodic faces must come in pairs";
        }
        HDomain hd{};
        hd.d = D;
        // Coarser block levels: halve the base grid while each halved size still tiles
        // by whole blocks.
        int nc[3] = {D.base_cells[0], dim > 1 ? D.base_cells[1] : 1, dim > 2 ? D.base_cells[2] : 1};
        int levels = 1;
        for (;;) {
            bool ok = true;
            for (int a = 0; a < dim; a++)
                if (nc[a] % 2 || (nc[a] / 2) % bs) ok = false;
            if (!ok) break;
            for (int a = 0; a < dim; a++) nc[a] /= 2;
            levels++;
        }
        for (int a = 0; a < 3; a++) hd.nblk_low[a] = a < dim ? nc[a] / bs : 1;
        hd.base = nt + levels - 1;
        hd.top = hd.base;
        if (hd.base + max_refine >= MAXLEV) return "too many levels";
        for (int a = 0; a < dim; a++)
            if ((int64_t)hd.nblk_low[a] << (hd.base + max_refine - nt) >= (1 << 17)) return "grid too large";
        T.doms.push_back(hd);
    }

    // Small coarse levels go below the block levels: while every domain's lowest
    // block level has at most kTailBig cells and lies below its base grid, that level
    // becomes a uniform grid of the single-workgroup coarse solver.
    for (;;) {
        bool ok = true;
        for (const HDomain &hd : T.doms) {
            int64_t c = 1;
            for (int a = 0; a < dim; a++) c *= (int64_t)hd.nblk_low[a] * bs;
            if (c > kTailBig || hd.base <= nt) ok = false;
        }
        if (!ok) break;
        nt++;
        for (HDomain &hd : T.doms)
            for (int a = 0; a < dim; a++) hd.nblk_low[a] *= 2;
    }
    T.nt = nt;

    Builder bld;
    bld.dim = dim; bld.bs = bs; bld.nt = nt; bld.doms = &T.doms;
    {
        size_t est = 0;   // blocks of the levels up to the base grids
        for (const HDomain &hd : T.doms) {
            size_t per = 1;
            for (int a = 0; a < dim; a++) per *= (size_t)hd.nblk_low[a];
            for (int l = nt; l <= hd.base; l++) est += per << (dim * (l - nt));
        }
        bld.at.reserve(est + est / 2);
        bld.B.reserve(est + est / 2);
    }
    // Every block of the levels up to the base grid exists.
    for (int i = 0; i < ndom; i++) {
        for (int l = nt; l <= T.doms[i].base; l++) {
            int n[3] = {bld.nblk(i, l, 0), bld.nblk(i, l, 1), bld.nblk(i, l, 2)};
            int b[3];
            for (b[2] = 0; b[2] < n[2]; b[2]++)
                for (b[1] = 0; b[1] < n[1]; b[1]++)
                    for (b[0] = 0; b[0] < n[0]; b[0]++) {
                        int par = -1;
                        if (l > nt) {
                            int q[3] = {b[0] / 2, b[1] / 2, dim == 3 ? b[2] / 2 : 0};
                            par = bld.find(i, l - 1, q);
                            bld.B[par].has_children = true;
                            int c = (b[0] & 1) | ((b[1] & 1) << 1) | (dim == 3 ? (b[2] & 1) << 2 : 0);
                            bld.B[par].child[c] = (int)bld.B.size();
                        }
                        bld.add(i, l, b, par);
                    }
        }
    }
    // Refinement closure: visit untested leaves below each domain's top allowed level
    // until no predicate fires any more.
    if (refine && max_refine > 0) {
        bool changed = true;
        while (changed) {
            changed = false;
            for (size_t l = 0; l < bld.by_level.size(); l++) {
                for (size_t q = 0; q < bld.by_level[l].size(); q++) {
                    int id = bld.by_level[l][q];
                    HBlock &hb = bld.B[id];
                    int rel = hb.lev - T.doms[hb.dom].base;
                    if (hb.has_children || hb.tested || rel < 0 || rel >= max_refine) continue;
                    hb.tested = true;
                    int32_t o[3] = {hb.bc[0] * bs, hb.bc[1] * bs, dim == 3 ? hb.bc[2] * bs : 0};
                    if (refine(ud, hb.dom, rel, o, bs)) {
                        bld.split(id);
                        changed = true;
                    }
                }
            }
        }
    }
    for (const HBlock &hb : bld.B) {
        T.doms[hb.dom].top = std::max(T.doms[hb.dom].top, hb.lev);
        if (hb.lev > T.doms[hb.dom].base) T.refined = true;
    }
    T.nlev = 0;
    for (auto &hd : T.doms) {
        hd.nblev = hd.top - nt + 1;
        T.nlev = std::max(T.nlev, hd.top + 1);
    }

    // Final numbering: level, domain, Morton order.
    std::vector<int> newid(bld.B.size(), -1);
    std::vector<std::vector<std::vector<int>>> groups(T.nlev, std::vector<std::vector<int>>(ndom));
    for (int id = 0; id < (int)bld.B.size(); id++) groups[bld.B[id].lev][bld.B[id].dom].push_back(id);
    std::vector<uint64_t> mcode(bld.B.size());
    for (size_t id = 0; id < bld.B.size(); id++) mcode[id] = morton_code(bld.B[id].bc, dim);
    for (int l = 0; l < T.nlev; l++)
        for (int i = 0; i < ndom; i++)
            std::sort(groups[l][i].begin(), groups[l][i].end(), [&](int a, int b) { return mcode[a] < mcode[b]; });
    T.lev_first.assign(T.nlev + 1, 0);
    int next = 0;
    for (int l = 0; l < T.nlev; l++) {
        T.lev_first[l] = next;
        for (int i = 0; i < ndom; i++)
            for (int id : groups[l][i]) newid[id] = next++;
    }
    T.lev_first[T.nlev] = next;
    int nb = next;
    // block indices travel as 8 b + face in the coarse-fine face lists
    if (nb >= (1 << 28)) return "too many blocks (at most 2^28)";
    T.org.assign(3 * (size_t)nb, 0);
    T.nbr.assign(6 * (size_t)nb, -1);
    T.cf.assign(6 * (size_t)nb, -1);
    T.parent.assign(nb, -1);
    T.dom.assign(nb, 0);
    T.lev.assign(nb, 0);
    T.parents_of_level.assign(T.nlev, {});
    T.cf_of_level.assign(T.nlev, {});
    for (int id = 0; id < (int)bld.B.size(); id++) {
        const HBlock &hb = bld.B[id];
        int n = newid[id];
        for (int a = 0; a < 3; a++) T.org[3 * n + a] = a < dim ? hb.bc[a] * bs : 0;
        T.dom[n] = hb.dom;
        T.lev[n] = hb.lev;
        T.parent[n] = hb.parent >= 0 ? newid[hb.parent] : -1;
        bool has_cf = false;
        for (int f = 0; f < 2 * dim; f++) {
            int a = f / 2;
            int q[3] = {hb.bc[0], hb.bc[1], hb.bc[2]};
            q[a] += (f & 1) ? 1 : -1;
            if (!bld.wrap(hb.dom, hb.lev, q)) {
                T.nbr[6 * n + f] = -1;
                continue;
            }
            int s = bld.find(hb.dom, hb.lev, q);
            if (s >= 0) {
                T.nbr[6 * n + f] = newid[s];
                continue;
            }
            int c[3] = {q[0] / 2, q[1] / 2, q[2] / 2};
            int cb = bld.find(hb.dom, hb.lev - 1, c);
            if (cb < 0) return "internal error: unbalanced tree";
            T.nbr[6 * n + f] = -2;
            T.cf[6 * n + f] = newid[cb];
            has_cf = true;
        }
        if (hb.has_children) T.parents_of_level[hb.lev].push_back(n);
        if (has_cf) T.cf_of_level[hb.lev].push_back(n);
    }
    for (auto &v : T.parents_of_level) std::sort(v.begin(), v.end());
    for (auto &v : T.cf_of_level) std::sort(v.begin(), v.end());
    // Leaf order: domain, level, Morton.
    T.leaf_first.assign(ndom + 1, 0);
    T.dom_leaf_cells.assign(ndom, 0);
    int64_t cells_per_block = 1;
    for (int a = 0; a < dim; a++) cells_per_block *= bs;
    for (int i = 0; i < ndom; i++) {
        T.leaf_first[i] = (int32_t)T.leaf_blk.size();
        for (int l = 0; l < T.nlev; l++)
            for (int id : groups[l][i])
                if (!bld.B[id].has_children) T.leaf_blk.push_back(newid[id]);
        T.dom_leaf_cells[i] = (int64_t)(T.leaf_blk.size() - T.leaf_first[i]) * cells_per_block;
    }
    T.leaf_first[ndom] = (int32_t)T.leaf_blk.size();
    T.nleaf_cells = (int64_t)T.leaf_blk.size() * cells_per_block;

    // Geometry per domain and level; tail grid offsets.
    T.h.assign((size_t)ndom * MAXLEV * 3, 1.0);
    T.ncell.assign((size_t)ndom * MAXLEV * 3, 1);
    T.tail_off.assign((size_t)ndom * MAXLEV, 0);
    int64_t off = 0;
    for (int i = 0; i < ndom; i++) {
        const HDomain &hd = T.doms[i];
        for (int l = 0; l < T.nlev; l++) {
            for (int a = 0; a < dim; a++) {
                int64_t n;
                if (l >= nt) n = (int64_t)hd.nblk_low[a] * bs << (l - nt);
                else n = ((int64_t)hd.nblk_low[a] * bs) >> (nt - l);
                T.ncell[((size_t)i * MAXLEV + l) * 3 + a] = (int32_t)n;
                T.h[((size_t)i * MAXLEV + l) * 3 + a] = (hd.d.hi[a] - hd.d.lo[a]) / (double)n;
            }
            if (l < nt) {
                int64_t p = 1;
                for (int a = 0; a < dim; a++) p *= T.ncell[((size_t)i * MAXLEV + l) * 3 + a] + 2;
                T.tail_off[(size_t)i * MAXLEV + l] = off;
                off += p;
            }
        }
    }
    T.tail_cells = off;
    // Large tail levels (more than kTailBig cells, all axes even so a sweep can push
    // its ghosts) run as multi-workgroup launches; the rest in one workgroup.
    T.tail_top.assign(ndom, nt - 1);
    for (int i = 0; i < ndom; i++) {
        int l = nt - 1;
        while (l > 0) {
            int64_t c = 1;
            bool even = true;
            for (int a = 0; a < dim; a++) {
                int n = T.ncell[((size_t)i * MAXLEV + l) * 3 + a];
                c *= n;
                even = even && n % 2 == 0;
            }
            if (c <= kTailBig || !even) break;
            l--;
        }
        T.tail_top[i] = l;
        int64_t c = 1;
        for (int a = 0; a < dim; a++) c *= T.ncell[((size_t)i * MAXLEV + l) * 3 + a];
        if (c >= (1 << 22)) return "coarse grid below the block levels too large (odd block counts)";
        if (l > 14) return "too many coarse grid levels below the block levels";
    }
    return "";
}

}  // namespace mgx
