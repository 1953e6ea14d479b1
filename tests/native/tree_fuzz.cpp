// Randomised host-side use of the C ABI (tree construction, storage sizing, leaf layout,
// destruction; no device) for a build with AddressSanitizer on the host code: trees in
// 2D and 3D, block sizes 4, 8 and 16, forests of up to three domains, random boundary
// kinds and random refinement predicates, and the boundary-face listing.  Exits non-zero
// if a valid tree is rejected, a singular one accepted, or a listed face is out of range.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "mg.h"
static unsigned rs = 12345;
static int rnd() { rs = rs * 1103515245u + 12345u; return (rs >> 16) & 0x7fff; }
static int pred(void *ud, int, int, const int32_t *, int) {
    const int p = *(int *)ud;
    return (rnd() % 100) < p;
}
int main() {
    int n = 0, bad = 0, sing = 0;
    for (int trial = 0; trial < 300; trial++) {
        int dim = 2 + (trial & 1);
        int bsopt[3] = {4, 8, 16};
        int bs = bsopt[rnd() % 3];
        int ndom = 1 + rnd() % 3;
        std::vector<mg_domain> d(ndom);
        for (int i = 0; i < ndom; i++) {
            d[i] = mg_domain{};
            d[i].dim = dim;
            for (int a = 0; a < 3; a++) {
                int mult = 1 + rnd() % (dim == 3 ? 4 : 8);
                d[i].base_cells[a] = a < dim ? bs * mult : 1;
                d[i].lo[a] = 0; d[i].hi[a] = 1 + a;
            }
            for (int f = 0; f < 6; f++) { d[i].bc.kind[f] = f < 2 * dim ? rnd() % 2 : MG_BC_PERIODIC; d[i].bc.value[f] = 0.5; }
            if (rnd() % 3 == 0) { d[i].bc.kind[0] = d[i].bc.kind[1] = MG_BC_PERIODIC; }
        }
        mg_params p; mg_default_params(&p);
        p.variable_eps = rnd() % 2; p.precision = rnd() % 2;
        int prob = rnd() % 40;
        int maxref = rnd() % (dim == 3 ? 3 : 4);
        // a domain without a Dirichlet face that is not fully periodic is singular and
        // must be rejected (no Helmholtz term here)
        bool singular = false;
        for (int i = 0; i < ndom; i++) {
            bool dir = false, per = true;
            for (int f = 0; f < 2 * dim; f++) {
                dir = dir || d[i].bc.kind[f] == MG_BC_DIRICHLET;
                per = per && d[i].bc.kind[f] == MG_BC_PERIODIC;
            }
            singular = singular || (!dir && !per);
        }
        mg_tree *t = nullptr;
        int rc = mg_tree_create(d.data(), ndom, bs, maxref, pred, &prob, &p, &t);
        if (singular) {
            if (rc != MG_ERR_ARG || t) bad++;
            else sing++;
            continue;
        }
        if (rc) { bad++; continue; }
        size_t bytes = 0; mg_tree_storage_bytes(t, &bytes);
        int64_t nl = 0; mg_num_leaf_cells(t, &nl);
        std::vector<int32_t> lay(5 * nl);
        mg_leaf_layout(t, lay.data());
        int nlev = 0; mg_num_levels(t, &nlev);
        int64_t nbf = 0; mg_boundary_faces(t, &nbf, nullptr, nullptr);
        std::vector<int64_t> cells(nbf);
        std::vector<int32_t> faces(nbf);
        mg_boundary_faces(t, &nbf, cells.data(), faces.data());
        for (int64_t q = 0; q < nbf; q++)
            if (cells[q] < 0 || cells[q] >= nl || faces[q] < 0 || faces[q] >= 2 * dim) bad++;
        mg_tree_destroy(t);
        n++;
    }
    printf("trees %d rejected %d singular %d\n", n, bad, sing);
    return bad ? 1 : 0;
}
