// Host check of the guard-cell source indices the stage and fill kernels
// use (same_cell, coarse_cell / coarse_child, fine_block / fine_cell in
// csrc/kernel_common.hpp) against the forest's own leaf geometry (Sec. 3.3,
// 3.5): for every leaf face, face point t and child, the source cell named by
// the indices must be, in physical space, the guard cell itself (neighbour
// of the same level, Eq. 15), the coarser cell whose child it is (Eq. 16),
// or the finer cell that is its child (Eq. 17).  The guard cell is the own
// face cell moved one cell width across the face.  Forests: random
// refinements (2:1 balanced by the forest's planner) of 2-D and 3-D root
// grids, periodic and outflow, N = 2 .. 8.  Prints one line per forest and
// "OK" at the end; exits non-zero on the first mismatch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2502_12620_amd/csrc/forest.hpp"
#include "../../paper_2502_12620_amd/csrc/kernel_common.hpp"

using namespace dgamr;

struct Box {
    double lo[3], h[3];
};

static double L_dom[3];
static bool periodic[3];

static Box cell_box(const LeafGeo &G, int cell, int N, int D)
{
    int ijk[3];
    dgk::cell_ijk(cell, N, D, ijk);
    Box b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = a < D ? G.lo[a] + ijk[a] * G.h[a] : 0.0;
        b.h[a] = a < D ? G.h[a] : 1.0;
    }
    return b;
}

static bool same_pos(double x, double y, int a)
{
    double d = x - y;
    if (periodic[a]) d -= L_dom[a] * std::round(d / L_dom[a]);
    return std::fabs(d) <= 1e-12 * L_dom[a];
}

static bool same_box(const Box &x, const Box &y, int D)
{
    for (int a = 0; a < D; ++a)
        if (!same_pos(x.lo[a], y.lo[a], a) || std::fabs(x.h[a] - y.h[a]) > 1e-12 * y.h[a]) return false;
    return true;
}

// the child ch (bit b: upper half along b) of a box
static Box child_box(const Box &b, int ch, int D)
{
    Box c = b;
    for (int a = 0; a < D; ++a) {
        c.h[a] = 0.5 * b.h[a];
        c.lo[a] = b.lo[a] + ((ch >> a) & 1) * c.h[a];
    }
    return c;
}

static int fail(const char *what, int leaf, int face, int t, int ch)
{
    std::fprintf(stderr, "MISMATCH %s: leaf %d face %d t %d child %d\n", what, leaf, face, t, ch);
    return 1;
}

static int check(Forest &f, long &counted)
{
    const int D = f.dim(), N = f.desc().n_cell, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const std::vector<LeafGeo> geo = f.geometry();
    const std::vector<FaceLink> &links = f.links();
    for (int i = 0; i < f.n(); ++i)
        for (int face = 0; face < 2 * D; ++face) {
            const int a = face / 2, side = (face & 1) ? 1 : -1;
            const FaceLink &L = links[size_t(i) * 2 * D + face];
            if (L.type == LINK_BOUNDARY) continue;
            for (int t = 0; t < nfc; ++t) {
                int ijk_t[3];
                // own cell next to the face, moved across it
                const int own = dgk::face_cell(a, side > 0 ? N - 1 : 0, t, N, D);
                Box guard = cell_box(geo[i], own, N, D);
                guard.lo[a] += side * guard.h[a];
                dgk::cell_ijk(own, N, D, ijk_t);
                if (dgk::face_t(ijk_t, a, N, D) != t) return fail("face_t", i, face, t, -1);
                if (L.type == LINK_SAME) {
                    const int c = dgk::same_cell(a, side, t, N, D);
                    if (c < 0 || c >= ncell || geo[L.nbr[0]].level != geo[i].level) return fail("same range", i, face, t, -1);
                    if (!same_box(cell_box(geo[L.nbr[0]], c, N, D), guard, D)) return fail("same", i, face, t, -1);
                    ++counted;
                } else if (L.type == LINK_COARSE) {
                    const int c = dgk::coarse_cell(a, side, t, L.off, N, D);
                    const int ch = dgk::coarse_child(a, side, t, N, D);
                    if (c < 0 || c >= ncell || ch < 0 || ch >= (1 << D) || geo[L.nbr[0]].level != geo[i].level - 1)
                        return fail("coarse range", i, face, t, ch);
                    if (!same_box(child_box(cell_box(geo[L.nbr[0]], c, N, D), ch, D), guard, D))
                        return fail("coarse", i, face, t, ch);
                    ++counted;
                } else if (L.type == LINK_FINE) {
                    const int h = dgk::fine_block(t, N, D);
                    if (h < 0 || h >= (1 << (D - 1))) return fail("fine block range", i, face, t, -1);
                    const int fl = dgk::link_nbr(L, h);
                    if (fl < 0 || fl >= f.n() || geo[fl].level != geo[i].level + 1) return fail("fine leaf", i, face, t, -1);
                    for (int ch = 0; ch < (1 << D); ++ch) {
                        const int c = dgk::fine_cell(a, side, t, ch, N, D);
                        if (c < 0 || c >= ncell) return fail("fine range", i, face, t, ch);
                        if (!same_box(cell_box(geo[fl], c, N, D), child_box(guard, ch, D), D))
                            return fail("fine", i, face, t, ch);
                        ++counted;
                    }
                } else {
                    return fail("link type", i, face, t, -1);
                }
            }
        }
    return 0;
}

int main()
{
    std::mt19937 rng(2502);
    int forests = 0;
    long counted = 0;
    for (int D = 2; D <= 3; ++D)
        for (int N = 2; N <= 8; N += 2)
            for (int bcase = 0; bcase < 2; ++bcase) {
                dgamr_forest_desc d{};
                d.dim = D;
                d.degree = 1;
                d.n_cell = N;
                for (int a = 0; a < 3; ++a) {
                    d.roots[a] = a < D ? 2 + (a == 0) : 1;
                    d.lo[a] = -1.0;
                    d.hi[a] = a < D ? -1.0 + 1.5 * d.roots[a] : 0.0;
                    d.bc[a] = bcase == 0 ? DGAMR_BC_PERIODIC : DGAMR_BC_OUTFLOW;
                    L_dom[a] = a < D ? d.hi[a] - d.lo[a] : 1.0;
                    periodic[a] = bcase == 0;
                }
                d.max_level = D == 2 ? 5 : 4;
                d.gamma = 1.4;
                std::string err;
                if (Forest::validate(d, err) != DGAMR_OK) {
                    std::fprintf(stderr, "descriptor: %s\n", err.c_str());
                    return 2;
                }
                Forest f(d);
                if (f.build_links(err) != DGAMR_OK) {
                    std::fprintf(stderr, "links: %s\n", err.c_str());
                    return 2;
                }
                for (int round = 0; round < 4; ++round) {
                    if (check(f, counted)) return 1;
                    ++forests;
                    std::vector<int8_t> flags(f.n());
                    for (auto &x : flags) x = int8_t(rng() % 3 == 0 ? 1 : (rng() % 4 == 0 ? -1 : 0));
                    std::vector<Inherit> inh;
                    if (f.plan(flags.data(), err) != DGAMR_OK || f.commit(inh, err) != DGAMR_OK) {
                        std::fprintf(stderr, "regrid: %s\n", err.c_str());
                        return 2;
                    }
                    std::printf("dim %d N %d %s round %d: %d leaves\n", D, N, bcase == 0 ? "periodic" : "outflow",
                                round, f.n());
                }
                if (check(f, counted)) return 1;
                ++forests;
            }
    std::printf("OK %d forests, %ld guard-cell sources checked\n", forests, counted);
    return 0;
}
