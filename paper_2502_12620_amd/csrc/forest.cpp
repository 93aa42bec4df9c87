// Host-side forest topology; see forest.hpp.
#include "forest.hpp"

#include <cmath>

#include <algorithm>
#include <numeric>

namespace dgamr {

namespace {
constexpr int kMaxLevel = 12; // idx < 2048 per axis: 11 bits each in the packed key
}

void frame_matrix(int dim, int code, int Q[3][3])
{
    for (int g = 0; g < 3; ++g)
        for (int l = 0; l < 3; ++l) Q[g][l] = 0;
    if (dim == 2) {
        static const int c[4] = {1, 0, -1, 0}, sn[4] = {0, 1, 0, -1};
        Q[0][0] = c[code];
        Q[0][1] = -sn[code];
        Q[1][0] = sn[code];
        Q[1][1] = c[code];
        Q[2][2] = 1;
        return;
    }
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int n = 0;
    for (int pi = 0; pi < 6; ++pi)
        for (int sg = 0; sg < 8; ++sg) {
            int M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int l = 0; l < 3; ++l) M[perms[pi][l]][l] = ((sg >> l) & 1) ? -1 : 1;
            const int det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                            M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                            M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            if (det != 1) continue;
            if (n++ == code) {
                for (int g = 0; g < 3; ++g)
                    for (int l = 0; l < 3; ++l) Q[g][l] = M[g][l];
                return;
            }
        }
}

Forest::Forest(const dgamr_forest_desc &d) : desc_(d)
{
    for (int a = desc_.dim; a < 3; ++a) {
        desc_.roots[a] = 1;
        desc_.bc[a] = DGAMR_BC_PERIODIC;
        desc_.lo[a] = 0.0;
        desc_.hi[a] = 1.0;
    }
    int ntree = desc_.roots[0] * desc_.roots[1] * desc_.roots[2];
    leaves_.resize(ntree);
    for (int t = 0; t < ntree; ++t) leaves_[t].tree = t;
    reindex();
}

int Forest::validate(const dgamr_forest_desc &d, std::string &err)
{
    if (d.dim != 2 && d.dim != 3) { err = "dim must be 2 or 3"; return DGAMR_EINVAL; }
    if (d.degree < 0 || d.degree > 3) { err = "degree must be 0..3"; return DGAMR_EUNSUPPORTED; }
    if (d.n_cell < 2 || d.n_cell % 2) { err = "n_cell must be even and >= 2"; return DGAMR_EINVAL; }
    int nmax = d.dim == 2 ? 16 : 8;
    if (d.n_cell > nmax) { err = "n_cell above the built limit (16 in 2-D, 8 in 3-D)"; return DGAMR_EUNSUPPORTED; }
    if (d.max_level < 1 || d.max_level > kMaxLevel) { err = "max_level must be 1..12"; return DGAMR_EINVAL; }
    long ntree = 1;
    for (int a = 0; a < d.dim; ++a) {
        if (d.roots[a] < 1) { err = "roots must be >= 1"; return DGAMR_EINVAL; }
        if (!(d.hi[a] > d.lo[a])) { err = "hi must exceed lo"; return DGAMR_EINVAL; }
        if (d.bc[a] != DGAMR_BC_PERIODIC && d.bc[a] != DGAMR_BC_OUTFLOW && d.bc[a] != DGAMR_BC_DIRICHLET) {
            err = "bad bc";
            return DGAMR_EINVAL;
        }
        if ((d.bc[a] == DGAMR_BC_DIRICHLET) != (d.equation == DGAMR_EQ_DIFFUSION && d.bc[a] != DGAMR_BC_PERIODIC)) {
            err = "Dirichlet faces belong to the diffusion equation, whose non-periodic faces are Dirichlet";
            return DGAMR_EINVAL;
        }
        ntree *= d.roots[a];
    }
    if (ntree >= (1L << 24)) { err = "too many roots"; return DGAMR_EUNSUPPORTED; }
    if (!(d.gamma > 1.0)) { err = "gamma must exceed 1"; return DGAMR_EINVAL; }
    if (d.precision != DGAMR_FP64 && d.precision != DGAMR_FP32) { err = "bad precision"; return DGAMR_EINVAL; }
    if (d.hanging != DGAMR_HANG_PAPER && d.hanging != DGAMR_HANG_CONSERVATIVE) { err = "bad hanging mode"; return DGAMR_EINVAL; }
    if (d.limiter != DGAMR_LIMITER_NONE && d.limiter != DGAMR_LIMITER_POSITIVITY) { err = "bad limiter"; return DGAMR_EINVAL; }
    if (d.equation != DGAMR_EQ_EULER && d.equation != DGAMR_EQ_ADVECTION && d.equation != DGAMR_EQ_DIFFUSION) {
        err = "bad equation";
        return DGAMR_EINVAL;
    }
    if (d.equation == DGAMR_EQ_DIFFUSION) {
        if (d.limiter != DGAMR_LIMITER_NONE) { err = "the positivity limiter is for the Euler equations"; return DGAMR_EINVAL; }
        if (d.precision != DGAMR_FP64) { err = "diffusion is built in FP64 only"; return DGAMR_EUNSUPPORTED; }
        if (d.hanging != DGAMR_HANG_PAPER) { err = "diffusion takes hanging faces from guard cells only"; return DGAMR_EUNSUPPORTED; }
        if (d.degree < 1) { err = "the interior-penalty method needs degree >= 1"; return DGAMR_EUNSUPPORTED; }
        if (!(d.diffusivity > 0.0) || !std::isfinite(d.diffusivity)) { err = "diffusivity must be positive"; return DGAMR_EINVAL; }
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d.exact_a[a])) { err = "exact_a must be finite"; return DGAMR_EINVAL; }
    }
    if (d.equation == DGAMR_EQ_ADVECTION) {
        if (d.limiter != DGAMR_LIMITER_NONE) { err = "the positivity limiter is for the Euler equations"; return DGAMR_EINVAL; }
        if (d.precision != DGAMR_FP64) { err = "scalar convection is built in FP64 only"; return DGAMR_EUNSUPPORTED; }
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d.velocity[a])) { err = "velocity must be finite"; return DGAMR_EINVAL; }
    }
    return DGAMR_OK;
}

uint64_t Forest::pack(int tree, int level, const int *idx) const
{
    return (uint64_t(tree) << 40) | (uint64_t(level) << 33) | (uint64_t(idx[2]) << 22) |
           (uint64_t(idx[1]) << 11) | uint64_t(idx[0]);
}

int Forest::find(int tree, int level, const int *idx) const
{
    if (level < 1) return -1;
    auto it = index_.find(pack(tree, level, idx));
    return it == index_.end() ? -1 : it->second;
}

void Forest::reindex()
{
    index_.clear();
    index_.reserve(leaves_.size() * 2);
    for (int i = 0; i < n(); ++i) index_[pack(leaves_[i].tree, leaves_[i].level, leaves_[i].idx)] = i;
}

// root adjacent to `tree` across (axis, side), wrapping periodic axes;
// false at an outflow boundary
bool Forest::neighbour_root(int tree, int axis, int side, int &out) const
{
    int r[3] = {tree % desc_.roots[0], (tree / desc_.roots[0]) % desc_.roots[1],
                tree / (desc_.roots[0] * desc_.roots[1])};
    r[axis] += side;
    if (r[axis] < 0 || r[axis] >= desc_.roots[axis]) {
        if (desc_.bc[axis] != DGAMR_BC_PERIODIC) return false;
        r[axis] = (r[axis] + desc_.roots[axis]) % desc_.roots[axis];
    }
    out = r[0] + desc_.roots[0] * (r[1] + desc_.roots[1] * r[2]);
    return true;
}

uint64_t Forest::morton(const Key &k) const
{
    int shift = desc_.max_level - k.level;
    uint64_t code = 0;
    for (int b = 0; b < kMaxLevel; ++b)
        for (int a = 0; a < desc_.dim; ++a)
            code |= uint64_t(((k.idx[a] << shift) >> b) & 1) << (desc_.dim * b + a);
    return code;
}

void Forest::sort_keys(std::vector<Key> &v) const
{
    std::stable_sort(v.begin(), v.end(), [this](const Key &x, const Key &y) {
        if (x.tree != y.tree) return x.tree < y.tree;
        return morton(x) < morton(y);
    });
}

int Forest::set_frames(const int32_t *codes, std::string &err)
{
    const int d = desc_.dim, ntree = desc_.roots[0] * desc_.roots[1] * desc_.roots[2];
    if (n() != ntree) {
        err = "root frames are set on the unrefined forest";
        return DGAMR_ESTATE;
    }
    bool any = false;
    for (int t = 0; t < ntree; ++t) {
        if (codes[t] < 0 || codes[t] >= (d == 2 ? 4 : 24)) {
            err = "frame codes are 0..3 (2-D) or 0..23 (3-D)";
            return DGAMR_EINVAL;
        }
        any = any || codes[t] != 0;
    }
    if (any) {
        for (int a = 1; a < d; ++a)
            if ((desc_.hi[a] - desc_.lo[a]) / desc_.roots[a] != (desc_.hi[0] - desc_.lo[0]) / desc_.roots[0]) {
                err = "rotated root frames need equal root edges";
                return DGAMR_EINVAL;
            }
        if (desc_.hanging == DGAMR_HANG_CONSERVATIVE) {
            err = "rotated root frames are built for the paper hanging mode";
            return DGAMR_EUNSUPPORTED;
        }
    }
    frame_.assign(codes, codes + ntree);
    rotated_ = any;
    return build_links(err);
}

int Forest::set_nodes(const double *xy, std::string &err)
{
    const int d = desc_.dim;
    if (d == 3 && desc_.degree > 2) {
        err = "trilinear root blocks are built for degree <= 2";
        return DGAMR_EUNSUPPORTED;
    }
    if (desc_.hanging == DGAMR_HANG_CONSERVATIVE || desc_.equation == DGAMR_EQ_DIFFUSION) {
        err = "bilinear / trilinear root blocks are built for the paper hanging mode, Euler and scalar convection";
        return DGAMR_EUNSUPPORTED;
    }
    const int n[3] = {desc_.roots[0] + 1, desc_.roots[1] + 1, d == 3 ? desc_.roots[2] + 1 : 1};
    const long total = long(n[0]) * n[1] * n[2];
    for (long k = 0; k < d * total; ++k)
        if (!std::isfinite(xy[k])) {
            err = "nodes must be finite";
            return DGAMR_EINVAL;
        }
    auto node = [&](int i, int j, int k) { return xy + long(d) * ((long(k) * n[1] + j) * n[0] + i); };
    // on a periodic axis the last node layer is the first moved by the period
    for (int a = 0; a < d; ++a) {
        if (desc_.bc[a] != DGAMR_BC_PERIODIC) continue;
        const double L = desc_.hi[a] - desc_.lo[a];
        for (long id = 0; id < total; ++id) {
            int idx[3] = {int(id % n[0]), int((id / n[0]) % n[1]), int(id / (long(n[0]) * n[1]))};
            if (idx[a] != 0) continue;
            int last[3] = {idx[0], idx[1], idx[2]};
            last[a] = n[a] - 1;
            const double *p0 = node(idx[0], idx[1], idx[2]), *p1 = node(last[0], last[1], last[2]);
            for (int b = 0; b < d; ++b)
                if (std::fabs(p1[b] - p0[b] - (b == a ? L : 0.0)) > 1e-12 * (desc_.hi[b] - desc_.lo[b])) {
                    err = "periodic axis: the last node layer must be the first one moved by the period";
                    return DGAMR_EINVAL;
                }
        }
    }
    // every root with a positive Jacobian at its corners: the d edges
    // leaving each corner, oriented along the reference axes
    const int nr = desc_.roots[0] * desc_.roots[1] * (d == 3 ? desc_.roots[2] : 1);
    for (int t = 0; t < nr; ++t) {
        const int r[3] = {t % desc_.roots[0], (t / desc_.roots[0]) % desc_.roots[1],
                          d == 3 ? t / (desc_.roots[0] * desc_.roots[1]) : 0};
        for (int b = 0; b < (1 << d); ++b) {
            double E[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            const int c0[3] = {r[0] + (b & 1), r[1] + ((b >> 1) & 1), r[2] + ((b >> 2) & 1)};
            const double *pc = node(c0[0], c0[1], d == 3 ? c0[2] : 0);
            for (int e = 0; e < d; ++e) {
                int c1[3] = {c0[0], c0[1], c0[2]};
                const bool up = !((b >> e) & 1);
                c1[e] += up ? 1 : -1;
                const double *pe = node(c1[0], c1[1], d == 3 ? c1[2] : 0);
                for (int a = 0; a < d; ++a) E[a][e] = (up ? 1.0 : -1.0) * (pe[a] - pc[a]);
            }
            const double det = d == 2 ? E[0][0] * E[1][1] - E[0][1] * E[1][0]
                                      : E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                                            E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                                            E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
            if (!(det > 0.0)) {
                err = "every root must have a positive Jacobian at its corners (nodes in the order of the axes)";
                return DGAMR_EINVAL;
            }
        }
    }
    nodes_.assign(xy, xy + d * total);
    return DGAMR_OK;
}

// Position of a leaf-level index (at `span` leaves per root edge) moved
// between a root's local frame and the global axes (relative to the root):
// along global axis g = pi(l) the local index l, reversed when Q[g][l] = -1.
static void local_to_root(const int Q[3][3], int d, int span, const int *loc, int *glob)
{
    for (int l = 0; l < d; ++l)
        for (int g = 0; g < d; ++g) {
            if (Q[g][l] == 1) glob[g] = loc[l];
            if (Q[g][l] == -1) glob[g] = span - 1 - loc[l];
        }
}
static void root_to_local(const int Q[3][3], int d, int span, const int *glob, int *loc)
{
    for (int l = 0; l < d; ++l)
        for (int g = 0; g < d; ++g) {
            if (Q[g][l] == 1) loc[l] = glob[g];
            if (Q[g][l] == -1) loc[l] = span - 1 - glob[g];
        }
}

int Forest::build_links(std::string &err)
{
    const int d = desc_.dim, nf = 2 * d;
    links_.assign(size_t(n()) * nf, FaceLink{});
    plans_.clear();
    for (int i = 0; i < n(); ++i) {
        const Key &k = leaves_[i];
        const int span = 1 << (k.level - 1);
        int Q[3][3];
        frame_matrix(d, frame_of(k.tree), Q);
        for (int face = 0; face < nf; ++face) {
            const int a = face / 2, s = (face % 2) ? 1 : -1;
            FaceLink &L = links_[size_t(i) * nf + face];
            for (int q = 0; q < 4; ++q) L.nbr[q] = -1;
            int tang[2] = {0, 0}, nt = 0;
            for (int b = 0; b < d; ++b)
                if (b != a) tang[nt++] = b;
            int nidx[3] = {k.idx[0], k.idx[1], k.idx[2]};
            int ntree = k.tree;
            // the neighbour's face toward this leaf, in the neighbour's frame
            int na = a, ns = -s;
            nidx[a] += s;
            if (nidx[a] < 0 || nidx[a] >= span) {
                // across the root face: global axis and side of the local face
                int ga = 0, gs = 0;
                for (int g = 0; g < d; ++g)
                    if (Q[g][a] != 0) {
                        ga = g;
                        gs = s * Q[g][a];
                    }
                if (!neighbour_root(k.tree, ga, gs, ntree)) {
                    L.type = LINK_BOUNDARY;
                    continue;
                }
                int glob[3] = {0, 0, 0}, Qn[3][3];
                local_to_root(Q, d, span, k.idx, glob);
                glob[ga] = gs > 0 ? 0 : span - 1;
                frame_matrix(d, frame_of(ntree), Qn);
                root_to_local(Qn, d, span, glob, nidx);
                nidx[2] = d == 3 ? nidx[2] : 0;
                for (int l = 0; l < d; ++l)
                    if (Qn[ga][l] != 0) {
                        na = l;
                        ns = -gs * Qn[ga][l];
                    }
            }
            const bool rot = frame_of(ntree) != frame_of(k.tree);
            int j = find(ntree, k.level, nidx);
            if (j >= 0) {
                L.type = LINK_SAME;
                L.nbr[0] = j;
            } else {
                int pidx[3] = {nidx[0] >> 1, nidx[1] >> 1, nidx[2] >> 1};
                j = find(ntree, k.level - 1, pidx);
                if (j >= 0) {
                    L.type = LINK_COARSE;
                    L.nbr[0] = j;
                    for (int q = 0; q < nt; ++q) L.off[q] = k.idx[tang[q]] & 1;
                } else {
                    // the 2^(d-1) children of the same-level position that touch
                    // the face, ordered by this leaf's tangential axes (in the
                    // neighbour's frame when the frames differ; rotated faces
                    // take their sources from the guard-cell plans)
                    int ntang[2] = {0, 0}, nnt = 0;
                    for (int b = 0; b < d; ++b)
                        if (b != na) ntang[nnt++] = b;
                    bool ok = k.level < desc_.max_level;
                    for (int c = 0; ok && c < (1 << (d - 1)); ++c) {
                        int cidx[3] = {2 * nidx[0], 2 * nidx[1], 2 * nidx[2]};
                        cidx[na] += (ns > 0) ? 1 : 0;
                        for (int q = 0; q < nnt; ++q) cidx[ntang[q]] += (c >> q) & 1;
                        int jj = find(ntree, k.level + 1, cidx);
                        if (jj < 0) ok = false;
                        L.nbr[c] = jj;
                    }
                    if (!ok) {
                        err = "forest violates 2:1 face balance";
                        return DGAMR_EBALANCE;
                    }
                    L.type = LINK_FINE;
                }
            }
            L.rot = 0;
            if (rot) {
                L.rot = 1 + int(plans_.size());
                if (!rot_plans(i, face, L)) {
                    err = "a guard cell across rotated roots is not covered by its neighbours";
                    return DGAMR_EBALANCE;
                }
            }
        }
    }
    return DGAMR_OK;
}

// Guard-cell plans of the rotated face (leaf i, face): for each guard cell
// t, its box in the neighbour root's local frame (finest-level units), the
// neighbour cells that cover it, and the relative frame.
bool Forest::rot_plans(int i, int face, const FaceLink &L)
{
    const int d = desc_.dim, N = desc_.n_cell;
    const Key &k = leaves_[i];
    const long unit = long(N) << (desc_.max_level - 1); // finest units per root edge
    const long edge = unit >> (k.level - 1), h = edge / N;
    const int a = face / 2, s = (face % 2) ? 1 : -1;
    int Q[3][3];
    frame_matrix(d, frame_of(k.tree), Q);
    const int src = L.nbr[0];
    int Qn[3][3];
    frame_matrix(d, frame_of(leaves_[src].tree), Qn);
    // m = Qn^T Q: source reference coordinates from destination ones
    int m[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int lp = 0; lp < d; ++lp)
        for (int l = 0; l < d; ++l)
            for (int g = 0; g < d; ++g) m[lp][l] += Qn[g][lp] * Q[g][l];
    int tang[2] = {0, 0}, nt = 0;
    for (int b = 0; b < d; ++b)
        if (b != a) tang[nt++] = b;
    auto leaf_lbox = [&](int j, long *lo) {
        const Key &q = leaves_[j];
        const long e = unit >> (q.level - 1);
        for (int b = 0; b < 3; ++b) lo[b] = b < d ? q.idx[b] * e : 0;
        return e;
    };
    const int nfc = d == 2 ? N : N * N;
    for (int t = 0; t < nfc; ++t) {
        // guard cell box in this root's local frame
        long lo[3] = {0, 0, 0};
        leaf_lbox(i, lo);
        int ijk[3] = {0, 0, 0};
        ijk[a] = s > 0 ? N - 1 : 0;
        ijk[tang[0]] = t % N;
        if (d == 3) ijk[tang[1]] = t / N;
        for (int b = 0; b < d; ++b) lo[b] += ijk[b] * h;
        lo[a] += s * h;
        // to the global axes relative to this root, then across into the
        // neighbour root (the face's global axis shifts by one root edge)
        long gl[3] = {0, 0, 0};
        int ga = 0, gs = 0;
        for (int l = 0; l < d; ++l)
            for (int g = 0; g < d; ++g) {
                if (Q[g][l] == 1) gl[g] = lo[l];
                if (Q[g][l] == -1) gl[g] = unit - lo[l] - h;
                if (l == a && Q[g][l] != 0) {
                    ga = g;
                    gs = s * Q[g][l];
                }
            }
        gl[ga] += gs > 0 ? -unit : unit;
        long nl[3] = {0, 0, 0}; // guard box in the neighbour's local frame
        for (int l = 0; l < d; ++l)
            for (int g = 0; g < d; ++g) {
                if (Qn[g][l] == 1) nl[l] = gl[g];
                if (Qn[g][l] == -1) nl[l] = unit - gl[g] - h;
            }
        RotPlan P{};
        for (int lp = 0; lp < 3; ++lp)
            for (int l = 0; l < 3; ++l) P.m[3 * lp + l] = (signed char)m[lp][l];
        auto cell_of = [&](int j, const long *pt, long &ch) {
            long blo[3];
            const long e = leaf_lbox(j, blo), hc = e / N;
            int c = 0, mul = 1;
            for (int b = 0; b < d; ++b) {
                c += int((pt[b] - blo[b]) / hc) * mul;
                mul *= N;
            }
            ch = hc;
            return c;
        };
        auto contains = [&](int j, const long *pt) {
            long blo[3];
            const long e = leaf_lbox(j, blo);
            for (int b = 0; b < d; ++b)
                if (pt[b] < blo[b] || pt[b] >= blo[b] + e) return false;
            return true;
        };
        if (L.type != LINK_FINE && !contains(src, nl)) return false;
        if (L.type == LINK_SAME) {
            long hc;
            P.type = PLAN_COPY;
            P.leaf[0] = src;
            P.cell[0] = cell_of(src, nl, hc);
        } else if (L.type == LINK_COARSE) {
            long hc;
            P.type = PLAN_SPLIT;
            P.leaf[0] = src;
            P.cell[0] = cell_of(src, nl, hc);
            long blo[3];
            leaf_lbox(src, blo);
            int child = 0;
            for (int b = 0; b < d; ++b) child |= int(((nl[b] - blo[b]) % hc) / (hc / 2)) << b;
            P.child = child;
        } else {
            P.type = PLAN_COMBINE;
            for (int c = 0; c < (1 << d); ++c) {
                long pt[3] = {0, 0, 0};
                for (int b = 0; b < d; ++b) pt[b] = nl[b] + ((c >> b) & 1) * (h / 2);
                int jf = -1;
                for (int q = 0; q < (1 << (d - 1)); ++q)
                    if (L.nbr[q] >= 0 && contains(L.nbr[q], pt)) jf = L.nbr[q];
                if (jf < 0) return false;
                long hc;
                P.leaf[c] = jf;
                P.cell[c] = cell_of(jf, pt, hc);
            }
        }
        plans_.push_back(P);
    }
    return true;
}

std::vector<LeafGeo> Forest::geometry() const
{
    const int d = desc_.dim;
    std::vector<LeafGeo> g(n());
    for (int i = 0; i < n(); ++i) {
        const Key &k = leaves_[i];
        int r[3] = {k.tree % desc_.roots[0], (k.tree / desc_.roots[0]) % desc_.roots[1],
                    k.tree / (desc_.roots[0] * desc_.roots[1])};
        int Q[3][3];
        frame_matrix(d, frame_of(k.tree), Q);
        LeafGeo &G = g[i];
        G.vol = 1.0;
        // local origin of the leaf: its local lower corner, mapped through the
        // root's frame (the root box maps onto itself)
        const int span = 1 << (k.level - 1);
        for (int a = 0; a < 3; ++a) {
            const double root = (desc_.hi[a] - desc_.lo[a]) / desc_.roots[a];
            G.lo[a] = desc_.lo[a] + r[a] * root;
        }
        for (int l = 0; l < 3; ++l) {
            const int ga = [&] {
                for (int gg = 0; gg < d; ++gg)
                    if (Q[gg][l] != 0) return gg;
                return l;
            }();
            const double root = (desc_.hi[ga] - desc_.lo[ga]) / desc_.roots[ga];
            const double edge = root / double(span);
            G.h[l] = edge / desc_.n_cell;
            G.scale[l] = 2.0 / G.h[l];
            if (l < d) {
                G.vol *= G.h[l];
                // the local coordinate k.idx[l] * edge from the root's local
                // origin, which sits at the root's far side when Q[ga][l] = -1
                G.lo[ga] += Q[ga][l] > 0 ? k.idx[l] * edge : root - k.idx[l] * edge;
            }
        }
        G.level = k.level;
        G.pad = 0;
        for (int b = 0; b < 8; ++b) G.node[b][0] = G.node[b][1] = G.node[b][2] = 0.0;
        if (mapped()) {
            // the leaf's corners: the root's multilinear map at the leaf's
            // corners in the root's unit box; the corner's local position
            // turned onto the node grid's axes by the root's frame
            const int nx = desc_.roots[0] + 1, ny = desc_.roots[1] + 1;
            for (int b = 0; b < (1 << d); ++b) {
                double sl[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < d; ++a) sl[a] = double(k.idx[a] + ((b >> a) & 1)) / span;
                for (int l = 0; l < d; ++l)
                    for (int a = 0; a < d; ++a) {
                        if (Q[a][l] == 1) s[a] = sl[l];
                        if (Q[a][l] == -1) s[a] = 1.0 - sl[l];
                    }
                for (int nn = 0; nn < (1 << d); ++nn) {
                    double w = 1.0;
                    int id[3] = {r[0], r[1], r[2]};
                    for (int a = 0; a < d; ++a) {
                        const int bit = (nn >> a) & 1;
                        w *= bit ? s[a] : 1.0 - s[a];
                        id[a] += bit;
                    }
                    const double *xy = nodes_.data() + long(d) * ((long(d == 3 ? id[2] : 0) * ny + id[1]) * nx + id[0]);
                    for (int a = 0; a < d; ++a) G.node[b][a] += w * xy[a];
                }
            }
        }
        for (int gg = 0; gg < 3; ++gg)
            for (int l = 0; l < 3; ++l) G.q[3 * gg + l] = (signed char)Q[gg][l];
        for (int x = 9; x < 12; ++x) G.q[x] = 0;
    }
    return g;
}

int Forest::plan(const int8_t *flags, std::string &err)
{
    const int d = desc_.dim, nf = 2 * d, nchild = 1 << d, nl = n();
    std::vector<int> r(nl, 0);
    for (int i = 0; i < nl; ++i) r[i] = (flags[i] > 0 && leaves_[i].level < desc_.max_level) ? 1 : 0;
    auto face_nbrs = [&](int i, int face, int *out) {
        const FaceLink &L = links_[size_t(i) * nf + face];
        if (L.type == LINK_BOUNDARY) return 0;
        if (L.type == LINK_FINE) {
            for (int c = 0; c < (1 << (d - 1)); ++c) out[c] = L.nbr[c];
            return 1 << (d - 1);
        }
        out[0] = L.nbr[0];
        return 1;
    };
    // refinement closed under 2:1 face balance (worklist)
    std::vector<int> work;
    for (int i = 0; i < nl; ++i)
        if (r[i]) work.push_back(i);
    while (!work.empty()) {
        int i = work.back();
        work.pop_back();
        for (int face = 0; face < nf; ++face) {
            int nb[4];
            int m = face_nbrs(i, face, nb);
            for (int q = 0; q < m; ++q) {
                int j = nb[q];
                if (!r[j] && leaves_[i].level + r[i] > leaves_[j].level + 1) {
                    r[j] = 1;
                    work.push_back(j);
                }
            }
        }
    }
    // coarsening families keyed by their parent
    std::unordered_map<uint64_t, std::vector<int>> fam;
    for (int i = 0; i < nl; ++i) {
        const Key &k = leaves_[i];
        if (k.level <= 1 || flags[i] >= 0 || r[i]) continue;
        int pidx[3] = {k.idx[0] >> 1, k.idx[1] >> 1, k.idx[2] >> 1};
        fam[pack(k.tree, k.level - 1, pidx)].push_back(i);
    }
    std::vector<int> grp(nl, -1);
    std::vector<uint64_t> gkey;
    for (auto &kv : fam) {
        if (int(kv.second.size()) != nchild) continue; // some sibling is not a flagged leaf
        int g = int(gkey.size());
        gkey.push_back(kv.first);
        for (int i : kv.second) grp[i] = g;
    }
    for (bool changed = true; changed;) {
        changed = false;
        for (int i = 0; i < nl; ++i) {
            if (grp[i] < 0) continue;
            bool bad = false;
            for (int face = 0; face < nf && !bad; ++face) {
                int nb[4];
                int m = face_nbrs(i, face, nb);
                for (int q = 0; q < m; ++q) {
                    int j = nb[q];
                    if (grp[j] == grp[i]) continue;
                    int lj = leaves_[j].level + r[j] - (grp[j] >= 0 ? 1 : 0);
                    if (lj > leaves_[i].level) bad = true;
                }
            }
            if (bad) {
                int g = grp[i];
                for (int j = 0; j < nl; ++j)
                    if (grp[j] == g) grp[j] = -1;
                changed = true;
            }
        }
    }
    // new leaves with their inheritance sources
    planned_.clear();
    planned_inh_.clear();
    std::vector<char> done(gkey.size(), 0);
    for (int i = 0; i < nl; ++i) {
        const Key &k = leaves_[i];
        if (r[i]) {
            for (int c = 0; c < nchild; ++c) {
                Key ch;
                ch.tree = k.tree;
                ch.level = k.level + 1;
                for (int a = 0; a < 3; ++a) ch.idx[a] = a < d ? 2 * k.idx[a] + ((c >> a) & 1) : 0;
                Inherit in{};
                in.type = INH_SPLIT;
                in.src[0] = i;
                in.child = c;
                planned_.push_back(ch);
                planned_inh_.push_back(in);
            }
        } else if (grp[i] >= 0) {
            if (done[grp[i]]) continue;
            done[grp[i]] = 1;
            Key pa;
            pa.tree = k.tree;
            pa.level = k.level - 1;
            for (int a = 0; a < 3; ++a) pa.idx[a] = k.idx[a] >> 1;
            Inherit in{};
            in.type = INH_COMBINE;
            for (int c = 0; c < nchild; ++c) {
                int cidx[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a) cidx[a] = 2 * pa.idx[a] + ((c >> a) & 1);
                in.src[c] = find(k.tree, k.level, cidx);
            }
            planned_.push_back(pa);
            planned_inh_.push_back(in);
        } else {
            Inherit in{};
            in.type = INH_COPY;
            in.src[0] = i;
            planned_.push_back(k);
            planned_inh_.push_back(in);
        }
    }
    // sort keys and inheritance together
    std::vector<int> perm(planned_.size());
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [this](int x, int y) {
        const Key &a = planned_[x], &b = planned_[y];
        if (a.tree != b.tree) return a.tree < b.tree;
        return morton(a) < morton(b);
    });
    std::vector<Key> ks(perm.size());
    std::vector<Inherit> is(perm.size());
    for (size_t q = 0; q < perm.size(); ++q) {
        ks[q] = planned_[perm[q]];
        is[q] = planned_inh_[perm[q]];
    }
    planned_.swap(ks);
    planned_inh_.swap(is);
    has_plan_ = true;
    (void)err;
    return DGAMR_OK;
}

int Forest::commit(std::vector<Inherit> &inh, std::string &err)
{
    if (!has_plan_) {
        err = "no refinement plan pending";
        return DGAMR_ESTATE;
    }
    leaves_.swap(planned_);
    inh.swap(planned_inh_);
    planned_.clear();
    planned_inh_.clear();
    has_plan_ = false;
    reindex();
    return build_links(err);
}

} // namespace dgamr
