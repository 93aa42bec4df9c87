/*
 * Oracle - forest of block trees (Sec. 3.1), block mesh and guard layer
 * (Sec. 3.3), refinement planning with level limits and 2:1 face balance,
 * and L2 inheritance on refinement/coarsening (Sec. 3.4, Eq. 11-14).
 * TEST INFRASTRUCTURE (see oracle.h).
 *
 * Geometry is kept in exact global integer units: one root edge is
 * unit = N * 2^(max_level-1) units, so every cell edge of every leaf is an
 * integer.  All neighbour relations are found by brute-force geometric
 * search over the leaves, which is slow and plainly correct.
 */
#include <stdio.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

static long ipow2(int e) { return 1L << e; }

long orc_domain_units(const orc_forest *f, int axis) { return f->unit * f->roots[axis]; }

int orc_ncell(const orc_forest *f)
{
    int n = 1;
    for (int a = 0; a < f->dim; ++a) n *= f->N;
    return n;
}

int orc_nface_cells(const orc_forest *f)
{
    int n = 1;
    for (int a = 0; a < f->dim - 1; ++a) n *= f->N;
    return n;
}

void orc_cell_ijk(const orc_forest *f, int cell, int *ijk)
{
    ijk[0] = cell % f->N;
    ijk[1] = (cell / f->N) % f->N;
    ijk[2] = (f->dim == 3) ? cell / (f->N * f->N) : 0;
}

int orc_cell_index(const orc_forest *f, const int *ijk)
{
    return ijk[0] + f->N * (ijk[1] + (f->dim == 3 ? f->N * ijk[2] : 0));
}

/* Frames of the root blocks (Sec. 3.1: neighbouring roots may be rotated
 * against each other; the relative rotation is what the guard fill of
 * Sec. 3.5 has to undo).  A root's frame is a rotation Q of its local axes,
 * global vector = Q local vector, Q a signed permutation matrix with
 * determinant +1.  2-D: code k is k quarter turns counter-clockwise.  3-D:
 * code k is the k-th such matrix when the permutations (pi(0), pi(1), pi(2))
 * of the local axes are taken in lexicographic order and, for each, the
 * signs of the local axes s_l (bit l of 0..7 set: s_l = -1) in increasing
 * order, with Q[pi(l)][l] = s_l. */
void orc_frame_matrix(const orc_forest *f, int tree, int Q[3][3])
{
    int code = f->frame ? f->frame[tree] : 0;
    memset(Q, 0, sizeof(int) * 9);
    if (f->dim == 2) {
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
            int M[3][3];
            memset(M, 0, sizeof(M));
            for (int l = 0; l < 3; ++l) M[perms[pi][l]][l] = (sg >> l) & 1 ? -1 : 1;
            int det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                      M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                      M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            if (det != 1) continue;
            if (n == code) {
                memcpy(Q, M, sizeof(M));
                return;
            }
            ++n;
        }
}

/* lower corner and edge of a leaf in its root's local frame */
void orc_leaf_lbox(const orc_forest *f, const orc_key *k, long *lo, long *size)
{
    long edge = f->unit / ipow2(k->level - 1);
    for (int a = 0; a < 3; ++a) lo[a] = (a < f->dim) ? k->idx[a] * edge : 0;
    *size = edge;
}

/* a local box [p, p + e) of root `tree` in global units: along global axis
 * pi(l) the local interval of axis l, reversed when Q[pi(l)][l] = -1 */
static void local_to_global(const orc_forest *f, int tree, const long *p, long e, long *g)
{
    int Q[3][3];
    orc_frame_matrix(f, tree, Q);
    int r[3];
    r[0] = tree % f->roots[0];
    r[1] = (tree / f->roots[0]) % f->roots[1];
    r[2] = tree / (f->roots[0] * f->roots[1]);
    for (int a = 0; a < 3; ++a) g[a] = 0;
    for (int l = 0; l < f->dim; ++l)
        for (int a = 0; a < f->dim; ++a) {
            if (Q[a][l] == 1) g[a] = r[a] * f->unit + p[l];
            if (Q[a][l] == -1) g[a] = r[a] * f->unit + f->unit - p[l] - e;
        }
}

/* lower corner and edge (global units) of a leaf */
void orc_leaf_box(const orc_forest *f, const orc_key *k, long *lo, long *size)
{
    long l[3];
    orc_leaf_lbox(f, k, l, size);
    local_to_global(f, k->tree, l, *size, lo);
}

void orc_cell_gbox(const orc_forest *f, const orc_key *k, const int *ijk, long *lo)
{
    long l[3], size;
    orc_leaf_lbox(f, k, l, &size);
    long h = size / f->N;
    for (int a = 0; a < f->dim; ++a) l[a] += ijk[a] * h;
    local_to_global(f, k->tree, l, h, lo);
}

/* Morton code of the leaf's lower corner at the finest level: bit b of x
 * goes to position d*b, y to d*b+1, z to d*b+2 (x fastest). */
static unsigned long long morton(const orc_forest *f, const orc_key *k)
{
    int shift = f->max_level - k->level;
    unsigned long long code = 0;
    for (int b = 0; b < 21; ++b)
        for (int a = 0; a < f->dim; ++a) {
            unsigned long long bit = ((unsigned long long)(k->idx[a] << shift) >> b) & 1ULL;
            code |= bit << (f->dim * b + a);
        }
    return code;
}

static const orc_forest *g_sort_forest;
static int key_cmp(const void *pa, const void *pb)
{
    const orc_key *a = pa, *b = pb;
    if (a->tree != b->tree) return a->tree < b->tree ? -1 : 1;
    unsigned long long ma = morton(g_sort_forest, a), mb = morton(g_sort_forest, b);
    if (ma != mb) return ma < mb ? -1 : 1;
    return a->level - b->level;
}

void orc_sort_leaves(const orc_forest *f, orc_key *leaves, int n)
{
    g_sort_forest = f;
    qsort(leaves, n, sizeof(orc_key), key_cmp);
}

static int box_contains(const long *lo, long size, int dim, const double *x)
{
    for (int a = 0; a < dim; ++a)
        if (x[a] < (double)lo[a] || x[a] >= (double)(lo[a] + size)) return 0;
    return 1;
}

int orc_find_leaf(const orc_forest *f, const orc_key *leaves, int n, const double *xin)
{
    double x[3] = {xin[0], xin[1], xin[2]};
    for (int a = 0; a < f->dim; ++a) {
        double L = (double)orc_domain_units(f, a);
        if (x[a] < 0 || x[a] >= L) {
            if (f->bc[a] != ORC_BC_PERIODIC) return -1;
            while (x[a] < 0) x[a] += L;
            while (x[a] >= L) x[a] -= L;
        }
    }
    for (int i = 0; i < n; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &leaves[i], lo, &size);
        if (box_contains(lo, size, f->dim, x)) return i;
    }
    return -1;
}

/* ---------------------------------------------------------------- topology */

/* overlap of [a0,a1) and [b0,b1) with positive length */
static int overlaps(long a0, long a1, long b0, long b1) { return a0 < b1 && b0 < a1; }

/* Face neighbours of leaf `i` across face (axis, side): all leaves B whose
 * opposite face lies in the same plane (mod the period) and whose
 * tangential extent overlaps.  Finer neighbours are ordered by their
 * tangential position, lower remaining axis fastest. */
static void find_face_nbrs(const orc_forest *f, int i, int axis, int side, orc_face_nbr *out)
{
    long lo[3], size;
    orc_leaf_box(f, &f->leaf[i], lo, &size);
    long plane = (side > 0) ? lo[axis] + size : lo[axis];
    long L = orc_domain_units(f, axis);
    memset(out, 0, sizeof(*out));
    if (plane == 0 || plane == L) {
        if (f->bc[axis] != ORC_BC_PERIODIC) {
            out->boundary = 1;
            return;
        }
    }
    long tlo[4][3];
    for (int j = 0; j < f->nleaves; ++j) {
        long blo[3], bsize;
        orc_leaf_box(f, &f->leaf[j], blo, &bsize);
        long bplane = (side > 0) ? blo[axis] : blo[axis] + bsize; /* B's opposite face */
        int touch = (bplane == plane) || (bplane - L == plane) || (bplane + L == plane) ||
                    (bplane == plane - L) || (bplane == plane + L);
        if (!touch) continue;
        int ok = 1;
        for (int b = 0; b < f->dim; ++b) {
            if (b == axis) continue;
            if (!overlaps(lo[b], lo[b] + size, blo[b], blo[b] + bsize)) ok = 0;
        }
        if (!ok) continue;
        if (out->nn >= 4) {
            fprintf(stderr, "oracle: too many face neighbours\n");
            abort();
        }
        out->nb[out->nn] = j;
        for (int b = 0; b < 3; ++b) tlo[out->nn][b] = blo[b];
        out->nn++;
        out->level_diff = f->leaf[j].level - f->leaf[i].level;
    }
    if (out->nn == 0) {
        fprintf(stderr, "oracle: leaf %d face (%d,%d) has no neighbour\n", i, axis, side);
        abort();
    }
    /* order finer neighbours by tangential position (lower axis fastest) */
    for (int x = 0; x < out->nn; ++x)
        for (int y = x + 1; y < out->nn; ++y) {
            long kx = 0, ky = 0;
            for (int b = f->dim - 1; b >= 0; --b) {
                if (b == axis) continue;
                kx = kx * 4 * L + tlo[x][b];
                ky = ky * 4 * L + tlo[y][b];
            }
            if (ky < kx) {
                int t = out->nb[x]; out->nb[x] = out->nb[y]; out->nb[y] = t;
                for (int b = 0; b < 3; ++b) { long s = tlo[x][b]; tlo[x][b] = tlo[y][b]; tlo[y][b] = s; }
            }
        }
}

/* tangential axes of a face axis, in increasing order */
static void tangential_axes(int dim, int axis, int *ta)
{
    int n = 0;
    for (int b = 0; b < dim; ++b)
        if (b != axis) ta[n++] = b;
}

/* global axis and side of the local face (axis, side) of a leaf of `tree` */
static void global_face(const orc_forest *f, int tree, int axis, int side, int *gaxis, int *gside)
{
    int Q[3][3];
    orc_frame_matrix(f, tree, Q);
    for (int a = 0; a < f->dim; ++a)
        if (Q[a][axis] != 0) {
            *gaxis = a;
            *gside = side * Q[a][axis];
        }
}

/* Guard plan for guard cell t of the local face (axis, side) of leaf i: the
 * guard cell is the cell of this leaf's level just outside the face
 * (Sec. 3.3); it is covered by cells of the face neighbours.  Boxes are
 * global; a neighbour in a root of another frame is found the same way. */
static void build_guard_plan(const orc_forest *f, int i, int axis, int side, int t,
                             const orc_face_nbr *fn, orc_guard_plan *gp)
{
    long lo[3], size;
    orc_leaf_box(f, &f->leaf[i], lo, &size);
    long h = size / f->N;
    int ta[2];
    tangential_axes(f->dim, axis, ta);
    int ijk[3] = {0, 0, 0};
    ijk[axis] = (side > 0) ? f->N - 1 : 0;
    ijk[ta[0]] = t % f->N;
    if (f->dim == 3) ijk[ta[1]] = t / f->N;
    long glo[3] = {0, 0, 0};
    orc_cell_gbox(f, &f->leaf[i], ijk, glo);
    int gaxis = axis, gside = side;
    global_face(f, f->leaf[i].tree, axis, side, &gaxis, &gside);
    glo[gaxis] += gside * h;
    axis = gaxis;
    gp->npiece = 0;
    gp->piece = NULL;
    if (fn->boundary) {
        gp->kind = 2;
        return;
    }
    long L = orc_domain_units(f, axis);
    gp->piece = calloc(8, sizeof(orc_piece));
    for (int n = 0; n < fn->nn; ++n) {
        int j = fn->nb[n];
        long blo[3], bsize;
        orc_leaf_box(f, &f->leaf[j], blo, &bsize);
        /* bring B next to the guard cell along the face axis (periodic wrap) */
        long shift = 0;
        if (glo[axis] < 0) shift = -L;
        if (glo[axis] >= L) shift = L;
        blo[axis] += shift;
        long bh = bsize / f->N;
        for (int c = 0; c < orc_ncell(f); ++c) {
            int cijk[3];
            orc_cell_ijk(f, c, cijk);
            long clo[3] = {0, 0, 0}, olo[3] = {0, 0, 0}, ohi[3] = {0, 0, 0};
            orc_cell_gbox(f, &f->leaf[j], cijk, clo);
            clo[axis] += shift;
            int ok = 1;
            for (int a = 0; a < f->dim; ++a) {
                olo[a] = clo[a] > glo[a] ? clo[a] : glo[a];
                ohi[a] = (clo[a] + bh) < (glo[a] + h) ? (clo[a] + bh) : (glo[a] + h);
                if (olo[a] >= ohi[a]) ok = 0;
            }
            if (!ok) continue;
            orc_piece *pc = &gp->piece[gp->npiece++];
            pc->leaf = j;
            pc->cell = c;
            for (int a = 0; a < 3; ++a) {
                pc->lo[a] = olo[a];
                pc->hi[a] = ohi[a];
                pc->src_lo[a] = clo[a];
            }
            pc->src_size = bh;
        }
    }
    int same_frame = (f->frame ? f->frame[f->leaf[fn->nb[0]].tree] : 0) == (f->frame ? f->frame[f->leaf[i].tree] : 0);
    if (gp->npiece == 1 && fn->level_diff == 0 && same_frame)
        gp->kind = 0; /* Eq. 15: same level, rotation identity: copy */
    else
        gp->kind = 1; /* Eq. 15-17 with a rotation, or split / combine: L2 projection */
}

void orc_free_topology(orc_forest *f)
{
    if (f->gp) {
        long ng = (long)f->nleaves * 2 * f->dim * orc_nface_cells(f);
        for (long g = 0; g < ng; ++g) free(f->gp[g].piece);
        free(f->gp);
        f->gp = NULL;
    }
    free(f->fn);
    f->fn = NULL;
}

void orc_build_topology(orc_forest *f)
{
    orc_free_topology(f);
    int nf = 2 * f->dim, nfc = orc_nface_cells(f);
    f->fn = calloc((size_t)f->nleaves * nf, sizeof(orc_face_nbr));
    f->gp = calloc((size_t)f->nleaves * nf * nfc, sizeof(orc_guard_plan));
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < f->nleaves; ++i)
        for (int face = 0; face < nf; ++face) {
            int axis = face / 2, side = (face % 2) ? 1 : -1;
            int gaxis = axis, gside = side;
            global_face(f, f->leaf[i].tree, axis, side, &gaxis, &gside);
            find_face_nbrs(f, i, gaxis, gside, &f->fn[i * nf + face]);
            if (abs(f->fn[i * nf + face].level_diff) > 1) {
                fprintf(stderr, "oracle: 2:1 balance violated\n");
                abort();
            }
            for (int t = 0; t < nfc; ++t)
                build_guard_plan(f, i, axis, side, t, &f->fn[i * nf + face],
                                 &f->gp[((long)i * nf + face) * nfc + t]);
        }
}

/* ---------------------------------------------------------------- create */

orc_forest *orc_create(int dim, int p, int n_cell, const int *roots, const double *lo,
                       const double *hi, const int *bc, int max_level, double gamma, int hanging)
{
    if ((dim != 2 && dim != 3) || p < 0 || p > 3 || n_cell < 2 || n_cell % 2 || max_level < 1)
        return NULL;
    orc_forest *f = calloc(1, sizeof(orc_forest));
    f->dim = dim;
    f->p = p;
    f->N = n_cell;
    f->nb = orc_num_modes(dim, p);
    f->nv = dim + 2;
    f->equation = ORC_EQ_EULER;
    f->q = p + 1;
    f->max_level = max_level;
    f->gamma = gamma;
    f->hanging = hanging;
    for (int a = 0; a < 3; ++a) {
        f->roots[a] = (a < dim) ? roots[a] : 1;
        f->lo[a] = (a < dim) ? lo[a] : 0.0;
        f->hi[a] = (a < dim) ? hi[a] : 1.0;
        f->bc[a] = (a < dim) ? bc[a] : ORC_BC_PERIODIC;
    }
    f->unit = (long)n_cell * ipow2(max_level - 1);
    f->exps = malloc(sizeof(int) * 3 * f->nb);
    orc_mode_exponents(dim, p, f->exps);
    f->nleaves = f->roots[0] * f->roots[1] * f->roots[2];
    f->leaf = calloc(f->nleaves, sizeof(orc_key));
    for (int t = 0; t < f->nleaves; ++t) {
        f->leaf[t].tree = t;
        f->leaf[t].level = 1;
    }
    orc_build_topology(f);
    return f;
}

void orc_set_advection(orc_forest *f, const double *vel)
{
    f->equation = ORC_EQ_ADVECTION;
    f->nv = 1;
    for (int a = 0; a < 3; ++a) f->vel[a] = a < f->dim ? vel[a] : 0.0;
}

void orc_set_diffusion(orc_forest *f, double nu, const double *avec)
{
    f->equation = ORC_EQ_DIFFUSION;
    f->nv = 1;
    f->nu = nu;
    for (int a = 0; a < 3; ++a) f->avec[a] = a < f->dim ? avec[a] : 0.0;
}

int orc_set_frames(orc_forest *f, const int *codes)
{
    int ntree = f->roots[0] * f->roots[1] * f->roots[2], ncode = f->dim == 2 ? 4 : 24;
    int any = 0;
    for (int t = 0; t < ntree; ++t) {
        if (codes[t] < 0 || codes[t] >= ncode) return -1;
        any |= codes[t] != 0;
    }
    /* a rotated root must map onto its own box: equal physical edges */
    if (any)
        for (int a = 1; a < f->dim; ++a)
            if ((f->hi[a] - f->lo[a]) / f->roots[a] != (f->hi[0] - f->lo[0]) / f->roots[0]) return -1;
    /* the mortar of the conservative mode is written along the global axes */
    if (any && f->hanging == ORC_HANG_CONSERVATIVE) return -1;
    free(f->frame);
    f->frame = malloc(sizeof(int) * ntree);
    memcpy(f->frame, codes, sizeof(int) * ntree);
    orc_build_topology(f);
    return 0;
}

/* Sec. 3.3, Eq. 6: root blocks as bilinear (3-D: trilinear) images of the
 * reference square (cube): xy holds the (roots_x + 1) x (roots_y + 1)
 * [x (roots_z + 1)] grid nodes, x fastest, d coordinates each; root (rx,
 * ry[, rz]) has the corner nodes (rx + bx, ry + by[, rz + bz]), b in {0,1}^d.
 * On a periodic axis the last node layer must be the first one moved by the
 * period.  Every root must have a positive Jacobian at its corners.  A
 * root with a rotated frame takes its local axes along the node grid's axes
 * as its frame turns them (its corner b is the grid node the frame maps it
 * to); on such forests the momentum is stored along the global axes, and
 * the guard fill turns only coordinates.  Not with the conservative mode
 * or the diffusion equation. */
int orc_set_nodes(orc_forest *f, const double *xy)
{
    if (f->hanging == ORC_HANG_CONSERVATIVE || f->equation == ORC_EQ_DIFFUSION) return -1;
    int d = f->dim, n[3] = {f->roots[0] + 1, f->roots[1] + 1, d == 3 ? f->roots[2] + 1 : 1};
    long total = (long)n[0] * n[1] * n[2];
#define NODE(i, j, k) (xy + (long)d * (((long)(k) * n[1] + (j)) * n[0] + (i)))
    for (int a = 0; a < d; ++a) {
        if (f->bc[a] != ORC_BC_PERIODIC) continue;
        double L = f->hi[a] - f->lo[a];
        for (long id = 0; id < total; ++id) {
            int idx[3] = {(int)(id % n[0]), (int)((id / n[0]) % n[1]), (int)(id / ((long)n[0] * n[1]))};
            if (idx[a] != 0) continue;
            int last[3] = {idx[0], idx[1], idx[2]};
            last[a] = n[a] - 1;
            const double *p0 = NODE(idx[0], idx[1], idx[2]), *p1 = NODE(last[0], last[1], last[2]);
            for (int b = 0; b < d; ++b) {
                double want = p0[b] + (b == a ? L : 0.0);
                if (fabs(p1[b] - want) > 1e-12 * (f->hi[b] - f->lo[b])) return -1;
            }
        }
    }
    int nr = f->roots[0] * f->roots[1] * (d == 3 ? f->roots[2] : 1);
    for (int t = 0; t < nr; ++t) {
        int r[3] = {t % f->roots[0], (t / f->roots[0]) % f->roots[1], d == 3 ? t / (f->roots[0] * f->roots[1]) : 0};
        /* the Jacobian at each corner: the d edges leaving it, oriented along
         * the reference axes */
        for (int b = 0; b < (1 << d); ++b) {
            double E[3][3] = {{0}};
            int c0[3] = {r[0] + (b & 1), r[1] + ((b >> 1) & 1), r[2] + ((b >> 2) & 1)};
            const double *pc = NODE(c0[0], c0[1], d == 3 ? c0[2] : 0);
            for (int e = 0; e < d; ++e) {
                int c1[3] = {c0[0], c0[1], c0[2]};
                int up = !((b >> e) & 1);
                c1[e] += up ? 1 : -1;
                const double *pe = NODE(c1[0], c1[1], d == 3 ? c1[2] : 0);
                for (int a = 0; a < d; ++a) E[a][e] = (up ? 1.0 : -1.0) * (pe[a] - pc[a]);
            }
            double det = d == 2 ? E[0][0] * E[1][1] - E[0][1] * E[1][0]
                                : E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                                      E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                                      E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
            if (!(det > 0.0)) return -1;
        }
    }
#undef NODE
    free(f->nodes);
    f->nodes = malloc(sizeof(double) * d * total);
    memcpy(f->nodes, xy, sizeof(double) * d * total);
    return 0;
}

void orc_set_time(orc_forest *f, double t) { f->time = f->stage_time = t; }
double orc_get_time(const orc_forest *f) { return f->time; }

void orc_destroy(orc_forest *f)
{
    if (!f) return;
    orc_free_topology(f);
    free(f->leaf);
    free(f->new_leaf);
    free(f->exps);
    free(f->frame);
    free(f->nodes);
    free(f);
}

int orc_num_leaves(const orc_forest *f) { return f->nleaves; }

void orc_leaf_keys(const orc_forest *f, int *keys)
{
    for (int i = 0; i < f->nleaves; ++i) {
        keys[5 * i + 0] = f->leaf[i].tree;
        keys[5 * i + 1] = f->leaf[i].level;
        keys[5 * i + 2] = f->leaf[i].idx[0];
        keys[5 * i + 3] = f->leaf[i].idx[1];
        keys[5 * i + 4] = f->leaf[i].idx[2];
    }
}

long orc_state_len(const orc_forest *f) { return (long)f->nleaves * f->nv * f->nb * orc_ncell(f); }

long orc_guard_len(const orc_forest *f)
{
    return (long)f->nleaves * 2 * f->dim * f->nv * f->nb * orc_nface_cells(f);
}

/* ---------------------------------------------------------------- adaptation */

static int same_parent(const orc_key *a, const orc_key *b)
{
    if (a->tree != b->tree || a->level != b->level) return 0;
    for (int x = 0; x < 3; ++x)
        if ((a->idx[x] >> 1) != (b->idx[x] >> 1)) return 0;
    return 1;
}

/* Refinement planning (Sec. 4.3 step 3 and Sec. 3.1).  Rules, applied in
 * this order:
 *   1. a refine flag counts only below max_level, a coarsen flag only above
 *      level 1;
 *   2. refinement is closed under 2:1 face balance: a leaf must refine when
 *      a face neighbour would end up two levels finer (refinement wins);
 *   3. a family of 2^d sibling leaves coarsens into its parent only if all
 *      of them are flagged -1 and none refines, and only if no face
 *      neighbour outside the family ends up finer than the family's level;
 *      families failing this are dropped until no more fail. */
int orc_plan_adapt(orc_forest *f, const signed char *flags)
{
    int n = f->nleaves, nf = 2 * f->dim, nchild = 1 << f->dim;
    int *r = calloc(n, sizeof(int));
    for (int i = 0; i < n; ++i)
        r[i] = (flags[i] > 0 && f->leaf[i].level < f->max_level) ? 1 : 0;
    for (int changed = 1; changed;) {
        changed = 0;
        for (int i = 0; i < n; ++i)
            for (int face = 0; face < nf; ++face) {
                const orc_face_nbr *fn = &f->fn[i * nf + face];
                for (int k = 0; k < fn->nn; ++k) {
                    int j = fn->nb[k];
                    if (f->leaf[i].level + r[i] > f->leaf[j].level + r[j] + 1 && !r[j]) {
                        r[j] = 1;
                        changed = 1;
                    }
                }
            }
    }
    /* coarsening families: group id = index of the first sibling found */
    int *grp = malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) grp[i] = -1;
    for (int i = 0; i < n; ++i) {
        if (grp[i] >= 0 || f->leaf[i].level <= 1 || flags[i] >= 0 || r[i]) continue;
        int members[8], nm = 0;
        for (int j = 0; j < n && nm < 8; ++j)
            if (same_parent(&f->leaf[i], &f->leaf[j])) members[nm++] = j;
        if (nm != nchild) continue;
        int ok = 1;
        for (int m = 0; m < nm; ++m)
            if (flags[members[m]] >= 0 || r[members[m]]) ok = 0;
        if (!ok) continue;
        for (int m = 0; m < nm; ++m) grp[members[m]] = i;
    }
    for (int changed = 1; changed;) {
        changed = 0;
        for (int i = 0; i < n; ++i) {
            if (grp[i] < 0) continue;
            int lvl = f->leaf[i].level;
            int bad = 0;
            for (int face = 0; face < nf && !bad; ++face) {
                const orc_face_nbr *fn = &f->fn[i * nf + face];
                for (int k = 0; k < fn->nn; ++k) {
                    int j = fn->nb[k];
                    if (grp[j] == grp[i]) continue;
                    int lj = f->leaf[j].level + r[j] - (grp[j] >= 0 ? 1 : 0);
                    if (lj > lvl) bad = 1;
                }
            }
            if (bad) {
                int g = grp[i];
                for (int j = 0; j < n; ++j)
                    if (grp[j] == g) grp[j] = -1;
                changed = 1;
            }
        }
    }
    /* new leaf list */
    free(f->new_leaf);
    f->new_leaf = malloc(sizeof(orc_key) * (size_t)n * nchild);
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const orc_key *k = &f->leaf[i];
        if (r[i]) {
            for (int c = 0; c < nchild; ++c) {
                orc_key ch = *k;
                ch.level = k->level + 1;
                for (int a = 0; a < 3; ++a)
                    ch.idx[a] = (a < f->dim) ? 2 * k->idx[a] + ((c >> a) & 1) : 0;
                f->new_leaf[m++] = ch;
            }
        } else if (grp[i] >= 0) {
            if (grp[i] == i) {
                orc_key pa = *k;
                pa.level = k->level - 1;
                for (int a = 0; a < 3; ++a) pa.idx[a] = k->idx[a] >> 1;
                f->new_leaf[m++] = pa;
            }
        } else {
            f->new_leaf[m++] = *k;
        }
    }
    orc_sort_leaves(f, f->new_leaf, m);
    f->new_n = m;
    free(r);
    free(grp);
    return m;
}

static int key_eq(const orc_key *a, const orc_key *b)
{
    return a->tree == b->tree && a->level == b->level && a->idx[0] == b->idx[0] &&
           a->idx[1] == b->idx[1] && a->idx[2] == b->idx[2];
}

/* defined in solver.c: L2 projection of one source cell's polynomial over
 * an overlap box into a destination cell's coefficients (accumulating) */
void orc_project_overlap(const orc_forest *f, const double *src, long src_stride,
                         const long *src_lo, long src_size, const long *dst_lo, long dst_size,
                         const long *olo, const long *ohi, int (*Qs)[3], int (*Qd)[3], double *acc);

/* Eq. 11-14: each new cell receives the L2 projection of the old piecewise
 * polynomial over its box; unchanged leaves are copied. */
void orc_apply_adapt(orc_forest *f, const double *u_old, double *u_new)
{
    int nc = orc_ncell(f), nv = f->nv, nb = f->nb;
    long per_leaf = (long)nv * nb * nc;
    int old_n = f->nleaves;
    orc_key *old = f->leaf;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < f->new_n; ++i) {
        const orc_key *k = &f->new_leaf[i];
        double *dst = u_new + i * per_leaf;
        int same = -1;
        for (int j = 0; j < old_n; ++j)
            if (key_eq(k, &old[j])) same = j;
        if (same >= 0) {
            memcpy(dst, u_old + same * per_leaf, sizeof(double) * per_leaf);
            continue;
        }
        memset(dst, 0, sizeof(double) * per_leaf);
        /* inheritance stays inside one tree: boxes in its local frame */
        long lo[3], size;
        orc_leaf_lbox(f, k, lo, &size);
        long h = size / f->N;
        for (int j = 0; j < old_n; ++j) {
            if (old[j].tree != k->tree) continue;
            long blo[3], bsize;
            orc_leaf_lbox(f, &old[j], blo, &bsize);
            int ok = 1;
            for (int a = 0; a < f->dim; ++a)
                if (!overlaps(lo[a], lo[a] + size, blo[a], blo[a] + bsize)) ok = 0;
            if (!ok) continue;
            long bh = bsize / f->N;
            for (int c = 0; c < nc; ++c) {
                int ijk[3];
                orc_cell_ijk(f, c, ijk);
                long clo[3] = {0, 0, 0};
                for (int a = 0; a < f->dim; ++a) clo[a] = lo[a] + ijk[a] * h;
                for (int sc = 0; sc < nc; ++sc) {
                    int sijk[3];
                    orc_cell_ijk(f, sc, sijk);
                    long slo[3] = {0, 0, 0}, olo[3] = {0, 0, 0}, ohi[3] = {0, 0, 0};
                    int ov = 1;
                    for (int a = 0; a < f->dim; ++a) {
                        slo[a] = blo[a] + sijk[a] * bh;
                        olo[a] = slo[a] > clo[a] ? slo[a] : clo[a];
                        ohi[a] = (slo[a] + bh) < (clo[a] + h) ? (slo[a] + bh) : (clo[a] + h);
                        if (olo[a] >= ohi[a]) ov = 0;
                    }
                    if (!ov) continue;
                    double acc[5 * 20];
                    memset(acc, 0, sizeof(acc));
                    orc_project_overlap(f, u_old + j * per_leaf + sc, nc, slo, bh, clo, h, olo, ohi, NULL, NULL, acc);
                    for (int v = 0; v < nv; ++v)
                        for (int l = 0; l < nb; ++l) dst[((long)v * nb + l) * nc + c] += acc[v * nb + l];
                }
            }
        }
    }
    orc_free_topology(f); /* sized by the old leaf count */
    free(f->leaf);
    f->leaf = f->new_leaf;
    f->nleaves = f->new_n;
    f->new_leaf = NULL;
    f->new_n = 0;
    orc_build_topology(f);
}
