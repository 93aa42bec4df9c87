/*
 * Oracle - DG solver pieces: initial-condition projection, guard-cell fill
 * (Sec. 3.5, Eq. 15-17), residual of the Galerkin weak form (Sec. 2,
 * Eq. 3-5), SSP-RK3 (Sec. 2), CFL time step (Sec. 4.3), conserved totals,
 * positivity limiter (named in Sec. 5.3.2), block indicator and errors.
 * TEST INFRASTRUCTURE (see oracle.h).
 *
 * Everything is plain loops in FP64, in physical units, one cell at a time.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_internal.h"

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* physical length of one global unit along an axis */
static double unit_len(const orc_forest *f, int a)
{
    return (f->hi[a] - f->lo[a]) / (double)orc_domain_units(f, a);
}

/* physical cell edge of leaf i along its local axis a (the global axis the
 * root's frame maps it to) */
static double local_h(const orc_forest *f, int i, int a)
{
    int Q[3][3];
    orc_frame_matrix(f, f->leaf[i].tree, Q);
    long lo[3], size;
    orc_leaf_box(f, &f->leaf[i], lo, &size);
    for (int g = 0; g < f->dim; ++g)
        if (Q[g][a] != 0) return (size / f->N) * unit_len(f, g);
    return 0.0;
}

/* the vector components (momentum) of a state: global = Q local, local =
 * Q^T global; scalar equations have none */
static void rotate_state(const orc_forest *f, int Q[3][3], int transpose, double *u)
{
    if (f->equation != ORC_EQ_EULER) return;
    double m[3] = {0, 0, 0};
    for (int a = 0; a < f->dim; ++a)
        for (int b = 0; b < f->dim; ++b) m[a] += (transpose ? Q[b][a] : Q[a][b]) * u[1 + b];
    for (int a = 0; a < f->dim; ++a) u[1 + a] = m[a];
}

static long sidx(const orc_forest *f, long leaf, int v, int m, int cell)
{
    return ((leaf * f->nv + v) * f->nb + m) * (long)orc_ncell(f) + cell;
}

static long gidx(const orc_forest *f, long leaf, int face, int v, int m, int t)
{
    return (((leaf * 2 * f->dim + face) * f->nv + v) * f->nb + m) * (long)orc_nface_cells(f) + t;
}

/* evaluate the cell polynomial with coefficients coef[v*stride_v + m*stride_m]
 * at reference point xi */
/* ---------------------------------------------------------------- bilinear / trilinear blocks
 * Sec. 3.3, Eq. 6: with root grid nodes set, a root is the bilinear (3-D:
 * trilinear) image of the reference square (cube) spanned by its corner
 * nodes.  A leaf's cells are images of equal squares (cubes) of that
 * reference box, so each cell is the multilinear image of its own reference
 * cell [-1,1]^d with the images of its corners as nodes.  The weak form
 * (Eq. 3-4) is then evaluated with the Jacobian J = dx/dxi of that map at
 * every quadrature point: volume term sum_q w_q grad_xi phi_m . adj(J) F
 * (adj(J) = det(J) J^-1, the contravariant flux), face term
 * sum_f w_f |N| Fhat(U-, U+; N/|N|) phi_m with N = side * (row a of adj(J))
 * the outward normal scaled by the face Jacobian, and the full mass matrix
 * M_mn = sum_q w_q det(J) phi_m phi_n (exact with p+1 points per axis:
 * det(J) has degree d-1 per axis). */
static int mapped(const orc_forest *f) { return f->nodes != NULL; }

/* physical corners of cell c of leaf i; corner k has reference coordinate
 * -1 or +1 along axis a by bit a of k */
static void cell_corners(const orc_forest *f, int i, int c, double cx[8][3])
{
    const orc_key *k = &f->leaf[i];
    int d = f->dim, nk = 1 << d;
    long lo[3], size;
    orc_leaf_lbox(f, k, lo, &size);
    int ijk[3];
    orc_cell_ijk(f, c, ijk);
    long hu = size / f->N;
    int nx = f->roots[0] + 1, ny = f->roots[1] + 1;
    int r[3] = {k->tree % f->roots[0], (k->tree / f->roots[0]) % f->roots[1], k->tree / (f->roots[0] * f->roots[1])};
    /* a rotated root's local axis l runs along the node grid's axis a with
     * Q[a][l] != 0, reversed where Q[a][l] = -1 */
    int Q[3][3];
    orc_frame_matrix(f, k->tree, Q);
    for (int b = 0; b < nk; ++b) {
        double sl[3] = {0, 0, 0}, s[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) sl[a] = (double)(lo[a] + (ijk[a] + ((b >> a) & 1)) * hu) / (double)f->unit;
        for (int l = 0; l < d; ++l)
            for (int a = 0; a < d; ++a) {
                if (Q[a][l] == 1) s[a] = sl[l];
                if (Q[a][l] == -1) s[a] = 1.0 - sl[l];
            }
        for (int a = 0; a < 3; ++a) cx[b][a] = 0.0;
        /* the root's multilinear map at s */
        for (int n = 0; n < nk; ++n) {
            double wgt = 1.0;
            int node[3] = {r[0], r[1], r[2]};
            for (int a = 0; a < d; ++a) {
                int bit = (n >> a) & 1;
                wgt *= bit ? s[a] : 1.0 - s[a];
                node[a] += bit;
            }
            const double *xy = f->nodes + d * ((d == 3 ? node[2] * ny : 0) * nx + node[1] * nx + node[0]);
            for (int a = 0; a < d; ++a) cx[b][a] += wgt * xy[a];
        }
    }
}

/* x(xi) of the multilinear cell map */
static void map_point(const orc_forest *f, const double cx[8][3], const double *xi, double *x)
{
    int d = f->dim;
    for (int a = 0; a < 3; ++a) x[a] = 0.0;
    for (int b = 0; b < (1 << d); ++b) {
        double wgt = 1.0;
        for (int a = 0; a < d; ++a) wgt *= 0.5 * (1.0 + (((b >> a) & 1) ? xi[a] : -xi[a]));
        for (int a = 0; a < d; ++a) x[a] += wgt * cx[b][a];
    }
}

/* J[a][e] = dx_a / dxi_e of the multilinear cell map; returns det J */
static double map_jacobian(const orc_forest *f, const double cx[8][3], const double *xi, double J[3][3])
{
    int d = f->dim;
    for (int a = 0; a < 3; ++a)
        for (int e = 0; e < 3; ++e) J[a][e] = 0.0;
    for (int b = 0; b < (1 << d); ++b)
        for (int e = 0; e < d; ++e) {
            double wgt = ((b >> e) & 1) ? 0.5 : -0.5;
            for (int c = 0; c < d; ++c)
                if (c != e) wgt *= 0.5 * (1.0 + (((b >> c) & 1) ? xi[c] : -xi[c]));
            for (int a = 0; a < d; ++a) J[a][e] += wgt * cx[b][a];
        }
    if (d == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* row e of adj(J) = det(J) J^-1: the contravariant direction of xi_e */
static void adj_row(const orc_forest *f, double J[3][3], int e, double *r)
{
    if (f->dim == 2) {
        if (e == 0) { r[0] = J[1][1]; r[1] = -J[0][1]; }
        else { r[0] = -J[1][0]; r[1] = J[0][0]; }
        r[2] = 0.0;
        return;
    }
    /* adj[e][a] = cofactor of J[a][e] */
    for (int a = 0; a < 3; ++a) {
        int a1 = (a + 1) % 3, a2 = (a + 2) % 3, e1 = (e + 1) % 3, e2 = (e + 2) % 3;
        r[a] = J[a1][e1] * J[a2][e2] - J[a1][e2] * J[a2][e1];
    }
}

/* solve the symmetric positive definite n x n system M X = B for nrhs
 * right-hand sides (B is nrhs x n, overwritten) by Cholesky */
static void spd_solve(int n, const double *M, double *B, int nrhs)
{
    double L[20 * 20];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c <= r; ++c) {
            double s = M[r * n + c];
            for (int k = 0; k < c; ++k) s -= L[r * 20 + k] * L[c * 20 + k];
            L[r * 20 + c] = (r == c) ? sqrt(s) : s / L[c * 20 + c];
        }
    for (int j = 0; j < nrhs; ++j) {
        double *b = B + j * n;
        for (int r = 0; r < n; ++r) {
            double s = b[r];
            for (int k = 0; k < r; ++k) s -= L[r * 20 + k] * b[k];
            b[r] = s / L[r * 20 + r];
        }
        for (int r = n - 1; r >= 0; --r) {
            double s = b[r];
            for (int k = r + 1; k < n; ++k) s -= L[k * 20 + r] * b[k];
            b[r] = s / L[r * 20 + r];
        }
    }
}

/* mass matrix of cell c of leaf i with the volume rule (xi, w: nq points) */
static void mapped_mass(const orc_forest *f, int i, int c, int nq, double (*xi)[3], const double *w, double *M)
{
    double cx[8][3];
    cell_corners(f, i, c, cx);
    int nb = f->nb;
    for (int k = 0; k < nb * nb; ++k) M[k] = 0.0;
    for (int iq = 0; iq < nq; ++iq) {
        double J[3][3], det = map_jacobian(f, cx, xi[iq], J);
        double ph[20];
        for (int m = 0; m < nb; ++m) ph[m] = orc_phi(f->dim, f->exps + 3 * m, xi[iq]);
        for (int m = 0; m < nb; ++m)
            for (int n = 0; n < nb; ++n) M[m * nb + n] += w[iq] * det * ph[m] * ph[n];
    }
}

/* numerical flux along the outward unit normal n (Eq. 5): the Rusanov flux
 * with alpha = max(|u.n| + c) over both traces; for scalar convection the
 * same formula with alpha = |vel.n| is the upwind flux */
static void num_flux_n(const orc_forest *f, const double *um, const double *up, const double *n, double *fh)
{
    int d = f->dim, nv = f->nv;
    if (f->equation == ORC_EQ_ADVECTION) {
        double vn = 0.0;
        for (int a = 0; a < d; ++a) vn += f->vel[a] * n[a];
        fh[0] = 0.5 * (vn * (um[0] + up[0]) - fabs(vn) * (up[0] - um[0]));
        return;
    }
    double fm[5] = {0, 0, 0, 0, 0}, fp[5] = {0, 0, 0, 0, 0};
    double vm = 0.0, vp = 0.0;
    for (int a = 0; a < d; ++a) {
        double fa[5], fb[5];
        orc_euler_flux(d, f->gamma, um, a, fa);
        orc_euler_flux(d, f->gamma, up, a, fb);
        for (int v = 0; v < nv; ++v) {
            fm[v] += fa[v] * n[a];
            fp[v] += fb[v] * n[a];
        }
        vm += um[1 + a] * n[a];
        vp += up[1 + a] * n[a];
    }
    double am = f->gamma * orc_pressure(d, f->gamma, um) / um[0];
    double ap = f->gamma * orc_pressure(d, f->gamma, up) / up[0];
    double cm = sqrt(am > 0.0 ? am : 0.0), cp = sqrt(ap > 0.0 ? ap : 0.0);
    double lm = fabs(vm / um[0]) + cm, lp = fabs(vp / up[0]) + cp;
    double alpha = lm > lp ? lm : lp;
    for (int v = 0; v < nv; ++v) fh[v] = 0.5 * ((fm[v] + fp[v]) - alpha * (up[v] - um[v]));
}

static void eval_poly(const orc_forest *f, const double *coef, long stride_v, long stride_m,
                      const double *xi, double *u)
{
    for (int v = 0; v < f->nv; ++v) {
        double s = 0.0;
        for (int m = 0; m < f->nb; ++m) s += coef[v * stride_v + m * stride_m] * orc_phi(f->dim, f->exps + 3 * m, xi);
        u[v] = s;
    }
}

/* the same with the basis values at the point given (ph[m] = phi_m) */
static void eval_with(const orc_forest *f, const double *coef, long stride_v, long stride_m,
                      const double *ph, double *u)
{
    for (int v = 0; v < f->nv; ++v) {
        double s = 0.0;
        for (int m = 0; m < f->nb; ++m) s += coef[v * stride_v + m * stride_m] * ph[m];
        u[v] = s;
    }
}

/* Tensor Gauss points of an nq-per-axis rule over [-1,1]^dim. */
static int tensor_points(int dim, int q, const double *gx, const double *gw, double (*xi)[3], double *w)
{
    int n = 1;
    for (int a = 0; a < dim; ++a) n *= q;
    for (int i = 0; i < n; ++i) {
        int rem = i;
        w[i] = 1.0;
        xi[i][0] = xi[i][1] = xi[i][2] = 0.0;
        for (int a = 0; a < dim; ++a) {
            xi[i][a] = gx[rem % q];
            w[i] *= gw[rem % q];
            rem /= q;
        }
    }
    return n;
}

/* L2 projection (Eq. 11-14 written for one overlap piece, with the rotation
 * of Sec. 3.5): accumulate into acc[v*nb+l] the contribution
 * (1/M_dst,l) int_{overlap} phi^dst_l u^src dV for a source cell (global
 * lower corner src_lo, edge src_size) and a destination cell (dst_lo,
 * dst_size).  Each cell's polynomial lives in its root's local frame: a
 * point's reference coordinates in a cell are Q^T times those taken along
 * the global axes of its box, and the source state's momentum is turned
 * into the destination frame, Qd^T Qs m (Qs, Qd null: identity; on
 * bilinear roots the momentum is stored along the global axes and only the
 * coordinates turn).  src
 * points at coefficient (v=0,m=0) with modes src_stride apart and
 * variables nb*src_stride apart.  Gauss rule with p+1 points per axis on
 * the overlap box (exact: degree <= 2p per axis). */
void orc_project_overlap(const orc_forest *f, const double *src, long src_stride,
                         const long *src_lo, long src_size, const long *dst_lo, long dst_size,
                         const long *olo, const long *ohi, int (*Qs)[3], int (*Qd)[3], double *acc)
{
    int q = f->p + 1;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double xi[512][3], w[512];
    int nq = tensor_points(f->dim, q, gx, gw, xi, w);
    double frac = 1.0; /* |overlap| / |dst| */
    for (int a = 0; a < f->dim; ++a) frac *= (double)(ohi[a] - olo[a]) / (double)dst_size;
    for (int iq = 0; iq < nq; ++iq) {
        double xs[3] = {0, 0, 0}, xd[3] = {0, 0, 0};
        for (int a = 0; a < f->dim; ++a) {
            double x = olo[a] + 0.5 * (xi[iq][a] + 1.0) * (double)(ohi[a] - olo[a]);
            xs[a] = 2.0 * (x - src_lo[a]) / (double)src_size - 1.0;
            xd[a] = 2.0 * (x - dst_lo[a]) / (double)dst_size - 1.0;
        }
        if (Qs) { /* global-axis reference coordinates -> the cells' local ones */
            double t[3] = {0, 0, 0}, r[3] = {0, 0, 0};
            for (int a = 0; a < f->dim; ++a)
                for (int b = 0; b < f->dim; ++b) {
                    t[a] += Qs[b][a] * xs[b];
                    r[a] += Qd[b][a] * xd[b];
                }
            for (int a = 0; a < f->dim; ++a) {
                xs[a] = t[a];
                xd[a] = r[a];
            }
        }
        double u[5];
        eval_poly(f, src, (long)f->nb * src_stride, src_stride, xs, u);
        if (Qs && !mapped(f)) { /* bilinear roots keep the momentum along the global axes */
            rotate_state(f, Qs, 0, u);
            rotate_state(f, Qd, 1, u);
        }
        for (int l = 0; l < f->nb; ++l) {
            double ph = orc_phi(f->dim, f->exps + 3 * l, xd);
            double c = frac * w[iq] * ph / orc_ref_mass(f->dim, f->exps + 3 * l);
            for (int v = 0; v < f->nv; ++v) acc[v * f->nb + l] += c * u[v];
        }
    }
}

/* ---------------------------------------------------------------- initial conditions */

static void prim_to_cons(int dim, double gamma, double rho, const double *vel, double p, double *u)
{
    double ke = 0.0;
    u[0] = rho;
    for (int a = 0; a < dim; ++a) {
        u[1 + a] = rho * vel[a];
        ke += vel[a] * vel[a];
    }
    u[dim + 1] = p / (gamma - 1.0) + 0.5 * rho * ke;
}

static double wrap_half(double d, double period)
{
    if (period <= 0.0) return d;
    while (d >= 0.5 * period) d -= period;
    while (d < -0.5 * period) d += period;
    return d;
}

/* Physical flux along axis a: Euler (Eq. 2, 23) or scalar convection
 * (Sec. 5.1, F = vel u, vel the velocity along the axes a is taken on). */
static void phys_flux(const orc_forest *f, const double *vel, const double *u, int a, double *fl)
{
    if (f->equation == ORC_EQ_ADVECTION) fl[0] = vel[a] * u[0];
    else orc_euler_flux(f->dim, f->gamma, u, a, fl);
}

/* Numerical flux for the outward normal side*e_axis (Eq. 5). */
static void num_flux(const orc_forest *f, const double *vel, const double *um, const double *up, int axis, int side,
                     double *fh)
{
    if (f->equation == ORC_EQ_ADVECTION) fh[0] = orc_upwind(vel, um[0], up[0], axis, side);
    else orc_rusanov(f->dim, f->gamma, um, up, axis, side, fh);
}

/* the convection velocity along the local axes of leaf i's root,
 * Q^T vel (Sec. 3.1 frames; the identity on aligned roots) */
static void local_velocity(const orc_forest *f, int i, double *vl)
{
    int Q[3][3];
    orc_frame_matrix(f, f->leaf[i].tree, Q);
    for (int l = 0; l < 3; ++l) {
        vl[l] = 0.0;
        for (int a = 0; a < f->dim; ++a) vl[l] += Q[a][l] * f->vel[a];
    }
}

/* Analytic states used as initial conditions and exact solutions.
 *  VORTEX  params: eps, xc, yc, u_inf, v_inf, period_x, period_y
 *          isentropic vortex with mean (rho,u,v,p) = (1,u_inf,v_inf,1),
 *          translated by (u_inf,v_inf) t; 3-D: extruded along z, w = 0.
 *  SEDOV   params: p_ambient, p_centre, cx, cy, cz
 *          rho = 1, u = 0; p = p_centre inside the 2^d cells of the finest
 *          level that share the centre vertex, p_ambient elsewhere.
 *  UNIFORM params: rho, u, v, w, p
 *  XWAVE   params: amplitude, u, period_x
 *          rho = 1 + A sin(2 pi (x - u t)/Lx), velocity (u,0,0), p = 1:
 *          an exact entropy wave.
 *  COSINE  (scalar convection, Sec. 5.1) params: k, period_x, period_y,
 *          period_z; u = prod_a [cos(2 pi k (x_a - vel_a t)/L_a) - 1].
 *  EXP     (diffusion, Sec. 5.2) u = exp(a . x + nu |a|^2 t) with the
 *          forest's a and nu (params unused): an exact solution of
 *          u_t = nu div grad u. */
static void analytic_state(const orc_forest *f, int kind, const double *prm, double t,
                           const double *x, double *u)
{
    const double pi = 3.14159265358979323846;
    double g = f->gamma;
    double vel[3] = {0, 0, 0};
    if (kind == ORC_IC_EXP) {
        double e = 0.0, a2 = 0.0;
        for (int a = 0; a < f->dim; ++a) {
            e += f->avec[a] * x[a];
            a2 += f->avec[a] * f->avec[a];
        }
        u[0] = exp(e + f->nu * a2 * t);
        return;
    }
    if (kind == ORC_IC_COSINE) {
        double prod = 1.0;
        for (int a = 0; a < f->dim; ++a)
            prod *= cos(2.0 * pi * prm[0] * (x[a] - f->vel[a] * t) / prm[1 + a]) - 1.0;
        u[0] = prod;
        return;
    }
    if (kind == ORC_IC_VORTEX) {
        double eps = prm[0];
        double dx = wrap_half(x[0] - prm[1] - prm[3] * t, prm[5]);
        double dy = wrap_half(x[1] - prm[2] - prm[4] * t, prm[6]);
        double r2 = dx * dx + dy * dy;
        double e1 = exp(0.5 * (1.0 - r2));
        vel[0] = prm[3] - eps / (2.0 * pi) * e1 * dy;
        vel[1] = prm[4] + eps / (2.0 * pi) * e1 * dx;
        double T = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * pi * pi) * exp(1.0 - r2);
        double rho = pow(T, 1.0 / (g - 1.0));
        double p = pow(rho, g);
        prim_to_cons(f->dim, g, rho, vel, p, u);
    } else if (kind == ORC_IC_SEDOV) {
        int inside = 1;
        for (int a = 0; a < f->dim; ++a) {
            double hmin = unit_len(f, a); /* one global unit = finest cell edge */
            if (fabs(x[a] - prm[2 + a]) >= hmin) inside = 0;
        }
        prim_to_cons(f->dim, g, 1.0, vel, inside ? prm[1] : prm[0], u);
    } else if (kind == ORC_IC_UNIFORM) {
        for (int a = 0; a < f->dim; ++a) vel[a] = prm[1 + a];
        prim_to_cons(f->dim, g, prm[0], vel, prm[4], u);
    } else { /* XWAVE */
        double rho = 1.0 + prm[0] * sin(2.0 * pi * (x[0] - prm[1] * t) / prm[2]);
        vel[0] = prm[1];
        prim_to_cons(f->dim, g, rho, vel, 1.0, u);
    }
}

/* physical coordinates of the (local) reference point xi in cell c of
 * leaf i */
static void cell_point(const orc_forest *f, int i, int c, const double *xi, double *x)
{
    if (mapped(f)) {
        double cx[8][3];
        cell_corners(f, i, c, cx);
        map_point(f, cx, xi, x);
        return;
    }
    long lo[3], size;
    orc_leaf_box(f, &f->leaf[i], lo, &size);
    long h = size / f->N;
    int ijk[3], Q[3][3];
    orc_cell_ijk(f, c, ijk);
    orc_cell_gbox(f, &f->leaf[i], ijk, lo);
    orc_frame_matrix(f, f->leaf[i].tree, Q);
    for (int a = 0; a < 3; ++a) x[a] = 0.0;
    for (int a = 0; a < f->dim; ++a) {
        double xg = 0.0; /* reference coordinate along global axis a */
        for (int b = 0; b < f->dim; ++b) xg += Q[a][b] * xi[b];
        double gl = lo[a] + 0.5 * (xg + 1.0) * h;
        x[a] = f->lo[a] + gl * unit_len(f, a);
    }
}

/* the analytic state at the local reference point xi of cell c of leaf i,
 * in the leaf's frame (on bilinear roots the momentum stays along the
 * global axes) */
static void analytic_local(const orc_forest *f, int i, int c, int kind, const double *params, double t,
                           const double *xi, double *u)
{
    double x[3];
    cell_point(f, i, c, xi, x);
    analytic_state(f, kind, params, t, x, u);
    if (mapped(f)) return;
    int Q[3][3];
    orc_frame_matrix(f, f->leaf[i].tree, Q);
    rotate_state(f, Q, 1, u);
}

/* L2 projection of an analytic state with p+3 Gauss points per axis:
 * K_l = (1/M_l) int phi_l U0 dV. */
void orc_project_ic(const orc_forest *f, int kind, const double *params, double t, double *u)
{
    int q = f->p + 3, nc = orc_ncell(f);
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double (*xi)[3] = malloc(sizeof(double) * 3 * 512);
    double *w = malloc(sizeof(double) * 512);
    int nq = tensor_points(f->dim, q, gx, gw, xi, w);
    /* the volume rule (p+1 points per axis) for the mass matrix of bilinear cells */
    double vx[8], vwt[8];
    orc_gauss_legendre(f->q, vx, vwt);
    double (*vxi)[3] = malloc(sizeof(double) * 3 * 512);
    double *vw = malloc(sizeof(double) * 512);
    int nvq = tensor_points(f->dim, f->q, vx, vwt, vxi, vw);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i)
        for (int c = 0; c < nc; ++c) {
            double acc[5 * 20];
            memset(acc, 0, sizeof(acc));
            for (int iq = 0; iq < nq; ++iq) {
                double s[5];
                analytic_local(f, i, c, kind, params, t, xi[iq], s);
                for (int l = 0; l < f->nb; ++l) {
                    double ph = orc_phi(f->dim, f->exps + 3 * l, xi[iq]);
                    for (int v = 0; v < f->nv; ++v) acc[v * f->nb + l] += w[iq] * ph * s[v];
                }
            }
            if (mapped(f)) {
                /* M K = int phi U det(J) dxi, M with the volume rule */
                double cx[8][3], M[400];
                cell_corners(f, i, c, cx);
                memset(acc, 0, sizeof(acc));
                for (int iq = 0; iq < nq; ++iq) {
                    double s[5], J[3][3], det = map_jacobian(f, cx, xi[iq], J);
                    analytic_local(f, i, c, kind, params, t, xi[iq], s);
                    for (int l = 0; l < f->nb; ++l) {
                        double ph = orc_phi(f->dim, f->exps + 3 * l, xi[iq]);
                        for (int v = 0; v < f->nv; ++v) acc[v * f->nb + l] += w[iq] * det * ph * s[v];
                    }
                }
                mapped_mass(f, i, c, nvq, vxi, vw, M);
                spd_solve(f->nb, M, acc, f->nv);
                for (int v = 0; v < f->nv; ++v)
                    for (int l = 0; l < f->nb; ++l) u[sidx(f, i, v, l, c)] = acc[v * f->nb + l];
                continue;
            }
            /* |J| cancels between the mass matrix and the quadrature */
            for (int v = 0; v < f->nv; ++v)
                for (int l = 0; l < f->nb; ++l)
                    u[sidx(f, i, v, l, c)] = acc[v * f->nb + l] / orc_ref_mass(f->dim, f->exps + 3 * l);
        }
    free(xi);
    free(w);
    free(vxi);
    free(vw);
}

/* ---------------------------------------------------------------- guard fill */

/* index of the own cell at face (axis, side) and tangential index t */
static int face_cell(const orc_forest *f, int axis, int side, int t)
{
    int ijk[3] = {0, 0, 0}, n = 0;
    ijk[axis] = side > 0 ? f->N - 1 : 0;
    for (int b = 0; b < f->dim; ++b) {
        if (b == axis) continue;
        ijk[b] = (n == 0) ? t % f->N : t / f->N;
        ++n;
    }
    return orc_cell_index(f, ijk);
}

/* Sec. 3.5: each guard cell receives, from the stage input that is never
 * modified during the stage, the copy of the same-level neighbour cell
 * (Eq. 15), the split of the coarser neighbour cell (Eq. 16) or the combine
 * of the finer neighbour cells (Eq. 17), all with the identity rotation.
 * Outflow domain faces (Sec. 5.3.1) take the mirror image of the own cell,
 * K_m (-1)^{m_axis}, so that both face traces coincide. */
void orc_fill_guards(const orc_forest *f, const double *u, double *g)
{
    int nf = 2 * f->dim, nfc = orc_nface_cells(f), nc = orc_ncell(f);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i)
        for (int face = 0; face < nf; ++face) {
            int axis = face / 2, side = (face % 2) ? 1 : -1;
            for (int t = 0; t < nfc; ++t) {
                const orc_guard_plan *gp = &f->gp[((long)i * nf + face) * nfc + t];
                if (gp->kind == 2) {
                    int c = face_cell(f, axis, side, t);
                    for (int v = 0; v < f->nv; ++v)
                        for (int m = 0; m < f->nb; ++m) {
                            double sgn = (f->exps[3 * m + axis] % 2) ? -1.0 : 1.0;
                            g[gidx(f, i, face, v, m, t)] = sgn * u[sidx(f, i, v, m, c)];
                        }
                } else if (gp->kind == 0) {
                    const orc_piece *pc = &gp->piece[0];
                    for (int v = 0; v < f->nv; ++v)
                        for (int m = 0; m < f->nb; ++m)
                            g[gidx(f, i, face, v, m, t)] = u[sidx(f, pc->leaf, v, m, pc->cell)];
                } else {
                    /* the guard cell's global box (in the pieces' unwrapped
                     * frame): the own cell's box moved across the face */
                    long lo[3], size;
                    orc_leaf_box(f, &f->leaf[i], lo, &size);
                    long h = size / f->N;
                    int c = face_cell(f, axis, side, t);
                    int ijk[3], Qd[3][3];
                    orc_cell_ijk(f, c, ijk);
                    long glo[3] = {0, 0, 0};
                    orc_cell_gbox(f, &f->leaf[i], ijk, glo);
                    orc_frame_matrix(f, f->leaf[i].tree, Qd);
                    for (int a = 0; a < f->dim; ++a) glo[a] += side * Qd[a][axis] * h;
                    double acc[5 * 20];
                    memset(acc, 0, sizeof(acc));
                    for (int k = 0; k < gp->npiece; ++k) {
                        const orc_piece *pc = &gp->piece[k];
                        int Qs[3][3];
                        orc_frame_matrix(f, f->leaf[pc->leaf].tree, Qs);
                        orc_project_overlap(f, u + sidx(f, pc->leaf, 0, 0, pc->cell), nc, pc->src_lo,
                                            pc->src_size, glo, h, pc->lo, pc->hi, Qs, Qd, acc);
                    }
                    for (int v = 0; v < f->nv; ++v)
                        for (int m = 0; m < f->nb; ++m) g[gidx(f, i, face, v, m, t)] = acc[v * f->nb + m];
                }
            }
        }
}

/* ---------------------------------------------------------------- residual */

/* R = M^{-1} [ int_cell F . grad(phi) dV - int_{boundary} Fhat phi dS ]
 * (Eq. 3-4, source G = 0) for every cell of every leaf.  The neighbour
 * state across a face is the adjacent cell inside the block, or the guard
 * cell at the block boundary (Sec. 3.3).  With the conservative hanging
 * mode, a coarse cell facing finer neighbours integrates instead over the
 * fine sub-faces, using the fine cells' own traces (mortar). */
static void diffusion_residual(const orc_forest *f, const double *u, const double *g, double *r);

/* The residual on bilinear cells (see the bilinear block helpers above):
 * the same cell loop as orc_residual with the metric terms at every point
 * and the full mass matrix.  The neighbour across a face is the adjacent
 * cell of the leaf or the guard cell (Sec. 3.5: copy, split, combine in the
 * reference space); its trace is taken at the shared reference face point. */
static void mapped_residual(const orc_forest *f, const double *u, const double *g, double *r)
{
    int d = f->dim, nf = 2 * d, nfc = orc_nface_cells(f), nc = orc_ncell(f), q = f->q, nb = f->nb, nv = f->nv;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double (*vxi)[3] = malloc(sizeof(double) * 3 * 512);
    double *vw = malloc(sizeof(double) * 512);
    int nq = tensor_points(d, q, gx, gw, vxi, vw);
    double (*fxi)[3] = malloc(sizeof(double) * 3 * 64);
    double *fw = malloc(sizeof(double) * 64);
    int nfq = tensor_points(d - 1, q, gx, gw, fxi, fw);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i)
        for (int c = 0; c < nc; ++c) {
            int ijk[3];
            orc_cell_ijk(f, c, ijk);
            double cx[8][3];
            cell_corners(f, i, c, cx);
            const double *K = u + sidx(f, i, 0, 0, c);
            double acc[5 * 20];
            memset(acc, 0, sizeof(acc));
            /* volume: sum_q w_q grad_xi phi_m . adj(J) F(U_q) */
            for (int iq = 0; iq < nq; ++iq) {
                double uq[5], J[3][3], A[3][3];
                eval_poly(f, K, (long)nb * nc, nc, vxi[iq], uq);
                map_jacobian(f, cx, vxi[iq], J);
                for (int e = 0; e < d; ++e) adj_row(f, J, e, A[e]);
                double F[3][5];
                for (int a = 0; a < d; ++a) phys_flux(f, f->vel, uq, a, F[a]);
                for (int m = 0; m < nb; ++m)
                    for (int e = 0; e < d; ++e) {
                        double de = orc_dphi(d, f->exps + 3 * m, vxi[iq], e);
                        for (int v = 0; v < nv; ++v) {
                            double ce = 0.0;
                            for (int a = 0; a < d; ++a) ce += A[e][a] * F[a][v];
                            acc[v * nb + m] += vw[iq] * de * ce;
                        }
                    }
            }
            /* faces: - sum_f w_f |N| Fhat(U-, U+; N/|N|) phi_m */
            for (int face = 0; face < nf; ++face) {
                int axis = face / 2, side = (face % 2) ? 1 : -1;
                int nijk[3] = {ijk[0], ijk[1], ijk[2]};
                nijk[axis] += side;
                int interior = nijk[axis] >= 0 && nijk[axis] < f->N;
                int t = 0, mul = 1;
                for (int b = 0; b < d; ++b) {
                    if (b == axis) continue;
                    t += ijk[b] * mul;
                    mul *= f->N;
                }
                const double *Kn;
                long nsv, nsm;
                if (interior) {
                    Kn = u + sidx(f, i, 0, 0, orc_cell_index(f, nijk));
                    nsv = (long)nb * nc;
                    nsm = nc;
                } else {
                    Kn = g + gidx(f, i, face, 0, 0, t);
                    nsv = (long)nb * nfc;
                    nsm = nfc;
                }
                for (int iq = 0; iq < nfq; ++iq) {
                    double xo[3] = {0, 0, 0}, xn[3] = {0, 0, 0};
                    int n = 0;
                    for (int b = 0; b < d; ++b) {
                        if (b == axis) continue;
                        xo[b] = xn[b] = fxi[iq][n++];
                    }
                    xo[axis] = side;
                    xn[axis] = -side;
                    double J[3][3], N[3], um[5], up[5], fh[5] = {0, 0, 0, 0, 0};
                    map_jacobian(f, cx, xo, J);
                    adj_row(f, J, axis, N);
                    double len = 0.0;
                    for (int a = 0; a < d; ++a) {
                        N[a] *= side;
                        len += N[a] * N[a];
                    }
                    len = sqrt(len);
                    double nn[3] = {N[0] / len, N[1] / len, N[2] / len};
                    eval_poly(f, K, (long)nb * nc, nc, xo, um);
                    eval_poly(f, Kn, nsv, nsm, xn, up);
                    num_flux_n(f, um, up, nn, fh);
                    for (int m = 0; m < nb; ++m) {
                        double ph = orc_phi(d, f->exps + 3 * m, xo);
                        for (int v = 0; v < nv; ++v) acc[v * nb + m] -= fw[iq] * len * fh[v] * ph;
                    }
                }
            }
            double M[400];
            mapped_mass(f, i, c, nq, vxi, vw, M);
            spd_solve(nb, M, acc, nv);
            for (int v = 0; v < nv; ++v)
                for (int m = 0; m < nb; ++m) r[sidx(f, i, v, m, c)] = acc[v * nb + m];
        }
    free(vxi);
    free(vw);
    free(fxi);
    free(fw);
}

void orc_residual(const orc_forest *f, const double *u, const double *g, double *r)
{
    if (f->equation == ORC_EQ_DIFFUSION) {
        diffusion_residual(f, u, g, r);
        return;
    }
    if (mapped(f)) {
        mapped_residual(f, u, g, r);
        return;
    }
    int d = f->dim, nf = 2 * d, nfc = orc_nface_cells(f), nc = orc_ncell(f), q = f->q;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double (*vxi)[3] = malloc(sizeof(double) * 3 * 512);
    double *vw = malloc(sizeof(double) * 512);
    int nq = tensor_points(d, q, gx, gw, vxi, vw);
    double (*fxi)[3] = malloc(sizeof(double) * 3 * 64);
    double *fw = malloc(sizeof(double) * 64);
    int nfq = tensor_points(d - 1, q, gx, gw, fxi, fw);
    /* basis values at the volume points and at the face points seen from
     * both sides of every face */
    int nb = f->nb;
    double *vphi = malloc(sizeof(double) * nq * nb);
    double *vdphi = malloc(sizeof(double) * nq * d * nb);
    double *fown = malloc(sizeof(double) * nf * nfq * nb);
    double *fnbr = malloc(sizeof(double) * nf * nfq * nb);
    for (int iq = 0; iq < nq; ++iq)
        for (int m = 0; m < nb; ++m) {
            vphi[iq * nb + m] = orc_phi(d, f->exps + 3 * m, vxi[iq]);
            for (int a = 0; a < d; ++a) vdphi[(iq * d + a) * nb + m] = orc_dphi(d, f->exps + 3 * m, vxi[iq], a);
        }
    for (int face = 0; face < nf; ++face) {
        int axis = face / 2, side = (face % 2) ? 1 : -1;
        for (int iq = 0; iq < nfq; ++iq) {
            double xo[3] = {0, 0, 0}, xn[3] = {0, 0, 0};
            int n = 0;
            for (int b = 0; b < d; ++b) {
                if (b == axis) continue;
                xo[b] = xn[b] = fxi[iq][n++];
            }
            xo[axis] = side;
            xn[axis] = -side;
            for (int m = 0; m < nb; ++m) {
                fown[(face * nfq + iq) * nb + m] = orc_phi(d, f->exps + 3 * m, xo);
                fnbr[(face * nfq + iq) * nb + m] = orc_phi(d, f->exps + 3 * m, xn);
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &f->leaf[i], lo, &size);
        long hu = size / f->N;
        double h[3] = {1, 1, 1};
        for (int a = 0; a < d; ++a) h[a] = local_h(f, i, a); /* local axes */
        double vl[3];
        local_velocity(f, i, vl);
        double J = 1.0;
        for (int a = 0; a < d; ++a) J *= 0.5 * h[a];
        for (int c = 0; c < nc; ++c) {
            int ijk[3];
            orc_cell_ijk(f, c, ijk);
            const double *K = u + sidx(f, i, 0, 0, c);
            double acc[5 * 20];
            memset(acc, 0, sizeof(acc));
            /* volume integral */
            for (int iq = 0; iq < nq; ++iq) {
                double uq[5];
                eval_with(f, K, (long)f->nb * nc, nc, vphi + iq * nb, uq);
                for (int a = 0; a < d; ++a) {
                    double fl[5] = {0, 0, 0, 0, 0};
                    phys_flux(f, vl, uq, a, fl);
                    for (int m = 0; m < f->nb; ++m) {
                        double dp = vdphi[(iq * d + a) * nb + m] * 2.0 / h[a];
                        for (int v = 0; v < f->nv; ++v) acc[v * f->nb + m] += vw[iq] * J * fl[v] * dp;
                    }
                }
            }
            /* surface integrals */
            for (int face = 0; face < nf; ++face) {
                int axis = face / 2, side = (face % 2) ? 1 : -1;
                double Jf = 1.0;
                for (int b = 0; b < d; ++b)
                    if (b != axis) Jf *= 0.5 * h[b];
                int nijk[3] = {ijk[0], ijk[1], ijk[2]};
                nijk[axis] += side;
                int interior = nijk[axis] >= 0 && nijk[axis] < f->N;
                const orc_face_nbr *fn = &f->fn[i * nf + face];
                /* tangential index of this cell on the block face */
                int t = 0, mul = 1;
                for (int b = 0; b < d; ++b) {
                    if (b == axis) continue;
                    t += ijk[b] * mul;
                    mul *= f->N;
                }
                if (!interior && !fn->boundary && fn->level_diff == 1 && f->hanging == ORC_HANG_CONSERVATIVE) {
                    /* mortar over the fine cells that touch this face */
                    const orc_guard_plan *gp = &f->gp[((long)i * nf + face) * nfc + t];
                    long plane = (side > 0) ? lo[axis] + (ijk[axis] + 1) * hu : lo[axis] + ijk[axis] * hu;
                    long clo[3] = {0, 0, 0};
                    for (int a = 0; a < d; ++a) clo[a] = lo[a] + ijk[a] * hu;
                    for (int k = 0; k < gp->npiece; ++k) {
                        const orc_piece *pc = &gp->piece[k];
                        long touch = (side > 0) ? pc->src_lo[axis] : pc->src_lo[axis] + pc->src_size;
                        if (touch != plane) continue;
                        double Jff = 1.0;
                        for (int b = 0; b < d; ++b)
                            if (b != axis) Jff *= 0.5 * pc->src_size * unit_len(f, b);
                        const double *Kf = u + sidx(f, pc->leaf, 0, 0, pc->cell);
                        for (int iq = 0; iq < nfq; ++iq) {
                            double xo[3] = {0, 0, 0}, xf[3] = {0, 0, 0};
                            int n = 0;
                            for (int b = 0; b < d; ++b) {
                                if (b == axis) continue;
                                double gxp = pc->src_lo[b] + 0.5 * (fxi[iq][n] + 1.0) * pc->src_size;
                                xf[b] = fxi[iq][n];
                                xo[b] = 2.0 * (gxp - clo[b]) / (double)hu - 1.0;
                                ++n;
                            }
                            xo[axis] = side;
                            xf[axis] = -side;
                            double um[5], up[5], fh[5];
                            eval_poly(f, K, (long)f->nb * nc, nc, xo, um);
                            eval_poly(f, Kf, (long)f->nb * nc, nc, xf, up);
                            num_flux(f, vl, um, up, axis, side, fh);
                            for (int m = 0; m < f->nb; ++m) {
                                double ph = orc_phi(d, f->exps + 3 * m, xo);
                                for (int v = 0; v < f->nv; ++v) acc[v * f->nb + m] -= fw[iq] * Jff * fh[v] * ph;
                            }
                        }
                    }
                    continue;
                }
                const double *Kn;
                long nsv, nsm;
                if (interior) {
                    Kn = u + sidx(f, i, 0, 0, orc_cell_index(f, nijk));
                    nsv = (long)f->nb * nc;
                    nsm = nc;
                } else {
                    Kn = g + gidx(f, i, face, 0, 0, t);
                    nsv = (long)f->nb * nfc;
                    nsm = nfc;
                }
                for (int iq = 0; iq < nfq; ++iq) {
                    const double *po = fown + (face * nfq + iq) * nb;
                    double um[5], up[5], fh[5];
                    eval_with(f, K, (long)f->nb * nc, nc, po, um);
                    eval_with(f, Kn, nsv, nsm, fnbr + (face * nfq + iq) * nb, up);
                    num_flux(f, vl, um, up, axis, side, fh);
                    for (int m = 0; m < f->nb; ++m) {
                        double ph = po[m];
                        for (int v = 0; v < f->nv; ++v) acc[v * f->nb + m] -= fw[iq] * Jf * fh[v] * ph;
                    }
                }
            }
            for (int v = 0; v < f->nv; ++v)
                for (int m = 0; m < f->nb; ++m)
                    r[sidx(f, i, v, m, c)] = acc[v * f->nb + m] / (J * orc_ref_mass(d, f->exps + 3 * m));
        }
    }
    free(vxi);
    free(vw);
    free(fxi);
    free(fw);
    free(vphi);
    free(vdphi);
    free(fown);
    free(fnbr);
}

/* Diffusion equation u_t = nu div grad u (Sec. 5.2), symmetric interior
 * penalty DG (the IPDG method the paper cites), per cell K and mode m:
 *   M_m du_m/dt = nu [ - int_K grad u . grad phi_m dV
 *       + sum_{faces f of K} int_f ( {grad u} . n phi_m
 *                                   + 1/2 (u- - u+) grad phi_m . n
 *                                   - sigma (u- - u+) phi_m ) dS ]
 * with n the outward normal, u-/u+ the own and neighbour traces, {.} the
 * mean of both sides and sigma = 2 (p+1)^2 / h_n (h_n the cell edge along
 * n).  The neighbour is the adjacent cell inside the block or the guard
 * cell (Sec. 3.5: a cell of the own size).  A non-periodic face is a
 * Dirichlet face with data gD = the exact solution at the stage time:
 *   int_f ( grad u- . n phi_m + (u- - gD) grad phi_m . n - sigma (u- - gD) phi_m ) dS. */
static void diffusion_residual(const orc_forest *f, const double *u, const double *g, double *r)
{
    int d = f->dim, nf = 2 * d, nfc = orc_nface_cells(f), nc = orc_ncell(f), q = f->q, nb = f->nb;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double (*vxi)[3] = malloc(sizeof(double) * 3 * 512);
    double *vw = malloc(sizeof(double) * 512);
    int nq = tensor_points(d, q, gx, gw, vxi, vw);
    double (*fxi)[3] = malloc(sizeof(double) * 3 * 64);
    double *fw = malloc(sizeof(double) * 64);
    int nfq = tensor_points(d - 1, q, gx, gw, fxi, fw);
    /* reference derivatives at the volume points; values and normal
     * derivatives at the face points seen from the own side (xi_a = side)
     * and from the neighbour (xi_a = -side) */
    double *vd = malloc(sizeof(double) * nq * d * nb);
    double *fo = malloc(sizeof(double) * nf * nfq * nb), *fod = malloc(sizeof(double) * nf * nfq * nb);
    double *fn_ = malloc(sizeof(double) * nf * nfq * nb), *fnd = malloc(sizeof(double) * nf * nfq * nb);
    double (*fpt)[3] = malloc(sizeof(double) * 3 * nf * nfq);
    for (int iq = 0; iq < nq; ++iq)
        for (int a = 0; a < d; ++a)
            for (int m = 0; m < nb; ++m) vd[(iq * d + a) * nb + m] = orc_dphi(d, f->exps + 3 * m, vxi[iq], a);
    for (int face = 0; face < nf; ++face) {
        int axis = face / 2, side = (face % 2) ? 1 : -1;
        for (int iq = 0; iq < nfq; ++iq) {
            double xo[3] = {0, 0, 0}, xn[3] = {0, 0, 0};
            int n2 = 0;
            for (int b = 0; b < d; ++b) {
                if (b == axis) continue;
                xo[b] = xn[b] = fxi[iq][n2++];
            }
            xo[axis] = side;
            xn[axis] = -side;
            for (int a = 0; a < 3; ++a) fpt[face * nfq + iq][a] = xo[a];
            for (int m = 0; m < nb; ++m) {
                long k = ((long)face * nfq + iq) * nb + m;
                fo[k] = orc_phi(d, f->exps + 3 * m, xo);
                fod[k] = orc_dphi(d, f->exps + 3 * m, xo, axis);
                fn_[k] = orc_phi(d, f->exps + 3 * m, xn);
                fnd[k] = orc_dphi(d, f->exps + 3 * m, xn, axis);
            }
        }
    }
    double sig0 = 2.0 * (f->p + 1) * (f->p + 1);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &f->leaf[i], lo, &size);
        double h[3] = {1, 1, 1};
        for (int a = 0; a < d; ++a) h[a] = local_h(f, i, a); /* local axes */
        double J = 1.0;
        for (int a = 0; a < d; ++a) J *= 0.5 * h[a];
        for (int c = 0; c < nc; ++c) {
            int ijk[3];
            orc_cell_ijk(f, c, ijk);
            const double *K = u + sidx(f, i, 0, 0, c);
            double acc[20];
            memset(acc, 0, sizeof(acc));
            /* volume: - int grad u . grad phi_m */
            for (int iq = 0; iq < nq; ++iq) {
                double gu[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a)
                    for (int n = 0; n < nb; ++n) gu[a] += K[(long)n * nc] * vd[(iq * d + a) * nb + n] * 2.0 / h[a];
                for (int m = 0; m < nb; ++m)
                    for (int a = 0; a < d; ++a) acc[m] -= vw[iq] * J * gu[a] * vd[(iq * d + a) * nb + m] * 2.0 / h[a];
            }
            /* faces */
            for (int face = 0; face < nf; ++face) {
                int axis = face / 2, side = (face % 2) ? 1 : -1;
                double Jf = 1.0;
                for (int b = 0; b < d; ++b)
                    if (b != axis) Jf *= 0.5 * h[b];
                double sigma = sig0 / h[axis], s2 = 2.0 / h[axis];
                int nijk[3] = {ijk[0], ijk[1], ijk[2]};
                nijk[axis] += side;
                int interior = nijk[axis] >= 0 && nijk[axis] < f->N;
                const orc_face_nbr *fnb = &f->fn[i * nf + face];
                int dirichlet = !interior && fnb->boundary;
                int t = 0, mul = 1;
                for (int b = 0; b < d; ++b) {
                    if (b == axis) continue;
                    t += ijk[b] * mul;
                    mul *= f->N;
                }
                const double *Kn = NULL;
                long nsm = 0;
                if (interior) {
                    Kn = u + sidx(f, i, 0, 0, orc_cell_index(f, nijk));
                    nsm = nc;
                } else if (!dirichlet) {
                    Kn = g + gidx(f, i, face, 0, 0, t);
                    nsm = nfc;
                }
                for (int iq = 0; iq < nfq; ++iq) {
                    long k0 = ((long)face * nfq + iq) * nb;
                    /* own trace and normal derivative d/dx_axis */
                    double um = 0.0, gm = 0.0;
                    for (int n = 0; n < nb; ++n) {
                        um += K[(long)n * nc] * fo[k0 + n];
                        gm += K[(long)n * nc] * fod[k0 + n] * s2;
                    }
                    double up = 0.0, gn = 0.0;
                    if (dirichlet) {
                        double x[3], ex[5];
                        cell_point(f, i, c, fpt[face * nfq + iq], x);
                        analytic_state(f, ORC_IC_EXP, NULL, f->stage_time, x, ex);
                        up = ex[0];
                    } else {
                        for (int n = 0; n < nb; ++n) {
                            up += Kn[(long)n * nsm] * fn_[k0 + n];
                            gn += Kn[(long)n * nsm] * fnd[k0 + n] * s2;
                        }
                    }
                    /* {grad u} . n; a Dirichlet face takes the own gradient */
                    double flux_n = side * (dirichlet ? gm : 0.5 * (gm + gn));
                    double jump = um - up;
                    double wsym = dirichlet ? 1.0 : 0.5;
                    for (int m = 0; m < nb; ++m) {
                        double dn = side * fod[k0 + m] * s2;
                        acc[m] += fw[iq] * Jf * (flux_n * fo[k0 + m] + wsym * jump * dn - sigma * jump * fo[k0 + m]);
                    }
                }
            }
            for (int m = 0; m < nb; ++m)
                r[sidx(f, i, 0, m, c)] = f->nu * acc[m] / (J * orc_ref_mass(d, f->exps + 3 * m));
        }
    }
    free(vxi);
    free(vw);
    free(fxi);
    free(fw);
    free(vd);
    free(fo);
    free(fod);
    free(fn_);
    free(fnd);
    free(fpt);
}

/* ---------------------------------------------------------------- time stepping */

/* Shu-Osher SSP-RK3 (Sec. 2, third order per Sec. 5.1):
 *   U1   = Un + dt R(Un)
 *   U2   = 3/4 Un + 1/4 (U1 + dt R(U1))
 *   Un+1 = 1/3 Un + 2/3 (U2 + dt R(U2))
 * stage s computes a_s Un + b_s (Us + dt R(Us)). */
void orc_rk_combine(long n, int stage, double dt, const double *un, const double *us,
                    const double *r, double *unext)
{
    double a = (stage == 0) ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
    double b = (stage == 0) ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) unext[k] = a * un[k] + b * (us[k] + dt * r[k]);
}

/* Largest sum over axes of (|mean u_a| + mean c) / h_a over all cells,
 * from the cell means (mode 0). */
static double mapped_max_rate(const orc_forest *f, const double *u);

double orc_max_rate(const orc_forest *f, const double *u)
{
    if (mapped(f)) return mapped_max_rate(f, u);
    int d = f->dim, nc = orc_ncell(f);
    double mx = 0.0;
    for (int i = 0; i < f->nleaves; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &f->leaf[i], lo, &size);
        if (f->equation == ORC_EQ_DIFFUSION) { /* nu sum_a 1 / h_a^2 */
            double rate = 0.0;
            for (int a = 0; a < d; ++a) {
                double h = (size / f->N) * unit_len(f, a);
                rate += f->nu / (h * h);
            }
            if (rate > mx) mx = rate;
            continue;
        }
        if (f->equation == ORC_EQ_ADVECTION) { /* sum_a |vel_a| / h_a */
            double rate = 0.0;
            for (int a = 0; a < d; ++a) rate += fabs(f->vel[a]) / ((size / f->N) * unit_len(f, a));
            if (rate > mx) mx = rate;
            continue;
        }
        for (int c = 0; c < nc; ++c) {
            double s[5];
            for (int v = 0; v < f->nv; ++v) s[v] = u[sidx(f, i, v, 0, c)];
            double cs = sqrt(f->gamma * orc_pressure(d, f->gamma, s) / s[0]);
            double rate = 0.0;
            for (int a = 0; a < d; ++a) rate += (fabs(s[1 + a] / s[0]) + cs) / local_h(f, i, a);
            if (rate > mx) mx = rate;
        }
    }
    return mx;
}

/* The rate on bilinear cells: the cell means of the state (integrals over
 * the physical cell with the volume rule, divided by its area), and for
 * each reference axis b the unit normal n_b and the width h_b = 2 det(J) /
 * |row b of adj(J)| at the cell centre (the edge lengths for a rectangle):
 * sum_b (|u.n_b| + c) / h_b; scalar convection sum_b |vel.n_b| / h_b. */
static double mapped_max_rate(const orc_forest *f, const double *u)
{
    int d = f->dim, nc = orc_ncell(f), nb = f->nb;
    double gx[8], gw[8];
    orc_gauss_legendre(f->q, gx, gw);
    double (*xi)[3] = malloc(sizeof(double) * 3 * 512);
    double *w = malloc(sizeof(double) * 512);
    int nq = tensor_points(d, f->q, gx, gw, xi, w);
    double mx = 0.0;
    for (int i = 0; i < f->nleaves; ++i)
        for (int c = 0; c < nc; ++c) {
            double cx[8][3], J[3][3];
            cell_corners(f, i, c, cx);
            double s[5] = {0, 0, 0, 0, 0}, vol = 0.0;
            for (int iq = 0; iq < nq; ++iq) {
                double det = map_jacobian(f, cx, xi[iq], J), uq[5];
                eval_poly(f, u + sidx(f, i, 0, 0, c), (long)nb * nc, nc, xi[iq], uq);
                vol += w[iq] * det;
                for (int v = 0; v < f->nv; ++v) s[v] += w[iq] * det * uq[v];
            }
            for (int v = 0; v < f->nv; ++v) s[v] /= vol;
            const double x0[3] = {0, 0, 0};
            double det0 = map_jacobian(f, cx, x0, J);
            double cs = f->equation == ORC_EQ_ADVECTION ? 0.0 : sqrt(f->gamma * orc_pressure(d, f->gamma, s) / s[0]);
            double rate = 0.0;
            for (int b = 0; b < d; ++b) {
                double A[3];
                adj_row(f, J, b, A);
                double len = 0.0;
                for (int a = 0; a < d; ++a) len += A[a] * A[a];
                len = sqrt(len);
                double h = 2.0 * det0 / len, un = 0.0;
                for (int a = 0; a < d; ++a)
                    un += (f->equation == ORC_EQ_ADVECTION ? f->vel[a] : s[1 + a] / s[0]) * A[a] / len;
                rate += (fabs(un) + cs) / h;
            }
            if (rate > mx) mx = rate;
        }
    free(xi);
    free(w);
    return mx;
}

/* Sec. 4.3 step 2(a): critical time increment over all blocks,
 * dt = CFL / max_cells sum_a (|u_a| + c) / h_a. */
double orc_dt(const orc_forest *f, const double *u, double cfl) { return cfl / orc_max_rate(f, u); }

/* T_v = sum over cells of |cell| * mean_v, leaf by leaf, cell by cell (the
 * momentum along the global axes). */
void orc_totals(const orc_forest *f, const double *u, double *totals)
{
    int nc = orc_ncell(f);
    for (int v = 0; v < f->nv; ++v) totals[v] = 0.0;
    if (mapped(f)) { /* sum over cells of the integral of U over the physical cell */
        double gx[8], gw[8];
        orc_gauss_legendre(f->q, gx, gw);
        double (*xi)[3] = malloc(sizeof(double) * 3 * 512);
        double *w = malloc(sizeof(double) * 512);
        int nq = tensor_points(f->dim, f->q, gx, gw, xi, w);
        for (int i = 0; i < f->nleaves; ++i)
            for (int c = 0; c < nc; ++c) {
                double cx[8][3], J[3][3], m[5] = {0, 0, 0, 0, 0};
                cell_corners(f, i, c, cx);
                for (int iq = 0; iq < nq; ++iq) {
                    double det = map_jacobian(f, cx, xi[iq], J), uq[5];
                    eval_poly(f, u + sidx(f, i, 0, 0, c), (long)f->nb * nc, nc, xi[iq], uq);
                    for (int v = 0; v < f->nv; ++v) m[v] += w[iq] * det * uq[v];
                }
                for (int v = 0; v < f->nv; ++v) totals[v] += m[v];
            }
        free(xi);
        free(w);
        return;
    }
    for (int i = 0; i < f->nleaves; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &f->leaf[i], lo, &size);
        double vol = 1.0;
        for (int a = 0; a < f->dim; ++a) vol *= (size / f->N) * unit_len(f, a);
        int Q[3][3];
        orc_frame_matrix(f, f->leaf[i].tree, Q);
        for (int c = 0; c < nc; ++c) {
            double m[5] = {0, 0, 0, 0, 0};
            for (int v = 0; v < f->nv; ++v) m[v] = u[sidx(f, i, v, 0, c)];
            rotate_state(f, Q, 0, m); /* momentum along the global axes */
            for (int v = 0; v < f->nv; ++v) totals[v] += vol * m[v];
        }
    }
}

/* Gauss-Lobatto nodes on [-1,1] with L points (L = 2, 3, 4): the end
 * points and the roots of P'_{L-1}, closed forms. */
static int lobatto_nodes(int L, double *x)
{
    if (L == 2) { x[0] = -1.0; x[1] = 1.0; }
    else if (L == 3) { x[0] = -1.0; x[1] = 0.0; x[2] = 1.0; }
    else { x[0] = -1.0; x[1] = -1.0 / sqrt(5.0); x[2] = 1.0 / sqrt(5.0); x[3] = 1.0; L = 4; }
    return L;
}

/* Positivity-preserving scaling limiter of Zhang and Shu (the paper's
 * references for the positivity limiter), written from the published
 * method.  The point set S is Zhang and Shu's for tensor cells: for every
 * axis a, the points whose a-coordinate is a node of the L-point
 * Gauss-Lobatto rule and whose other coordinates are nodes of the (p+1)-point
 * Gauss rule, with L the smallest number of points such that the Lobatto
 * rule is exact for degree p (2L - 3 >= p, L >= 2).  The cell mean is a
 * convex combination of the values at S (their positivity is what the
 * positivity of the next cell means needs); S contains the face Gauss
 * points.  The volume Gauss points, where the volume integral evaluates the
 * flux, are added to S.  For each cell, with eps = min(1e-13, mean rho,
 * p(mean)):
 *   1. theta1 = min(1, (rho_mean - eps)/(rho_mean - min_S rho)); the
 *      non-mean density modes are scaled by theta1;
 *   2. for every point of S with p(U) < eps, t = (pbar - eps)/(pbar - p(U)),
 *      where the chord from (0, pbar) to (1, p(U)) reaches eps; pressure
 *      is a concave function of the conserved variables where rho > 0, so
 *      p(Ubar + t (U - Ubar)) >= eps there (the chord bound instead of the
 *      exact root of the quadratic p(Ubar + t (U - Ubar)) = eps: the root
 *      takes a square root of a discriminant that vanishes when the
 *      pressure along the segment touches eps, where rounding of order
 *      u becomes sqrt(u) in t; the chord is Lipschitz in the state);
 *      theta2 = min t (1 where p >= eps); all non-mean modes are scaled by
 *      theta2.  Cell means are unchanged.
 * On bilinear / trilinear roots the mean is the one over the physical cell,
 * Ubar = int U |J| / int |J| with the volume rule, which differs from the
 * mode-0 coefficient; each scaling is then U <- Ubar + theta (U - Ubar),
 * which (phi_0 = 1) also moves mode 0 and keeps the physical mean. */
void orc_limit_positivity(const orc_forest *f, double *u)
{
    if (f->equation != ORC_EQ_EULER) return; /* density and pressure only exist for Euler */
    int d = f->dim, nc = orc_ncell(f), q = f->q, nv = f->nv;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    int L = 2;
    while (2 * L - 3 < f->p) ++L;
    double lx[4];
    L = lobatto_nodes(L, lx);
    int nq = 1, nfq = 1;
    for (int a = 0; a < d; ++a) nq *= q;
    for (int a = 0; a < d - 1; ++a) nfq *= q;
    int npts = nq + d * L * nfq;
    double (*pts)[3] = malloc(sizeof(double) * 3 * npts);
    int np = 0;
    /* volume Gauss points */
    for (int k = 0; k < nq; ++k) {
        int rem = k;
        pts[np][0] = pts[np][1] = pts[np][2] = 0.0;
        for (int a = 0; a < d; ++a) {
            pts[np][a] = gx[rem % q];
            rem /= q;
        }
        ++np;
    }
    /* Zhang-Shu points: Lobatto along axis a, Gauss along the others */
    for (int a = 0; a < d; ++a)
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < nfq; ++k) {
                int rem = k;
                pts[np][0] = pts[np][1] = pts[np][2] = 0.0;
                for (int b = 0; b < d; ++b) {
                    if (b == a) {
                        pts[np][b] = lx[l];
                    } else {
                        pts[np][b] = gx[rem % q];
                        rem /= q;
                    }
                }
                ++np;
            }
    double g = f->gamma;
    /* the volume rule, for the physical mean of bilinear / trilinear cells */
    double (*vxi)[3] = malloc(sizeof(double) * 3 * 512);
    double *vw = malloc(sizeof(double) * 512);
    int nvq = tensor_points(d, q, gx, gw, vxi, vw);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f->nleaves; ++i)
        for (int c = 0; c < nc; ++c) {
            double *K = u + sidx(f, i, 0, 0, c);
            long sv = (long)f->nb * nc, sm = nc;
            double mean[5];
            for (int v = 0; v < nv; ++v) mean[v] = K[v * sv];
            if (mapped(f)) {
                double cx[8][3], vol = 0.0, acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                cell_corners(f, i, c, cx);
                for (int iq = 0; iq < nvq; ++iq) {
                    double J[3][3], det = map_jacobian(f, cx, vxi[iq], J), uq[5];
                    eval_poly(f, K, sv, sm, vxi[iq], uq);
                    vol += vw[iq] * det;
                    for (int v = 0; v < nv; ++v) acc[v] += vw[iq] * det * uq[v];
                }
                for (int v = 0; v < nv; ++v) mean[v] = acc[v] / vol;
            }
            double pbar = orc_pressure(d, g, mean);
            double eps = 1e-13;
            if (mean[0] < eps) eps = mean[0];
            if (pbar < eps) eps = pbar;
            /* density */
            double rmin = mean[0];
            for (int k = 0; k < npts; ++k) {
                double uq[5];
                eval_poly(f, K, sv, sm, pts[k], uq);
                if (uq[0] < rmin) rmin = uq[0];
            }
            double th1 = 1.0;
            if (rmin < mean[0]) {
                th1 = (mean[0] - eps) / (mean[0] - rmin);
                if (th1 > 1.0) th1 = 1.0;
            }
            if (th1 < 1.0) {
                for (int m = 1; m < f->nb; ++m) K[m * sm] *= th1;
                if (mapped(f)) K[0] = mean[0] + th1 * (K[0] - mean[0]);
            }
            /* pressure */
            double th2 = 1.0;
            for (int k = 0; k < npts; ++k) {
                double uq[5];
                eval_poly(f, K, sv, sm, pts[k], uq);
                double pq = orc_pressure(d, g, uq);
                if (pq >= eps) continue;
                /* p is concave in U where rho > 0, so along the segment
                 * p(Ubar + t (U - Ubar)) >= (1 - t) pbar + t p(U): the
                 * chord reaches eps at t = (pbar - eps) / (pbar - p(U)) */
                double t = (pbar - eps) / (pbar - pq);
                if (t > 1.0) t = 1.0;
                if (t < 0.0) t = 0.0;
                if (t < th2) th2 = t;
            }
            if (th2 < 1.0)
                for (int v = 0; v < nv; ++v) {
                    for (int m = 1; m < f->nb; ++m) K[v * sv + m * sm] *= th2;
                    if (mapped(f)) K[v * sv] = mean[v] + th2 * (K[v * sv] - mean[v]);
                }
        }
    free(pts);
    free(vxi);
    free(vw);
}

/* Block indicator: ratio of the largest to the smallest density cell mean
 * over the block's cells and its face guard cells. */
void orc_indicator(const orc_forest *f, const double *u, double *eta)
{
    int nc = orc_ncell(f), nfc = orc_nface_cells(f);
    double *g = malloc(sizeof(double) * orc_guard_len(f));
    orc_fill_guards(f, u, g);
    for (int i = 0; i < f->nleaves; ++i) {
        double mx = -1e300, mn = 1e300;
        for (int c = 0; c < nc; ++c) {
            double r = u[sidx(f, i, 0, 0, c)];
            if (r > mx) mx = r;
            if (r < mn) mn = r;
        }
        for (int face = 0; face < 2 * f->dim; ++face)
            for (int t = 0; t < nfc; ++t) {
                double r = g[gidx(f, i, face, 0, 0, t)];
                if (r > mx) mx = r;
                if (r < mn) mn = r;
            }
        /* Euler: density ratio over the block and its face guards; scalar
         * convection and diffusion (Sec. 5.1, 5.2): the largest cell
         * average there */
        eta[i] = f->equation == ORC_EQ_EULER ? mx / mn : mx;
    }
    free(g);
}

double orc_step(const orc_forest *f, double cfl, double dt_fixed, int limiter, double *u)
{
    long n = orc_state_len(f);
    double dt = dt_fixed > 0.0 ? dt_fixed : orc_dt(f, u, cfl);
    double *un = malloc(sizeof(double) * n);
    double *us = malloc(sizeof(double) * n);
    double *r = malloc(sizeof(double) * n);
    double *g = malloc(sizeof(double) * orc_guard_len(f));
    memcpy(un, u, sizeof(double) * n);
    memcpy(us, u, sizeof(double) * n);
    /* stage input times of SSP-RK3: t, t + dt, t + dt/2 (Dirichlet data) */
    const double ct[3] = {0.0, 1.0, 0.5};
    orc_forest *fm = (orc_forest *)f;
    for (int s = 0; s < 3; ++s) {
        fm->stage_time = f->time + ct[s] * dt;
        orc_fill_guards(f, us, g);
        orc_residual(f, us, g, r);
        orc_rk_combine(n, s, dt, un, us, r, u);
        if (limiter) orc_limit_positivity(f, u);
        memcpy(us, u, sizeof(double) * n);
    }
    fm->time += dt;
    fm->stage_time = fm->time;
    free(un);
    free(us);
    free(r);
    free(g);
    return dt;
}

void orc_errors(const orc_forest *f, const double *u, int kind, const double *params, double t,
                double *l1, double *l2)
{
    int q = f->p + 3, nc = orc_ncell(f);
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    double (*xi)[3] = malloc(sizeof(double) * 3 * 512);
    double *w = malloc(sizeof(double) * 512);
    int nq = tensor_points(f->dim, q, gx, gw, xi, w);
    for (int v = 0; v < f->nv; ++v) l1[v] = l2[v] = 0.0;
    for (int i = 0; i < f->nleaves; ++i) {
        long lo[3], size;
        orc_leaf_box(f, &f->leaf[i], lo, &size);
        double J = 1.0;
        for (int a = 0; a < f->dim; ++a) J *= 0.5 * (size / f->N) * unit_len(f, a);
        for (int c = 0; c < nc; ++c)
            for (int iq = 0; iq < nq; ++iq) {
                double ex[5], uh[5];
                if (mapped(f)) {
                    double cx[8][3], Jm[3][3];
                    cell_corners(f, i, c, cx);
                    J = map_jacobian(f, cx, xi[iq], Jm);
                }
                analytic_local(f, i, c, kind, params, t, xi[iq], ex);
                eval_poly(f, u + sidx(f, i, 0, 0, c), (long)f->nb * nc, nc, xi[iq], uh);
                for (int v = 0; v < f->nv; ++v) {
                    double e = uh[v] - ex[v];
                    l1[v] += w[iq] * J * fabs(e);
                    l2[v] += w[iq] * J * e * e;
                }
            }
    }
    for (int v = 0; v < f->nv; ++v) l2[v] = sqrt(l2[v]);
    free(xi);
    free(w);
}
