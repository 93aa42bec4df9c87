/*
 * Oracle - basis, quadrature, inheritance operators, Euler and Rusanov
 * fluxes.  TEST INFRASTRUCTURE (see oracle.h).
 *
 * Basis (Sec. 2, "complete set of basis functions in P^K"): total-degree
 * products of unnormalised Legendre polynomials on the reference cell
 * [-1,1]^d, phi_m(xi) = prod_k P_{m_k}(xi_k), |m| <= p.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

/* Legendre polynomial by the three-term recurrence
 * (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}. */
double orc_legendre(int n, double x)
{
    if (n == 0) return 1.0;
    double pm = 1.0, pc = x;
    for (int k = 1; k < n; ++k) {
        double pn = ((2.0 * k + 1.0) * x * pc - k * pm) / (k + 1.0);
        pm = pc;
        pc = pn;
    }
    return pc;
}

/* Derivative via P'_{n+1} = P'_{n-1} + (2n+1) P_n, valid on all of [-1,1]. */
double orc_legendre_deriv(int n, double x)
{
    if (n == 0) return 0.0;
    double dm = 0.0, dc = 1.0; /* P'_0, P'_1 */
    for (int k = 1; k < n; ++k) {
        double dn = dm + (2.0 * k + 1.0) * orc_legendre(k, x);
        dm = dc;
        dc = dn;
    }
    return dc;
}

/* Gauss-Legendre nodes (ascending) and weights: roots of P_q by Newton
 * iteration from the Chebyshev-like guess, w = 2 / ((1-x^2) P'_q(x)^2). */
void orc_gauss_legendre(int q, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < q; ++i) {
        double z = cos(pi * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double dz = orc_legendre(q, z) / orc_legendre_deriv(q, z);
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        double d = orc_legendre_deriv(q, z);
        x[q - 1 - i] = z;
        w[q - 1 - i] = 2.0 / ((1.0 - z * z) * d * d);
    }
    if (q % 2 == 1) x[q / 2] = 0.0; /* the middle root is exactly zero */
}

int orc_num_modes(int dim, int p)
{
    int n = 0;
    for (int s = 0; s <= p; ++s)
        n += (dim == 2) ? (s + 1) : (s + 1) * (s + 2) / 2;
    return n;
}

/* Graded order: s = |m| ascending; inside s, m_x descending, then m_y
 * descending, m_z = s - m_x - m_y. */
void orc_mode_exponents(int dim, int p, int *exps)
{
    int n = 0;
    for (int s = 0; s <= p; ++s) {
        for (int mx = s; mx >= 0; --mx) {
            if (dim == 2) {
                exps[3 * n + 0] = mx;
                exps[3 * n + 1] = s - mx;
                exps[3 * n + 2] = 0;
                ++n;
            } else {
                for (int my = s - mx; my >= 0; --my) {
                    exps[3 * n + 0] = mx;
                    exps[3 * n + 1] = my;
                    exps[3 * n + 2] = s - mx - my;
                    ++n;
                }
            }
        }
    }
}

double orc_phi(int dim, const int *e, const double *xi)
{
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= orc_legendre(e[a], xi[a]);
    return v;
}

double orc_dphi(int dim, const int *e, const double *xi, int axis)
{
    double v = 1.0;
    for (int a = 0; a < dim; ++a)
        v *= (a == axis) ? orc_legendre_deriv(e[a], xi[a]) : orc_legendre(e[a], xi[a]);
    return v;
}

/* Reference mass of mode m: integral of phi_m^2 over [-1,1]^d. */
double orc_ref_mass(int dim, const int *e)
{
    double v = 1.0;
    for (int a = 0; a < dim; ++a) v *= 2.0 / (2.0 * e[a] + 1.0);
    return v;
}

/* Eq. 11-12: child coefficients K_C solve M_C K_C = int_{child} phi^C phi^P K_P.
 * Written out by tensor Gauss quadrature over the child cell (exact: the
 * integrand has degree <= 2p per axis).  The child cell is the half of the
 * parent with lower corner (bit_a(child) - 1)/... in parent coordinates. */
void orc_split_matrix(int dim, int p, int child, double *S)
{
    int nb = orc_num_modes(dim, p);
    int *ex = malloc(sizeof(int) * 3 * nb);
    orc_mode_exponents(dim, p, ex);
    int q = p + 1;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    memset(S, 0, sizeof(double) * nb * nb);
    int nq = 1;
    for (int a = 0; a < dim; ++a) nq *= q;
    for (int iq = 0; iq < nq; ++iq) {
        double xc[3] = {0, 0, 0}, xp[3] = {0, 0, 0}, w = 1.0;
        int rem = iq;
        for (int a = 0; a < dim; ++a) {
            int ia = rem % q;
            rem /= q;
            double s = ((child >> a) & 1) ? 0.5 : -0.5; /* child centre in parent coords */
            xc[a] = gx[ia];
            xp[a] = s + 0.5 * gx[ia];
            w *= gw[ia];
        }
        for (int l = 0; l < nb; ++l) {
            double pc = orc_phi(dim, ex + 3 * l, xc);
            for (int j = 0; j < nb; ++j)
                S[l * nb + j] += w * pc * orc_phi(dim, ex + 3 * j, xp);
        }
    }
    /* divide by the child reference mass (child Jacobian cancels on both sides) */
    for (int l = 0; l < nb; ++l) {
        double m = orc_ref_mass(dim, ex + 3 * l);
        for (int j = 0; j < nb; ++j) S[l * nb + j] /= m;
    }
    free(ex);
}

/* Eq. 13-14: M_P K_P = sum_i int_{Omega_i} phi^P phi^C K^C_i.  Matrix of the
 * contribution of child `child`: C[l][j] = int_{Omega_child} phi^P_l phi^C_j / M_P,l.
 * With |Omega_child| = 2^-d |Omega_P| the integral in child reference
 * coordinates carries a factor 2^-d. */
void orc_combine_matrix(int dim, int p, int child, double *C)
{
    int nb = orc_num_modes(dim, p);
    int *ex = malloc(sizeof(int) * 3 * nb);
    orc_mode_exponents(dim, p, ex);
    int q = p + 1;
    double gx[8], gw[8];
    orc_gauss_legendre(q, gx, gw);
    memset(C, 0, sizeof(double) * nb * nb);
    int nq = 1;
    for (int a = 0; a < dim; ++a) nq *= q;
    double jac = 1.0;
    for (int a = 0; a < dim; ++a) jac *= 0.5;
    for (int iq = 0; iq < nq; ++iq) {
        double xc[3] = {0, 0, 0}, xp[3] = {0, 0, 0}, w = 1.0;
        int rem = iq;
        for (int a = 0; a < dim; ++a) {
            int ia = rem % q;
            rem /= q;
            double s = ((child >> a) & 1) ? 0.5 : -0.5;
            xc[a] = gx[ia];
            xp[a] = s + 0.5 * gx[ia];
            w *= gw[ia];
        }
        for (int l = 0; l < nb; ++l) {
            double pp = orc_phi(dim, ex + 3 * l, xp);
            for (int j = 0; j < nb; ++j)
                C[l * nb + j] += jac * w * pp * orc_phi(dim, ex + 3 * j, xc);
        }
    }
    for (int l = 0; l < nb; ++l) {
        double m = orc_ref_mass(dim, ex + 3 * l);
        for (int j = 0; j < nb; ++j) C[l * nb + j] /= m;
    }
    free(ex);
}

/* Ideal-gas pressure, Eq. 23: p = (gamma-1) rho e, rho e = E - |rho u|^2/(2 rho). */
double orc_pressure(int dim, double gamma, const double *u)
{
    double ke = 0.0;
    for (int a = 0; a < dim; ++a) ke += u[1 + a] * u[1 + a];
    return (gamma - 1.0) * (u[dim + 1] - 0.5 * ke / u[0]);
}

/* Euler flux F_axis (Eq. 2 and its 3-D analogue):
 * (rho u_a, rho u_a u + p e_a, u_a (E + p)). */
void orc_euler_flux(int dim, double gamma, const double *u, int axis, double *f)
{
    double rho = u[0];
    double ua = u[1 + axis] / rho;
    double p = orc_pressure(dim, gamma, u);
    f[0] = u[1 + axis];
    for (int b = 0; b < dim; ++b) f[1 + b] = u[1 + b] * ua;
    f[1 + axis] += p;
    f[dim + 1] = ua * (u[dim + 1] + p);
}

/* Eq. 5 with the dissipative sign: for the outward normal n = sign*e_axis,
 * Fhat = 1/2 [ (F(U-) + F(U+)) . n - alpha (U+ - U-) ],
 * alpha = max(|u-.n| + c-, |u+.n| + c+) evaluated pointwise. */
void orc_rusanov(int dim, double gamma, const double *um, const double *up,
                 int axis, int sign, double *fhat)
{
    double fm[5], fp[5];
    orc_euler_flux(dim, gamma, um, axis, fm);
    orc_euler_flux(dim, gamma, up, axis, fp);
    double am = gamma * orc_pressure(dim, gamma, um) / um[0];
    double ap = gamma * orc_pressure(dim, gamma, up) / up[0];
    /* a trace with gamma p / rho < 0 enters with zero sound speed */
    double cm = sqrt(am > 0.0 ? am : 0.0);
    double cp = sqrt(ap > 0.0 ? ap : 0.0);
    double lm = fabs(um[1 + axis] / um[0]) + cm;
    double lp = fabs(up[1 + axis] / up[0]) + cp;
    double alpha = lm > lp ? lm : lp;
    int nv = dim + 2;
    for (int v = 0; v < nv; ++v)
        fhat[v] = 0.5 * ((double)sign * (fm[v] + fp[v]) - alpha * (up[v] - um[v]));
}

/* Sec. 5.1: F(u) = vel u.  The Rusanov flux with alpha = |vel . n| for the
 * outward normal n = sign*e_axis is the upwind flux:
 * Fhat = 1/2 [ vn (u- + u+) - |vn| (u+ - u-) ],  vn = sign*vel_axis. */
double orc_upwind(const double *vel, double um, double up, int axis, int sign)
{
    double vn = (double)sign * vel[axis];
    return 0.5 * (vn * (um + up) - fabs(vn) * (up - um));
}
