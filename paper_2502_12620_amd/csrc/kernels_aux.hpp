// Auxiliary HIP kernels: positivity limiter, block indicator, analytic
// initial-condition projection and L2 inheritance on refinement.
#pragma once

#include "kernels.hpp"  // split_any

namespace dgk {

template <int D, int P>
__global__ __launch_bounds__(256) void k_limit(double *u, int N, long ncell_total, double gamma)
{
    constexpr int NV = D + 2, NB = Tab<D, P>::NB;
    const int ncell = D == 2 ? N * N : N * N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const long leaf = gid / ncell;
    const int c = int(gid % ncell);
    const long sv = long(NB) * ncell, base = leaf * NV * sv + c;
    double K[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) K[v][m] = u[base + v * sv + m * ncell];
    limit_cell<D, P>(K, gamma);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 1; m < NB; ++m) u[base + v * sv + m * ncell] = K[v][m];
}

// ------------------------------------------------------------------ initial conditions
// Analytic states (same definitions as the test workloads):
//  VORTEX  eps, xc, yc, u_inf, v_inf, period_x, period_y: isentropic vortex
//          with mean (rho,u,v,p) = (1,u_inf,v_inf,1), extruded in 3-D
//  SEDOV   p_ambient, p_centre, cx, cy, cz: rho = 1, u = 0, p = p_centre
//          within one finest cell edge of the centre along every axis
//  UNIFORM rho, u, v, w, p
//  XWAVE   amplitude, u, period_x: rho = 1 + A sin(2 pi (x - u t)/Lx),
//          velocity (u,0,0), p = 1
//  COSINE  (scalar convection, Sec. 5.1) k, period_x, period_y, period_z,
//          vel_x, vel_y, vel_z: u = prod_a [cos(2 pi k (x_a - vel_a t)/L_a) - 1]
//  EXP     (diffusion, Sec. 5.2) a_x, a_y, a_z, nu: u = exp(a . x + nu |a|^2 t)
__device__ __forceinline__ double wrap_half(double d, double period)
{
    if (period <= 0.0) return d;
    while (d >= 0.5 * period) d -= period;
    while (d < -0.5 * period) d += period;
    return d;
}

template <int D>
__device__ void analytic(int kind, const IcParams &P, double t, double gamma, const double *x, const double *hmin,
                         double *U)
{
    const double pi = 3.14159265358979323846;
    double vel[3] = {0.0, 0.0, 0.0}, rho = 1.0, p = 1.0;
    if (kind == DGAMR_IC_EXP) { // diffusion (Sec. 5.2): a = p[0..2], nu = p[3]
        double e = 0.0, a2 = 0.0;
        for (int a = 0; a < D; ++a) {
            e += P.p[a] * x[a];
            a2 += P.p[a] * P.p[a];
        }
        U[0] = exp(e + P.p[3] * a2 * t);
        return;
    }
    if (kind == DGAMR_IC_COSINE) {
        double prod = 1.0;
        for (int a = 0; a < D; ++a) prod *= cos(2.0 * pi * P.p[0] * (x[a] - P.p[4 + a] * t) / P.p[1 + a]) - 1.0;
        U[0] = prod;
        return;
    }
    if (kind == DGAMR_IC_VORTEX) {
        double eps = P.p[0];
        double dx = wrap_half(x[0] - P.p[1] - P.p[3] * t, P.p[5]);
        double dy = wrap_half(x[1] - P.p[2] - P.p[4] * t, P.p[6]);
        double r2 = dx * dx + dy * dy;
        double e1 = exp(0.5 * (1.0 - r2));
        vel[0] = P.p[3] - eps / (2.0 * pi) * e1 * dy;
        vel[1] = P.p[4] + eps / (2.0 * pi) * e1 * dx;
        double T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * pi * pi) * exp(1.0 - r2);
        rho = pow(T, 1.0 / (gamma - 1.0));
        p = pow(rho, gamma);
    } else if (kind == DGAMR_IC_SEDOV) {
        bool inside = true;
        for (int a = 0; a < D; ++a) inside = inside && fabs(x[a] - P.p[2 + a]) < hmin[a];
        p = inside ? P.p[1] : P.p[0];
    } else if (kind == DGAMR_IC_UNIFORM) {
        rho = P.p[0];
        for (int a = 0; a < D; ++a) vel[a] = P.p[1 + a];
        p = P.p[4];
    } else {
        rho = 1.0 + P.p[0] * sin(2.0 * pi * (x[0] - P.p[1] * t) / P.p[2]);
        vel[0] = P.p[1];
    }
    double ke = 0.0;
    U[0] = rho;
    for (int a = 0; a < D; ++a) {
        U[1 + a] = rho * vel[a];
        ke += vel[a] * vel[a];
    }
    U[D + 1] = p / (gamma - 1.0) + 0.5 * rho * ke;
}

// Gauss points (p+3 per axis) and Legendre values there, for the
// initial-condition projection.
template <int P>
struct IcTab {
    static constexpr int QI = P + 3;
    double x[QI] = {}, w[QI] = {}, leg1[QI][P + 1] = {};
    constexpr IcTab()
    {
        for (int q = 0; q < QI; ++q) {
            x[q] = gl_x(QI, q);
            w[q] = gl_w(QI, q);
            for (int n = 0; n <= P; ++n) leg1[q][n] = leg(n, x[q]);
        }
    }
};
template <int P>
inline constexpr IcTab<P> kIcTab{};

// K_m = (1/M_m) int phi_m U0 dV with p+3 Gauss points per axis
template <int D, int P, int NV = D + 2>
__global__ __launch_bounds__(256) void k_project_ic(double *u, const LeafGeo *geo, int N, long ncell_total, int kind,
                                                    IcParams prm, double t, double gamma, double hmin0, double hmin1,
                                                    double hmin2)
{
    constexpr int NB = Tab<D, P>::NB, QI = P + 3;
    const int ncell = D == 2 ? N * N : N * N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const long leaf = gid / ncell;
    const int c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    const LeafGeo G = geo[leaf];
    const double hmin[3] = {hmin0, hmin1, hmin2};
    double acc[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) acc[v][m] = 0.0;
    constexpr int NQI = ipow(QI, D);
#pragma unroll 1
    for (int q = 0; q < NQI; ++q) {
        const int qi[3] = {q % QI, (q / QI) % QI, q / (QI * QI)};
        double x[3] = {0, 0, 0}, xi[3] = {0, 0, 0}, w = 1.0;
        for (int a = 0; a < D; ++a) {
            w *= kIcTab<P>.w[qi[a]];
            xi[a] = kIcTab<P>.x[qi[a]];
        }
        leaf_point<D>(G, ijk, xi, x);
        double U[D + 2];
        analytic<D>(kind, prm, t, gamma, x, hmin, U);
        if constexpr (NV == D + 2) { // momentum into the leaf's frame: Q^T m
            double m[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int l = 0; l < D; ++l)
#pragma unroll
                for (int g2 = 0; g2 < D; ++g2) m[l] += double(G.q[3 * g2 + l]) * U[1 + g2];
#pragma unroll
            for (int l = 0; l < D; ++l) U[1 + l] = m[l];
        }
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            double ph = w;
#pragma unroll
            for (int a = 0; a < D; ++a) ph *= kIcTab<P>.leg1[qi[a]][kTab<D, P>.e[m][a]];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v][m] = fma(ph, U[v], acc[v][m]);
        }
    }
    const long sv = long(NB) * ncell, base = leaf * NV * sv + c;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) u[base + v * sv + m * ncell] = acc[v][m] * kTab<D, P>.inv_mass[m];
}

// ------------------------------------------------------------------ inheritance
// Eq. 11-14 on a refinement switch: copy, split (child cells of a refined
// leaf from the parent cells) or combine (cells of a coarsened parent from
// its 2^d children's cells).
template <int D, int P, int NV = D + 2>
__global__ __launch_bounds__(256) void k_inherit(const double *uold, double *unew, const Inherit *inh, int N,
                                                 long ncell_total)
{
    constexpr int NB = Tab<D, P>::NB;
    const int ncell = D == 2 ? N * N : N * N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const long leaf = gid / ncell;
    const int c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    const Inherit I = inh[leaf];
    const long sv = long(NB) * ncell;
    double *out = unew + leaf * NV * sv + c;
    if (I.type == dgamr::INH_COPY) {
        const double *src = uold + long(I.src[0]) * NV * sv + c;
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) out[v * sv + m * ncell] = src[v * sv + m * ncell];
    } else if (I.type == dgamr::INH_SPLIT) {
        int pijk[3] = {0, 0, 0}, child = 0;
        for (int a = 0; a < D; ++a) {
            const int gi = ((I.child >> a) & 1) * N + ijk[a];
            pijk[a] = gi >> 1;
            child |= (gi & 1) << a;
        }
        const int pc = pijk[0] + N * (pijk[1] + N * pijk[2]);
        const double *src = uold + long(I.src[0]) * NV * sv + pc;
        for (int v = 0; v < NV; ++v) {
            double ks[NB], gk[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) ks[n] = src[v * sv + n * ncell];
            split_any<D, P, double>(child, ks, gk);
#pragma unroll
            for (int m = 0; m < NB; ++m) out[v * sv + m * ncell] = gk[m];
        }
    } else {
        int cl = 0, fbase[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            const int gi = 2 * ijk[a];
            cl |= (gi / N) << a;
            fbase[a] = gi % N;
        }
        const double *src = uold + long(I.src[cl]) * NV * sv;
        for (int v = 0; v < NV; ++v) {
            double acc[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) acc[m] = 0.0;
#pragma unroll
            for (int ch = 0; ch < (1 << D); ++ch) {
                const int fc = (fbase[0] + (ch & 1)) +
                               N * ((fbase[1] + ((ch >> 1) & 1)) + (D == 3 ? N * (fbase[2] + ((ch >> 2) & 1)) : 0));
                double ks[NB];
#pragma unroll
                for (int n = 0; n < NB; ++n) ks[n] = src[v * sv + n * ncell + fc];
#pragma unroll
                for (int m = 0; m < NB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        const double cc = kTab<D, P>.comb[ch][m][n];
                        if (cc != 0.0) acc[m] = fma(cc, ks[n], acc[m]);
                    }
            }
#pragma unroll
            for (int m = 0; m < NB; ++m) out[v * sv + m * ncell] = acc[m];
        }
    }
}

} // namespace dgk
