// Bilinear root blocks (Sec. 3.3, Eq. 6), 2-D: a root is the bilinear image
// of the reference square spanned by its four corner nodes, and every cell
// of its leaves the bilinear image of the cell's reference square with the
// images of its corners as nodes.  The weak form (Sec. 2, Eq. 3-4) then
// carries the map's Jacobian J = dx/dxi at every quadrature point:
//   volume  sum_q w_q grad_xi phi_m . adj(J) F(U_q)   (adj(J) = det(J) J^-1:
//           the contravariant flux),
//   faces   - sum_f w_f |N| Fhat(U-, U+; N / |N|) phi_m with N = side * (row
//           a of adj(J)) on the face xi_a = side (the outward normal scaled
//           by the face Jacobian),
// and the residual is M^-1 of that with the full mass matrix M_mn =
// sum_q w_q det(J_q) phi_m phi_n (exact with p+1 points per axis: det(J) is
// bilinear), solved per cell by Cholesky.  The neighbour across a block
// face is the guard cell (coefficients from the fill kernel: copy, split,
// combine in the reference space, Eq. 15-17); its trace is taken at the
// shared reference face point.
//
// One thread per cell; these forests step through the fill, this kernel
// and the stage update as separate launches.
#pragma once

#include "kernels_aux.hpp"  // analytic states, IC quadrature
#include "kernels_ipdg.hpp" // DiffTab: basis derivatives and weights at the volume points

namespace dgk {

// corners of cell (i, j) of a leaf: the leaf's bilinear map at the cell's
// corners in the leaf's unit square; (xi, eta) = (-1,-1), (1,-1), (-1,1), (1,1)
__device__ __forceinline__ void mapped_cell_corners(const LeafGeo &G, int i, int j, int N, double cx[4][2])
{
    const double inv = 1.0 / N;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const double s0 = (i + (b & 1)) * inv, s1 = (j + (b >> 1)) * inv;
#pragma unroll
        for (int a = 0; a < 2; ++a)
            cx[b][a] = (1.0 - s0) * (1.0 - s1) * G.node[0][a] + s0 * (1.0 - s1) * G.node[1][a] +
                       (1.0 - s0) * s1 * G.node[2][a] + s0 * s1 * G.node[3][a];
    }
}

// J[a][b] = dx_a / dxi_b of the bilinear cell map at (e, h); returns det J
__device__ __forceinline__ double mapped_jacobian(const double cx[4][2], double e, double h, double J[2][2])
{
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        J[a][0] = 0.25 * ((1.0 - h) * (cx[1][a] - cx[0][a]) + (1.0 + h) * (cx[3][a] - cx[2][a]));
        J[a][1] = 0.25 * ((1.0 - e) * (cx[2][a] - cx[0][a]) + (1.0 + e) * (cx[3][a] - cx[1][a]));
    }
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
}

// physical point of the bilinear cell map at (e, h)
__device__ __forceinline__ void mapped_point(const double cx[4][2], double e, double h, double *x)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
        x[a] = 0.25 * ((1.0 - e) * (1.0 - h) * cx[0][a] + (1.0 + e) * (1.0 - h) * cx[1][a] +
                       (1.0 - e) * (1.0 + h) * cx[2][a] + (1.0 + e) * (1.0 + h) * cx[3][a]);
    x[2] = 0.0;
}

// numerical flux along the outward unit normal (n0, n1) (Eq. 5): Rusanov
// with alpha = max(|u.n| + c) over both traces; for scalar convection the
// same formula with alpha = |vel.n| (upwind)
template <int EQ>
__device__ __forceinline__ void mapped_flux(const MappedArgs &g, const double *UL, const double *UR, double n0,
                                            double n1, double *Phi)
{
    if constexpr (EQ == EQ_ADVECTION) {
        const double vn = g.vel[0] * n0 + g.vel[1] * n1;
        Phi[0] = 0.5 * (vn * (UL[0] + UR[0]) - fabs(vn) * (UR[0] - UL[0]));
    } else {
        const double gm1 = g.gamma - 1.0;
        const double rl = recip(UL[0]), rr = recip(UR[0]);
        const double pl = pressure_r<2>(UL, gm1, rl), pr = pressure_r<2>(UR, gm1, rr);
        const double unl = (UL[1] * n0 + UL[2] * n1) * rl, unr = (UR[1] * n0 + UR[2] * n1) * rr;
        const double al = fabs(unl) + sqrt_nn(g.gamma * pl * rl), ar = fabs(unr) + sqrt_nn(g.gamma * pr * rr);
        const double alpha = al > ar ? al : ar;
        const double FL[4] = {UL[0] * unl, UL[1] * unl + pl * n0, UL[2] * unl + pl * n1, (UL[3] + pl) * unl};
        const double FR[4] = {UR[0] * unr, UR[1] * unr + pr * n0, UR[2] * unr + pr * n1, (UR[3] + pr) * unr};
#pragma unroll
        for (int v = 0; v < 4; ++v) Phi[v] = 0.5 * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
    }
}

// physical flux along the x (A = 0) or y (A = 1) axis
template <int EQ, int A>
__device__ __forceinline__ void mapped_phys_flux(const MappedArgs &g, const double *U, double *F)
{
    if constexpr (EQ == EQ_ADVECTION) {
        F[0] = g.vel[A] * U[0];
    } else {
        const double rinv = recip(U[0]);
        const double p = pressure_r<2>(U, g.gamma - 1.0, rinv);
        euler_flux<2, A, double>(U, U[1 + A] * rinv, p, F);
    }
}

// X <- M^-1 X for NV right-hand sides, M symmetric positive definite (NB x NB)
template <int NB, int NV>
__device__ __forceinline__ void mapped_solve(const double (&M)[NB][NB], double (&X)[NV][NB])
{
    double L[NB][NB];
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            double s = M[r][c];
#pragma unroll
            for (int k = 0; k < c; ++k) s -= L[r][k] * L[c][k];
            L[r][c] = r == c ? sqrt(s) : s / L[c][c];
        }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            double s = X[v][r];
#pragma unroll
            for (int k = 0; k < r; ++k) s -= L[r][k] * X[v][k];
            X[v][r] = s / L[r][r];
        }
#pragma unroll
        for (int r = NB - 1; r >= 0; --r) {
            double s = X[v][r];
#pragma unroll
            for (int k = r + 1; k < NB; ++k) s -= L[k][r] * X[v][k];
            X[v][r] = s / L[r][r];
        }
    }
}

// mass matrix of a bilinear cell with the volume rule
template <int P>
__device__ __forceinline__ void mapped_mass(const double cx[4][2], double (&M)[Tab<2, P>::NB][Tab<2, P>::NB])
{
    constexpr int NB = Tab<2, P>::NB, NQ = Tab<2, P>::NQ, Q = P + 1;
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) M[m][n] = 0.0;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        double J[2][2];
        const double wd = kDiffTab<2, P>.wv[q] * mapped_jacobian(cx, gl_x(Q, q % Q), gl_x(Q, q / Q), J);
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int n = 0; n <= m; ++n) M[m][n] = fma(wd * kTab<2, P>.phi_v[q][m], kTab<2, P>.phi_v[q][n], M[m][n]);
    }
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = m + 1; n < NB; ++n) M[m][n] = M[n][m];
}

template <int P, int EQ, int OM>
__global__ __launch_bounds__(128) void k_mapped(MappedArgs g)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : 4, NB = Tab<2, P>::NB, NQ = Tab<2, P>::NQ, Q = P + 1;
    const int N = g.N, ncell = N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= g.ncell_total) return;
    const int leaf = int(gid / ncell), c = int(gid % ncell);
    const int ci = c % N, cj = c / N;
    double cx[4][2];
    mapped_cell_corners(g.geo[leaf], ci, cj, N, cx);
    const long sv = long(NB) * ncell;
    const double *K0 = g.us + long(leaf) * NV * sv + c;
    double K[NV][NB], R[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            K[v][m] = K0[v * sv + long(m) * ncell];
            R[v][m] = 0.0;
        }
    // ---- volume: sum_q w_q grad_xi phi_m . adj(J) F(U_q)
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        double J[2][2];
        mapped_jacobian(cx, gl_x(Q, q % Q), gl_x(Q, q / Q), J);
        const double a00 = J[1][1], a01 = -J[0][1], a10 = -J[1][0], a11 = J[0][0]; // rows of adj(J)
        double U[NV], Fx[NV], Fy[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) s = fma(kTab<2, P>.phi_v[q][m], K[v][m], s);
            U[v] = s;
        }
        mapped_phys_flux<EQ, 0>(g, U, Fx);
        mapped_phys_flux<EQ, 1>(g, U, Fy);
        const double w = kDiffTab<2, P>.wv[q];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double c0 = w * (a00 * Fx[v] + a01 * Fy[v]), c1 = w * (a10 * Fx[v] + a11 * Fy[v]);
#pragma unroll
            for (int m = 0; m < NB; ++m)
                R[v][m] = fma(kDiffTab<2, P>.dphi_v[0][q][m], c0, fma(kDiffTab<2, P>.dphi_v[1][q][m], c1, R[v][m]));
        }
    }
    // ---- faces
    static_for<0, 2>([&](auto Ai) __attribute__((always_inline)) {
        constexpr int A = Ai;
        const int stride = A == 0 ? 1 : N;
        const int ia = A == 0 ? ci : cj, t = A == 0 ? cj : ci;
#pragma unroll 1
        for (int si = 0; si < 2; ++si) {
            const int s = si ? 1 : -1;
            const int face = 2 * A + si;
            const bool interior = s > 0 ? ia < N - 1 : ia > 0;
            const double *Kn;
            long nsv, nsm;
            if (interior) {
                Kn = K0 + s * stride;
                nsv = sv;
                nsm = ncell;
            } else {
                Kn = g.guard + (long(leaf) * 4 + face) * NV * NB * N + t;
                nsv = long(NB) * N;
                nsm = N;
            }
            double KN[NV][NB];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) KN[v][m] = Kn[v * nsv + m * nsm];
#pragma unroll 1
            for (int f = 0; f < Q; ++f) {
                const double xt = gl_x(Q, f);
                double J[2][2];
                if (A == 0) mapped_jacobian(cx, double(s), xt, J);
                else mapped_jacobian(cx, xt, double(s), J);
                // outward normal scaled by the face Jacobian: side * row A of adj(J)
                const double N0 = s * (A == 0 ? J[1][1] : -J[1][0]), N1 = s * (A == 0 ? -J[0][1] : J[0][0]);
                const double len = sqrt(N0 * N0 + N1 * N1), il = 1.0 / len;
                double UL[NV], UR[NV], Phi[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double a = 0.0, b = 0.0;
#pragma unroll
                    for (int m = 0; m < NB; ++m) {
                        a = fma(face_phi<2, P, A>(m, f, s), K[v][m], a);
                        b = fma(face_phi<2, P, A>(m, f, -s), KN[v][m], b);
                    }
                    UL[v] = a;
                    UR[v] = b;
                }
                mapped_flux<EQ>(g, UL, UR, N0 * il, N1 * il, Phi);
                const double w = gl_w(Q, f) * len;
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int m = 0; m < NB; ++m) R[v][m] = fma(-w * Phi[v], face_phi<2, P, A>(m, f, s), R[v][m]);
            }
        }
    });
    // ---- M^-1
    double M[NB][NB];
    mapped_mass<P>(cx, M);
    mapped_solve<NB, NV>(M, R);
    double *o = g.out + long(leaf) * NV * sv + c;
    if constexpr (OM == OUT_RES64) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) o[v * sv + long(m) * ncell] = R[v][m];
    } else {
        const double dt = *g.dt, a = g.rk_a, b = g.rk_b;
        const double *U0 = g.un + long(leaf) * NV * sv + c;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m)
                o[v * sv + long(m) * ncell] = a * U0[v * sv + long(m) * ncell] + b * (K[v][m] + dt * R[v][m]);
    }
}

// CFL rate of the leaves of a bilinear forest (one workgroup per leaf): per
// cell the means of the state over the physical cell (volume rule), and for
// each reference axis b the unit normal n_b and the width h_b = 2 det(J) /
// |row b of adj(J)| at the cell centre (the edge lengths of a rectangle):
// sum_b (|u.n_b| + c) / h_b (scalar convection: sum_b |vel.n_b| / h_b).
template <int P, int EQ>
__global__ __launch_bounds__(256) void k_mapped_rate(MappedArgs g, double *leaf_max)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : 4, NB = Tab<2, P>::NB, NQ = Tab<2, P>::NQ, Q = P + 1;
    __shared__ double red[256];
    const int leaf = blockIdx.x, N = g.N, ncell = N * N;
    const long sv = long(NB) * ncell;
    double mx = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        double cx[4][2], J[2][2];
        mapped_cell_corners(g.geo[leaf], c % N, c / N, N, cx);
        const double *K0 = g.us + long(leaf) * NV * sv + c;
        double s[NV], area = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] = 0.0;
        for (int q = 0; q < NQ; ++q) {
            const double wd = kDiffTab<2, P>.wv[q] * mapped_jacobian(cx, gl_x(Q, q % Q), gl_x(Q, q / Q), J);
            area += wd;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double u = 0.0;
#pragma unroll
                for (int m = 0; m < NB; ++m) u = fma(kTab<2, P>.phi_v[q][m], K0[v * sv + long(m) * ncell], u);
                s[v] += wd * u;
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] /= area;
        const double det0 = mapped_jacobian(cx, 0.0, 0.0, J);
        double cs = 0.0;
        if constexpr (EQ != EQ_ADVECTION) cs = sqrt(g.gamma * pressure_r<2>(s, g.gamma - 1.0, 1.0 / s[0]) / s[0]);
        double rate = 0.0;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double A0 = b == 0 ? J[1][1] : -J[1][0], A1 = b == 0 ? -J[0][1] : J[0][0];
            const double len = sqrt(A0 * A0 + A1 * A1), h = 2.0 * det0 / len;
            const double n0 = A0 / len, n1 = A1 / len;
            double un;
            if constexpr (EQ == EQ_ADVECTION) un = g.vel[0] * n0 + g.vel[1] * n1;
            else un = (s[1] * n0 + s[2] * n1) / s[0];
            rate += (fabs(un) + cs) / h;
        }
        mx = rate > mx ? rate : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) leaf_max[leaf] = red[0];
}

// Integrals of the state over the physical cells of a leaf (volume rule),
// one workgroup per leaf (a power of two of threads): part[leaf * NV + v]
template <int P, int EQ>
__global__ __launch_bounds__(256) void k_mapped_totals_leaf(MappedArgs g, double *part)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : 4, NB = Tab<2, P>::NB, NQ = Tab<2, P>::NQ, Q = P + 1;
    __shared__ double red[NV][256];
    const int leaf = blockIdx.x, N = g.N, ncell = N * N;
    const long sv = long(NB) * ncell;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        double cx[4][2], J[2][2];
        mapped_cell_corners(g.geo[leaf], c % N, c / N, N, cx);
        const double *K0 = g.us + long(leaf) * NV * sv + c;
        for (int q = 0; q < NQ; ++q) {
            const double wd = kDiffTab<2, P>.wv[q] * mapped_jacobian(cx, gl_x(Q, q % Q), gl_x(Q, q / Q), J);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double u = 0.0;
#pragma unroll
                for (int m = 0; m < NB; ++m) u = fma(kTab<2, P>.phi_v[q][m], K0[v * sv + long(m) * ncell], u);
                s[v] = fma(wd, u, s[v]);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w)
#pragma unroll
            for (int v = 0; v < NV; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) part[long(leaf) * NV + v] = red[v][0];
}

// Initial state on bilinear cells: M K = int phi_m U0 det(J) dxi with p+3
// Gauss points per axis for the right-hand side and the volume rule for M.
template <int P, int NV>
__global__ __launch_bounds__(128) void k_mapped_project_ic(double *u, const LeafGeo *geo, int N, long ncell_total,
                                                           int kind, IcParams prm, double t, double gamma)
{
    constexpr int NB = Tab<2, P>::NB, QI = P + 3, NQI = QI * QI;
    const int ncell = N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const long leaf = gid / ncell;
    const int c = int(gid % ncell);
    double cx[4][2];
    mapped_cell_corners(geo[leaf], c % N, c / N, N, cx);
    const double hmin[3] = {0.0, 0.0, 0.0};
    double acc[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) acc[v][m] = 0.0;
#pragma unroll 1
    for (int q = 0; q < NQI; ++q) {
        const int q0 = q % QI, q1 = q / QI;
        double J[2][2], x[3];
        const double e = kIcTab<P>.x[q0], h = kIcTab<P>.x[q1];
        const double wd = kIcTab<P>.w[q0] * kIcTab<P>.w[q1] * mapped_jacobian(cx, e, h, J);
        mapped_point(cx, e, h, x);
        double U[4];
        analytic<2>(kind, prm, t, gamma, x, hmin, U);
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const double ph = wd * kIcTab<P>.leg1[q0][kTab<2, P>.e[m][0]] * kIcTab<P>.leg1[q1][kTab<2, P>.e[m][1]];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v][m] = fma(ph, U[v], acc[v][m]);
        }
    }
    double M[NB][NB];
    mapped_mass<P>(cx, M);
    mapped_solve<NB, NV>(M, acc);
    const long sv = long(NB) * ncell, base = leaf * NV * sv + c;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) u[base + v * sv + m * ncell] = acc[v][m];
}

} // namespace dgk
