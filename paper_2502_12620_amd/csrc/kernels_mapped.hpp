// Bilinear (3-D: trilinear) root blocks (Sec. 3.3, Eq. 6): a root is the
// multilinear image of the reference square (cube) spanned by its corner
// nodes, and every cell of its leaves the multilinear image of the cell's
// reference box with the images of its corners as nodes.  The weak form
// (Sec. 2, Eq. 3-4) then carries the map's Jacobian J = dx/dxi at every
// quadrature point:
//   volume  sum_q w_q grad_xi phi_m . adj(J) F(U_q)   (adj(J) = det(J) J^-1:
//           the contravariant flux),
//   faces   - sum_f w_f |N| Fhat(U-, U+; N / |N|) phi_m with N = side * (row
//           a of adj(J)) on the face xi_a = side (the outward normal scaled
//           by the face Jacobian),
// and the residual is M^-1 of that with the full mass matrix M_mn =
// sum_q w_q det(J_q) phi_m phi_n (exact with p+1 points per axis: det(J)
// has degree d-1 per axis), solved per cell by Cholesky.  The neighbour
// across a block face is the guard cell (coefficients from the fill kernel:
// copy, split, combine in the reference space, Eq. 15-17); its trace is
// taken at the shared reference face point.
//
// One thread per cell; these forests step through the fill, this kernel
// and the stage update as separate launches.
#pragma once

#include "kernels_aux.hpp"  // analytic states, IC quadrature
#include "kernels_ipdg.hpp" // DiffTab: basis derivatives and weights at the volume points

namespace dgk {

// corners of cell ijk of a leaf: the leaf's multilinear map at the cell's
// corners in the leaf's unit box; corner b lies at reference coordinate
// -1 or +1 along axis a by bit a of b
template <int D>
__device__ __forceinline__ void mapped_cell_corners(const LeafGeo &G, const int *ijk, int N, double (&cx)[1 << D][3])
{
    const double inv = 1.0 / N;
#pragma unroll
    for (int b = 0; b < (1 << D); ++b) {
        double s[3];
#pragma unroll
        for (int a = 0; a < D; ++a) s[a] = (ijk[a] + ((b >> a) & 1)) * inv;
#pragma unroll
        for (int a = 0; a < 3; ++a) cx[b][a] = 0.0;
#pragma unroll
        for (int n = 0; n < (1 << D); ++n) {
            double w = 1.0;
#pragma unroll
            for (int a = 0; a < D; ++a) w *= ((n >> a) & 1) ? s[a] : 1.0 - s[a];
#pragma unroll
            for (int a = 0; a < D; ++a) cx[b][a] = fma(w, G.node[n][a], cx[b][a]);
        }
    }
}

// J[a][e] = dx_a / dxi_e of the multilinear cell map at xi; returns det J
template <int D>
__device__ __forceinline__ double mapped_jacobian(const double (&cx)[1 << D][3], const double *xi, double (&J)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int e = 0; e < 3; ++e) J[a][e] = 0.0;
#pragma unroll
    for (int b = 0; b < (1 << D); ++b)
#pragma unroll
        for (int e = 0; e < D; ++e) {
            double w = ((b >> e) & 1) ? 0.5 : -0.5;
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (c != e) w *= 0.5 * (1.0 + (((b >> c) & 1) ? xi[c] : -xi[c]));
#pragma unroll
            for (int a = 0; a < D; ++a) J[a][e] = fma(w, cx[b][a], J[a][e]);
        }
    if constexpr (D == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// row e of adj(J) = det(J) J^-1: the contravariant direction of xi_e
template <int D>
__device__ __forceinline__ void mapped_adj_row(const double (&J)[3][3], int e, double *r)
{
    if constexpr (D == 2) {
        r[0] = e == 0 ? J[1][1] : -J[1][0];
        r[1] = e == 0 ? -J[0][1] : J[0][0];
        r[2] = 0.0;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, e1 = (e + 1) % 3, e2 = (e + 2) % 3;
            r[a] = J[a1][e1] * J[a2][e2] - J[a1][e2] * J[a2][e1];
        }
    }
}

// physical point of the multilinear cell map at xi
template <int D>
__device__ __forceinline__ void mapped_point(const double (&cx)[1 << D][3], const double *xi, double *x)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = 0.0;
#pragma unroll
    for (int b = 0; b < (1 << D); ++b) {
        double w = 1.0;
#pragma unroll
        for (int a = 0; a < D; ++a) w *= 0.5 * (1.0 + (((b >> a) & 1) ? xi[a] : -xi[a]));
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = fma(w, cx[b][a], x[a]);
    }
}

// reference coordinates of volume point q (x fastest)
template <int D, int P>
__device__ __forceinline__ void mapped_vpoint(int q, double *xi)
{
    constexpr int Q = P + 1;
    xi[0] = gl_x(Q, q % Q);
    xi[1] = gl_x(Q, (q / Q) % Q);
    xi[2] = D == 3 ? gl_x(Q, q / (Q * Q)) : 0.0;
}

// numerical flux along the outward unit normal n (Eq. 5): Rusanov with
// alpha = max(|u.n| + c) over both traces; for scalar convection the same
// formula with alpha = |vel.n| (upwind)
template <int D, int EQ>
__device__ __forceinline__ void mapped_flux(const MappedArgs &g, const double *UL, const double *UR, const double *n,
                                            double *Phi)
{
    if constexpr (EQ == EQ_ADVECTION) {
        double vn = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) vn = fma(g.vel[a], n[a], vn);
        Phi[0] = 0.5 * (vn * (UL[0] + UR[0]) - fabs(vn) * (UR[0] - UL[0]));
    } else {
        constexpr int NV = D + 2;
        const double gm1 = g.gamma - 1.0;
        const double rl = recip(UL[0]), rr = recip(UR[0]);
        const double pl = pressure_r<D>(UL, gm1, rl), pr = pressure_r<D>(UR, gm1, rr);
        double ml = 0.0, mr = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            ml = fma(UL[1 + a], n[a], ml);
            mr = fma(UR[1 + a], n[a], mr);
        }
        const double unl = ml * rl, unr = mr * rr;
        const double al = fabs(unl) + sqrt_nn(g.gamma * pl * rl), ar = fabs(unr) + sqrt_nn(g.gamma * pr * rr);
        const double alpha = al > ar ? al : ar;
        double FL[NV], FR[NV];
        FL[0] = UL[0] * unl;
        FR[0] = UR[0] * unr;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            FL[1 + a] = UL[1 + a] * unl + pl * n[a];
            FR[1 + a] = UR[1 + a] * unr + pr * n[a];
        }
        FL[D + 1] = (UL[D + 1] + pl) * unl;
        FR[D + 1] = (UR[D + 1] + pr) * unr;
#pragma unroll
        for (int v = 0; v < NV; ++v) Phi[v] = 0.5 * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
    }
}

// physical flux along axis A
template <int D, int EQ, int A>
__device__ __forceinline__ void mapped_phys_flux(const MappedArgs &g, const double *U, double *F)
{
    if constexpr (EQ == EQ_ADVECTION) {
        F[0] = g.vel[A] * U[0];
    } else {
        const double rinv = recip(U[0]);
        const double p = pressure_r<D>(U, g.gamma - 1.0, rinv);
        euler_flux<D, A, double>(U, U[1 + A] * rinv, p, F);
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

// the state's mean over the physical cell from the mass matrix: with
// phi_0 = 1, M[n][0] = int phi_n det J and M[0][0] is the cell's volume
template <int NB, int NV>
__device__ __forceinline__ void mapped_mean(const double (&M)[NB][NB], const double (&K)[NV][NB], double (&mean)[NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int n = 0; n < NB; ++n) s = fma(M[n][0], K[v][n], s);
        mean[v] = s / M[0][0];
    }
}

// mass matrix of a multilinear cell with the volume rule
template <int D, int P>
__device__ __forceinline__ void mapped_mass(const double (&cx)[1 << D][3], double (&M)[Tab<D, P>::NB][Tab<D, P>::NB])
{
    constexpr int NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ;
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) M[m][n] = 0.0;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        double J[3][3], xi[3];
        mapped_vpoint<D, P>(q, xi);
        const double wd = kDiffTab<D, P>.wv[q] * mapped_jacobian<D>(cx, xi, J);
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int n = 0; n <= m; ++n) M[m][n] = fma(wd * kTab<D, P>.phi_v[q][m], kTab<D, P>.phi_v[q][n], M[m][n]);
    }
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = m + 1; n < NB; ++n) M[m][n] = M[n][m];
}

// LIM: the positivity limiter on the new state, about the cell's mean over
// the physical cell (Euler, OUT_RK)
template <int D, int P, int EQ, int OM, bool LIM = false>
__global__ __launch_bounds__(128) void k_mapped(MappedArgs g)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : D + 2, NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ, NF = Tab<D, P>::NF;
    constexpr int Q = P + 1;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= g.ncell_total) return;
    const int leaf = int(gid / ncell), c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    double cx[1 << D][3];
    mapped_cell_corners<D>(g.geo[leaf], ijk, N, cx);
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
        double J[3][3], xi[3], A[D][3];
        mapped_vpoint<D, P>(q, xi);
        mapped_jacobian<D>(cx, xi, J);
#pragma unroll
        for (int e = 0; e < D; ++e) mapped_adj_row<D>(J, e, A[e]);
        double U[NV], F[D][NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) s = fma(kTab<D, P>.phi_v[q][m], K[v][m], s);
            U[v] = s;
        }
        static_for<0, D>([&](auto Ai) __attribute__((always_inline)) { mapped_phys_flux<D, EQ, Ai>(g, U, F[Ai]); });
        const double w = kDiffTab<D, P>.wv[q];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int e = 0; e < D; ++e) {
                double ce = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) ce = fma(A[e][a], F[a][v], ce);
                ce *= w;
#pragma unroll
                for (int m = 0; m < NB; ++m) R[v][m] = fma(kDiffTab<D, P>.dphi_v[e][q][m], ce, R[v][m]);
            }
    }
    // ---- faces
    static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
        constexpr int A = Ai;
        constexpr int TA = A == 0 ? 1 : 0, TB = A == 2 ? 1 : 2; // tangential axes, lower first
        const int stride = A == 0 ? 1 : (A == 1 ? N : N * N);
        const int ia = ijk[A], t = face_t(ijk, A, N, D);
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
                Kn = g.guard + (long(leaf) * 2 * D + face) * NV * NB * nfc + t;
                nsv = long(NB) * nfc;
                nsm = nfc;
            }
            double KN[NV][NB];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) KN[v][m] = Kn[v * nsv + m * nsm];
#pragma unroll 1
            for (int f = 0; f < NF; ++f) {
                double xi[3] = {0.0, 0.0, 0.0};
                xi[A] = double(s);
                xi[TA] = gl_x(Q, f % Q);
                if (D == 3) xi[TB] = gl_x(Q, f / Q);
                double J[3][3], Nv[3];
                mapped_jacobian<D>(cx, xi, J);
                mapped_adj_row<D>(J, A, Nv);
                double len2 = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    Nv[a] *= s;
                    len2 = fma(Nv[a], Nv[a], len2);
                }
                const double len = sqrt(len2), il = 1.0 / len;
                double n[3];
#pragma unroll
                for (int a = 0; a < D; ++a) n[a] = Nv[a] * il;
                double UL[NV], UR[NV], Phi[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double a = 0.0, b = 0.0;
#pragma unroll
                    for (int m = 0; m < NB; ++m) {
                        a = fma(face_phi<D, P, A>(m, f, s), K[v][m], a);
                        b = fma(face_phi<D, P, A>(m, f, -s), KN[v][m], b);
                    }
                    UL[v] = a;
                    UR[v] = b;
                }
                mapped_flux<D, EQ>(g, UL, UR, n, Phi);
                const double w = kDiffTab<D, P>.wf[f] * len;
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int m = 0; m < NB; ++m) R[v][m] = fma(-w * Phi[v], face_phi<D, P, A>(m, f, s), R[v][m]);
            }
        }
    });
    // ---- M^-1
    double M[NB][NB];
    mapped_mass<D, P>(cx, M);
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
        if constexpr (LIM && EQ == EQ_EULER) {
            double Kn[NV][NB], mean[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[v][m] = a * U0[v * sv + long(m) * ncell] + b * (K[v][m] + dt * R[v][m]);
            mapped_mean<NB, NV>(M, Kn, mean);
            limit_cell<D, P, true>(Kn, g.gamma, mean);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) o[v * sv + long(m) * ncell] = Kn[v][m];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m)
                    o[v * sv + long(m) * ncell] = a * U0[v * sv + long(m) * ncell] + b * (K[v][m] + dt * R[v][m]);
        }
    }
}

// the positivity limiter alone on bilinear / trilinear roots: one thread
// per cell, about the cell's mean over the physical cell
template <int D, int P>
__global__ __launch_bounds__(128) void k_mapped_limit(double *u, const LeafGeo *geo, int N, long ncell_total,
                                                      double gamma)
{
    constexpr int NV = D + 2, NB = Tab<D, P>::NB;
    const int ncell = D == 2 ? N * N : N * N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const int leaf = int(gid / ncell), c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    double cx[1 << D][3];
    mapped_cell_corners<D>(geo[leaf], ijk, N, cx);
    double M[NB][NB];
    mapped_mass<D, P>(cx, M);
    const long sv = long(NB) * ncell;
    double *K0 = u + long(leaf) * NV * sv + c;
    double K[NV][NB], mean[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) K[v][m] = K0[v * sv + long(m) * ncell];
    mapped_mean<NB, NV>(M, K, mean);
    limit_cell<D, P, true>(K, gamma, mean);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) K0[v * sv + long(m) * ncell] = K[v][m];
}

// the integrals of the state over the physical cell (volume rule) and the
// cell's volume
template <int D, int P, int NV>
__device__ __forceinline__ double mapped_cell_integrals(const double (&cx)[1 << D][3], const double *K0, long sv,
                                                        int ncell, double *s)
{
    constexpr int NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ;
    double vol = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int q = 0; q < NQ; ++q) {
        double J[3][3], xi[3];
        mapped_vpoint<D, P>(q, xi);
        const double wd = kDiffTab<D, P>.wv[q] * mapped_jacobian<D>(cx, xi, J);
        vol += wd;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double u = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) u = fma(kTab<D, P>.phi_v[q][m], K0[v * sv + long(m) * ncell], u);
            s[v] = fma(wd, u, s[v]);
        }
    }
    return vol;
}

// CFL rate of the leaves of a mapped forest (one workgroup per leaf, a
// power of two of threads): per cell the means over the physical cell, and
// for each reference axis b the unit normal n_b and the width h_b =
// 2 det(J) / |row b of adj(J)| at the cell centre (the edge lengths of a
// box): sum_b (|u.n_b| + c) / h_b (scalar convection: sum_b |vel.n_b| / h_b).
template <int D, int P, int EQ>
__global__ __launch_bounds__(256) void k_mapped_rate(MappedArgs g, double *leaf_max)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : D + 2, NB = Tab<D, P>::NB;
    __shared__ double red[256];
    const int leaf = blockIdx.x, N = g.N, ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(NB) * ncell;
    double mx = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        int ijk[3];
        cell_ijk(c, N, D, ijk);
        double cx[1 << D][3], J[3][3], s[NV];
        mapped_cell_corners<D>(g.geo[leaf], ijk, N, cx);
        const double vol = mapped_cell_integrals<D, P, NV>(cx, g.us + long(leaf) * NV * sv + c, sv, ncell, s);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] /= vol;
        const double x0[3] = {0.0, 0.0, 0.0};
        const double det0 = mapped_jacobian<D>(cx, x0, J);
        double cs = 0.0;
        if constexpr (EQ != EQ_ADVECTION) cs = sqrt(g.gamma * pressure_r<D>(s, g.gamma - 1.0, 1.0 / s[0]) / s[0]);
        double rate = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            double A[3];
            mapped_adj_row<D>(J, b, A);
            double len2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) len2 += A[a] * A[a];
            const double len = sqrt(len2), h = 2.0 * det0 / len;
            double un = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) un += (EQ == EQ_ADVECTION ? g.vel[a] : s[1 + a] / s[0]) * (A[a] / len);
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
template <int D, int P, int EQ>
__global__ __launch_bounds__(256) void k_mapped_totals_leaf(MappedArgs g, double *part)
{
    constexpr int NV = EQ == EQ_ADVECTION ? 1 : D + 2, NB = Tab<D, P>::NB;
    __shared__ double red[NV][256];
    const int leaf = blockIdx.x, N = g.N, ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(NB) * ncell;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        int ijk[3];
        cell_ijk(c, N, D, ijk);
        double cx[1 << D][3], sc[NV];
        mapped_cell_corners<D>(g.geo[leaf], ijk, N, cx);
        mapped_cell_integrals<D, P, NV>(cx, g.us + long(leaf) * NV * sv + c, sv, ncell, sc);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] += sc[v];
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

// Initial state on mapped cells: M K = int phi_m U0 det(J) dxi with p+3
// Gauss points per axis for the right-hand side and the volume rule for M.
template <int D, int P, int NV>
__global__ __launch_bounds__(128) void k_mapped_project_ic(double *u, const LeafGeo *geo, int N, long ncell_total,
                                                           int kind, IcParams prm, double t, double gamma)
{
    constexpr int NB = Tab<D, P>::NB, QI = P + 3, NQI = ipow(QI, D);
    const int ncell = D == 2 ? N * N : N * N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    const long leaf = gid / ncell;
    const int c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    double cx[1 << D][3];
    mapped_cell_corners<D>(geo[leaf], ijk, N, cx);
    const double hmin[3] = {0.0, 0.0, 0.0};
    double acc[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) acc[v][m] = 0.0;
#pragma unroll 1
    for (int q = 0; q < NQI; ++q) {
        const int qi[3] = {q % QI, (q / QI) % QI, q / (QI * QI)};
        double J[3][3], x[3], xi[3] = {0.0, 0.0, 0.0}, w = 1.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xi[a] = kIcTab<P>.x[qi[a]];
            w *= kIcTab<P>.w[qi[a]];
        }
        const double wd = w * mapped_jacobian<D>(cx, xi, J);
        mapped_point<D>(cx, xi, x);
        double U[D + 2];
        analytic<D>(kind, prm, t, gamma, x, hmin, U);
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            double ph = wd;
#pragma unroll
            for (int a = 0; a < D; ++a) ph *= kIcTab<P>.leg1[qi[a]][kTab<D, P>.e[m][a]];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v][m] = fma(ph, U[v], acc[v][m]);
        }
    }
    double M[NB][NB];
    mapped_mass<D, P>(cx, M);
    mapped_solve<NB, NV>(M, acc);
    const long sv = long(NB) * ncell, base = leaf * NV * sv + c;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) u[base + v * sv + m * ncell] = acc[v][m];
}

} // namespace dgk
