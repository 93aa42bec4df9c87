// Diffusion equation u_t = nu div grad u (Sec. 5.2) with the symmetric
// interior-penalty DG discretisation the paper cites, on the same forest,
// guard cells and SSP-RK3 stages as the Euler path.
//
// One thread per cell.  Per mode m of the cell (outward normal n, own and
// neighbour traces u-/u+, {.} the mean of both sides, sigma = 2 (p+1)^2/h_n):
//   M_m du_m/dt = nu [ - int_K grad u . grad phi_m
//       + sum_faces int_f ( {grad u} . n phi_m + 1/2 (u- - u+) grad phi_m . n
//                           - sigma (u- - u+) phi_m ) ].
// The neighbour across a face is the adjacent cell of the block or, at a
// block face, the guard cell (coefficients written by the fill kernel:
// copy, split or combine, Eq. 15-17).  A domain face (LINK_BOUNDARY) is a
// Dirichlet face with data from the exact solution exp(a . x + nu |a|^2 t)
// at the stage time: its terms are int_f ( grad u- . n phi_m
// + (u- - gD) grad phi_m . n - sigma (u- - gD) phi_m ).
#pragma once

#include "kernels.hpp"

namespace dgk {

// Basis derivatives for the diffusion operator: d phi_m / d xi_a at the
// volume Gauss points, and at the face points of axis a on the side
// xi_a = +1 the normal derivative (the -1 side follows by parity: P_n'(-1)
// = (-1)^(n+1) P_n'(1)).
template <int D, int P>
struct DiffTab {
    static constexpr int NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ, NF = Tab<D, P>::NF, Q = P + 1;
    double dphi_v[D][NQ][NB] = {}; // d phi_m / d xi_a at volume point q
    double wv[NQ] = {};            // volume weights
    double dn_f[D][NF][NB] = {};   // d phi_m / d xi_a at the face point, xi_a = +1
    double wf[NF] = {};            // face weights
    constexpr DiffTab()
    {
        for (int q = 0; q < NQ; ++q) {
            const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
            double w = 1.0;
            for (int a = 0; a < D; ++a) w *= gl_w(Q, qi[a]);
            wv[q] = w;
            for (int ax = 0; ax < D; ++ax)
                for (int m = 0; m < NB; ++m) {
                    double v = 1.0;
                    for (int a = 0; a < D; ++a) {
                        const int e = kTab<D, P>.e[m][a];
                        v *= a == ax ? dleg(e, gl_x(Q, qi[a])) : leg(e, gl_x(Q, qi[a]));
                    }
                    dphi_v[ax][q][m] = v;
                }
        }
        for (int f = 0; f < NF; ++f) wf[f] = gl_w(Q, f % Q) * (D == 3 ? gl_w(Q, f / Q) : 1.0);
        for (int ax = 0; ax < D; ++ax)
            for (int f = 0; f < NF; ++f)
                for (int m = 0; m < NB; ++m) {
                    const int e = kTab<D, P>.e[m][ax];
                    dn_f[ax][f][m] = kTab<D, P>.phi_f[ax][f][m] * (0.5 * e * (e + 1)); // P_e'(1) = e(e+1)/2
                }
    }
};
template <int D, int P>
inline constexpr DiffTab<D, P> kDiffTab{};


// phi_m and d phi_m / d xi_A at face point f of axis A on side s: the +1
// side's tables, with P_e(-1) = (-1)^e and P_e'(-1) = (-1)^(e+1) P_e'(1)
template <int D, int P, int A>
__device__ __forceinline__ double face_phi(int m, int f, int s)
{
    const int e = kTab<D, P>.e[m][A];
    return (s < 0 && (e & 1)) ? -kTab<D, P>.phi_f[A][f][m] : kTab<D, P>.phi_f[A][f][m];
}
template <int D, int P, int A>
__device__ __forceinline__ double face_dphi(int m, int f, int s)
{
    const int e = kTab<D, P>.e[m][A];
    return (s < 0 && !(e & 1)) ? -kDiffTab<D, P>.dn_f[A][f][m] : kDiffTab<D, P>.dn_f[A][f][m];
}

// value and normal derivative (d/dxi_A) of the polynomial k at face point f
// of axis A on side s
template <int D, int P, int A>
__device__ __forceinline__ void face_val_dn(const double *k, int f, int s, double &val, double &dn)
{
    constexpr int NB = Tab<D, P>::NB;
    val = 0.0;
    dn = 0.0;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        val = fma(face_phi<D, P, A>(m, f, s), k[m], val);
        dn = fma(face_dphi<D, P, A>(m, f, s), k[m], dn);
    }
}

template <int D, int P, int OM>
__global__ __launch_bounds__(256) void k_ipdg(IpdgArgs g)
{
    constexpr int NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ, NF = Tab<D, P>::NF, Q = P + 1;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= g.ncell_total) return;
    const int leaf = int(gid / ncell), c = int(gid % ncell);
    int ijk[3];
    cell_ijk(c, N, D, ijk);
    const LeafGeo G = g.geo[leaf];
    const double *K0 = g.us + long(leaf) * NB * ncell + c;
    double K[NB], R[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        K[m] = K0[long(m) * ncell];
        R[m] = 0.0;
    }
    // ---- volume: - int grad u . grad phi_m  (|J| divided out: the factors
    // (2/h_a)^2 remain)
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
            constexpr int A = Ai;
            double gq = 0.0;
#pragma unroll
            for (int n = 0; n < NB; ++n) gq = fma(kDiffTab<D, P>.dphi_v[A][q][n], K[n], gq);
            const double s2 = G.scale[A] * G.scale[A] * kDiffTab<D, P>.wv[q];
#pragma unroll
            for (int m = 0; m < NB; ++m) R[m] = fma(-s2 * kDiffTab<D, P>.dphi_v[A][q][m], gq, R[m]);
        });
    }
    // ---- faces (J_f / |J| = 2/h_a)
    static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
        constexpr int A = Ai;
        const double sc = G.scale[A];                       // 2/h_A
        const double sigma = 2.0 * (P + 1) * (P + 1) * 0.5 * sc; // 2 (p+1)^2 / h_A
        const int stride = A == 0 ? 1 : (A == 1 ? N : N * N);
        const int t = face_t(ijk, A, N, D);
#pragma unroll 1
        for (int si = 0; si < 2; ++si) {
            const int s = si ? 1 : -1;
            const int face = 2 * A + si;
            const bool interior = s > 0 ? ijk[A] < N - 1 : ijk[A] > 0;
            const FaceLink L = g.links[leaf * 2 * D + face];
            const bool dirichlet = !interior && L.type == dgamr::LINK_BOUNDARY;
            double Kn[NB];
            if (interior) {
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[m] = K0[long(m) * ncell + s * stride];
            } else if (!dirichlet) {
                const double *gk = g.guard + (long(leaf) * 2 * D + face) * NB * nfc + t;
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[m] = gk[long(m) * nfc];
            } else {
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[m] = 0.0;
            }
#pragma unroll 1
            for (int f = 0; f < NF; ++f) {
                double um, dm, up, dp;
                face_val_dn<D, P, A>(K, f, s, um, dm);
                if (dirichlet) {
                    // physical face point
                    double x[3] = {0.0, 0.0, 0.0}, xi[3] = {0.0, 0.0, 0.0};
                    const int f0 = f % Q, f1 = f / Q;
                    int k = 0;
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        if (b == A) xi[b] = double(s);
                        else xi[b] = gl_x(Q, k++ == 0 ? f0 : f1);
                    }
                    leaf_point<D>(G, ijk, xi, x);
                    double e = 0.0, a2 = 0.0;
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        e = fma(g.avec[b], x[b], e);
                        a2 = fma(g.avec[b], g.avec[b], a2);
                    }
                    up = exp(e + g.nu * a2 * g.t);
                    dp = dm;
                } else {
                    face_val_dn<D, P, A>(Kn, f, -s, up, dp);
                }
                // normal derivatives in physical units, times the normal's sign
                const double gm = sc * dm, gp = sc * dp;
                const double flux_n = s * (dirichlet ? gm : 0.5 * (gm + gp));
                const double jump = um - up;
                const double wsym = dirichlet ? 1.0 : 0.5;
                const double w = kDiffTab<D, P>.wf[f] * sc;
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const double ph = face_phi<D, P, A>(m, f, s);
                    const double dnm = sc * face_dphi<D, P, A>(m, f, s); // d phi_m / dx_A
                    R[m] = fma(w, flux_n * ph + wsym * jump * s * dnm - sigma * jump * ph, R[m]);
                }
            }
        }
    });
#pragma unroll
    for (int m = 0; m < NB; ++m) R[m] *= g.nu * kTab<D, P>.inv_mass[m];
    double *o = g.out + long(leaf) * NB * ncell + c;
    if constexpr (OM == OUT_RES64) {
#pragma unroll
        for (int m = 0; m < NB; ++m) o[long(m) * ncell] = R[m];
    } else {
        const double dt = *g.dt, a = g.rk_a, b = g.rk_b;
        const double *U0 = g.un + long(leaf) * NB * ncell + c;
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            double v = b * (K[m] + dt * R[m]);
            if (a != 0.0) v = fma(a, U0[long(m) * ncell], v);
            o[long(m) * ncell] = v;
        }
    }
}

} // namespace dgk
