// 2-D DG stage kernel with one lane per (cell, variable).
//
// The four conserved variables of a cell live in the four lanes of one
// DPP quad: each lane keeps only its variable's coefficients and residual,
// contracts them with the basis tables, and fetches the other three
// variables' point values with quad broadcasts when the Euler flux or the
// Rusanov flux needs the full state.  A workgroup covers a slab of rows of
// one leaf (all of it for large forests), so a small forest still spreads
// over every compute unit with several waves per SIMD.  Faces inside the
// slab are computed once and shared through LDS; faces on a slab edge that
// lies inside the leaf are recomputed from the neighbouring row, and faces
// on the leaf boundary take the far side from the guard buffer or, inline,
// from the neighbour leaf (copy, split, combine, outflow mirror).
#pragma once

#include "kernels.hpp"

namespace dgk {

// value of x held by lane K of this lane's quad
template <int K>
__device__ __forceinline__ double quad_bcast(double x)
{
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6); // DPP quad_perm
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Full state of the cell from the four lanes' values of their variable.
__device__ __forceinline__ void quad_state(double x, double *U)
{
    U[0] = quad_bcast<0>(x);
    U[1] = quad_bcast<1>(x);
    U[2] = quad_bcast<2>(x);
    U[3] = quad_bcast<3>(x);
}

// Euler flux component of variable v along axis A (Eq. 2): F_v = U_v u_A
// + p [v = 1 + A] + p u_A [v = E].
template <int A>
__device__ __forceinline__ double flux_v(double uv, double ua, double p, double isM, double isE)
{
    return fma(uv, ua, p * (isM + isE * ua));
}

// Rusanov flux (Eq. 5, dissipative sign, +e_A direction) of this lane's
// variable between left value tl and right value tr; the other variables
// come from the quad.
template <int A>
__device__ __forceinline__ double rusanov_v(double tl, double tr, double gamma, double isM, double isE)
{
    double L[4], R[4];
    quad_state(tl, L);
    quad_state(tr, R);
    const double gm1 = gamma - 1.0;
    const double rl = recip(L[0]), rr = recip(R[0]);
    const double pl = pressure_r<2>(L, gm1, rl), pr = pressure_r<2>(R, gm1, rr);
    const double ul = L[1 + A] * rl, ur = R[1 + A] * rr;
    const double al = fabs(ul) + sqrt_nn(gamma * pl * rl), ar = fabs(ur) + sqrt_nn(gamma * pr * rr);
    const double alpha = al > ar ? al : ar;
    const double fl = flux_v<A>(tl, ul, pl, isM, isE), fr = flux_v<A>(tr, ur, pr, isM, isE);
    return 0.5 * ((fl + fr) - alpha * (tr - tl));
}

// trace of one variable's polynomial at face point f of axis A on side s
template <int P, int A>
__device__ __forceinline__ double trace1(const double *k, int f, int s)
{
    double e, o;
    trace_eo<2, P>(k, A, f, e, o);
    return s > 0 ? e + o : e - o;
}

// Far-side polynomial (this lane's variable) of leaf face (A, side) for the
// cell with tangential index t: the stored guard cell, or inline the
// same-level neighbour cell (Eq. 15), the split of the coarser neighbour
// cell (Eq. 16), the combine of the four finer cells (Eq. 17), or at an
// outflow boundary the mirror image K_m (-1)^{m_A}.
template <int P, int A, int GM>
__device__ __forceinline__ void far_coeffs_v(const StageArgs &g, const double *K, int v, int leaf, int side, int t,
                                             const FaceLink &L, double *kv)
{
    constexpr int NV = 4, NB = Tab<2, P>::NB;
    const int N = g.N, ncell = N * N;
    const long sv = long(NB) * ncell;
    const int face = 2 * A + (side > 0);
    if (GM == GUARD_BUFFER) {
        const double *gk = g.guard + ((long(leaf) * 4 + face) * NV * NB) * N + long(v) * NB * N + t;
#pragma unroll
        for (int m = 0; m < NB; ++m) kv[m] = gk[m * N];
    } else if (L.type == dgamr::LINK_BOUNDARY) {
#pragma unroll
        for (int m = 0; m < NB; ++m) kv[m] = (kTab<2, P>.e[m][A] % 2) ? -K[m] : K[m];
    } else if (L.type == dgamr::LINK_SAME) {
        const int c = same_cell(A, side, t, N, 2);
        const double *nk = g.us + long(L.nbr[0]) * NV * sv + v * sv + c;
#pragma unroll
        for (int m = 0; m < NB; ++m) kv[m] = nk[m * ncell];
    } else if (L.type == dgamr::LINK_COARSE) {
        const int c = coarse_cell(A, side, t, L.off, N, 2);
        const int child = coarse_child(A, side, t, N, 2);
        const double *ck = g.us + long(L.nbr[0]) * NV * sv + v * sv + c;
        double kc[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) kc[m] = ck[m * ncell];
        split_any<2, P>(child, kc, kv);
    } else { // LINK_FINE
        const double *fk = g.us + long(link_nbr(L, fine_block(t, N, 2))) * NV * sv + v * sv;
        double kf[4][NB];
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const int fc = fine_cell(A, side, t, ch, N, 2);
#pragma unroll
            for (int n = 0; n < NB; ++n) kf[ch][n] = fk[n * ncell + fc];
        }
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            double s = 0.0;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    const double cc = kTab<2, P>.comb[ch][m][n];
                    if (cc != 0.0) s = fma(cc, kf[ch][n], s);
                }
            kv[m] = s;
        }
    }
}

// Conservative hanging face, this lane's variable: Rusanov flux at the
// fine sub-faces' Gauss points with the fine cells' own traces, lifted with
// the own basis at the mapped points.
template <int P, int A>
__device__ __forceinline__ void mortar_lift_v(const StageArgs &g, const double *K, double *R, int v, int side, const FaceLink L,
                              int t, double scale, double isM, double isE)
{
    constexpr int NV = 4, NB = Tab<2, P>::NB, Q = P + 1;
    constexpr int TA = 1 - A;
    const int N = g.N, ncell = N * N;
    const long sv = long(NB) * ncell;
    const double *fk0 = g.us + long(link_nbr(L, fine_block(t, N, 2))) * NV * sv + v * sv;
    // the fine cells touching the face: children with the half along A
    // nearest to this block
    const int near = (side > 0 ? 0 : 1) << A;
#pragma unroll 1
    for (int S = 0; S < 2; ++S) {
        const double *fk = fk0 + fine_cell(A, side, t, near | (S << TA), N, 2);
        double kf[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) kf[m] = fk[m * ncell];
#pragma unroll 1
        for (int F = 0; F < Q; ++F) {
            const double x0 = 0.5 * (gl_x(Q, F) + (S ? 1.0 : -1.0));
            const double uf = trace1<P, A>(kf, F, -side);
            double ec = 0.0, oc = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = leg(kTab<2, P>.e[m][TA], x0);
                if (kTab<2, P>.e[m][A] % 2 == 0) ec = fma(c, K[m], ec);
                else oc = fma(c, K[m], oc);
            }
            const double uc = side > 0 ? ec + oc : ec - oc;
            const double phi = side > 0 ? rusanov_v<A>(uc, uf, g.gamma, isM, isE)
                                        : rusanov_v<A>(uf, uc, g.gamma, isM, isE);
            const double f = scale * 0.5 * gl_w(Q, F) * phi;
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = leg(kTab<2, P>.e[m][TA], x0) * kTab<2, P>.inv_mass[m];
                const double sg = side > 0 ? -1.0 : ((kTab<2, P>.e[m][A] % 2) ? -1.0 : 1.0);
                R[m] = fma(sg * c, f, R[m]);
            }
        }
    }
}

// grid: nleaves * (N / rows) workgroups of rows*N*4 threads (<= 512)
template <int P, int GM, int OM>
__global__ __launch_bounds__(512) void k_stage2v(StageArgs g, int rows)
{
    constexpr int NV = 4, NB = Tab<2, P>::NB, NQ = Tab<2, P>::NQ, NF = P + 1;
    extern __shared__ double lds[];
    const int N = g.N, ncell = N * N;
    const int slabs = N / rows;
    const int wg = xcd_leaf(blockIdx.x, g.nleaves * slabs);
    const int li = wg / slabs, j0 = (wg % slabs) * rows;
    const int leaf = g.work ? g.work[li] : li; // listed leaves of a pool, or all
    const int lane = threadIdx.x, v = lane & 3;
    const int lc = lane >> 2;             // cell inside the slab
    const int i = lc % N, j = j0 + lc / N;
    const int cell = i + N * j;
    const int nslab = rows * N;           // cells in the slab
    const bool x_in_wave = 64 % (4 * N) == 0; // uniform
    const double isE = v == 3 ? 1.0 : 0.0;
    const double scale[2] = {g.geo[leaf].scale[0], g.geo[leaf].scale[1]};
    const long sv = long(NB) * ncell;
    const long vbase = long(leaf) * NV * sv + v * sv;
    const long idx0 = vbase + cell;

    // ---- every global read up front, so one memory round trip overlaps the
    // volume integral: own coefficients, the RK base state, and the
    // polynomial across each face of this cell that is not inside the slab
    double K[NB], R[NB], Un[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        K[m] = g.us[idx0 + m * ncell];
        R[m] = 0.0;
    }
    if constexpr (OM == OUT_RK) {
        if (g.rk_a != 0.0) { // uniform: stages 2 and 3
#pragma unroll
            for (int m = 0; m < NB; ++m) Un[m] = g.un[idx0 + m * ncell];
        } else {
#pragma unroll
            for (int m = 0; m < NB; ++m) Un[m] = 0.0;
        }
    }
    const FaceLink Lxm = g.links[leaf * 4 + 0], Lxp = g.links[leaf * 4 + 1];
    const FaceLink Lym = g.links[leaf * 4 + 2], Lyp = g.links[leaf * 4 + 3];
    const bool mort_xm = g.conservative && i == 0 && Lxm.type == dgamr::LINK_FINE;
    const bool mort_xp = g.conservative && i == N - 1 && Lxp.type == dgamr::LINK_FINE;
    const bool mort_ym = g.conservative && j == 0 && Lym.type == dgamr::LINK_FINE;
    const bool mort_yp = g.conservative && j == N - 1 && Lyp.type == dgamr::LINK_FINE;
    double far_xm[NB], far_xp[NB], far_ym[NB], far_yp[NB];
    if (i == 0 && !mort_xm) far_coeffs_v<P, 0, GM>(g, K, v, leaf, -1, j, Lxm, far_xm);
    if (i == N - 1 && !mort_xp) far_coeffs_v<P, 0, GM>(g, K, v, leaf, +1, j, Lxp, far_xp);
    if (j == j0) {
        if (j > 0) { // slab edge inside the leaf: the row below
#pragma unroll
            for (int m = 0; m < NB; ++m) far_ym[m] = g.us[idx0 + m * ncell - N];
        } else if (!mort_ym) {
            far_coeffs_v<P, 1, GM>(g, K, v, leaf, -1, i, Lym, far_ym);
        }
    }
    if (j == j0 + rows - 1) {
        if (j < N - 1) { // slab edge inside the leaf: the row above
#pragma unroll
            for (int m = 0; m < NB; ++m) far_yp[m] = g.us[idx0 + m * ncell + N];
        } else if (!mort_yp) {
            far_coeffs_v<P, 1, GM>(g, K, v, leaf, +1, i, Lyp, far_yp);
        }
    }

    // ---- volume integral
    const double gm1 = g.gamma - 1.0;
    const double isMx = v == 1 ? 1.0 : 0.0, isMy = v == 2 ? 1.0 : 0.0;
    static_for<0, NQ>([&](auto Qi) {
        constexpr int q = Qi;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const double c = kTab<2, P>.phi_v[q][m];
            if (c != 0.0) s = fma(c, K[m], s);
        }
        double U[4];
        quad_state(s, U);
        const double rinv = recip(U[0]);
        const double p = pressure_r<2>(U, gm1, rinv);
        const double fx = scale[0] * flux_v<0>(s, U[1] * rinv, p, isMx, isE);
        const double fy = scale[1] * flux_v<1>(s, U[2] * rinv, p, isMy, isE);
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const double cx = kTab<2, P>.dproj[0][q][m], cy = kTab<2, P>.dproj[1][q][m];
            if (cx != 0.0) R[m] = fma(cx, fx, R[m]);
            if (cy != 0.0) R[m] = fma(cy, fy, R[m]);
        }
    });

    // ---- surface integrals; LDS slot of (face point f, slab cell, var)
    auto slot = [&](int f, int c) { return (f * nslab + c) * 4 + v; };
    static_for<0, 2>([&](auto Ai) {
        constexpr int A = Ai;
        // x faces join cells of one row; when whole rows fill whole waves
        // (4 N divides 64) the x exchange stays inside a wave
        auto sync_axis = [&]() __attribute__((always_inline)) {
            if (A == 0 && x_in_wave) wave_lds_sync();
            else __syncthreads();
        };
        const double isM = v == 1 + A ? 1.0 : 0.0;
        const int ia = A == 0 ? i : j;
        const int t = A == 0 ? j : i;
        const int stride = A == 0 ? 1 : N;
        // the neighbour across a face is in this slab unless the face is on
        // the leaf boundary or (A = 1) on the slab's edge
        const bool lds_m = A == 0 ? i > 0 : j > j0;
        const bool lds_p = A == 0 ? i < N - 1 : j < j0 + rows - 1;
        const bool mort_m = A == 0 ? mort_xm : mort_ym;
        const bool mort_p = A == 0 ? mort_xp : mort_yp;
        const auto &far_m = [&]() -> const double(&)[NB] {
            if constexpr (A == 0) return far_xm;
            else return far_ym;
        }();
        const auto &far_p = [&]() -> const double(&)[NB] {
            if constexpr (A == 0) return far_xp;
            else return far_yp;
        }();
        const double sc = scale[A];
        if (mort_m) mortar_lift_v<P, A>(g, K, R, v, -1, A == 0 ? Lxm : Lym, t, sc, isM, isE);
        if (mort_p) mortar_lift_v<P, A>(g, K, R, v, +1, A == 0 ? Lxp : Lyp, t, sc, isM, isE);
        double Tm[NF], Fm[NF], Fp[NF];
        sync_axis();
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double e, o;
            trace_eo<2, P>(K, A, f, e, o);
            lds[slot(f, lc)] = e + o;
            Tm[f] = e - o;
        }
        sync_axis();
        // - face: left state = the + trace of the polynomial below
        if (mort_m) {
#pragma unroll
            for (int f = 0; f < NF; ++f) Fm[f] = 0.0;
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double tl = lds_m ? lds[slot(f, lc - stride)] : trace1<P, A>(far_m, f, +1);
                Fm[f] = rusanov_v<A>(tl, Tm[f], g.gamma, isM, isE);
            }
        }
        sync_axis();
#pragma unroll
        for (int f = 0; f < NF; ++f) lds[slot(f, lc)] = Fm[f];
        sync_axis();
        // + face: computed by the cell above, unless that cell is outside the slab
        if (lds_p) {
#pragma unroll
            for (int f = 0; f < NF; ++f) Fp[f] = lds[slot(f, lc + stride)];
        } else if (mort_p) {
#pragma unroll
            for (int f = 0; f < NF; ++f) Fp[f] = 0.0;
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                Fp[f] = rusanov_v<A>(trace1<P, A>(K, f, +1), trace1<P, A>(far_p, f, -1), g.gamma, isM, isE);
        }
        // lift
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double dm = sc * Fm[f], dp = sc * Fp[f];
            const double even = dm - dp, odd = -(dm + dp);
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = kTab<2, P>.lift_f[A][f][m];
                if (c != 0.0) R[m] = fma(c, (kTab<2, P>.e[m][A] % 2 == 0) ? even : odd, R[m]);
            }
        }
    });

    // ---- output (this lane's variable)
    static_assert(OM == OUT_RES64 || OM == OUT_RK, "the FP32 residual runs one thread per cell");
    if constexpr (OM == OUT_RES64) {
#pragma unroll
        for (int m = 0; m < NB; ++m) g.out64[idx0 + m * ncell] = R[m];
    } else {
        double dt;
        if (g.rate_in) {
            dt = g.cfl / __longlong_as_double((long long)*g.rate_in);
            if (blockIdx.x == 0 && threadIdx.x == 0) *g.dt_out = dt;
        } else {
            dt = g.dt[g.leaf_member ? g.leaf_member[leaf] : 0];
        }
        if (g.rate_clear && blockIdx.x == 0 && threadIdx.x == 0) *g.rate_clear = 0ULL;
        const double a = g.rk_a, b = g.rk_b;
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            K[m] = a * Un[m] + b * (K[m] + dt * R[m]);
            g.out64[idx0 + m * ncell] = K[m];
        }
        if (g.rate_out) {
            double U[4];
            quad_state(K[0], U);
            const double rinv = 1.0 / U[0];
            const double cs = sqrt(g.gamma * pressure_r<2>(U, gm1, rinv) * rinv);
            const double rate = (fabs(U[1] * rinv) + cs) / g.geo[leaf].h[0] + (fabs(U[2] * rinv) + cs) / g.geo[leaf].h[1];
            block_max_to(rate, lds, g.rate_out); // the four lanes of a cell hold the same rate
        }
    }
}

} // namespace dgk
