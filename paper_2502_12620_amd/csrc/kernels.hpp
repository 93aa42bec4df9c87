// HIP kernels of the DG stage for gfx950: guard-cell fill (Sec. 3.5,
// Eq. 15-17) and the residual of the Galerkin weak form (Sec. 2, Eq. 3-5),
// optionally fused with the SSP-RK3 stage update.
//
// One workgroup per leaf, one thread per cell.  The thread keeps its cell's
// coefficients K[var][mode] and residual R[var][mode] in registers; the
// basis tables are compile-time constants, so after full unrolling every
// table entry is an immediate and structural zeros disappear.  The flux of
// each face inside the block is computed once: the + trace of every cell
// goes through LDS to its + neighbour, which computes the Rusanov flux and
// sends it back through LDS.
#pragma once

#include <type_traits>

#include "kernel_common.hpp"

namespace dgk {

// one cell's coefficients (or residual) per variable and mode
template <int D, int P>
using CellCoef = double[D + 2][Tab<D, P>::NB];

// Number of face points exchanged through LDS at once: all of them in 2-D,
// one at a time in 3-D (keeps the register budget to one cell's state and
// residual).
template <int D, int P>
constexpr int face_chunk() { return D == 2 ? (P == 3 ? 2 : Tab<D, P>::NF) : 1; }

// Full unrolling over the quadrature points makes every table entry an
// immediate.  In 3-D the unrolled code and its live ranges outgrow the
// register file (one cell's state and residual already take 4 NB VGPRs per
// variable), so there the point loops stay loops over tables read with
// scalar loads.
template <int D, int P>
constexpr bool unroll_points() { return D == 2; }

// Whether to apply table entry c taken at a point of such a loop: unrolled,
// c is an immediate and its structural zeros drop out; in a loop, c is a
// runtime value and a multiply by zero costs less than a branch on it.
template <int D, int P>
__device__ __forceinline__ bool use_entry(double c) { return !unroll_points<D, P>() || c != 0.0; }

// even / odd parts (in the normal mode index) of the trace of K at face
// point f of axis a: the trace at xi_a = +1 is e + o, at xi_a = -1 it is e - o.
template <int D, int P, typename T>
__device__ __forceinline__ void trace_eo(const T *K, int a, int f, T &e, T &o)
{
    e = T(0);
    o = T(0);
#pragma unroll
    for (int m = 0; m < Tab<D, P>::NB; ++m) {
        const double c = kTab<D, P>.phi_f[a][f][m];
        if (use_entry<D, P>(c)) {
            if (kTab<D, P>.e[m][a] % 2 == 0) e = fma(T(c), K[m], e);
            else o = fma(T(c), K[m], o);
        }
    }
}

// the same for coefficients streamed from memory (coef[m*sm])
template <int D, int P, typename T>
__device__ __forceinline__ void trace_eo_mem(const double *__restrict__ coef, long sm, int a, int f, T &e, T &o)
{
    e = T(0);
    o = T(0);
#pragma unroll
    for (int m = 0; m < Tab<D, P>::NB; ++m) {
        const double c = kTab<D, P>.phi_f[a][f][m];
        if (use_entry<D, P>(c)) {
            const T k = T(coef[m * sm]);
            if (kTab<D, P>.e[m][a] % 2 == 0) e = fma(T(c), k, e);
            else o = fma(T(c), k, o);
        }
    }
}

// Conservative hanging-face flux: the coarse cell integrates the Rusanov
// flux over the 2^(d-1) fine sub-faces at the fine Gauss points, with the
// fine cells' own traces, and lifts it with its own basis evaluated at the
// mapped points (tangential xi = (xi_fine + sigma)/2).
template <int D, int P, int A, int EQ, typename T>
__device__ __forceinline__ void mortar_lift(const StageArgs &g, const T (&K)[nvar<D, EQ>()][Tab<D, P>::NB],
                                            T (&R)[nvar<D, EQ>()][Tab<D, P>::NB], int side, const FaceLink L, int t,
                                            T scale)
{
    constexpr int NV = nvar<D, EQ>(), NB = Tab<D, P>::NB, Q = P + 1, NF = Tab<D, P>::NF;
    constexpr int TA = A == 0 ? 1 : 0, TBX = A == 2 ? 1 : 2; // tangential axes, lower first
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(NB) * ncell;
    const int fleaf = link_nbr(L, fine_block(t, N, D));
    // the fine cells touching the face: children with the half along A
    // nearest to this block
    const int near = (side > 0 ? 0 : 1) << A;
    const double sub = D == 2 ? 0.5 : 0.25; // fine face Jacobian / coarse face Jacobian
    // runs only on hanging faces: kept as loops (table values computed on
    // the fly) to keep the code small
#pragma unroll 1
    for (int S = 0; S < (1 << (D - 1)); ++S) {
        const int s0 = S & 1, s1 = (S >> 1) & 1;
        const int fcell = fine_cell(A, side, t, near | (s0 << TA) | (s1 << TBX), N, D);
        const double *fk = g.us + long(fleaf) * NV * sv + fcell;
#pragma unroll 1
        for (int F = 0; F < NF; ++F) {
            const int q0 = F % Q, q1 = F / Q;
            const double x0 = 0.5 * (gl_x(Q, q0) + (s0 ? 1.0 : -1.0));
            const double x1 = 0.5 * (gl_x(Q, q1) + (s1 ? 1.0 : -1.0));
            const double w = gl_w(Q, q0) * (D == 3 ? gl_w(Q, q1) : 1.0);
            T Uf[NV], Uc[NV], Phi[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T e, o;
                trace_eo_mem<D, P, T>(fk + v * sv, ncell, A, F, e, o);
                Uf[v] = side > 0 ? e - o : e + o; // the fine cell touches the face with its -side side
                T ec = T(0), oc = T(0);
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const double c = leg(kTab<D, P>.e[m][TA], x0) * (D == 3 ? leg(kTab<D, P>.e[m][TBX], x1) : 1.0);
                    if (c != 0.0) {
                        if (kTab<D, P>.e[m][A] % 2 == 0) ec = fma(T(c), K[v][m], ec);
                        else oc = fma(T(c), K[v][m], oc);
                    }
                }
                Uc[v] = side > 0 ? ec + oc : ec - oc;
            }
            if (side > 0) num_flux<D, A, EQ, T>(g, Uc, Uf, T(g.gamma), Phi);
            else num_flux<D, A, EQ, T>(g, Uf, Uc, T(g.gamma), Phi);
            // +face: -int Phi phi ; -face: +int Phi phi with phi(-1) = (-1)^{m_A} phi(+1)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const T f = scale * T(sub * w) * Phi[v];
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const double c = leg(kTab<D, P>.e[m][TA], x0) * (D == 3 ? leg(kTab<D, P>.e[m][TBX], x1) : 1.0) *
                                     kTab<D, P>.inv_mass[m];
                    if (c != 0.0) {
                        const double sg = side > 0 ? -1.0 : ((kTab<D, P>.e[m][A] % 2) ? -1.0 : 1.0);
                        R[v][m] = fma(T(sg * c), f, R[v][m]);
                    }
                }
            }
        }
    }
}

// Coefficients of the split of a coarse cell for child CH (Eq. 11-12):
// g = S_CH k, one variable at a time.
template <int D, int P, int CH, typename T>
__host__ __device__ __forceinline__ void split_coeffs(const T *k, T *gk)
{
    constexpr int NB = Tab<D, P>::NB;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        T s = T(0);
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const double c = kTab<D, P>.split[CH][m][n];
            if (c != 0.0) s = fma(T(c), k[n], s);
        }
        gk[m] = s;
    }
}

template <int D, int P, typename T>
__host__ __device__ __forceinline__ void split_any(int child, const T *k, T *gk)
{
    switch (child) {
    case 0: split_coeffs<D, P, 0, T>(k, gk); break;
    case 1: split_coeffs<D, P, 1, T>(k, gk); break;
    case 2: split_coeffs<D, P, 2, T>(k, gk); break;
    case 3: split_coeffs<D, P, 3, T>(k, gk); break;
    case 4: if constexpr (D == 3) split_coeffs<D, P, 4, T>(k, gk); break;
    case 5: if constexpr (D == 3) split_coeffs<D, P, 5, T>(k, gk); break;
    case 6: if constexpr (D == 3) split_coeffs<D, P, 6, T>(k, gk); break;
    default: if constexpr (D == 3) split_coeffs<D, P, 7, T>(k, gk); break;
    }
}

// Adds the combine contribution of child CH (Eq. 13-14): gk += C_CH k.
template <int D, int P, int CH>
__device__ __forceinline__ void comb_coeffs(const double *k, double *gk)
{
    constexpr int NB = Tab<D, P>::NB;
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const double c = kTab<D, P>.comb[CH][m][n];
            if (c != 0.0) gk[m] = fma(c, k[n], gk[m]);
        }
}

template <int D, int P>
__device__ __forceinline__ void comb_any(int child, const double *k, double *gk)
{
    switch (child) {
    case 0: comb_coeffs<D, P, 0>(k, gk); break;
    case 1: comb_coeffs<D, P, 1>(k, gk); break;
    case 2: comb_coeffs<D, P, 2>(k, gk); break;
    case 3: comb_coeffs<D, P, 3>(k, gk); break;
    case 4: if constexpr (D == 3) comb_coeffs<D, P, 4>(k, gk); break;
    case 5: if constexpr (D == 3) comb_coeffs<D, P, 5>(k, gk); break;
    case 6: if constexpr (D == 3) comb_coeffs<D, P, 6>(k, gk); break;
    default: if constexpr (D == 3) comb_coeffs<D, P, 7>(k, gk); break;
    }
}

// Far-side traces of block face (A, side) at the FCH face points starting
// at f0, for the cell with tangential index t (the far polynomial touches
// the face with its -side side):
//  - guard-buffer mode: the stored guard cell;
//  - inline mode: the same-level neighbour cell (Eq. 15), the split of the
//    coarser neighbour cell (Eq. 16), the combine of the 2^d finer cells
//    (Eq. 17), or at an outflow boundary the mirror image, whose trace is
//    the own trace.
template <int D, int P, int A, int GM, int FCH, int NV, typename T>
__device__ __forceinline__ void far_traces(const StageArgs &g, const T (&K)[NV][Tab<D, P>::NB], int leaf, int side,
                                           int t, const FaceLink &L, int f0, T (&Tr)[FCH][NV])
{
    constexpr int NB = Tab<D, P>::NB;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long sv = long(NB) * ncell;
    const int face = 2 * A + (side > 0);
    auto traces_of = [&](const T *kv, int v, int poly_side) {
#pragma unroll
        for (int fi = 0; fi < FCH; ++fi) {
            T e, o;
            trace_eo<D, P, T>(kv, A, f0 + fi, e, o);
            Tr[fi][v] = poly_side > 0 ? e + o : e - o;
        }
    };
    if (GM == GUARD_TRACE) {
        constexpr int NF = Tab<D, P>::NF;
        const double *gt = g.guard + ((long(leaf) * 2 * D + face) * NV * NF) * nfc + t;
#pragma unroll
        for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
            for (int v = 0; v < NV; ++v) Tr[fi][v] = T(gt[(long(v) * NF + f0 + fi) * nfc]);
        return;
    }
    if (GM == GUARD_BUFFER) {
        const double *gk = g.guard + ((long(leaf) * 2 * D + face) * NV * NB) * nfc + t;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T kv[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) kv[m] = T(gk[(long(v) * NB + m) * nfc]);
            traces_of(kv, v, -side);
        }
        return;
    }
    if (L.type == dgamr::LINK_BOUNDARY) {
#pragma unroll
        for (int v = 0; v < NV; ++v) traces_of(K[v], v, side);
    } else if (L.type == dgamr::LINK_SAME) {
        const int c = same_cell(A, side, t, N, D);
        const double *nk = g.us + long(L.nbr[0]) * NV * sv + c;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T kv[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) kv[m] = T(nk[v * sv + m * ncell]);
            traces_of(kv, v, -side);
        }
    } else if (L.type == dgamr::LINK_COARSE) {
        const int c = coarse_cell(A, side, t, L.off, N, D);
        const int child = coarse_child(A, side, t, N, D);
        const double *ck = g.us + long(L.nbr[0]) * NV * sv + c;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T kv[NB], gv[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) kv[m] = T(ck[v * sv + m * ncell]);
            split_any<D, P, T>(child, kv, gv);
            traces_of(gv, v, -side);
        }
    } else { // LINK_FINE
        const double *fk = g.us + long(link_nbr(L, fine_block(t, N, D))) * NV * sv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T gv[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) gv[m] = T(0);
#pragma unroll
            for (int ch = 0; ch < (1 << D); ++ch) {
                const int fc = fine_cell(A, side, t, ch, N, D);
                T kv[NB];
#pragma unroll
                for (int n = 0; n < NB; ++n) kv[n] = T(fk[v * sv + n * ncell + fc]);
#pragma unroll
                for (int m = 0; m < NB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        const double cc = kTab<D, P>.comb[ch][m][n];
                        if (cc != 0.0) gv[m] = fma(T(cc), kv[n], gv[m]);
                    }
            }
            traces_of(gv, v, -side);
        }
    }
}

// Far-side polynomial of block face (A, side) for the cell with tangential
// index t, per variable (its traces at the face are taken at -side):
//  - guard-buffer mode: the stored guard cell;
//  - inline mode: the same-level neighbour cell (Eq. 15), the split of the
//    coarser neighbour cell (Eq. 16), the combine of the 2^d finer cells
//    (Eq. 17), or at an outflow boundary the mirror image K_m (-1)^{m_A}.
template <int D, int P, int A, int GM, int NV, typename T>
__host__ __device__ __forceinline__ void far_poly(const StageArgs &g, const T (&K)[NV][Tab<D, P>::NB], int leaf, int side,
                                         int t, const FaceLink &L, T (&Kf)[NV][Tab<D, P>::NB])
{
    constexpr int NB = Tab<D, P>::NB;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long sv = long(NB) * ncell;
    const int face = 2 * A + (side > 0);
    if constexpr (GM == GUARD_BUFFER) {
        const double *gk = g.guard + ((long(leaf) * 2 * D + face) * NV * NB) * nfc + t;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) Kf[v][m] = T(gk[(long(v) * NB + m) * nfc]);
        return;
    }
    if (L.type == dgamr::LINK_BOUNDARY) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) Kf[v][m] = (kTab<D, P>.e[m][A] % 2) ? -K[v][m] : K[v][m];
    } else if (L.type == dgamr::LINK_SAME) {
        const int c = same_cell(A, side, t, N, D);
        const double *nk = g.us + long(L.nbr[0]) * NV * sv + c;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) Kf[v][m] = T(nk[v * sv + m * ncell]);
    } else if (L.type == dgamr::LINK_COARSE) {
        const int c = coarse_cell(A, side, t, L.off, N, D);
        const int child = coarse_child(A, side, t, N, D);
        const double *ck = g.us + long(L.nbr[0]) * NV * sv + c;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T kv[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) kv[m] = T(ck[v * sv + m * ncell]);
            split_any<D, P, T>(child, kv, Kf[v]);
        }
    } else { // LINK_FINE
        const double *fk = g.us + long(link_nbr(L, fine_block(t, N, D))) * NV * sv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int m = 0; m < NB; ++m) Kf[v][m] = T(0);
#pragma unroll
            for (int ch = 0; ch < (1 << D); ++ch) {
                const int fc = fine_cell(A, side, t, ch, N, D);
                T kv[NB];
#pragma unroll
                for (int n = 0; n < NB; ++n) kv[n] = T(fk[v * sv + n * ncell + fc]);
#pragma unroll
                for (int m = 0; m < NB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        const double cc = kTab<D, P>.comb[ch][m][n];
                        if (cc != 0.0) Kf[v][m] = fma(T(cc), kv[n], Kf[v][m]);
                    }
            }
        }
    }
}

// ------------------------------------------------------------------ positivity limiter
// Gauss-Lobatto rule of Zhang and Shu's point set: the fewest points L
// (L >= 2) whose rule is exact for degree P (2L - 3 >= P); its nodes are
// -1, +1 and, for L = 3, 0.
template <int P>
constexpr int lobatto_points() { return P <= 1 ? 2 : 3; }

// Interior Lobatto nodes that are not Gauss nodes of the (P+1)-point rule
// (0 for L = 3 with an even number of Gauss points): 1 at degree 3, else 0.
template <int P>
constexpr int lobatto_extra() { return (lobatto_points<P>() == 3 && (P + 1) % 2 == 0) ? 1 : 0; }

// Point set of the limiter: the volume Gauss points, then the face Gauss
// points of every face (basis values with the face side's sign), then for
// every axis a the points with xi_a = 0 and Gauss nodes on the other axes
// when 0 is a Lobatto node but not a Gauss node.  Together these are
// Zhang and Shu's points (Lobatto nodes along one axis, Gauss nodes along
// the others, over all axes) plus the volume Gauss points.
template <int D, int P>
struct LimiterPoints {
    static constexpr int NQ = Tab<D, P>::NQ, NF = Tab<D, P>::NF, NB = Tab<D, P>::NB;
    static constexpr int NPT = NQ + 2 * D * NF + lobatto_extra<P>() * D * NF;
    double phi[NPT][NB] = {};
    constexpr LimiterPoints()
    {
        for (int q = 0; q < NQ; ++q)
            for (int m = 0; m < NB; ++m) phi[q][m] = kTab<D, P>.phi_v[q][m];
        int n = NQ;
        for (int face = 0; face < 2 * D; ++face) {
            const int a = face / 2;
            const bool minus = (face & 1) == 0;
            for (int f = 0; f < NF; ++f, ++n)
                for (int m = 0; m < NB; ++m)
                    phi[n][m] = kTab<D, P>.phi_f[a][f][m] * ((minus && kTab<D, P>.e[m][a] % 2) ? -1.0 : 1.0);
        }
        if (lobatto_extra<P>())
            for (int a = 0; a < D; ++a)
                for (int f = 0; f < NF; ++f, ++n)
                    for (int m = 0; m < NB; ++m) // the face point's tangential values times P_{m_a}(0)
                        phi[n][m] = kTab<D, P>.phi_f[a][f][m] * leg(kTab<D, P>.e[m][a], 0.0);
    }
};
template <int D, int P>
inline constexpr LimiterPoints<D, P> kLimPts{};

// Zhang-Shu scaling limiter (named in Sec. 5.3.2) on one cell, in place,
// with eps = min(1e-13, mean rho, p(mean)):
//   theta1 = min(1, (rho_mean - eps)/(rho_mean - min_S rho)) scales the
//   non-mean density modes; then theta2 = min over S of the chord bound
//   t = (p(mean) - eps)/(p(mean) - p(U)) at the points with p(U) < eps
//   (pressure is concave in the conserved variables where rho > 0, so the
//   scaled state keeps p >= eps there) scales all non-mean modes.  The cell
//   mean is never changed.  MEAN_GIVEN: the cell mean is given (a bilinear /
//   trilinear cell, whose full mass matrix makes the mean differ from the
//   mode-0 coefficient), and the scalings U <- mean + theta (U - mean) move
//   mode 0 as well.
template <int D, int P, bool MEAN_GIVEN = false>
__device__ __forceinline__ void limit_cell(CellCoef<D, P> &K, double gamma, const double *given_mean = nullptr)
{
    constexpr int NV = D + 2, NB = Tab<D, P>::NB, NPT = LimiterPoints<D, P>::NPT;
    const double gm1 = gamma - 1.0;
    double mean[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) mean[v] = MEAN_GIVEN ? given_mean[v] : K[v][0];
    const double pbar = pressure<D>(mean, gm1);
    double eps = 1e-13;
    eps = mean[0] < eps ? mean[0] : eps;
    eps = pbar < eps ? pbar : eps;
    double rmin = mean[0];
#pragma unroll 1
    for (int pt = 0; pt < NPT; ++pt) {
        double r = 0.0;
#pragma unroll
        for (int m = 0; m < NB; ++m) r = fma(kLimPts<D, P>.phi[pt][m], K[0][m], r);
        rmin = r < rmin ? r : rmin;
    }
    if (rmin < mean[0]) {
        double th1 = (mean[0] - eps) / (mean[0] - rmin);
        if (th1 < 1.0) {
#pragma unroll
            for (int m = 1; m < NB; ++m) K[0][m] *= th1;
            if constexpr (MEAN_GIVEN) K[0][0] = mean[0] + th1 * (K[0][0] - mean[0]);
        }
    }
    double th2 = 1.0;
#pragma unroll 1
    for (int pt = 0; pt < NPT; ++pt) {
        double U[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) s = fma(kLimPts<D, P>.phi[pt][m], K[v][m], s);
            U[v] = s;
        }
        const double pq = pressure<D>(U, gm1);
        if (pq < eps) {
            double tq = (pbar - eps) / (pbar - pq);
            tq = tq > 1.0 ? 1.0 : (tq < 0.0 ? 0.0 : tq);
            th2 = tq < th2 ? tq : th2;
        }
    }
    if (th2 < 1.0)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int m = 1; m < NB; ++m) K[v][m] *= th2;
            if constexpr (MEAN_GIVEN) K[v][0] = mean[v] + th2 * (K[v][0] - mean[v]);
        }
}

// ------------------------------------------------------------------ stage kernel
// One thread per cell.  A workgroup covers a slab of `rows` layers of the
// leaf along its last axis (the whole leaf in 2-D; in 3-D slabs of at most
// 256 cells, so a thread may keep its cell's state and residual in up to
// 512 registers); faces on a slab edge inside the leaf read the adjacent
// layer straight from the stage input.
// threads per workgroup: 3-D degree <= 1 keeps whole 512-cell leaves (the
// state fits 256 registers); every other case uses slabs of <= 256 cells
// (3-D degree 2 in FP32 at 512 threads spills ~600 bytes per lane)
template <int D, int P, typename T = double>
constexpr int stage_threads() { return (D == 3 && P <= 1) ? 512 : 256; }
// default slab (cells per workgroup) when the caller does not choose one:
// the whole budget, except 3-D degree <= 1 and 2-D degree 1 and 2, where
// 128-cell slabs let several workgroups share a compute unit and hide each
// other's barriers (measured on 8^3 blocks at degree 1: 512-cell slabs
// 671 us, 256: 582 us, 128: 564 us; 16^2 blocks at degree 2: 256-cell
// slabs 184 us, 128: 171 us; 128^2 roots of 16^2 cells at degree 1:
// 256-cell slabs 330 us, 128: 311 us, 64: 323 us; 16^3 roots of 8^3 cells
// at degree 2 in FP64: 256-cell slabs 2.68 ms, 128: 2.53 ms, while in FP32
// 2.18 against 2.21 ms; 64^2 roots of 16^2 cells at degree 3 in FP64: 256
// cells 596 us, 128: 508 us, 64: 514 us, while in FP32 801 against 817 us)
template <int D, int P, typename T = double>
constexpr int stage_default_cells()
{
    return ((D == 3 && P <= 1) || (D == 3 && P == 2 && sizeof(T) == 8) || (D == 2 && (P == 1 || P == 2)) ||
            (D == 2 && P == 3 && sizeof(T) == 8))
               ? 128
               : stage_threads<D, P, T>();
}
// waves per SIMD the register budget is cut for, chosen by measurement on
// large forests: 2-D degree 1 in FP32 fits 128 registers (four waves);
// 2-D degree 2 in FP64 spills 44 bytes per lane to run two waves per SIMD
// instead of one (-20% time); 2-D degree 3 in FP32 runs two waves with 212
// bytes of spills (-18%), while in FP64 (536 bytes) that is slower; 3-D
// degree 1 in FP32 fits 164 registers (three waves; four: 335 -> 550 us on
// 16^3 roots); 3-D degree 2 in FP32 runs two waves with 268 bytes of
// spills (16^3 roots: 3.46 -> 2.17 ms), while three waves (more spills)
// take 7.0 ms and in FP64 two waves spill 936 bytes (2.69 -> 10.0 ms); 2-D
// degree 2 in FP32 fits 227 registers (two waves; three: 159 -> 263 us on
// 64^2 roots)
template <int D, int P, typename T = double>
constexpr int stage_min_waves()
{
    if (D != 2) return (D == 3 && P == 1 && sizeof(T) == 4) ? 3 : ((D == 3 && P == 2 && sizeof(T) == 4) ? 2 : 1);
    if (P == 1) return sizeof(T) == 4 ? 4 : 1;
    if (P == 2) return 2;
    return P == 3 && sizeof(T) == 4 ? 2 : 1;
}

// T is the arithmetic type of the residual: double, or float for the FP32
// path (state read as FP64 and rounded; the stage update, limiter and CFL
// rate stay FP64).
// One work item: slab `item` of the leaf list (all leaves, or the listed
// ones), for the thread's cell.
template <int D, int P>
__device__ __forceinline__ void volume_mfma(const float (&K)[D + 2][Tab<D, P>::NB], float (&R)[D + 2][Tab<D, P>::NB],
                                            float *lds, const float *scale, float gm1);
template <int D, int P>
constexpr int mfma_lds_floats();

// MF: the volume integral on the matrix cores (FP32 Euler, whole waves of
// cells; kernels_mfma.hpp)
template <int D, int P, int GM, int OM, bool LIM, typename T, int EQ, bool MF = false>
__device__ __forceinline__ void stage_item(const StageArgs &g, int rows, int item, int total)
{
    constexpr int NV = nvar<D, EQ>(), NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ, NF = Tab<D, P>::NF;
    constexpr int FCH = face_chunk<D, P>();
    extern __shared__ double lds_d[];
    T *lds = reinterpret_cast<T *>(lds_d);

    const int N = g.N, ncell = D == 2 ? N * N : N * N * N;
    const int layer = D == 2 ? N : N * N; // cells per layer of the last axis
    const int slabs = N / rows;
    const int wg = xcd_leaf(item, total);
    const int li = wg / slabs, k0 = (wg % slabs) * rows;
    const int leaf = g.work ? g.work[li] : li;
    const int lc = threadIdx.x, nslab = rows * layer;
    const int cell = lc + k0 * layer;
    int ijk[3];
    cell_ijk(cell, N, D, ijk);
    const T scale[3] = {T(g.geo[leaf].scale[0]), T(g.geo[leaf].scale[1]), T(g.geo[leaf].scale[2])};
    const long sv = long(NB) * ncell;
    const long base = long(leaf) * NV * sv + cell;
    // (v, m) plane of this leaf in array X: a workgroup-uniform address, so
    // the per-lane part of every state access is the one 32-bit cell offset
    const long lbase = long(leaf) * NV * sv;
    const unsigned uc = unsigned(cell);
    auto plane = [&](auto *X, int v, int m) __attribute__((always_inline)) { return X + (lbase + v * sv + long(m) * ncell); };

    T K[NV][NB], R[NV][NB];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            K[v][m] = T(plane(g.us, v, m)[uc]);
            R[v][m] = T(0);
        }

    // ---- volume integral: sum_q w_q F_a(U_q) (2/h_a) dphi_m/dxi_a / M_m
    const T gamma = T(g.gamma), gm1 = T(g.gamma - 1.0);
    // scalar convection: the velocity along the leaf's local axes, Q^T vel
    // (Sec. 3.1 frames; the identity on aligned roots)
    struct {
        double vel[3];
    } gv;
    if constexpr (EQ == EQ_ADVECTION) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) s += double(g.geo[leaf].q[3 * a + l]) * g.vel[a];
            gv.vel[l] = s;
        }
    } else {
        gv.vel[0] = gv.vel[1] = gv.vel[2] = 0.0;
    }
    auto vol_point = [&](auto qv) __attribute__((always_inline)) {
        const int q = qv;
        T U[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T s = T(0);
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = kTab<D, P>.phi_v[q][m];
                if (use_entry<D, P>(c)) s = fma(T(c), K[v][m], s);
            }
            U[v] = s;
        }
        T rinv = T(0), p = T(0);
        if constexpr (EQ == EQ_EULER) {
            rinv = recip(U[0]);
            p = pressure_r<D, T>(U, gm1, rinv);
        }
        static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
            constexpr int A = Ai;
            T F[NV];
            if constexpr (EQ == EQ_ADVECTION) F[0] = T(gv.vel[A]) * U[0];
            else euler_flux<D, A, T>(U, U[1 + A] * rinv, p, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] *= scale[A];
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = kTab<D, P>.dproj[A][q][m];
                // a mode of degree 0 along A has no derivative along A
                if (kTab<D, P>.e[m][A] != 0 && use_entry<D, P>(c)) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) R[v][m] = fma(T(c), F[v], R[v][m]);
                }
            }
        });
    };
    if constexpr (MF) {
        static_assert(std::is_same<T, float>::value && EQ == EQ_EULER, "matrix-core volume: FP32 Euler");
        float *wave_lds = reinterpret_cast<float *>(lds_d) + (threadIdx.x >> 6) * mfma_lds_floats<D, P>();
        // the per-wave regions alias the face exchange and the CFL fold of
        // the previous work item of a persistent workgroup: every wave
        // leaves them before any wave writes here
        __syncthreads();
        volume_mfma<D, P>(K, R, wave_lds, scale, gm1);
    } else if constexpr (unroll_points<D, P>()) {
        static_for<0, NQ>(vol_point);
    } else {
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) vol_point(q);
    }

    // ---- surface integrals, one axis at a time
    static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
        constexpr int A = Ai;
        const int stride = A == 0 ? 1 : (A == 1 ? N : N * N);
        const int ia = ijk[A];
        // neighbours reachable through LDS (inside this slab)
        const bool in_m = A == D - 1 ? ia > k0 : ia > 0;
        const bool in_p = A == D - 1 ? ia < k0 + rows - 1 : ia < N - 1;
        const int t = face_t(ijk, A, N, D);
        const T sc = scale[A];
        const FaceLink Lm = g.links[leaf * 2 * D + 2 * A];
        const FaceLink Lp = g.links[leaf * 2 * D + 2 * A + 1];
        const bool mort_m = g.conservative && ia == 0 && Lm.type == dgamr::LINK_FINE;
        const bool mort_p = g.conservative && ia == N - 1 && Lp.type == dgamr::LINK_FINE;
        if (mort_m) mortar_lift<D, P, A, EQ, T>(g, K, R, -1, Lm, t, sc);
        if (mort_p) mortar_lift<D, P, A, EQ, T>(g, K, R, +1, Lp, t, sc);
        // In 3-D a cell has at most one side along A whose neighbour is not
        // in the slab (slabs hold at least two layers or the whole leaf); the
        // polynomial across it (the neighbour cell at a slab edge, or the
        // far side of a block face: guard coefficients, or inline copy /
        // split / combine / mirror) is built once here and its traces taken
        // per face point.  Read per face point, the compiler hoists both
        // sides' loads out of the point loop and holds them (3-D degree 1 with
        // slab edges: 255 registers and a spill -> 213).  Mortar faces and
        // block faces read as traces keep their own paths.  In 2-D
        // (unrolled points) the per-point reads spill less.
        constexpr bool FAR_REGS = D == 3;
        const bool edge_m = FAR_REGS ? (!in_m && !mort_m && (ia > 0 || GM != GUARD_TRACE))
                                     : (A == D - 1 && !in_m && ia > 0);
        const bool edge_p = FAR_REGS ? (!in_p && !mort_p && (ia < N - 1 || GM != GUARD_TRACE))
                                     : (A == D - 1 && !in_p && ia < N - 1);
        constexpr int NBE = FAR_REGS ? NB : 1;
        T nb[NV][NBE];
        if constexpr (FAR_REGS) {
            if (edge_m || edge_p) {
                const int side = edge_m ? -1 : 1;
                if (edge_m ? ia > 0 : ia < N - 1) { // slab edge: the neighbour cell
                    const double *nk = g.us + base + side * stride;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int m = 0; m < NB; ++m) nb[v][m] = T(nk[v * sv + m * ncell]);
                } else if (edge_m) { // (a link chosen at run time would go to scratch)
                    far_poly<D, P, A, GM, NV, T>(g, K, leaf, -1, t, Lm, nb);
                } else {
                    far_poly<D, P, A, GM, NV, T>(g, K, leaf, +1, t, Lp, nb);
                }
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int m = 0; m < NB; ++m) nb[v][m] = T(0);
            }
        }
        auto face_chunk_body = [&](auto cv) __attribute__((always_inline)) {
            const int f0 = int(cv) * FCH;
            // own traces of this chunk: + side to LDS, - side kept
            T Tm[FCH][NV];
            __syncthreads();
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    T e, o;
                    trace_eo<D, P, T>(K[v], A, f0 + fi, e, o);
                    lds[(v * FCH + fi) * nslab + lc] = e + o;
                    Tm[fi][v] = e - o;
                }
            __syncthreads();
            // flux on the - face: left state = the left neighbour's + trace
            T Fm[FCH][NV];
            if (in_m) {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) {
                    T TL[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) TL[v] = lds[(v * FCH + fi) * nslab + lc - stride];
                    num_flux<D, A, EQ, T>(gv, TL, Tm[fi], gamma, Fm[fi]);
                }
            } else if (edge_m) { // slab edge inside the leaf: the layer below
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) {
                    T TL[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        T e, o;
                        if constexpr (FAR_REGS) trace_eo<D, P, T>(nb[v], A, f0 + fi, e, o);
                        else trace_eo_mem<D, P, T>(g.us + base - stride + v * sv, ncell, A, f0 + fi, e, o);
                        TL[v] = e + o;
                    }
                    num_flux<D, A, EQ, T>(gv, TL, Tm[fi], gamma, Fm[fi]);
                }
            } else if (!mort_m) {
                T TL[FCH][NV];
                far_traces<D, P, A, GM, FCH, NV, T>(g, K, leaf, -1, t, Lm, f0, TL);
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) num_flux<D, A, EQ, T>(gv, TL[fi], Tm[fi], gamma, Fm[fi]);
            } else {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fm[fi][v] = T(0);
            }
            __syncthreads();
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
                for (int v = 0; v < NV; ++v) lds[(v * FCH + fi) * nslab + lc] = Fm[fi][v];
            __syncthreads();
            T Fp[FCH][NV];
            if (in_p) {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fp[fi][v] = lds[(v * FCH + fi) * nslab + lc + stride];
            } else if (edge_p) { // slab edge inside the leaf: the layer above
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) {
                    T TL[NV], TR[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        T e, o;
                        trace_eo<D, P, T>(K[v], A, f0 + fi, e, o);
                        TL[v] = e + o;
                        if constexpr (FAR_REGS) trace_eo<D, P, T>(nb[v], A, f0 + fi, e, o);
                        else trace_eo_mem<D, P, T>(g.us + base + stride + v * sv, ncell, A, f0 + fi, e, o);
                        TR[v] = e - o;
                    }
                    num_flux<D, A, EQ, T>(gv, TL, TR, gamma, Fp[fi]);
                }
            } else if (!mort_p) {
                T TR[FCH][NV];
                far_traces<D, P, A, GM, FCH, NV, T>(g, K, leaf, +1, t, Lp, f0, TR);
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) {
                    T TL[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        T e, o;
                        trace_eo<D, P, T>(K[v], A, f0 + fi, e, o);
                        TL[v] = e + o;
                    }
                    num_flux<D, A, EQ, T>(gv, TL, TR[fi], gamma, Fp[fi]);
                }
            } else {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi)
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fp[fi][v] = T(0);
            }
            // lift: R_m += s_a w phi_m(+1)/M_m ((-1)^{m_A} Phi_- - Phi_+)
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi) {
                const int F = f0 + fi;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T dm = sc * Fm[fi][v], dp = sc * Fp[fi][v];
                    const T even = dm - dp, odd = -(dm + dp);
#pragma unroll
                    for (int m = 0; m < NB; ++m) {
                        const double c = kTab<D, P>.lift_f[A][F][m];
                        if (use_entry<D, P>(c)) R[v][m] = fma(T(c), (kTab<D, P>.e[m][A] % 2 == 0) ? even : odd, R[v][m]);
                    }
                }
            }
        };
        if constexpr (unroll_points<D, P>()) {
            static_for<0, NF / FCH>(face_chunk_body);
        } else {
#pragma unroll 1
            for (int ci = 0; ci < NF / FCH; ++ci) face_chunk_body(ci);
        }
    });

    // ---- output
    if constexpr (OM == OUT_RES64) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) plane(g.out64, v, m)[uc] = double(R[v][m]);
    } else if constexpr (OM == OUT_RES32) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) plane(g.out32, v, m)[uc] = float(R[v][m]);
    } else {
        double dt;
        if (g.rate_in) {
            const double rate = __longlong_as_double((long long)*g.rate_in);
            dt = g.cfl / rate;
            if (item == 0 && threadIdx.x == 0) *g.dt_out = dt;
        } else {
            dt = g.dt[g.leaf_member ? g.leaf_member[leaf] : 0];
        }
        if (g.rate_clear && item == 0 && threadIdx.x == 0) *g.rate_clear = 0ULL;
        const double a = g.rk_a, b = g.rk_b;
        // FP64 update; the FP32 path re-reads U_s at full precision
        double Kn[NV][NB];
        if constexpr (std::is_same<T, double>::value) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[v][m] = b * (K[v][m] + dt * R[v][m]);
        } else if (b != 0.0) {
            // FP32 path: U_s again at full precision; inside a (uniform)
            // branch so that its loads are issued here, not held in
            // registers through the residual
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[v][m] = b * (plane(g.us, v, m)[uc] + dt * double(R[v][m]));
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[v][m] = 0.0;
        }
        // stages 2 and 3 add the RK base state; a uniform branch keeps its
        // loads here, after the residual, instead of live through it
        if (a != 0.0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int m = 0; m < NB; ++m) Kn[v][m] = fma(a, plane(g.un, v, m)[uc], Kn[v][m]);
        }
        if constexpr (LIM && EQ == EQ_EULER) limit_cell<D, P>(Kn, g.gamma);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int m = 0; m < NB; ++m) plane(g.out64, v, m)[uc] = Kn[v][m];
        if (g.rate_out) {
            // CFL rate of the new state from its cell mean, folded over the block
            double rate = 0.0;
            if constexpr (EQ == EQ_ADVECTION) {
#pragma unroll
                for (int a2 = 0; a2 < D; ++a2) rate += fabs(g.vel[a2]) / g.geo[leaf].h[a2];
            } else {
                double U[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) U[v] = Kn[v][0];
                const double rinv = 1.0 / U[0];
                const double cs = sqrt(g.gamma * pressure_r<D>(U, g.gamma - 1.0, rinv) * rinv);
#pragma unroll
                for (int a2 = 0; a2 < D; ++a2) rate += (fabs(U[1 + a2] * rinv) + cs) / g.geo[leaf].h[a2];
            }
            block_max_to(rate, lds_d, g.rate_out);
        }
    }
}

// The stage kernel: one workgroup per (leaf, slab) work item, or (PERSIST,
// a grid smaller than the item count) each workgroup walks the items with
// a stride of the grid size.  With a grid that is a
// multiple of the XCD count every item a workgroup takes maps to the same
// XCD's leaf range.
template <int D, int P, int GM, int OM, bool LIM, typename T = double, int EQ = EQ_EULER, bool PERSIST = false,
          bool MF = false>
__global__ __launch_bounds__((stage_threads<D, P, T>()), (stage_min_waves<D, P, T>())) void k_stage(StageArgs g,
                                                                                                     int rows)
{
    const int total = g.nleaves * (g.N / rows);
    if constexpr (PERSIST) {
        for (int item = blockIdx.x; item < total; item += gridDim.x)
            stage_item<D, P, GM, OM, LIM, T, EQ, MF>(g, rows, item, total);
    } else { // one item per workgroup: no loop to hold values across items
        stage_item<D, P, GM, OM, LIM, T, EQ, MF>(g, rows, blockIdx.x, total);
    }
}

// ------------------------------------------------------------------ guard fill
// One thread per guard cell (leaf, face, t): Eq. 15 copy, Eq. 16 split of the
// coarser neighbour cell, Eq. 17 combine of the 2^d finer cells, outflow
// mirror K_m (-1)^{m_axis}; written as coefficients or as face traces.
template <int D, int P, int NV = D + 2>
__global__ __launch_bounds__(256) void k_fill(FillArgs g)
{
    constexpr int NB = Tab<D, P>::NB, NF = Tab<D, P>::NF;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= long(g.nfaces) * nfc) return;
    const int fi = int(gid / nfc), t = int(gid % nfc);
    const int lf = g.work ? g.work[fi / (2 * D)] * 2 * D + fi % (2 * D) : fi;
    const int leaf = lf / (2 * D), face = lf % (2 * D);
    const int a = face / 2, side = (face & 1) ? 1 : -1;
    const FaceLink L = g.links[lf];
    const long sv = long(NB) * ncell;
    // one variable of the guard cell -> coefficients, or its values at the
    // face points (the guard cell touches the face with its -side side)
    auto emit = [&](int v, const double *gk) __attribute__((always_inline)) {
        if (g.traces) {
            double *out = g.guard + (long(lf) * NV * NF) * nfc + t;
            for (int f = 0; f < NF; ++f) {
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const int ex = kTab<D, P>.e[m][0] * (a == 0) + kTab<D, P>.e[m][1] * (a == 1) +
                                   kTab<D, P>.e[m][2] * (a == 2);
                    const double c = kTab<D, P>.phi_f[a][f][m];
                    s = fma((side > 0 && (ex % 2)) ? -c : c, gk[m], s);
                }
                out[(v * NF + f) * nfc] = s;
            }
        } else {
            double *out = g.guard + (long(lf) * NV * NB) * nfc + t;
#pragma unroll
            for (int m = 0; m < NB; ++m) out[(v * NB + m) * nfc] = gk[m];
        }
    };
    if (L.rot > 0) {
        // a neighbour root of another frame (Sec. 3.5): copy, split or combine
        // in the source frame, then the rotation R^n into this leaf's frame
        const RotPlan Rp = g.plans[L.rot - 1 + t];
        double ks[NV][NB];
        for (int v = 0; v < NV; ++v) {
            double kv[NB];
            if (Rp.type == dgamr::PLAN_COMBINE) {
#pragma unroll
                for (int m = 0; m < NB; ++m) kv[m] = 0.0;
                for (int ch = 0; ch < (1 << D); ++ch) {
                    const double *src = g.u + long(Rp.leaf[ch]) * NV * sv + long(v) * sv + Rp.cell[ch];
                    double kf[NB];
#pragma unroll
                    for (int n = 0; n < NB; ++n) kf[n] = src[long(n) * ncell];
                    comb_any<D, P>(ch, kf, kv);
                }
            } else {
                const double *src = g.u + long(Rp.leaf[0]) * NV * sv + long(v) * sv + Rp.cell[0];
                double kc[NB];
#pragma unroll
                for (int n = 0; n < NB; ++n) kc[n] = src[long(n) * ncell];
                if (Rp.type == dgamr::PLAN_SPLIT) split_any<D, P, double>(Rp.child, kc, kv);
                else
#pragma unroll
                    for (int n = 0; n < NB; ++n) kv[n] = kc[n];
            }
            // modes: phi_n(m xi) = sign * phi_n'(xi), exponent l of n' = exponent
            // l' of n where m[l'][l] != 0
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                int e2[3] = {0, 0, 0};
                double sg = 1.0;
                for (int lp = 0; lp < D; ++lp)
                    for (int l = 0; l < D; ++l) {
                        const int mm = Rp.m[3 * lp + l];
                        if (mm != 0) {
                            e2[l] = kTab<D, P>.e[n][lp];
                            if (mm < 0 && (kTab<D, P>.e[n][lp] & 1)) sg = -sg;
                        }
                    }
                int idx = 0;
                for (int q = 0; q < NB; ++q)
                    if (kTab<D, P>.e[q][0] == e2[0] && kTab<D, P>.e[q][1] == e2[1] && kTab<D, P>.e[q][2] == e2[2])
                        idx = q;
                ks[v][idx] = sg * kv[n];
            }
        }
        if (NV == D + 2 && !g.global_vectors) { // momentum into this leaf's frame: m_dst[l] = sum_l' m[l'][l] m_src[l']
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                double mv[3] = {0.0, 0.0, 0.0};
                for (int l = 0; l < D; ++l)
                    for (int lp = 0; lp < D; ++lp) mv[l] += double(Rp.m[3 * lp + l]) * ks[1 + lp][n];
                for (int l = 0; l < D; ++l) ks[1 + l][n] = mv[l];
            }
        }
        for (int v = 0; v < NV; ++v) emit(v, ks[v]);
        return;
    }
    if (L.type == dgamr::LINK_SAME) {
        const int c = same_cell(a, side, t, N, D);
        const double *src = g.u + long(L.nbr[0]) * NV * sv + c;
        for (int v = 0; v < NV; ++v) {
            double gk[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) gk[m] = src[v * sv + m * ncell];
            emit(v, gk);
        }
    } else if (L.type == dgamr::LINK_BOUNDARY) {
        const int c = face_cell(a, side > 0 ? N - 1 : 0, t, N, D);
        const double *src = g.u + long(leaf) * NV * sv + c;
        for (int v = 0; v < NV; ++v) {
            double gk[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double k = src[v * sv + m * ncell];
                const int ex = kTab<D, P>.e[m][0] * (a == 0) + kTab<D, P>.e[m][1] * (a == 1) +
                               kTab<D, P>.e[m][2] * (a == 2);
                gk[m] = (ex % 2) ? -k : k;
            }
            emit(v, gk);
        }
    } else if (L.type == dgamr::LINK_COARSE) {
        // the guard cell (fine size) lies in one coarse cell; along a it is
        // the half nearest to this leaf
        const int c = coarse_cell(a, side, t, L.off, N, D);
        const int child = coarse_child(a, side, t, N, D);
        const double *src = g.u + long(L.nbr[0]) * NV * sv + c;
        for (int v = 0; v < NV; ++v) {
            double ks[NB], gk[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) ks[n] = src[v * sv + n * ncell];
            split_any<D, P, double>(child, ks, gk);
            emit(v, gk);
        }
    } else { // LINK_FINE: 2^d fine cells, 2 along a and 2^(d-1) tangential
        const double *base = g.u + long(link_nbr(L, fine_block(t, N, D))) * NV * sv;
        for (int v = 0; v < NV; ++v) {
            double acc[NB];
#pragma unroll
            for (int m = 0; m < NB; ++m) acc[m] = 0.0;
#pragma unroll
            for (int ch = 0; ch < (1 << D); ++ch) {
                const int c = fine_cell(a, side, t, ch, N, D);
                double ks[NB];
#pragma unroll
                for (int n = 0; n < NB; ++n) ks[n] = base[v * sv + n * ncell + c];
#pragma unroll
                for (int m = 0; m < NB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        const double cc = kTab<D, P>.comb[ch][m][n];
                        if (cc != 0.0) acc[m] = fma(cc, ks[n], acc[m]);
                    }
            }
            emit(v, acc);
        }
    }
}

} // namespace dgk
