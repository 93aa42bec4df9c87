// 3-D DG stage kernel with one lane per (cell, variable).
//
// Twelve cells of five conserved variables fill lanes 0..59 of a wave
// (lanes 60..63 repeat the last cell's lanes and store nothing).  Each lane
// keeps only its variable's coefficients and residual, so a cell's state
// and residual take 4 N_b registers per lane instead of 20 N_b in one
// thread; the full state at a point, needed by the Euler and Rusanov
// fluxes, is gathered from the cell's five lanes with ds_bpermute.  A
// workgroup covers a slab of layers (along z) of one leaf; faces inside the
// slab exchange traces and fluxes through LDS in chunks of face points,
// faces on a slab edge inside the leaf are recomputed from the adjacent
// layer, and leaf faces read the far side as traces from the guard buffer
// (the fill kernel writes them before each stage: copy, split, combine,
// outflow mirror).  Runs the fused RK stage in FP64 for the Euler
// equations without the limiter and without mortar faces; everything else
// takes the thread-per-cell kernel.
#pragma once

#include "kernels_2d.hpp"
#include "launch.hpp"

namespace dgk {

// face points exchanged through LDS at once
template <int P>
constexpr int face_chunk_3v() { return P == 0 ? 1 : (P == 1 ? 4 : (P == 2 ? 3 : 2)); }

// value of x held by the lane at byte address addr (4 * lane)
__device__ __forceinline__ double lane_get(double x, int addr)
{
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

// full state of the cell from its five lanes' values (addr0: byte address
// of the cell's first lane)
__device__ __forceinline__ void cell_state5(double x, int addr0, double *U)
{
#pragma unroll
    for (int j = 0; j < 5; ++j) U[j] = lane_get(x, addr0 + 4 * j);
}

// Rusanov flux (Eq. 5, dissipative sign, +e_A direction) of this lane's
// variable between left value tl and right value tr
template <int A>
__device__ __forceinline__ double rusanov_5(double tl, double tr, int addr0, double gamma, double isM, double isE)
{
    double L[5], R[5];
    cell_state5(tl, addr0, L);
    cell_state5(tr, addr0, R);
    const double gm1 = gamma - 1.0;
    const double rl = recip(L[0]), rr = recip(R[0]);
    const double pl = pressure_r<3>(L, gm1, rl), pr = pressure_r<3>(R, gm1, rr);
    const double ul = L[1 + A] * rl, ur = R[1 + A] * rr;
    const double al = fabs(ul) + sqrt_nn(gamma * pl * rl), ar = fabs(ur) + sqrt_nn(gamma * pr * rr);
    const double alpha = al > ar ? al : ar;
    const double fl = flux_v<A>(tl, ul, pl, isM, isE), fr = flux_v<A>(tr, ur, pr, isM, isE);
    return 0.5 * ((fl + fr) - alpha * (tr - tl));
}

// even / odd parts (in the normal mode index) of the trace at face point f
// of axis A (a constant after unrolling: zero table entries drop out)
template <int P, int A>
__device__ __forceinline__ void trace3(const double *K, int f, double &e, double &o)
{
    e = 0.0;
    o = 0.0;
#pragma unroll
    for (int m = 0; m < Tab<3, P>::NB; ++m) {
        const double c = kTab<3, P>.phi_f[A][f][m];
        if (c != 0.0) {
            if (kTab<3, P>.e[m][A] % 2 == 0) e = fma(c, K[m], e);
            else o = fma(c, K[m], o);
        }
    }
}

// An empty asm that takes and returns x: everything x depends on is computed
// before it, and a scheduling barrier after it keeps later work below.
// Without these the scheduler hoists the lane gathers and the table
// constants of every quadrature point ahead and holds them in registers.
#define DG_PIN(x) asm volatile("" : "+v"(x))

// The point loops are unrolled at every degree (table entries become
// constants).  At degree 3 loops over the tables read with scalar loads
// spill less (92 against 260 bytes per lane) but wait on a scalar load at
// every point: 2.13 ms against 1.30 ms per stage on 8^3 roots of 8^3 cells.

// grid: one workgroup per (leaf, slab of `rows` layers); block: 64 lanes per
// 12 cells of the slab (rows * N * N <= 144 cells)
template <int P>
__global__ __launch_bounds__(kThreads3v) void k_stage3v(StageArgs g, int rows)
{
    constexpr int NV = 5, NB = Tab<3, P>::NB, NQ = Tab<3, P>::NQ, NF = Tab<3, P>::NF;
    constexpr int FCH = face_chunk_3v<P>();
    static_assert(NF % FCH == 0, "face points come in whole chunks");
    extern __shared__ double lds[];
    const int N = g.N, layer = N * N, ncell = layer * N;
    const int slabs = N / rows;
    const int wg = xcd_leaf(blockIdx.x, g.nleaves * slabs);
    const int li = wg / slabs, k0 = (wg % slabs) * rows;
    const int leaf = g.work ? g.work[li] : li; // listed leaves of a pool, or all
    const int nslab = rows * layer;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lv = lane < 5 * kCells3v ? lane : lane - 5; // lanes 60..63 repeat lanes 55..58
    const int cw = lv / 5, v = lv - 5 * cw;
    const int addr0 = 4 * 5 * cw;                          // byte address of the cell's first lane
    const int lraw = wave * kCells3v + cw;
    const bool live = lane < 5 * kCells3v && lraw < nslab; // slots past the slab repeat its last cell
    const int lc = lraw < nslab ? lraw : nslab - 1;
    const int cell = lc + k0 * layer;
    const int ijk[3] = {cell % N, (cell / N) % N, cell / layer};
    const double isE = v == 4 ? 1.0 : 0.0;
    const double scale[3] = {g.geo[leaf].scale[0], g.geo[leaf].scale[1], g.geo[leaf].scale[2]};
    const long sv = long(NB) * ncell;
    const long vbase = long(leaf) * NV * sv + v * sv; // this variable's planes in this leaf
    const long idx0 = vbase + cell;

    double K[NB], R[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        K[m] = g.us[idx0 + long(m) * ncell];
        R[m] = 0.0;
    }

    // ---- volume integral
    const double gm1 = g.gamma - 1.0;
    auto vol_point = [&](auto qv) __attribute__((always_inline)) {
        const int q = qv;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const double c = kTab<3, P>.phi_v[q][m];
            if (c != 0.0) s = fma(c, K[m], s);
        }
        double U[5];
        cell_state5(s, addr0, U);
        const double rinv = recip(U[0]);
        const double p = pressure_r<3>(U, gm1, rinv);
        static_for<0, 3>([&](auto Ai) __attribute__((always_inline)) {
            constexpr int A = Ai;
            const double isM = v == 1 + A ? 1.0 : 0.0;
            const double F = scale[A] * flux_v<A>(s, U[1 + A] * rinv, p, isM, isE);
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const double c = kTab<3, P>.dproj[A][q][m];
                // a mode of degree 0 along A has no derivative along A
                if (kTab<3, P>.e[m][A] != 0 && c != 0.0) R[m] = fma(c, F, R[m]);
            }
        });
#pragma unroll
        for (int m = 0; m < NB; ++m) DG_PIN(R[m]);
        __builtin_amdgcn_sched_barrier(0);
    };
    static_for<0, NQ>(vol_point);

    // ---- surface integrals, one axis at a time; LDS slot of (chunk point,
    // slab cell, variable)
    auto slot = [&](int fi, int c) { return (fi * nslab + c) * NV + v; };
    static_for<0, 3>([&](auto Ai) __attribute__((always_inline)) {
        constexpr int A = Ai;
        const double isM = v == 1 + A ? 1.0 : 0.0;
        const int stride = A == 0 ? 1 : (A == 1 ? N : layer);
        const int ia = ijk[A];
        const bool in_m = A == 2 ? ia > k0 : ia > 0;            // - neighbour inside the slab
        const bool in_p = A == 2 ? ia < k0 + rows - 1 : ia < N - 1;
        const int t = face_t(ijk, A, N, 3);
        const double sc = scale[A];
        // far-side traces of the leaf faces: G[leaf][face][var][point][t]
        const double *gt_m = g.guard + ((long(leaf) * 6 + 2 * A) * NV * NF + long(v) * NF) * layer + t;
        const double *gt_p = g.guard + ((long(leaf) * 6 + 2 * A + 1) * NV * NF + long(v) * NF) * layer + t;
        // slabs hold whole layers of at least two rows, so only a z face
        // can be a slab edge, and a cell has at most one: its neighbour's
        // coefficients across it, read once
        const bool edge_m = A == 2 && !in_m && ia > 0, edge_p = A == 2 && !in_p && ia < N - 1;
        double nb[NB];
        if (A == 2 && (edge_m || edge_p)) {
            const double *nk = g.us + idx0 + (edge_m ? -stride : stride);
#pragma unroll
            for (int m = 0; m < NB; ++m) nb[m] = nk[long(m) * ncell];
        } else {
#pragma unroll
            for (int m = 0; m < NB; ++m) nb[m] = 0.0;
        }
        auto chunk = [&](auto cv) __attribute__((always_inline)) {
            const int f0 = int(cv) * FCH;
            double Tm[FCH], Fm[FCH], Fp[FCH];
            __syncthreads();
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi) {
                double e, o;
                trace3<P, A>(K, f0 + fi, e, o);
                if (live) lds[slot(fi, lc)] = e + o;
                Tm[fi] = e - o;
            }
            __syncthreads();
            // - face: left state = the + trace of the cell below
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi) {
                double tl;
                if (in_m) {
                    tl = lds[slot(fi, lc - stride)];
                } else if (edge_m) { // slab edge inside the leaf: the layer below
                    double e, o;
                    trace3<P, A>(nb, f0 + fi, e, o);
                    tl = e + o;
                } else {
                    tl = gt_m[long(f0 + fi) * layer];
                }
                Fm[fi] = rusanov_5<A>(tl, Tm[fi], addr0, g.gamma, isM, isE);
                DG_PIN(Fm[fi]);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi)
                if (live) lds[slot(fi, lc)] = Fm[fi];
            __syncthreads();
            // + face: computed by the cell above unless it is outside the slab
            if (in_p) {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) Fp[fi] = lds[slot(fi, lc + stride)];
            } else {
#pragma unroll
                for (int fi = 0; fi < FCH; ++fi) {
                    double e, o, tr;
                    if (edge_p) { // slab edge inside the leaf: the layer above
                        trace3<P, A>(nb, f0 + fi, e, o);
                        tr = e - o;
                    } else {
                        tr = gt_p[long(f0 + fi) * layer];
                    }
                    trace3<P, A>(K, f0 + fi, e, o);
                    Fp[fi] = rusanov_5<A>(e + o, tr, addr0, g.gamma, isM, isE);
                    DG_PIN(Fp[fi]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // lift: R_m += s_a w phi_m(+1)/M_m ((-1)^{m_A} Phi_- - Phi_+)
#pragma unroll
            for (int fi = 0; fi < FCH; ++fi) {
                const double dm = sc * Fm[fi], dp = sc * Fp[fi];
                const double even = dm - dp, odd = -(dm + dp);
#pragma unroll
                for (int m = 0; m < NB; ++m) {
                    const double c = kTab<3, P>.lift_f[A][f0 + fi][m];
                    if (c != 0.0) R[m] = fma(c, (kTab<3, P>.e[m][A] % 2 == 0) ? even : odd, R[m]);
                }
            }
#pragma unroll
            for (int m = 0; m < NB; ++m) DG_PIN(R[m]);
            __builtin_amdgcn_sched_barrier(0);
        };
        static_for<0, NF / FCH>(chunk);
    });

    // ---- fused RK stage (FP64), as the thread-per-cell kernel rounds it
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
    for (int m = 0; m < NB; ++m) K[m] = b * (K[m] + dt * R[m]);
    if (a != 0.0) { // uniform: stages 2 and 3 add the RK base state
#pragma unroll
        for (int m = 0; m < NB; ++m) K[m] = fma(a, g.un[idx0 + long(m) * ncell], K[m]);
    }
    if (live) {
#pragma unroll
        for (int m = 0; m < NB; ++m) g.out64[idx0 + long(m) * ncell] = K[m];
    }
    if (g.rate_out) {
        // CFL rate of the new state from its cell mean, folded over the slab
        double U[5];
        cell_state5(K[0], addr0, U);
        const double rinv = 1.0 / U[0];
        const double cs = sqrt(g.gamma * pressure_r<3>(U, gm1, rinv) * rinv);
        double rate = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) rate += (fabs(U[1 + a2] * rinv) + cs) / g.geo[leaf].h[a2];
        // every lane holds its cell's rate (unused lanes repeat a cell of the slab)
        block_max_to(rate, lds, g.rate_out);
    }
}

} // namespace dgk
