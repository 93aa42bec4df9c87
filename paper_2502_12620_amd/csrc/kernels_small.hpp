// Small HIP kernels that do not depend on the polynomial degree: SSP-RK3
// update, CFL reduction, conserved totals and the state check.
#pragma once

#include "kernel_common.hpp"

namespace dgk {

// ------------------------------------------------------------------ RK update
struct RkArgs {
    const double *un, *us;
    const void *r;
    double *out;
    const double *dt;
    double a, b;
    long n;
    int r32;
};

static __global__ __launch_bounds__(256) void k_rk(RkArgs g)
{
    const double dt = *g.dt;
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < g.n; i += long(gridDim.x) * blockDim.x) {
        double r = g.r32 ? double(static_cast<const float *>(g.r)[i]) : static_cast<const double *>(g.r)[i];
        double un = g.a != 0.0 ? g.un[i] : 0.0;
        g.out[i] = g.a * un + g.b * (g.us[i] + dt * r);
    }
}

// ------------------------------------------------------------------ CFL, totals, checks
// Per leaf: max over cells of sum_a (|u_a| + c)/h_a from the cell means.
// One workgroup per leaf (or per listed leaf of `work`).
template <int D>
__global__ __launch_bounds__(256) void k_rate(const double *u, const LeafGeo *geo, int N, int nb, double gamma,
                                              double *leaf_max, const int *work)
{
    constexpr int NV = D + 2;
    __shared__ double red[256];
    const int leaf = work ? work[blockIdx.x] : int(blockIdx.x), ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(nb) * ncell, base = long(leaf) * NV * sv;
    const LeafGeo G = geo[leaf];
    double mx = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        double U[NV];
        for (int v = 0; v < NV; ++v) U[v] = u[base + v * sv + c];
        double rinv = 1.0 / U[0];
        double cs = sqrt(gamma * pressure<D>(U, gamma - 1.0) * rinv);
        double rate = 0.0;
        for (int a = 0; a < D; ++a) rate += (fabs(U[1 + a] * rinv) + cs) / G.h[a];
        mx = rate > mx ? rate : mx;  // NaN never wins; caught by the state check
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) leaf_max[leaf] = red[0];
}

// dt = cfl / max over leaves (one workgroup; max is order independent)
static __global__ __launch_bounds__(1024) void k_dt_final(const double *leaf_max, int n, double cfl, double *dt)
{
    __shared__ double red[1024];
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = leaf_max[i] > mx ? leaf_max[i] : mx;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dt = cfl / red[0];
}

// The max over leaves of the CFL rate, stored as the bit pattern of the
// (non-negative) double in a rate slot of the fused-time-step scheme.
static __global__ __launch_bounds__(1024) void k_rate_slot(const double *leaf_max, int n, unsigned long long *slot)
{
    __shared__ double red[1024];
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = leaf_max[i] > mx ? leaf_max[i] : mx;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *slot = (unsigned long long)__double_as_longlong(red[0]);
}

// Per member forest of a pool: dt_m = cfl_m / max over the member's leaf
// range [first, first + count) (one workgroup per member; count 0 = empty
// member slot, left alone).
struct MemberDesc {
    int first, count;
    double cfl;
};

static __global__ __launch_bounds__(256) void k_dt_members(const double *leaf_max, const MemberDesc *members, double *dt)
{
    __shared__ double red[256];
    const MemberDesc M = members[blockIdx.x];
    if (M.count == 0) return;
    double mx = 0.0;
    for (int i = threadIdx.x; i < M.count; i += blockDim.x) {
        const double v = leaf_max[M.first + i];
        mx = v > mx ? v : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dt[blockIdx.x] = M.cfl / red[0];
}

// Per leaf partial totals sum_cells vol * mean_v, fixed tree order.
template <int D, int NV = D + 2>
__global__ __launch_bounds__(256) void k_totals_leaf(const double *u, const LeafGeo *geo, int N, int nb, double *part)
{
    __shared__ double red[NV][256];
    const int leaf = blockIdx.x, ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(nb) * ncell, base = long(leaf) * NV * sv;
    double s[NV];
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x)
        for (int v = 0; v < NV; ++v) s[v] += u[base + v * sv + c];
    for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int v = 0; v < NV; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double tv[NV];
        for (int v = 0; v < NV; ++v) tv[v] = red[v][0] * geo[leaf].vol;
        if constexpr (NV == D + 2) { // momentum along the global axes: Q m
            double m[3] = {0.0, 0.0, 0.0};
            for (int g = 0; g < D; ++g)
                for (int l = 0; l < D; ++l) m[g] += double(geo[leaf].q[3 * g + l]) * tv[1 + l];
            for (int g = 0; g < D; ++g) tv[1 + g] = m[g];
        }
        for (int v = 0; v < NV; ++v) part[long(leaf) * NV + v] = tv[v];
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_totals_final(const double *part, int n, double *tot)
{
    __shared__ double red[NV][256];
    double s[NV];
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        for (int v = 0; v < NV; ++v) s[v] += part[long(i) * NV + v];
    for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int v = 0; v < NV; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int v = 0; v < NV; ++v) tot[v] = red[v][0];
}

// counts cells with a non-finite coefficient or (Euler) a non-positive mean
// density or pressure
template <int D, int NV = D + 2>
__global__ __launch_bounds__(256) void k_check(const double *u, int N, int nb, long ncell_total, double gamma,
                                               unsigned long long *bad)
{
    const int ncell = D == 2 ? N * N : N * N * N;
    long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= ncell_total) return;
    long leaf = gid / ncell;
    int c = int(gid % ncell);
    const long sv = long(nb) * ncell, base = leaf * NV * sv + c;
    bool ok = true;
    for (int v = 0; v < NV; ++v)
        for (int m = 0; m < nb; ++m) ok = ok && isfinite(u[base + v * sv + m * ncell]);
    if constexpr (NV == D + 2) {
        double U[NV];
        for (int v = 0; v < NV; ++v) U[v] = u[base + v * sv];
        ok = ok && U[0] > 0.0 && pressure<D>(U, gamma - 1.0) > 0.0;
    }
    if (!ok) atomicAdd(bad, 1ULL);
}

// ------------------------------------------------------------------ indicator
// Euler: eta = max / min density mean over the block's cells and face-guard
// cells; scalar convection (Sec. 5.1): the largest cell mean there
template <int D, int NV = D + 2>
__global__ __launch_bounds__(256) void k_indicator_leaf(const double *u, const double *guard, int N, int nb, double *eta)
{
    __shared__ double smax[256], smin[256];
    const int leaf = blockIdx.x, ncell = D == 2 ? N * N : N * N * N, nfc = D == 2 ? N : N * N;
    const long sv = long(nb) * ncell, base = long(leaf) * NV * sv;
    double mx = -1e300, mn = 1e300;
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        double r = u[base + c];
        mx = r > mx ? r : mx;
        mn = r < mn ? r : mn;
    }
    for (int i = threadIdx.x; i < 2 * D * nfc; i += blockDim.x) {
        int face = i / nfc, t = i % nfc;
        double r = guard[((long(leaf) * 2 * D + face) * NV * nb) * nfc + t];
        mx = r > mx ? r : mx;
        mn = r < mn ? r : mn;
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + s] ? smax[threadIdx.x] : smax[threadIdx.x + s];
            smin[threadIdx.x] = smin[threadIdx.x] < smin[threadIdx.x + s] ? smin[threadIdx.x] : smin[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) eta[leaf] = NV == 1 ? smax[0] : smax[0] / smin[0];
}

// Scalar convection: per leaf sum_a |vel_a| / h_a (the CFL rate does not
// depend on the state); one thread per leaf (or listed leaf).
static __global__ __launch_bounds__(256) void k_rate_adv(const LeafGeo *geo, int n, double v0, double v1, double v2,
                                                         int dim, double *leaf_max)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v[3] = {v0, v1, v2};
    double rate = 0.0;
    for (int a = 0; a < dim; ++a) rate += fabs(v[a]) / geo[i].h[a];
    leaf_max[i] = rate;
}

// y = recip(x) (fn 0) or sqrt_nn(x) (fn 1), the stage kernels' FP64
// reciprocal and wave-speed square root, for their accuracy check
static __global__ __launch_bounds__(256) void k_math_probe(int fn, const double *x, double *y, long n)
{
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = fn == 0 ? recip(x[i]) : sqrt_nn(x[i]);
}

// *p = v (one thread): a host-computed value put on the device in stream
// order (the diffusion time step)
static __global__ void k_set_value(double *p, double v) { *p = v; }

} // namespace dgk
