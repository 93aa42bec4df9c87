// Device helpers and kernel argument blocks shared by the HIP kernels.
//
// Layout in HBM (block-major SoA): U[leaf][var][mode][cell], cell index x
// fastest, so the N^d threads of one workgroup (one leaf, one thread per
// cell) read every (var, mode) plane as one contiguous, coalesced run.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_tables.hpp"
#include "forest.hpp"

namespace dgk {

using dgamr::FaceLink;
using dgamr::Inherit;
using dgamr::LeafGeo;
using dgamr::RotPlan;

constexpr int kXcds = 8; // MI355X: 8 XCDs, workgroups dispatched round-robin

// Workgroup index -> leaf such that each XCD owns one contiguous range of
// leaves (neighbouring leaves in Morton order share that XCD's L2).
__device__ __forceinline__ int xcd_leaf(int bid, int n)
{
    int q = n / kXcds, r = n % kXcds;
    int x = bid % kXcds, slot = bid / kXcds;
    return x * q + (x < r ? x : r) + slot;
}

__host__ __device__ __forceinline__ void cell_ijk(int cell, int N, int D, int *ijk)
{
    ijk[0] = cell % N;
    ijk[1] = (cell / N) % N;
    ijk[2] = D == 3 ? cell / (N * N) : 0;
}

// physical position of the local point (ijk + (xi + 1)/2) h of a leaf:
// its local origin plus the frame Q applied to the local offset
template <int D>
__device__ __forceinline__ void leaf_point(const LeafGeo &G, const int *ijk, const double *xi, double *x)
{
    for (int g = 0; g < 3; ++g) x[g] = g < D ? G.lo[g] : 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const double off = (ijk[l] + 0.5 * (xi[l] + 1.0)) * G.h[l];
#pragma unroll
        for (int g = 0; g < D; ++g) x[g] += double(G.q[3 * g + l]) * off;
    }
}

// tangential index t of a cell on the face normal to axis a (the lower of
// the remaining axes fastest)
__host__ __device__ __forceinline__ int face_t(const int *ijk, int a, int N, int D)
{
    if (D == 2) return a == 0 ? ijk[1] : ijk[0];
    return a == 0 ? ijk[1] + N * ijk[2] : (a == 1 ? ijk[0] + N * ijk[2] : ijk[0] + N * ijk[1]);
}

// cell index of (normal index n along a, tangential index t)
__host__ __device__ __forceinline__ int face_cell(int a, int n, int t, int N, int D)
{
    int t0 = t % N, t1 = t / N;
    int i, j, k;
    if (a == 0) { i = n; j = t0; k = t1; }
    else if (a == 1) { i = t0; j = n; k = t1; }
    else { i = t0; j = t1; k = n; }
    return i + N * (j + N * k);
}

// k-th neighbour of a face link, selected without indexing the struct (a
// runtime index into a local copy would put it in scratch memory)
__host__ __device__ __forceinline__ int link_nbr(const FaceLink &L, int k)
{
    return k == 0 ? L.nbr[0] : (k == 1 ? L.nbr[1] : (k == 2 ? L.nbr[2] : L.nbr[3]));
}

// Where the guard cell at face point t of a block face comes from (Sec.
// 3.5).  a: the face's axis; side: +1 for the face on the + side (the
// neighbour lies along +a), -1 otherwise; t: the tangential index
// (face_t).  The guard cell has this block's cell size and sits next to the
// face on the neighbour's side.
//
// Neighbour of the same level (Eq. 15): its cell next to the face.
__host__ __device__ __forceinline__ int same_cell(int a, int side, int t, int N, int D)
{
    return face_cell(a, side > 0 ? 0 : N - 1, t, N, D);
}

// Coarser neighbour (Eq. 16): the guard cell is child coarse_child() (bit b:
// upper half along axis b) of the neighbour's cell coarse_cell(); off is the
// link's position of this block on the coarse face, in block edges.
__host__ __device__ __forceinline__ int coarse_cell(int a, int side, int t, const int *off, int N, int D)
{
    const int t0 = t % N, t1 = t / N;
    const int c0 = (off[0] * N + t0) / 2, c1 = D == 3 ? (off[1] * N + t1) / 2 : 0;
    return face_cell(a, side > 0 ? 0 : N - 1, c0 + N * c1, N, D);
}
__host__ __device__ __forceinline__ int coarse_child(int a, int side, int t, int N, int D)
{
    const int ta = a == 0 ? 1 : 0, tb = a == 2 ? 1 : 2; // tangential axes, lower first
    const int t0 = t % N, t1 = t / N;
    return ((side > 0 ? 0 : 1) << a) | ((t0 & 1) << ta) | (D == 3 ? ((t1 & 1) << tb) : 0);
}

// Finer neighbours (Eq. 17): the guard cell is covered by 2^d cells of one
// of the 2^(d-1) finer blocks on the face: the link's neighbour slot
// fine_block() (bit 0: upper half along the lower tangential axis, bit 1:
// along the other), and in it the cell fine_cell() under child ch of the
// guard cell (bit b of ch: upper half along axis b).
__host__ __device__ __forceinline__ int fine_block(int t, int N, int D)
{
    const int t0 = t % N, t1 = t / N;
    return (2 * t0) / N + (D == 3 ? 2 * ((2 * t1) / N) : 0);
}
__host__ __device__ __forceinline__ int fine_cell(int a, int side, int t, int ch, int N, int D)
{
    const int ta = a == 0 ? 1 : 0, tb = a == 2 ? 1 : 2;
    const int t0 = t % N, t1 = t / N;
    const int na = (ch >> a) & 1, n0 = (ch >> ta) & 1, n1 = D == 3 ? (ch >> tb) & 1 : 0;
    const int f0 = (2 * t0) % N + n0, f1 = D == 3 ? (2 * t1) % N + n1 : 0;
    return face_cell(a, side > 0 ? na : N - 2 + na, f0 + N * f1, N, D);
}

// 1/x for the state's normal positive densities: the hardware reciprocal
// estimate refined by Newton-Raphson steps r <- r + r (1 - x r), two in
// FP64 (quadratic convergence takes the estimate to full precision), one in
// FP32.  Within an ulp of the correctly rounded quotient, at half the
// instructions of the IEEE division sequence.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// sqrt(a) for a >= 0 (wave speeds): Goldschmidt's iteration from the
// hardware reciprocal-square-root estimate y (s = a y, h = y/2,
// r = 1/2 - s h, s <- s + s r, h <- h + h r, twice), then one Newton
// correction s <- s + h (a - s^2); zero for a = 0.  FP32 uses the hardware
// square root.
__device__ __forceinline__ double sqrt_nn(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double s = a * y, h = 0.5 * y;
    double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    s = fma(fma(-s, s, a), h, s);
    return a > 0.0 ? s : 0.0;
}
__device__ __forceinline__ float sqrt_nn(float a) { return __builtin_amdgcn_sqrtf(a > 0.0f ? a : 0.0f); }

// Euler flux along axis A (Eq. 2 and its 3-D analogue; EOS Eq. 23), in the
// arithmetic type T of the residual (FP64, or FP32 for the FP32 path).
template <int D, int A, typename T = double>
__device__ __forceinline__ void euler_flux(const T *U, T ua, T p, T *F)
{
    F[0] = U[1 + A];
#pragma unroll
    for (int b = 0; b < D; ++b) F[1 + b] = U[1 + b] * ua;
    F[1 + A] += p;
    F[D + 1] = ua * (U[D + 1] + p);
}

template <int D>
__device__ __forceinline__ double pressure(const double *U, double gm1)
{
    double ke = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) ke += U[1 + b] * U[1 + b];
    return gm1 * (U[D + 1] - 0.5 * ke / U[0]);
}

// the same with 1/rho already known
template <int D, typename T = double>
__device__ __forceinline__ T pressure_r(const T *U, T gm1, T rinv)
{
    T ke = T(0);
#pragma unroll
    for (int b = 0; b < D; ++b) ke += U[1 + b] * U[1 + b];
    return gm1 * (U[D + 1] - T(0.5) * ke * rinv);
}

// Eq. 5, dissipative sign, flux in the +e_A direction between the left
// state UL and the right state UR; alpha = max(|u_A| + c) of both sides.
template <int D, int A, typename T = double>
__device__ __forceinline__ void rusanov(const T *UL, const T *UR, T gamma, T *Phi)
{
    constexpr int NV = D + 2;
    const T gm1 = gamma - T(1);
    const T rl = recip(UL[0]), rr = recip(UR[0]);
    const T pl = pressure_r<D, T>(UL, gm1, rl), pr = pressure_r<D, T>(UR, gm1, rr);
    const T ul = UL[1 + A] * rl, ur = UR[1 + A] * rr;
    // a pressure rounded below zero (FP32 traces of a near-vacuum state)
    // enters the wave speed as zero; exact arithmetic never takes this branch
    // on a state the positivity limiter has passed
    const T cl = sqrt_nn(gamma * pl * rl), cr = sqrt_nn(gamma * pr * rr);
    const T al = fabs(ul) + cl, ar = fabs(ur) + cr;
    const T alpha = al > ar ? al : ar;
    T FL[NV], FR[NV];
    euler_flux<D, A, T>(UL, ul, pl, FL);
    euler_flux<D, A, T>(UR, ur, pr, FR);
#pragma unroll
    for (int v = 0; v < NV; ++v) Phi[v] = T(0.5) * ((FL[v] + FR[v]) - alpha * (UR[v] - UL[v]));
}

// ------------------------------------------------------------------ argument blocks
enum GuardMode : int {
    GUARD_BUFFER = 0, // every block face from the guard buffer (coefficients)
    GUARD_INLINE = 1, // every block face straight from the neighbours' cells:
                      // copy, split of the coarser cell or combine of the
                      // finer cells computed on the fly (no guard buffer)
    GUARD_TRACE = 2   // every block face from the guard buffer holding the
                      // guard cells' traces at the face points
};
enum OutMode : int { OUT_RES64 = 0, OUT_RES32 = 1, OUT_RK = 2 };

// conservation law: the Euler equations (Sec. 2) or the linear scalar
// convection equation u_t + vel . grad u = 0 (Sec. 5.1)
enum Equation : int { EQ_EULER = 0, EQ_ADVECTION = 1 };
template <int D, int EQ>
constexpr int nvar() { return EQ == EQ_ADVECTION ? 1 : D + 2; }

// max of two non-negative values in which a NaN wins
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// *out = max(*out, bits of m) for a non-negative m (or a NaN).  The value
// only grows, so a plain read that already holds at least m proves the
// atomic unnecessary: after the first workgroups most skip it, which keeps
// hundreds of same-address atomics off the memory system.
__device__ __forceinline__ void atomic_max_bits(unsigned long long *out, double m)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(m);
    if (__hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b) atomicMax(out, b);
}

// Orders this wave's LDS accesses before and after it: enough in place of a
// workgroup barrier when every lane that exchanges data through LDS
// belongs to the same wave (a wave executes its LDS instructions in order)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Folds the workgroup's maximum of x (non-negative; a NaN wins) into *out
// with an atomic max on the bit pattern.  A workgroup of whole waves takes
// the maximum across each wave with lane exchanges and combines one value
// per wave through LDS (two barriers); otherwise a tree over LDS (one
// barrier per level).  Every thread of the workgroup calls it; lds holds at
// least blockDim.x doubles and is free.
__device__ __forceinline__ void block_max_to(double x, double *lds, unsigned long long *out)
{
    const int tid = int(threadIdx.x), n = int(blockDim.x);
    if ((n & 63) == 0) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x = nan_max(x, __shfl_xor(x, off));
        __syncthreads();
        if ((tid & 63) == 0) lds[tid >> 6] = x;
        __syncthreads();
        if (tid == 0) {
            double m = lds[0];
            for (int w = 1; w < (n >> 6); ++w) m = nan_max(m, lds[w]);
            atomic_max_bits(out, m);
        }
    } else {
        __syncthreads();
        lds[tid] = x;
        __syncthreads();
        for (int s = 1; s < n; s <<= 1) {
            if ((tid % (2 * s)) == 0 && tid + s < n) lds[tid] = nan_max(lds[tid], lds[tid + s]);
            __syncthreads();
        }
        if (tid == 0) atomic_max_bits(out, lds[0]);
    }
}

struct StageArgs {
    const double *us;     // stage input (read-only during the stage)
    const double *un;     // RK base state (OUT_RK)
    const double *guard;  // guard buffer
    double *out64;        // residual (OUT_RES64) or next state (OUT_RK)
    float *out32;         // residual (OUT_RES32)
    const LeafGeo *geo;
    const FaceLink *links;
    const double *dt;     // device dt (OUT_RK), per member when leaf_member is set
    double rk_a, rk_b;
    double gamma;
    double vel[3];        // advection velocity (EQ_ADVECTION)
    int nleaves, N;       // work items: leaves listed in work (or all leaves)
    const int *work;      // leaf indices to process (null: 0 .. nleaves-1)
    const int *leaf_member; // member forest of each leaf (indexes dt), or null
    int conservative;     // mortar on hanging coarse faces
    // CFL time step fused into the stages (OUT_RK only): when rate_in is
    // set, dt = cfl / max rate read from *rate_in (written by the previous
    // step's last stage) and workgroup 0 stores it to dt_out; otherwise dt
    // is read from *dt.  When rate_clear is set, workgroup 0 zeroes it (the
    // slot this step's last stage will fill).  When rate_out is set, every
    // workgroup folds the max over its cells of sum_a (|u_a| + c)/h_a of the
    // new state into *rate_out (atomic max on the bit pattern of a
    // non-negative double).
    double cfl;
    const unsigned long long *rate_in;
    unsigned long long *rate_clear;
    double *dt_out;
    unsigned long long *rate_out;
};

// Numerical flux in the +e_A direction between the left state UL and the
// right state UR: Rusanov for Euler (Eq. 5); for scalar convection the same
// formula with alpha = |vel_A| is the upwind flux.
template <int D, int A, int EQ, typename T, class Args>
__device__ __forceinline__ void num_flux(const Args &g, const T *UL, const T *UR, T gamma, T *Phi)
{
    if constexpr (EQ == EQ_ADVECTION) {
        const T a = T(g.vel[A]);
        Phi[0] = T(0.5) * (a * (UL[0] + UR[0]) - fabs(a) * (UR[0] - UL[0]));
    } else {
        rusanov<D, A, T>(UL, UR, gamma, Phi);
    }
}

struct FillArgs {
    const double *u;
    double *guard;
    const FaceLink *links;
    const RotPlan *plans; // guard cells of faces between roots of different frames
    const int *work;   // leaves whose 2d faces are filled (null: all leaves)
    int nfaces;        // number of faces to fill (2d per listed leaf)
    int N;
    int traces;        // 0: guard coefficients G[leaf][face][var][mode][t];
                       // 1: their traces on the face, G[leaf][face][var][point][t]
    int global_vectors; // 1: momentum along the global axes (bilinear / trilinear
                        // roots): across rotated frames only the coordinates turn
};

struct IcParams {
    double p[8];
};

// Bilinear-root stage (2-D, Sec. 3.3 Eq. 6): residual over guard
// coefficients, optionally fused with the SSP-RK3 stage update
struct MappedArgs {
    const double *us;    // stage input (read-only)
    const double *un;    // RK base state (OUT_RK)
    const double *guard; // guard coefficients G[leaf][face][var][mode][t]
    double *out;         // residual (OUT_RES64) or next state (OUT_RK)
    const LeafGeo *geo;  // node[4][2]: each leaf's corners
    const double *dt;    // device dt (OUT_RK)
    double rk_a, rk_b;
    double gamma;
    double vel[3];       // convection velocity (EQ_ADVECTION)
    long ncell_total;
    int N;
};

// Diffusion stage (Sec. 5.2): interior-penalty residual, optionally fused
// with the SSP-RK3 stage update.
struct IpdgArgs {
    const double *us;    // stage input (read-only)
    const double *un;    // RK base state (OUT_RK)
    const double *guard; // guard coefficients G[leaf][face][0][mode][t]
    double *out;         // residual (OUT_RES64) or next state (OUT_RK)
    const LeafGeo *geo;
    const FaceLink *links;
    const double *dt;    // device dt (OUT_RK)
    double rk_a, rk_b;
    double nu;
    double avec[3];      // exact solution exp(a . x + nu |a|^2 t)
    double t;            // time of the stage input (Dirichlet data)
    long ncell_total;
    int N;
};

} // namespace dgk
