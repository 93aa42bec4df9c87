// Launch entry points of the degree-templated kernels.  Each (dim, degree)
// pair is compiled in its own translation unit (inst.hip with DG_D, DG_P),
// so the host API sees only these declarations.
#pragma once

#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace dgk {

// Launch shape of the stage kernel.  variant (FP64 without the limiter;
// 2-D any output, 3-D the fused stage without mortar faces): 0 = one lane
// per (cell, variable) in slabs of rows (2-D) or layers (3-D), 1 = one
// thread per cell.  rows: layers of the last axis per workgroup (0 = the
// kernel's own choice); grid: workgroups of a persistent launch of the
// thread-per-cell kernel (0 = one per work item).
struct StageShape {
    int variant = 1;
    int rows = 0;
    int grid = 0;
    int mfma = 0; // FP32 residual: 1 = the volume integral on the matrix cores where built
};

// 3-D lane-per-(cell, variable) kernel: 12 cells per wave, at most 12 waves
// per workgroup; a slab is whole layers, at least two of them (so that only
// z faces can be slab edges and a cell has at most one) unless it is the
// whole leaf
constexpr int kCells3v = 12;
constexpr int kThreads3v = 768;
inline bool rows_ok_3v(int N, int rows)
{
    return rows >= 1 && N % rows == 0 && (rows >= 2 || rows == N) && rows * N * N <= kCells3v * (kThreads3v / 64);
}

// largest slab height the 3-D lane kernel takes for block size N (0: none)
inline int rows_3v(int N)
{
    for (int r = N; r >= 1; --r)
        if (rows_ok_3v(N, r)) return r;
    return 0;
}

// Whether the fused stage of a 3-D Euler forest runs the lane kernel, which
// reads the far side of block faces as traces written by the fill kernel
// before the stage (the thread-per-cell kernel computes it inline): the
// lane kernel is asked for (variant 0) and takes the case.
inline bool stage_reads_traces(int dim, const StageShape &sh, bool limiter, bool fp32, bool conservative,
                               bool advection, int N)
{
    return dim == 3 && !advection && !fp32 && !limiter && !conservative && sh.variant == 0 &&
           (sh.rows == 0 ? rows_3v(N) > 0 : rows_ok_3v(N, sh.rows));
}

// residual / fused stage.  fp32: residual arithmetic in FP32 (out_mode
// OUT_RES32 or OUT_RK).
template <int D, int P>
hipError_t launch_stage(const StageArgs &a, int guard_mode, int out_mode, bool limiter, bool fp32,
                        const StageShape &shape, hipStream_t s, int equation = EQ_EULER);
// rows the thread-per-cell stage kernel accepts for block size N: divisors
// of N whose slab fits the kernel's thread budget, largest first
template <int D, int P>
int stage_rows_options(int N, int *rows, int max_options, bool fp32);
// guard fill: one thread per guard cell of the listed faces
template <int D, int P>
hipError_t launch_fill(const FillArgs &a, int nfc, hipStream_t s, int nv = D + 2);
// diffusion stage: one thread per cell; out_mode OUT_RES64 or OUT_RK
template <int D, int P>
hipError_t launch_ipdg(const IpdgArgs &a, int out_mode, hipStream_t s);

// Bilinear / trilinear roots (2-D any degree, 3-D degree <= 2): the
// residual or fused RK stage (out_mode OUT_RES64 / OUT_RK; eq EQ_EULER or
// EQ_ADVECTION; lim: the positivity limiter fused, Euler OUT_RK only), the
// positivity limiter alone, the CFL rate per leaf, the per-leaf totals (one
// workgroup of `block` threads per leaf, a power of two), and the initial
// projection (nv variables).
template <int D, int P>
hipError_t launch_mapped(const MappedArgs &a, int eq, int out_mode, bool lim, hipStream_t s);
template <int D, int P>
hipError_t launch_mapped_limit(double *u, const LeafGeo *geo, int N, long ncell_total, double gamma, hipStream_t s);
template <int D, int P>
hipError_t launch_mapped_rate(const MappedArgs &a, int eq, int nleaves, int block, double *leaf_max, hipStream_t s);
template <int D, int P>
hipError_t launch_mapped_totals(const MappedArgs &a, int eq, int nleaves, int block, double *part, hipStream_t s);
template <int D, int P>
hipError_t launch_mapped_ic(double *u, const LeafGeo *geo, int N, long total, int kind, const IcParams &prm,
                            double t, double gamma, int nv, hipStream_t s);
template <int D, int P>
hipError_t launch_limit(double *u, int N, long ncell_total, double gamma, hipStream_t s);
template <int D, int P>
hipError_t launch_project_ic(double *u, const LeafGeo *geo, int N, long ncell_total, int kind, const IcParams &prm,
                             double t, double gamma, const double *hmin, hipStream_t s, int nv = D + 2);
template <int D, int P>
hipError_t launch_inherit(const double *uold, double *unew, const Inherit *inh, int N, long ncell_total,
                          hipStream_t s, int nv = D + 2);

} // namespace dgk
