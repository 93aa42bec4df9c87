// One (dim, degree) instantiation of the degree-templated kernels and their
// launchers; compiled once per pair with -DDG_D=<dim> -DDG_P=<degree> and
// -DDG_PART=<part>, the heavy kernels split over parts so that the units
// compile in parallel:
//   part 0  the dispatcher launch_stage, the lane-per-(cell, variable)
//           kernels, scalar convection, fill, limiter, projection, inheritance
//   part 1  the thread-per-cell Euler stage kernels in FP64
//   part 2  the thread-per-cell Euler stage kernels with FP32 arithmetic
//   part 3  the diffusion stage
//   part 4  the thread-per-cell Euler stage kernels with FP32 arithmetic and
//           the volume integral on the matrix cores (degree >= 2)
#include "kernels.hpp"
#include "kernels_2d.hpp"
#include "kernels_3d.hpp"
#include "kernels_aux.hpp"
#include "kernels_ipdg.hpp"
#include "kernels_mapped.hpp"
#include "kernels_mfma.hpp"
#include "launch.hpp"

#ifndef DG_D
#error "DG_D must be defined"
#endif
#ifndef DG_P
#error "DG_P must be defined"
#endif
#ifndef DG_PART
#error "DG_PART must be defined"
#endif

namespace dgk {

// 2-D without the limiter: one lane per (cell, variable), a slab of rows
// per workgroup, with enough slabs to give every compute unit work.
template <int P>
hipError_t launch_stage_2v(const StageArgs &a, int gm, int om, hipStream_t s, int rows_req)
{
    int rows = a.N;
    if (rows_req > 0) {
        if (a.N % rows_req != 0 || rows_req * a.N * 4 > 512) return hipErrorInvalidValue;
        rows = rows_req;
    } else {
        while (rows * a.N * 4 > 512) rows /= 2;
        while (rows % 2 == 0 && rows > 1 && long(a.nleaves) * (a.N / rows) < 256) rows /= 2;
    }
    const int slabs = a.N / rows;
    const size_t lds = sizeof(double) * (P + 1) * rows * a.N * 4;
    const dim3 grid(unsigned(a.nleaves * slabs)), block(rows * a.N * 4);
    if (gm == GUARD_BUFFER && om == OUT_RES64)
        hipLaunchKernelGGL((k_stage2v<P, GUARD_BUFFER, OUT_RES64>), grid, block, lds, s, a, rows);
    else if (gm == GUARD_INLINE && om == OUT_RK)
        hipLaunchKernelGGL((k_stage2v<P, GUARD_INLINE, OUT_RK>), grid, block, lds, s, a, rows);
    else if (gm == GUARD_BUFFER && om == OUT_RK) // far side from the (rotated) guard fill
        hipLaunchKernelGGL((k_stage2v<P, GUARD_BUFFER, OUT_RK>), grid, block, lds, s, a, rows);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// 3-D fused FP64 stage with one lane per (cell, variable)
template <int P>
hipError_t launch_stage_3v(const StageArgs &a, hipStream_t s, int rows_req)
{
    const int N = a.N, layer = N * N;
    int rows = rows_req;
    if (rows > 0) {
        if (!rows_ok_3v(N, rows)) return hipErrorInvalidValue;
    } else {
        rows = rows_3v(N);
        if (rows == 0) return hipErrorInvalidValue;
        // small forests: thinner slabs until every compute unit has work
        while (rows % 2 == 0 && rows_ok_3v(N, rows / 2) && long(a.nleaves) * (N / rows) < 256) rows /= 2;
    }
    const int nslab = rows * layer;
    const int waves = (nslab + kCells3v - 1) / kCells3v;
    const size_t lds = sizeof(double) * size_t(face_chunk_3v<P>()) * nslab * 5;
    const dim3 grid(unsigned(long(a.nleaves) * (N / rows))), block(64 * waves);
    hipLaunchKernelGGL((k_stage3v<P>), grid, block, lds, s, a, rows);
    return hipGetLastError();
}

template <int D, int P, typename T>
bool rows_ok(int N, int rows)
{
    const int layer = D == 2 ? N : N * N;
    // 3-D: at least two layers unless the whole leaf (a cell has at most one
    // slab edge)
    return rows >= 1 && N % rows == 0 && (D == 2 || rows >= 2 || rows == N) && rows * layer <= stage_threads<D, P, T>();
}

template <int D, int P>
int stage_rows_options(int N, int *rows, int max_options, bool fp32)
{
    int n = 0;
    for (int r = N; r >= 1 && n < max_options; --r)
        if (fp32 ? rows_ok<D, P, float>(N, r) : rows_ok<D, P, double>(N, r)) rows[n++] = r;
    return n;
}

template <int D, int P, typename T, int EQ = EQ_EULER, bool MF = false>
hipError_t launch_stage_cell(const StageArgs &a, int gm, int om, bool lim, const StageShape &sh, hipStream_t s)
{
    // slab of `rows` layers along the last axis within the thread budget
    const int layer = D == 2 ? a.N : a.N * a.N;
    int rows = sh.rows;
    if (rows == 0) {
        rows = a.N;
        while (rows % 2 == 0 && rows * layer > stage_default_cells<D, P, T>()) rows /= 2;
    }
    if (!rows_ok<D, P, T>(a.N, rows)) return hipErrorInvalidValue;
    const int nslab = rows * layer;
    const long items = long(a.nleaves) * (a.N / rows);
    size_t lds = sizeof(double) * (D + 2) * face_chunk<D, P>() * nslab;
    if constexpr (MF) {
        // whole waves only; the volume phase's per-wave LDS regions alias the
        // face exchange's buffer
        if (nslab % 64 != 0) return hipErrorNotSupported;
        const size_t mf = sizeof(float) * size_t(mfma_lds_floats<D, P>()) * (nslab / 64);
        lds = mf > lds ? mf : lds;
    }
    const bool persist = sh.grid > 0 && sh.grid < items;
    // the persistent shape applies to the fused Euler stage (pools); every
    // other launch takes one workgroup per item
    const dim3 grid(unsigned(persist ? sh.grid : items)), block(nslab);
    const dim3 grid_all = dim3(unsigned(items));
    // the fused stage takes the far side of block faces inline (copy,
    // split, combine, mirror of the neighbour cells), or on forests with
    // rotated root frames from the guard fill; the residual entry point
    // reads guard coefficients
    if constexpr (EQ == EQ_ADVECTION) {
        // one variable: the far side is always taken inline
        if (gm == GUARD_INLINE && om == OUT_RK) {
            hipLaunchKernelGGL((k_stage<D, P, GUARD_INLINE, OUT_RK, false, T, EQ>), grid_all, block, lds, s, a, rows);
            return hipGetLastError();
        }
        if (gm == GUARD_BUFFER && om == OUT_RES64) {
            hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RES64, false, T, EQ>), grid_all, block, lds, s, a, rows);
            return hipGetLastError();
        }
        if (gm == GUARD_BUFFER && om == OUT_RK) { // rotated root frames
            hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RK, false, T, EQ>), grid_all, block, lds, s, a, rows);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    constexpr int GMRK = GUARD_INLINE; // the fused stage takes the far side inline
    if (gm == GMRK && om == OUT_RK) {
        if (persist && lim)
            hipLaunchKernelGGL((k_stage<D, P, GMRK, OUT_RK, true, T, EQ_EULER, true, MF>), grid, block, lds, s, a, rows);
        else if (persist)
            hipLaunchKernelGGL((k_stage<D, P, GMRK, OUT_RK, false, T, EQ_EULER, true, MF>), grid, block, lds, s, a, rows);
        else if (lim)
            hipLaunchKernelGGL((k_stage<D, P, GMRK, OUT_RK, true, T, EQ_EULER, false, MF>), grid, block, lds, s, a, rows);
        else
            hipLaunchKernelGGL((k_stage<D, P, GMRK, OUT_RK, false, T, EQ_EULER, false, MF>), grid, block, lds, s, a, rows);
        return hipGetLastError();
    }
    if (gm == GUARD_BUFFER && om == OUT_RK) {
        // the fused stage reading the far side from the guard fill (forests
        // with rotated root frames), one workgroup per item, on the vector
        // unit
        if constexpr (MF) {
            return hipErrorNotSupported;
        } else {
            if (lim)
                hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RK, true, T>), grid_all, block, lds, s, a, rows);
            else
                hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RK, false, T>), grid_all, block, lds, s, a, rows);
            return hipGetLastError();
        }
    }
    if constexpr (std::is_same<T, float>::value) {
        if (gm == GUARD_BUFFER && om == OUT_RES32) {
            hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RES32, false, T, EQ_EULER, false, MF>), grid_all, block,
                               lds, s, a, rows);
            return hipGetLastError();
        }
    } else if constexpr (D == 3) { // the 2-D FP64 residual runs one lane per (cell, variable)
        if (gm == GUARD_BUFFER && om == OUT_RES64) {
            hipLaunchKernelGGL((k_stage<D, P, GUARD_BUFFER, OUT_RES64, false, T>), grid_all, block, lds, s, a, rows);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

#if DG_PART == 0
// defined here, instantiated in parts 1 and 2
extern template hipError_t launch_stage_cell<DG_D, DG_P, double, EQ_EULER>(const StageArgs &, int, int, bool,
                                                                          const StageShape &, hipStream_t);
extern template hipError_t launch_stage_cell<DG_D, DG_P, float, EQ_EULER>(const StageArgs &, int, int, bool,
                                                                         const StageShape &, hipStream_t);
#if DG_P >= 2 && !(DG_D == 3 && DG_P == 3)
extern template hipError_t launch_stage_cell<DG_D, DG_P, float, EQ_EULER, true>(const StageArgs &, int, int, bool,
                                                                               const StageShape &, hipStream_t);
#endif

template <int D, int P>
hipError_t launch_stage(const StageArgs &a, int gm, int om, bool lim, bool fp32, const StageShape &sh, hipStream_t s,
                        int eq)
{
    if (a.nleaves == 0) return hipSuccess;
    if (eq == EQ_ADVECTION) return fp32 ? hipErrorInvalidValue : launch_stage_cell<D, P, double, EQ_ADVECTION>(a, gm, om, lim, sh, s);
    if (fp32) {
        if constexpr (mfma_volume<D, P>()) {
            // the volume integral on the matrix cores where the slab is whole
            // waves; otherwise (small blocks) on the vector unit
            if (sh.mfma) {
                const hipError_t e = launch_stage_cell<D, P, float, EQ_EULER, true>(a, gm, om, lim, sh, s);
                if (e != hipErrorNotSupported) return e;
            }
        }
        return launch_stage_cell<D, P, float>(a, gm, om, lim, sh, s);
    }
    if constexpr (D == 2) {
        // one lane per (cell, variable) unless the caller asks for one
        // thread per cell (variant 1) or needs the limiter
        if (!lim && (sh.variant == 0 || om != OUT_RK)) return launch_stage_2v<P>(a, gm, om, s, sh.rows);
    } else {
        // the fused stage reading guard traces is the lane kernel (the
        // caller filled the traces because stage_reads_traces holds)
        if (gm == GUARD_TRACE && om == OUT_RK) {
            if (!stage_reads_traces(3, sh, lim, false, a.conservative != 0, false, a.N)) return hipErrorInvalidValue;
            return launch_stage_3v<P>(a, s, sh.rows);
        }
    }
    return launch_stage_cell<D, P, double>(a, gm, om, lim, sh, s);
}

template <int D, int P>
hipError_t launch_fill(const FillArgs &a, int nfc, hipStream_t s, int nv)
{
    const long threads = long(a.nfaces) * nfc;
    const dim3 grid(unsigned((threads + 255) / 256)), block(256);
    if (nv == 1) hipLaunchKernelGGL((k_fill<D, P, 1>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_fill<D, P>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int D, int P>
hipError_t launch_limit(double *u, int N, long total, double gamma, hipStream_t s)
{
    hipLaunchKernelGGL((k_limit<D, P>), dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, u, N, total, gamma);
    return hipGetLastError();
}

template <int D, int P>
hipError_t launch_project_ic(double *u, const LeafGeo *geo, int N, long total, int kind, const IcParams &prm,
                             double t, double gamma, const double *hmin, hipStream_t s, int nv)
{
    const dim3 grid(unsigned((total + 255) / 256)), block(256);
    if (nv == 1)
        hipLaunchKernelGGL((k_project_ic<D, P, 1>), grid, block, 0, s, u, geo, N, total, kind, prm, t, gamma, hmin[0],
                           hmin[1], hmin[2]);
    else
        hipLaunchKernelGGL((k_project_ic<D, P>), grid, block, 0, s, u, geo, N, total, kind, prm, t, gamma, hmin[0],
                           hmin[1], hmin[2]);
    return hipGetLastError();
}

template <int D, int P>
hipError_t launch_inherit(const double *uold, double *unew, const Inherit *inh, int N, long total, hipStream_t s,
                          int nv)
{
    const dim3 grid(unsigned((total + 255) / 256)), block(256);
    if (nv == 1) hipLaunchKernelGGL((k_inherit<D, P, 1>), grid, block, 0, s, uold, unew, inh, N, total);
    else hipLaunchKernelGGL((k_inherit<D, P>), grid, block, 0, s, uold, unew, inh, N, total);
    return hipGetLastError();
}

template hipError_t launch_stage<DG_D, DG_P>(const StageArgs &, int, int, bool, bool, const StageShape &, hipStream_t,
                                             int);
template int stage_rows_options<DG_D, DG_P>(int, int *, int, bool);
template hipError_t launch_fill<DG_D, DG_P>(const FillArgs &, int, hipStream_t, int);
template hipError_t launch_limit<DG_D, DG_P>(double *, int, long, double, hipStream_t);
template hipError_t launch_project_ic<DG_D, DG_P>(double *, const LeafGeo *, int, long, int, const IcParams &, double,
                                                   double, const double *, hipStream_t, int);
template hipError_t launch_inherit<DG_D, DG_P>(const double *, double *, const Inherit *, int, long, hipStream_t, int);
#elif DG_PART == 3
template <int D, int P>
hipError_t launch_ipdg(const IpdgArgs &a, int om, hipStream_t s)
{
    if (a.ncell_total == 0) return hipSuccess;
    const dim3 grid(unsigned((a.ncell_total + 255) / 256)), block(256);
    if (om == OUT_RES64) hipLaunchKernelGGL((k_ipdg<D, P, OUT_RES64>), grid, block, 0, s, a);
    else if (om == OUT_RK) hipLaunchKernelGGL((k_ipdg<D, P, OUT_RK>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
template hipError_t launch_ipdg<DG_D, DG_P>(const IpdgArgs &, int, hipStream_t);
#if DG_D == 2 || DG_P <= 2
template <int D, int P>
hipError_t launch_mapped(const MappedArgs &a, int eq, int om, bool lim, hipStream_t s)
{
    if (a.ncell_total == 0) return hipSuccess;
    const dim3 grid(unsigned((a.ncell_total + 127) / 128)), block(128);
    if (lim) {
        if (eq != EQ_EULER || om != OUT_RK) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_mapped<D, P, EQ_EULER, OUT_RK, true>), grid, block, 0, s, a);
    } else if (eq == EQ_ADVECTION) {
        if (om == OUT_RES64) hipLaunchKernelGGL((k_mapped<D, P, EQ_ADVECTION, OUT_RES64>), grid, block, 0, s, a);
        else if (om == OUT_RK) hipLaunchKernelGGL((k_mapped<D, P, EQ_ADVECTION, OUT_RK>), grid, block, 0, s, a);
        else return hipErrorInvalidValue;
    } else {
        if (om == OUT_RES64) hipLaunchKernelGGL((k_mapped<D, P, EQ_EULER, OUT_RES64>), grid, block, 0, s, a);
        else if (om == OUT_RK) hipLaunchKernelGGL((k_mapped<D, P, EQ_EULER, OUT_RK>), grid, block, 0, s, a);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <int D, int P>
hipError_t launch_mapped_limit(double *u, const LeafGeo *geo, int N, long total, double gamma, hipStream_t s)
{
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mapped_limit<D, P>), dim3(unsigned((total + 127) / 128)), dim3(128), 0, s, u, geo, N, total,
                       gamma);
    return hipGetLastError();
}
template <int D, int P>
hipError_t launch_mapped_rate(const MappedArgs &a, int eq, int nleaves, int block, double *leaf_max, hipStream_t s)
{
    if (eq == EQ_ADVECTION)
        hipLaunchKernelGGL((k_mapped_rate<D, P, EQ_ADVECTION>), dim3(nleaves), dim3(block), 0, s, a, leaf_max);
    else
        hipLaunchKernelGGL((k_mapped_rate<D, P, EQ_EULER>), dim3(nleaves), dim3(block), 0, s, a, leaf_max);
    return hipGetLastError();
}
template <int D, int P>
hipError_t launch_mapped_totals(const MappedArgs &a, int eq, int nleaves, int block, double *part, hipStream_t s)
{
    if (eq == EQ_ADVECTION)
        hipLaunchKernelGGL((k_mapped_totals_leaf<D, P, EQ_ADVECTION>), dim3(nleaves), dim3(block), 0, s, a, part);
    else
        hipLaunchKernelGGL((k_mapped_totals_leaf<D, P, EQ_EULER>), dim3(nleaves), dim3(block), 0, s, a, part);
    return hipGetLastError();
}
template <int D, int P>
hipError_t launch_mapped_ic(double *u, const LeafGeo *geo, int N, long total, int kind, const IcParams &prm,
                            double t, double gamma, int nv, hipStream_t s)
{
    const dim3 grid(unsigned((total + 127) / 128)), block(128);
    if (nv == 1)
        hipLaunchKernelGGL((k_mapped_project_ic<D, P, 1>), grid, block, 0, s, u, geo, N, total, kind, prm, t, gamma);
    else
        hipLaunchKernelGGL((k_mapped_project_ic<D, P, D + 2>), grid, block, 0, s, u, geo, N, total, kind, prm, t,
                           gamma);
    return hipGetLastError();
}
template hipError_t launch_mapped<DG_D, DG_P>(const MappedArgs &, int, int, bool, hipStream_t);
template hipError_t launch_mapped_limit<DG_D, DG_P>(double *, const LeafGeo *, int, long, double, hipStream_t);
template hipError_t launch_mapped_rate<DG_D, DG_P>(const MappedArgs &, int, int, int, double *, hipStream_t);
template hipError_t launch_mapped_totals<DG_D, DG_P>(const MappedArgs &, int, int, int, double *, hipStream_t);
template hipError_t launch_mapped_ic<DG_D, DG_P>(double *, const LeafGeo *, int, long, int, const IcParams &, double,
                                                 double, int, hipStream_t);
#endif
#elif DG_PART == 1
template hipError_t launch_stage_cell<DG_D, DG_P, double, EQ_EULER>(const StageArgs &, int, int, bool,
                                                                   const StageShape &, hipStream_t);
#elif DG_PART == 2
template hipError_t launch_stage_cell<DG_D, DG_P, float, EQ_EULER>(const StageArgs &, int, int, bool,
                                                                  const StageShape &, hipStream_t);
#else
#if DG_P >= 2 && !(DG_D == 3 && DG_P == 3)
template hipError_t launch_stage_cell<DG_D, DG_P, float, EQ_EULER, true>(const StageArgs &, int, int, bool,
                                                                        const StageShape &, hipStream_t);
#endif
#endif

} // namespace dgk
