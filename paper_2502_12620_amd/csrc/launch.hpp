// Launch entry points of the degree-templated kernels.  Each (dim, degree)
// pair is compiled in its own translation unit (inst.hip with DG_D, DG_P),
// so the host API sees only these declarations.
#pragma once

#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace dgk {

// residual / fused stage.  variant (2-D FP64, fused stage without limiter):
// 0 = one lane per (cell, variable) in row slabs, 1 = one thread per cell.
// fp32: residual arithmetic in FP32 (out_mode OUT_RES32 or OUT_RK).
template <int D, int P>
hipError_t launch_stage(const StageArgs &a, int guard_mode, int out_mode, bool limiter, int variant, bool fp32,
                        hipStream_t s);
// guard fill: one thread per guard cell of the listed faces
template <int D, int P>
hipError_t launch_fill(const FillArgs &a, int nfc, hipStream_t s);
template <int D, int P>
hipError_t launch_limit(double *u, int N, long ncell_total, double gamma, hipStream_t s);
template <int D, int P>
hipError_t launch_project_ic(double *u, const LeafGeo *geo, int N, long ncell_total, int kind, const IcParams &prm,
                             double t, double gamma, const double *hmin, hipStream_t s);
template <int D, int P>
hipError_t launch_inherit(const double *uold, double *unew, const Inherit *inh, int N, long ncell_total,
                          hipStream_t s);

} // namespace dgk
