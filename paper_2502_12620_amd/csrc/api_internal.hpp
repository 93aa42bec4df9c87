// Internal helpers shared by the C-ABI translation units: error reporting,
// HIP error checks, the (dim, degree) dispatch, and the forest handle.
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "forest.hpp"

namespace dgapi {

inline thread_local std::string g_err;

inline int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(DGAMR_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- dispatch
template <class Fn>
int dispatch(int d, int p, Fn &&fn)
{
    switch (d * 10 + p) {
    case 20: return fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{});
    case 21: return fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    case 22: return fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
    case 23: return fn(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
    case 30: return fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 0>{});
    case 31: return fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{});
    case 32: return fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{});
    case 33: return fn(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{});
    default: return fail(DGAMR_EUNSUPPORTED, "unsupported (dim, degree)");
    }
}

inline int check_ptr(const void *p, const char *name)
{
    if (!p) return fail(DGAMR_EINVAL, std::string(name) + " is null");
    return DGAMR_OK;
}

#define CHECK(x)                      \
    do {                              \
        int rc_ = (x);                \
        if (rc_ != DGAMR_OK) return rc_; \
    } while (0)

#define GUARD_API(...)                                                      \
    try {                                                                   \
        __VA_ARGS__                                                         \
    } catch (const std::exception &e) {                                     \
        return fail(DGAMR_EINVAL, std::string("internal error: ") + e.what()); \
    } catch (...) {                                                         \
        return fail(DGAMR_EINVAL, "internal error");                        \
    }

} // namespace dgapi

struct dgamr_forest {
    dgamr::Forest topo;
    int device = 0;
    dgamr::LeafGeo *d_geo = nullptr;
    dgamr::FaceLink *d_links = nullptr;
    dgamr::RotPlan *d_plans = nullptr; // guard-cell plans of rotated faces
    size_t plans_cap = 0;
    int cap = 0;             // leaves the device tables can hold
    bool prof = false;       // bracket stage launches with events
    int stage_variant = -1;  // 2-D stage kernel: -1 auto, 0 lane per (cell, var), 1 thread per cell
    long var_split_max_cells = 131072; // auto: lane per (cell, var) up to this many cells
    int slab_rows = 0;       // layers of the last axis per stage workgroup, 0 = automatic
    int mfma = 0;            // FP32 residual: 1 = volume integral on the matrix cores where built
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec;
    long version = 0;        // bumped by every topology change
    double time = 0.0;       // time of the state (Dirichlet data of a diffusion forest)
    explicit dgamr_forest(const dgamr_forest_desc &d) : topo(d) {}
};

namespace dgapi {
// one dgamr_step with `work` as the work buffer (at least work_bytes_of(f)
// bytes), recording no events
int step_in_work(dgamr_forest *f, double cfl, double *u, void *work, double *dt_dev, hipStream_t stream);
size_t work_bytes_of(const dgamr_forest *f);
} // namespace dgapi

// A captured HIP graph of steps (of one forest, or of several pools).  It
// records the version counters of what it was captured from; launching it
// after any of them changed is refused.
struct dgamr_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<const long *, long>> versions;
    ~dgamr_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

