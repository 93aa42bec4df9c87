// C-ABI of the block-AMR DG library: forest handles, buffer sizes,
// refinement, and the launches of the HIP kernels.  See include/dgamr.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <type_traits>
#include <vector>

#include "api_internal.hpp"
#include "kernels_small.hpp"
#include "launch.hpp"

using dgamr::FaceLink;
using dgamr::Forest;
using dgamr::Inherit;
using dgamr::LeafGeo;
using namespace dgapi;

namespace {

int ncell_of(const dgamr_forest *f)
{
    int n = f->topo.desc().n_cell;
    return f->topo.dim() == 2 ? n * n : n * n * n;
}
int nfc_of(const dgamr_forest *f)
{
    int n = f->topo.desc().n_cell;
    return f->topo.dim() == 2 ? n : n * n;
}
int nb_of(const dgamr_forest *f) { return dgk::num_modes(f->topo.dim(), f->topo.desc().degree); }
int nv_of(const dgamr_forest *f) { return f->topo.nv(); }
size_t state_elems(const dgamr_forest *f) { return size_t(f->topo.n()) * nv_of(f) * nb_of(f) * ncell_of(f); }
size_t guard_elems(const dgamr_forest *f)
{
    return size_t(f->topo.n()) * 2 * f->topo.dim() * nv_of(f) * nb_of(f) * nfc_of(f);
}
// work layout: [U1 | U2 | guard | residual | leaf maxima | leaf partials | scalars]
struct Work {
    double *u1, *u2, *guard, *res, *leafmax, *part, *scal;
};
Work carve(const dgamr_forest *f, void *work)
{
    Work w;
    size_t s = state_elems(f), gsz = guard_elems(f), n = f->topo.n();
    double *p = static_cast<double *>(work);
    w.u1 = p;
    w.u2 = w.u1 + s;
    w.guard = w.u2 + s;
    w.res = w.guard + gsz;
    w.leafmax = w.res + s;
    w.part = w.leafmax + n;
    w.scal = w.part + n * 8;
    return w;
}
size_t work_elems(const dgamr_forest *f)
{
    size_t s = state_elems(f), gsz = guard_elems(f), n = f->topo.n();
    return 3 * s + gsz + n + n * 8 + 64;
}

int upload(dgamr_forest *f)
{
    int n = f->topo.n(), nf = 2 * f->topo.dim();
    HIP_TRY(hipSetDevice(f->device));
    if (n > f->cap) {
        if (f->d_geo) HIP_TRY(hipFree(f->d_geo));
        if (f->d_links) HIP_TRY(hipFree(f->d_links));
        int cap = n + n / 2 + 16;
        HIP_TRY(hipMalloc(&f->d_geo, sizeof(LeafGeo) * cap));
        HIP_TRY(hipMalloc(&f->d_links, sizeof(FaceLink) * size_t(cap) * nf));
        f->cap = cap;
    }
    std::vector<LeafGeo> geo = f->topo.geometry();
    HIP_TRY(hipMemcpy(f->d_geo, geo.data(), sizeof(LeafGeo) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_links, f->topo.links().data(), sizeof(FaceLink) * size_t(n) * nf, hipMemcpyHostToDevice));
    const auto &plans = f->topo.plans();
    if (plans.size() > f->plans_cap) {
        if (f->d_plans) HIP_TRY(hipFree(f->d_plans));
        f->plans_cap = plans.size() + plans.size() / 2 + 16;
        HIP_TRY(hipMalloc(&f->d_plans, sizeof(dgamr::RotPlan) * f->plans_cap));
    }
    if (!plans.empty())
        HIP_TRY(hipMemcpy(f->d_plans, plans.data(), sizeof(dgamr::RotPlan) * plans.size(), hipMemcpyHostToDevice));
    return DGAMR_OK;
}

// guard cells of every block face, as coefficients or (traces) as their
// values at the face points
int launch_fill(dgamr_forest *f, const double *u, double *guard, bool traces, hipStream_t s)
{
    int nf = 2 * f->topo.dim();
    dgk::FillArgs a{u,       guard, f->d_links, f->d_plans, nullptr, f->topo.n() * nf, f->topo.desc().n_cell,
                    traces ? 1 : 0, f->topo.mapped() ? 1 : 0};
    if (a.nfaces == 0) return DGAMR_OK;
    return dispatch(f->topo.dim(), f->topo.desc().degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_fill<D, P>(a, nfc_of(f), s, nv_of(f))));
        return DGAMR_OK;
    });
}

int stage_variant(const dgamr_forest *f)
{
    if (f->stage_variant >= 0) return f->stage_variant;
    // 3-D: one lane per (cell, variable) at degree 3, where one thread per
    // cell runs out of registers; one thread per cell below (measured)
    if (f->topo.dim() == 3) return f->topo.desc().degree >= 3 ? 0 : 1;
    return long(f->topo.n()) * ncell_of(f) <= f->var_split_max_cells ? 0 : 1;
}

dgk::StageShape stage_shape(const dgamr_forest *f)
{
    dgk::StageShape sh;
    sh.variant = stage_variant(f);
    sh.rows = f->slab_rows;
    sh.mfma = f->mfma;
    return sh;
}

// the fused stage of this forest reads guard traces (the 3-D lane kernel)
bool fused_reads_traces(const dgamr_forest *f)
{
    if (f->topo.unfused()) return false;
    return dgk::stage_reads_traces(f->topo.dim(), stage_shape(f), f->topo.desc().limiter == DGAMR_LIMITER_POSITIVITY,
                                   f->topo.desc().precision == DGAMR_FP32,
                                   f->topo.desc().hanging == DGAMR_HANG_CONSERVATIVE, f->topo.advection(),
                                   f->topo.desc().n_cell);
}

int launch_stage(dgamr_forest *f, dgk::StageArgs a, int gm, int om, hipStream_t s, bool lim = false)
{
    a.nleaves = f->topo.n();
    a.N = f->topo.desc().n_cell;
    a.gamma = f->topo.desc().gamma;
    a.geo = f->d_geo;
    a.links = f->d_links;
    a.conservative = f->topo.desc().hanging == DGAMR_HANG_CONSERVATIVE;
    for (int k = 0; k < 3; ++k) a.vel[k] = f->topo.desc().velocity[k];
    if (a.nleaves == 0) return DGAMR_OK;
    const bool fp32 = f->topo.desc().precision == DGAMR_FP32;
    const int eq = f->topo.advection() ? dgk::EQ_ADVECTION : dgk::EQ_EULER;
    const dgk::StageShape sh = stage_shape(f);
    return dispatch(f->topo.dim(), f->topo.desc().degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_stage<D, P>(a, gm, om, lim, fp32, sh, s, eq)));
        return DGAMR_OK;
    });
}

// arguments of the bilinear-root kernels
dgk::MappedArgs mapped_args(const dgamr_forest *f, const double *us, const double *un, const double *guard,
                            double *out, const double *dt, double a, double b)
{
    dgk::MappedArgs m{};
    m.us = us;
    m.un = un;
    m.guard = guard;
    m.out = out;
    m.geo = f->d_geo;
    m.dt = dt;
    m.rk_a = a;
    m.rk_b = b;
    m.gamma = f->topo.desc().gamma;
    for (int k = 0; k < 3; ++k) m.vel[k] = f->topo.desc().velocity[k];
    m.ncell_total = long(f->topo.n()) * ncell_of(f);
    m.N = f->topo.desc().n_cell;
    return m;
}

// dimension and degree of a mapped forest as compile-time constants (the
// built cases: 2-D any degree, 3-D degree <= 2)
template <class Fn>
int dispatch_mapped(const dgamr_forest *f, Fn &&fn)
{
    using std::integral_constant;
    const int p = f->topo.desc().degree;
    if (f->topo.dim() == 3) {
        switch (p) {
        case 0: return fn(integral_constant<int, 3>{}, integral_constant<int, 0>{});
        case 1: return fn(integral_constant<int, 3>{}, integral_constant<int, 1>{});
        case 2: return fn(integral_constant<int, 3>{}, integral_constant<int, 2>{});
        default: return fail(DGAMR_EUNSUPPORTED, "trilinear root blocks are built for degree <= 2");
        }
    }
    switch (p) {
    case 0: return fn(integral_constant<int, 2>{}, integral_constant<int, 0>{});
    case 1: return fn(integral_constant<int, 2>{}, integral_constant<int, 1>{});
    case 2: return fn(integral_constant<int, 2>{}, integral_constant<int, 2>{});
    default: return fn(integral_constant<int, 2>{}, integral_constant<int, 3>{});
    }
}

int launch_limit(dgamr_forest *f, double *u, hipStream_t s)
{
    if (f->topo.scalar()) return fail(DGAMR_EINVAL, "the positivity limiter is for the Euler equations");
    long total = long(f->topo.n()) * ncell_of(f);
    if (total == 0) return DGAMR_OK;
    if (f->topo.mapped())
        // bilinear / trilinear roots: scaled about the mean over the physical cell
        return dispatch_mapped(f, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_mapped_limit<D, P>(u, f->d_geo, f->topo.desc().n_cell, total, f->topo.desc().gamma, s)));
            return DGAMR_OK;
        });
    return dispatch(f->topo.dim(), f->topo.desc().degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_limit<D, P>(u, f->topo.desc().n_cell, total, f->topo.desc().gamma, s)));
        return DGAMR_OK;
    });
}

int launch_dt(dgamr_forest *f, double cfl, const double *u, double *dt_dev, const Work &w, hipStream_t s)
{
    int n = f->topo.n();
    if (n == 0) return fail(DGAMR_EINVAL, "empty forest");
    int ncell = ncell_of(f), block = 1;
    while (block < ncell && block < 256) block <<= 1; // power of two for the tree reduction
    const double *vel = f->topo.desc().velocity;
    if (f->topo.mapped()) {
        dgk::MappedArgs a = mapped_args(f, u, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0);
        const int eq = f->topo.advection() ? dgk::EQ_ADVECTION : dgk::EQ_EULER;
        CHECK(dispatch_mapped(f, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_mapped_rate<D, P>(a, eq, n, block, w.leafmax, s)));
            return DGAMR_OK;
        }));
    } else if (f->topo.advection())
        hipLaunchKernelGGL(dgk::k_rate_adv, dim3((n + 255) / 256), dim3(256), 0, s, f->d_geo, n, vel[0], vel[1],
                           vel[2], f->topo.dim(), w.leafmax);
    else if (f->topo.dim() == 2)
        hipLaunchKernelGGL(dgk::k_rate<2>, dim3(n), dim3(block), 0, s, u, f->d_geo, f->topo.desc().n_cell, nb_of(f),
                           f->topo.desc().gamma, w.leafmax, nullptr);
    else
        hipLaunchKernelGGL(dgk::k_rate<3>, dim3(n), dim3(block), 0, s, u, f->d_geo, f->topo.desc().n_cell, nb_of(f),
                           f->topo.desc().gamma, w.leafmax, nullptr);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(dgk::k_dt_final, dim3(1), dim3(1024), 0, s, w.leafmax, n, cfl, dt_dev);
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

int take_event(dgamr_forest *f, hipEvent_t &e)
{
    if (f->ev_free.empty()) {
        HIP_TRY(hipEventCreate(&e));
    } else {
        e = f->ev_free.back();
        f->ev_free.pop_back();
    }
    return DGAMR_OK;
}

// Diffusion: dt = cfl / max over cells of nu sum_a 1/h_a^2 (the finest
// cells), on the host.
double diffusion_dt(const dgamr_forest *f, double cfl)
{
    const auto &d = f->topo.desc();
    int lmax = 1;
    for (const auto &k : f->topo.leaves()) lmax = k.level > lmax ? k.level : lmax;
    double rate = 0.0;
    for (int a = 0; a < f->topo.dim(); ++a) {
        const double h = (d.hi[a] - d.lo[a]) / (double(d.roots[a]) * d.n_cell * double(1L << (lmax - 1)));
        rate += d.diffusivity / (h * h);
    }
    return cfl / rate;
}

int launch_ipdg(dgamr_forest *f, const double *us, const double *un, const double *guard, double *out,
                const double *dt_dev, double rk_a, double rk_b, double t, int om, hipStream_t s)
{
    const auto &d = f->topo.desc();
    dgk::IpdgArgs a{};
    a.us = us;
    a.un = un;
    a.guard = guard;
    a.out = out;
    a.geo = f->d_geo;
    a.links = f->d_links;
    a.dt = dt_dev;
    a.rk_a = rk_a;
    a.rk_b = rk_b;
    a.nu = d.diffusivity;
    for (int k = 0; k < 3; ++k) a.avec[k] = k < f->topo.dim() ? d.exact_a[k] : 0.0;
    a.t = t;
    a.ncell_total = long(f->topo.n()) * ncell_of(f);
    a.N = d.n_cell;
    return dispatch(f->topo.dim(), d.degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_ipdg<D, P>(a, om, s)));
        return DGAMR_OK;
    });
}

// One SSP-RK3 step of a diffusion forest: dt from the host, per stage the
// guard fill (coefficients) and the fused interior-penalty stage with the
// Dirichlet data at the stage time (t, t + dt, t + dt/2).
int step_diffusion(dgamr_forest *f, double cfl, double *u, const Work &w, double *dt_dev, hipStream_t s)
{
    if (!(cfl > 0.0)) return fail(DGAMR_EINVAL, "a diffusion step needs cfl > 0 (its time step is set on the host)");
    const double dt = diffusion_dt(f, cfl);
    hipLaunchKernelGGL(dgk::k_set_value, dim3(1), dim3(1), 0, s, dt_dev, dt);
    HIP_TRY(hipGetLastError());
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0}, C[3] = {0.0, 1.0, 0.5};
    const double *us = u;
    double *outs[3] = {w.u1, w.u2, u};
    for (int st = 0; st < 3; ++st) {
        CHECK(launch_fill(f, us, w.guard, false, s));
        CHECK(launch_ipdg(f, us, u, w.guard, outs[st], dt_dev, A[st], B[st], f->time + C[st] * dt, dgk::OUT_RK, s));
        us = outs[st];
    }
    f->time += dt;
    return DGAMR_OK;
}

} // namespace

extern "C" {

const char *dgamr_last_error(void) { return dgapi::g_err.c_str(); }

int dgamr_create_forest(const dgamr_forest_desc *desc, dgamr_forest **out)
{
    GUARD_API({
        CHECK(check_ptr(desc, "desc"));
        CHECK(check_ptr(out, "out"));
        *out = nullptr;
        std::string err;
        int rc = Forest::validate(*desc, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        auto *f = new dgamr_forest(*desc);
        HIP_TRY(hipGetDevice(&f->device));
        rc = f->topo.build_links(err);
        if (rc != DGAMR_OK) {
            delete f;
            return fail(rc, err);
        }
        rc = upload(f);
        if (rc != DGAMR_OK) {
            delete f;
            return rc;
        }
        *out = f;
        return DGAMR_OK;
    })
}

int dgamr_destroy_forest(dgamr_forest *f)
{
    if (!f) return DGAMR_OK;
    for (auto e : f->ev_free) (void)hipEventDestroy(e);
    for (auto &pr : f->ev_rec) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    (void)hipFree(f->d_geo);
    (void)hipFree(f->d_links);
    (void)hipFree(f->d_plans);
    delete f;
    return DGAMR_OK;
}

int dgamr_num_leaves(const dgamr_forest *f, int64_t *n)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(n, "n"));
    *n = f->topo.n();
    return DGAMR_OK;
}

int dgamr_leaf_keys(const dgamr_forest *f, int32_t *keys)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(keys, "keys"));
    for (int i = 0; i < f->topo.n(); ++i) {
        const auto &k = f->topo.leaves()[i];
        keys[5 * i + 0] = k.tree;
        keys[5 * i + 1] = k.level;
        keys[5 * i + 2] = k.idx[0];
        keys[5 * i + 3] = k.idx[1];
        keys[5 * i + 4] = k.idx[2];
    }
    return DGAMR_OK;
}

int dgamr_state_bytes(const dgamr_forest *f, size_t *u_bytes, size_t *guard_bytes, size_t *residual_bytes,
                      size_t *work_bytes)
{
    CHECK(check_ptr(f, "forest"));
    if (u_bytes) *u_bytes = state_elems(f) * sizeof(double);
    if (guard_bytes) *guard_bytes = guard_elems(f) * sizeof(double);
    if (residual_bytes)
        *residual_bytes = state_elems(f) * (f->topo.desc().precision == DGAMR_FP32 ? sizeof(float) : sizeof(double));
    if (work_bytes) *work_bytes = work_elems(f) * sizeof(double);
    return DGAMR_OK;
}

int dgamr_set_refinement(dgamr_forest *f, const int8_t *flags, int64_t *n_new)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(flags, "flags"));
        std::string err;
        int rc = f->topo.plan(flags, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        if (n_new) *n_new = f->topo.planned_n();
        return DGAMR_OK;
    })
}

int dgamr_apply_refinement(dgamr_forest *f, const double *u_old, double *u_new, hipStream_t stream)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        if (!f->topo.has_plan()) return fail(DGAMR_ESTATE, "no refinement plan pending");
        CHECK(check_ptr(u_old, "u_old"));
        CHECK(check_ptr(u_new, "u_new"));
        std::string err;
        std::vector<Inherit> inh;
        int rc = f->topo.commit(inh, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        int n = f->topo.n();
        Inherit *d_inh = nullptr;
        HIP_TRY(hipMalloc(reinterpret_cast<void **>(&d_inh), sizeof(Inherit) * n));
        HIP_TRY(hipMemcpyAsync(d_inh, inh.data(), sizeof(Inherit) * n, hipMemcpyHostToDevice, stream));
        long total = long(n) * ncell_of(f);
        rc = dispatch(f->topo.dim(), f->topo.desc().degree, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_inherit<D, P>(u_old, u_new, d_inh, f->topo.desc().n_cell, total, stream, nv_of(f))));
            return DGAMR_OK;
        });
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipFree(d_inh));
        f->version += 1;
        if (rc != DGAMR_OK) return rc;
        return upload(f);
    })
}

int dgamr_fill_guardcells(dgamr_forest *f, const double *u, double *guard, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(guard, "guard"));
    return launch_fill(f, u, guard, false, stream);
}

int dgamr_dg_residual(dgamr_forest *f, const double *u, const double *guard, void *r, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(guard, "guard"));
    CHECK(check_ptr(r, "r"));
    if (f->topo.diffusion())
        return launch_ipdg(f, u, nullptr, guard, static_cast<double *>(r), nullptr, 0.0, 1.0, f->time, dgk::OUT_RES64,
                           stream);
    if (f->topo.mapped()) {
        dgk::MappedArgs a = mapped_args(f, u, nullptr, guard, static_cast<double *>(r), nullptr, 0.0, 1.0);
        const int eq = f->topo.advection() ? dgk::EQ_ADVECTION : dgk::EQ_EULER;
        return dispatch_mapped(f, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_mapped<D, P>(a, eq, dgk::OUT_RES64, false, stream)));
            return DGAMR_OK;
        });
    }
    dgk::StageArgs a{};
    a.us = u;
    a.guard = guard;
    bool r32 = f->topo.desc().precision == DGAMR_FP32;
    a.out64 = r32 ? nullptr : static_cast<double *>(r);
    a.out32 = r32 ? static_cast<float *>(r) : nullptr;
    return launch_stage(f, a, dgk::GUARD_BUFFER, r32 ? dgk::OUT_RES32 : dgk::OUT_RES64, stream);
}

int dgamr_rk_stage(dgamr_forest *f, int stage, const double *dt_dev, const double *u_n, const double *u_s,
                   const void *r, double *u_next, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    if (stage < 0 || stage > 2) return fail(DGAMR_EINVAL, "stage must be 0, 1 or 2");
    CHECK(check_ptr(dt_dev, "dt_dev"));
    CHECK(check_ptr(u_s, "u_s"));
    CHECK(check_ptr(r, "r"));
    CHECK(check_ptr(u_next, "u_next"));
    if (stage > 0) CHECK(check_ptr(u_n, "u_n"));
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
    dgk::RkArgs a{u_n, u_s, r, u_next, dt_dev, A[stage], B[stage], long(state_elems(f)),
                  f->topo.desc().precision == DGAMR_FP32 ? 1 : 0};
    if (a.n == 0) return DGAMR_OK;
    long blocks = (a.n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(dgk::k_rk, dim3(unsigned(blocks)), dim3(256), 0, stream, a);
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

int dgamr_compute_dt(dgamr_forest *f, double cfl, const double *u, double *dt_dev, void *work, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(dt_dev, "dt_dev"));
    CHECK(check_ptr(work, "work"));
    if (!(cfl > 0.0)) return fail(DGAMR_EINVAL, "cfl must be positive");
    if (f->topo.diffusion()) {
        hipLaunchKernelGGL(dgk::k_set_value, dim3(1), dim3(1), 0, stream, dt_dev, diffusion_dt(f, cfl));
        HIP_TRY(hipGetLastError());
        return DGAMR_OK;
    }
    return launch_dt(f, cfl, u, dt_dev, carve(f, work), stream);
}

// Measurement hook: events before and after one stage's launches
int prof_begin(dgamr_forest *f, hipStream_t stream, hipEvent_t &e1)
{
    e1 = nullptr;
    if (!f->prof) return DGAMR_OK;
    hipEvent_t e0 = nullptr;
    CHECK(take_event(f, e0));
    CHECK(take_event(f, e1));
    f->ev_rec.emplace_back(e0, e1);
    HIP_TRY(hipEventRecord(e0, stream));
    return DGAMR_OK;
}

int prof_end(dgamr_forest *f, hipStream_t stream, hipEvent_t e1)
{
    if (e1) HIP_TRY(hipEventRecord(e1, stream));
    return DGAMR_OK;
}

// One SSP-RK3 step as three fused stage launches (far side of block faces
// inline, or from guard traces for the 3-D lane kernel; limiter fused).  rate_in / rate_clear / rate_out select the CFL
// time step folded into the stages (see StageArgs).
int run_step(dgamr_forest *f, double cfl, double *u, const Work &w, double *dt_dev,
             const unsigned long long *rate_in, unsigned long long *rate_clear, unsigned long long *rate_out,
             hipStream_t stream)
{
    const bool lim = f->topo.desc().limiter == DGAMR_LIMITER_POSITIVITY;
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
    const double *us = u;
    double *outs[3] = {w.u1, w.u2, u};
    if (f->topo.mapped()) {
        // bilinear roots: the guard fill (reference-space copy, split,
        // combine), then the residual with the metric terms fused with the
        // stage update (and the limiter about the physical cell mean)
        const int eq = f->topo.advection() ? dgk::EQ_ADVECTION : dgk::EQ_EULER;
        for (int s = 0; s < 3; ++s) {
            hipEvent_t e1;
            CHECK(prof_begin(f, stream, e1));
            CHECK(launch_fill(f, us, w.guard, false, stream));
            dgk::MappedArgs a = mapped_args(f, us, u, w.guard, outs[s], dt_dev, A[s], B[s]);
            CHECK(dispatch_mapped(f, [&](auto D, auto P) -> int {
                HIP_TRY((dgk::launch_mapped<D, P>(a, eq, dgk::OUT_RK, lim, stream)));
                return DGAMR_OK;
            }));
            CHECK(prof_end(f, stream, e1));
            us = outs[s];
        }
        return DGAMR_OK;
    }
    if (f->topo.rotated()) {
        // roots of different frames: the guard fill applies the rotation of
        // each guard cell (Sec. 3.5) into the guard buffer; the stage kernel
        // reads the far side of block faces from there, fused with the stage
        // update and the limiter (dt from the step's CFL reduction)
        for (int s = 0; s < 3; ++s) {
            hipEvent_t e1;
            CHECK(prof_begin(f, stream, e1));
            CHECK(launch_fill(f, us, w.guard, false, stream));
            dgk::StageArgs a{};
            a.us = us;
            a.un = u;
            a.guard = w.guard;
            a.out64 = outs[s];
            a.dt = dt_dev;
            a.rk_a = A[s];
            a.rk_b = B[s];
            a.cfl = cfl;
            a.dt_out = dt_dev;
            CHECK(launch_stage(f, a, dgk::GUARD_BUFFER, dgk::OUT_RK, stream, lim));
            CHECK(prof_end(f, stream, e1));
            us = outs[s];
        }
        return DGAMR_OK;
    }
    for (int s = 0; s < 3; ++s) {
        dgk::StageArgs a{};
        a.us = us;
        a.un = u;
        a.out64 = outs[s];
        a.dt = dt_dev;
        a.rk_a = A[s];
        a.rk_b = B[s];
        a.cfl = cfl;
        a.rate_in = s == 0 ? rate_in : nullptr;
        a.rate_clear = s == 0 ? rate_clear : nullptr;
        a.dt_out = dt_dev;
        a.rate_out = s == 2 ? rate_out : nullptr;
        // the 3-D lane kernel reads the far side of every block face as
        // traces from the guard buffer; the other stage kernels compute it
        // inline
        const bool guard3 = fused_reads_traces(f);
        if (guard3) {
            a.guard = w.guard;
            CHECK(launch_fill(f, us, w.guard, true, stream));
        }
        hipEvent_t e1;
        CHECK(prof_begin(f, stream, e1));
        CHECK(launch_stage(f, a, guard3 ? dgk::GUARD_TRACE : dgk::GUARD_INLINE, dgk::OUT_RK, stream, lim));
        CHECK(prof_end(f, stream, e1));
        us = outs[s];
    }
    return DGAMR_OK;
}

int dgamr_step(dgamr_forest *f, double cfl, double *u, void *work, double *dt_dev, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(work, "work"));
    CHECK(check_ptr(dt_dev, "dt_dev"));
    Work w = carve(f, work);
    if (f->topo.diffusion()) return step_diffusion(f, cfl, u, w, dt_dev, stream);
    if (cfl > 0.0) CHECK(launch_dt(f, cfl, u, dt_dev, w, stream));
    return run_step(f, cfl, u, w, dt_dev, nullptr, nullptr, nullptr, stream);
}

int dgamr_math_probe(int fn, const double *x, double *y, int64_t n, hipStream_t stream)
{
    if (fn != 0 && fn != 1) return fail(DGAMR_EINVAL, "fn must be 0 (reciprocal) or 1 (square root)");
    CHECK(check_ptr(x, "x"));
    CHECK(check_ptr(y, "y"));
    if (n < 0) return fail(DGAMR_EINVAL, "n must be >= 0");
    if (n == 0) return DGAMR_OK;
    hipLaunchKernelGGL(dgk::k_math_probe, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, fn, x, y, long(n));
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

int dgamr_set_root_frames(dgamr_forest *f, const int32_t *codes)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(codes, "codes"));
        std::string err;
        int rc = f->topo.set_frames(codes, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        f->version += 1;
        return upload(f);
    })
}

int dgamr_set_root_nodes(dgamr_forest *f, const double *xy)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(xy, "xy"));
        if (f->topo.desc().precision != DGAMR_FP64)
            return fail(DGAMR_EUNSUPPORTED, "bilinear roots are built for the FP64 residual");
        std::string err;
        int rc = f->topo.set_nodes(xy, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        f->version += 1;
        return upload(f);
    })
}

int dgamr_set_time(dgamr_forest *f, double t)
{
    CHECK(check_ptr(f, "forest"));
    if (!std::isfinite(t)) return fail(DGAMR_EINVAL, "time must be finite");
    f->time = t;
    return DGAMR_OK;
}

int dgamr_get_time(const dgamr_forest *f, double *t)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(t, "t"));
    *t = f->time;
    return DGAMR_OK;
}

} // extern "C"

// dgamr_step with a work area the caller does not own (the static one of
// dgamr_step_static): the same launches, no events recorded.
int dgapi::step_in_work(dgamr_forest *f, double cfl, double *u, void *work, double *dt_dev, hipStream_t stream)
{
    Work w = carve(f, work);
    if (f->topo.diffusion()) return step_diffusion(f, cfl, u, w, dt_dev, stream);
    if (cfl > 0.0) CHECK(launch_dt(f, cfl, u, dt_dev, w, stream));
    const bool prof_was = f->prof;
    f->prof = false;
    const int rc = run_step(f, cfl, u, w, dt_dev, nullptr, nullptr, nullptr, stream);
    f->prof = prof_was;
    return rc;
}

size_t dgapi::work_bytes_of(const dgamr_forest *f) { return work_elems(f) * sizeof(double); }

extern "C" {

int dgamr_run(dgamr_forest *f, double cfl, int nsteps, double *u, void *work, double *dt_dev, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(work, "work"));
    CHECK(check_ptr(dt_dev, "dt_dev"));
    if (nsteps < 0) return fail(DGAMR_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return DGAMR_OK;
    Work w = carve(f, work);
    if (f->topo.diffusion()) {
        for (int s = 0; s < nsteps; ++s) CHECK(step_diffusion(f, cfl, u, w, dt_dev, stream));
        return DGAMR_OK;
    }
    auto *slot = reinterpret_cast<unsigned long long *>(w.scal + 2);
    if (cfl <= 0.0 || f->topo.unfused()) { // rotated frames, bilinear roots: dt from a reduction per step
        for (int s = 0; s < nsteps; ++s) {
            if (cfl > 0.0) CHECK(launch_dt(f, cfl, u, dt_dev, w, stream));
            CHECK(run_step(f, cfl, u, w, dt_dev, nullptr, nullptr, nullptr, stream));
        }
        return DGAMR_OK;
    }
    CHECK(launch_dt(f, cfl, u, dt_dev, w, stream));
    for (int s = 0; s < nsteps; ++s) {
        const int rd = s & 1, wr = rd ^ 1;
        const bool last = s == nsteps - 1;
        CHECK(run_step(f, cfl, u, w, dt_dev, s == 0 ? nullptr : slot + rd, last ? nullptr : slot + wr,
                       last ? nullptr : slot + wr, stream));
    }
    return DGAMR_OK;
}

int dgamr_run_capture(dgamr_forest *f, double cfl, int nsteps, double *u, void *work, double *dt_dev,
                      dgamr_graph **out)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(u, "u"));
        CHECK(check_ptr(work, "work"));
        CHECK(check_ptr(dt_dev, "dt_dev"));
        CHECK(check_ptr(out, "out"));
        *out = nullptr;
        if (!(cfl > 0.0)) return fail(DGAMR_EINVAL, "cfl must be positive");
        if (nsteps <= 0) return fail(DGAMR_EINVAL, "nsteps must be positive");
        if (f->topo.diffusion())
            return fail(DGAMR_EUNSUPPORTED, "diffusion steps take their stage times from the host: not captured");
        Work w = carve(f, work);
        auto *slot = reinterpret_cast<unsigned long long *>(w.scal + 2);
        hipStream_t s;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        auto *g = new dgamr_graph;
        const bool prof_was = f->prof;
        f->prof = false; // no event records inside a graph
        int rc = DGAMR_OK;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(DGAMR_EHIP, "hipStreamBeginCapture failed");
        } else {
            // CFL rate of the input state into slot 0, then every step takes
            // its dt from the slot its predecessor's last stage filled
            rc = launch_dt(f, cfl, u, dt_dev, w, s);
            if (rc == DGAMR_OK) {
                hipLaunchKernelGGL(dgk::k_rate_slot, dim3(1), dim3(1024), 0, s, w.leafmax, f->topo.n(), slot);
                if (hipGetLastError() != hipSuccess) rc = fail(DGAMR_EHIP, "k_rate_slot launch failed");
            }
            for (int st = 0; st < nsteps && rc == DGAMR_OK; ++st) {
                const int rd = st & 1, wr = rd ^ 1;
                const bool last = st == nsteps - 1;
                if (f->topo.unfused()) { // fill + stage kernel per stage: the CFL reduction of every step
                    if (st > 0) rc = launch_dt(f, cfl, u, dt_dev, w, s);
                    if (rc == DGAMR_OK) rc = run_step(f, cfl, u, w, dt_dev, nullptr, nullptr, nullptr, s);
                    continue;
                }
                rc = run_step(f, cfl, u, w, dt_dev, slot + rd, slot + wr, last ? nullptr : slot + wr, s);
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc == DGAMR_OK && e != hipSuccess) rc = fail(DGAMR_EHIP, "hipStreamEndCapture failed");
            g->graph = graph;
            if (rc == DGAMR_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(DGAMR_EHIP, "hipGraphInstantiate failed");
        }
        f->prof = prof_was;
        (void)hipStreamDestroy(s);
        if (rc != DGAMR_OK) {
            delete g;
            return rc;
        }
        g->versions.emplace_back(&f->version, f->version);
        *out = g;
        return DGAMR_OK;
    })
}

int dgamr_conserved_totals(dgamr_forest *f, const double *u, double *totals_dev, void *work, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(totals_dev, "totals_dev"));
    CHECK(check_ptr(work, "work"));
    Work w = carve(f, work);
    int n = f->topo.n(), block = ncell_of(f) < 256 ? ncell_of(f) : 256;
    if (n == 0) return fail(DGAMR_EINVAL, "empty forest");
    int bp = 1;
    while (bp < block) bp <<= 1; // power of two for the tree reduction
    if (f->topo.mapped()) {
        dgk::MappedArgs a = mapped_args(f, u, nullptr, nullptr, nullptr, nullptr, 0.0, 1.0);
        const bool adv = f->topo.advection();
        CHECK(dispatch_mapped(f, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_mapped_totals<D, P>(a, adv ? dgk::EQ_ADVECTION : dgk::EQ_EULER, n, bp, w.part, stream)));
            return DGAMR_OK;
        }));
        if (adv) hipLaunchKernelGGL(dgk::k_totals_final<1>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
        else if (f->topo.dim() == 2)
            hipLaunchKernelGGL(dgk::k_totals_final<4>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
        else hipLaunchKernelGGL(dgk::k_totals_final<5>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
        HIP_TRY(hipGetLastError());
        return DGAMR_OK;
    }
    if (f->topo.scalar()) {
        if (f->topo.dim() == 2)
            hipLaunchKernelGGL((dgk::k_totals_leaf<2, 1>), dim3(n), dim3(bp), 0, stream, u, f->d_geo,
                               f->topo.desc().n_cell, nb_of(f), w.part);
        else
            hipLaunchKernelGGL((dgk::k_totals_leaf<3, 1>), dim3(n), dim3(bp), 0, stream, u, f->d_geo,
                               f->topo.desc().n_cell, nb_of(f), w.part);
        hipLaunchKernelGGL(dgk::k_totals_final<1>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
    } else if (f->topo.dim() == 2) {
        hipLaunchKernelGGL(dgk::k_totals_leaf<2>, dim3(n), dim3(bp), 0, stream, u, f->d_geo, f->topo.desc().n_cell,
                           nb_of(f), w.part);
        hipLaunchKernelGGL(dgk::k_totals_final<4>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
    } else {
        hipLaunchKernelGGL(dgk::k_totals_leaf<3>, dim3(n), dim3(bp), 0, stream, u, f->d_geo, f->topo.desc().n_cell,
                           nb_of(f), w.part);
        hipLaunchKernelGGL(dgk::k_totals_final<5>, dim3(1), dim3(256), 0, stream, w.part, n, totals_dev);
    }
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

int dgamr_limit_positivity(dgamr_forest *f, double *u, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    return launch_limit(f, u, stream);
}

int dgamr_indicator(dgamr_forest *f, const double *u, double *eta_dev, void *work, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(eta_dev, "eta_dev"));
    CHECK(check_ptr(work, "work"));
    Work w = carve(f, work);
    CHECK(launch_fill(f, u, w.guard, false, stream));
    int n = f->topo.n();
    if (n == 0) return DGAMR_OK;
    if (f->topo.scalar() && f->topo.dim() == 2)
        hipLaunchKernelGGL((dgk::k_indicator_leaf<2, 1>), dim3(n), dim3(256), 0, stream, u, w.guard,
                           f->topo.desc().n_cell, nb_of(f), eta_dev);
    else if (f->topo.scalar())
        hipLaunchKernelGGL((dgk::k_indicator_leaf<3, 1>), dim3(n), dim3(256), 0, stream, u, w.guard,
                           f->topo.desc().n_cell, nb_of(f), eta_dev);
    else if (f->topo.dim() == 2)
        hipLaunchKernelGGL(dgk::k_indicator_leaf<2>, dim3(n), dim3(256), 0, stream, u, w.guard, f->topo.desc().n_cell,
                           nb_of(f), eta_dev);
    else
        hipLaunchKernelGGL(dgk::k_indicator_leaf<3>, dim3(n), dim3(256), 0, stream, u, w.guard, f->topo.desc().n_cell,
                           nb_of(f), eta_dev);
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

int dgamr_project_ic(dgamr_forest *f, int kind, const double *params, double t, double *u, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(params, "params"));
    CHECK(check_ptr(u, "u"));
    if (kind < DGAMR_IC_VORTEX || kind > DGAMR_IC_EXP) return fail(DGAMR_EINVAL, "unknown initial condition");
    if ((kind == DGAMR_IC_COSINE) != f->topo.advection() || (kind == DGAMR_IC_EXP) != f->topo.diffusion())
        return fail(DGAMR_EINVAL, "DGAMR_IC_COSINE is the scalar convection state, DGAMR_IC_EXP the diffusion "
                                  "state, the others are Euler states");
    dgk::IcParams prm;
    std::memcpy(prm.p, params, sizeof(prm.p));
    const auto &d = f->topo.desc();
    if (kind == DGAMR_IC_COSINE)
        for (int a = 0; a < 3; ++a) prm.p[4 + a] = d.velocity[a]; // translation of the exact solution
    if (kind == DGAMR_IC_EXP) { // the forest's exact solution
        for (int a = 0; a < 3; ++a) prm.p[a] = d.exact_a[a];
        prm.p[3] = d.diffusivity;
    }
    double hmin[3];
    for (int a = 0; a < 3; ++a)
        hmin[a] = (d.hi[a] - d.lo[a]) / (double(d.roots[a]) * d.n_cell * double(1 << (d.max_level - 1)));
    long total = long(f->topo.n()) * ncell_of(f);
    if (total == 0) return DGAMR_OK;
    if (f->topo.mapped())
        return dispatch_mapped(f, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_mapped_ic<D, P>(u, f->d_geo, d.n_cell, total, kind, prm, t, d.gamma, nv_of(f), stream)));
            return DGAMR_OK;
        });
    return dispatch(f->topo.dim(), d.degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_project_ic<D, P>(u, f->d_geo, d.n_cell, total, kind, prm, t, d.gamma, hmin, stream,
                                              nv_of(f))));
        return DGAMR_OK;
    });
}

int dgamr_check_state(dgamr_forest *f, const double *u, int64_t *bad, void *work, hipStream_t stream)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(u, "u"));
    CHECK(check_ptr(bad, "bad"));
    CHECK(check_ptr(work, "work"));
    Work w = carve(f, work);
    auto *cnt = reinterpret_cast<unsigned long long *>(w.scal);
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), stream));
    long total = long(f->topo.n()) * ncell_of(f);
    if (total > 0) {
        dim3 grid(unsigned((total + 255) / 256)), block(256);
        if (f->topo.scalar() && f->topo.dim() == 2)
            hipLaunchKernelGGL((dgk::k_check<2, 1>), grid, block, 0, stream, u, f->topo.desc().n_cell, nb_of(f), total,
                               f->topo.desc().gamma, cnt);
        else if (f->topo.scalar())
            hipLaunchKernelGGL((dgk::k_check<3, 1>), grid, block, 0, stream, u, f->topo.desc().n_cell, nb_of(f), total,
                               f->topo.desc().gamma, cnt);
        else if (f->topo.dim() == 2)
            hipLaunchKernelGGL(dgk::k_check<2>, grid, block, 0, stream, u, f->topo.desc().n_cell, nb_of(f), total,
                               f->topo.desc().gamma, cnt);
        else
            hipLaunchKernelGGL(dgk::k_check<3>, grid, block, 0, stream, u, f->topo.desc().n_cell, nb_of(f), total,
                               f->topo.desc().gamma, cnt);
        HIP_TRY(hipGetLastError());
    }
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *bad = int64_t(h);
    return h ? fail(DGAMR_ENONPHYSICAL, "non-physical state: " + std::to_string(h) + " cells") : DGAMR_OK;
}

int dgamr_set_tuning(dgamr_forest *f, int knob, long value)
{
    CHECK(check_ptr(f, "forest"));
    if (knob == DGAMR_TUNE_STAGE_VARIANT) {
        if (value < -1 || value > 1) return fail(DGAMR_EINVAL, "stage variant must be -1, 0 or 1");
        f->stage_variant = int(value);
    } else if (knob == DGAMR_TUNE_VAR_SPLIT_MAX_CELLS) {
        if (value < 0) return fail(DGAMR_EINVAL, "cell count must be >= 0");
        f->var_split_max_cells = value;
    } else if (knob == DGAMR_TUNE_MFMA) {
        if (value != 0 && value != 1) return fail(DGAMR_EINVAL, "mfma must be 0 or 1");
        f->mfma = int(value);
    } else if (knob == DGAMR_TUNE_SLAB_ROWS) {
        const int N = f->topo.desc().n_cell;
        if (value < 0 || value > N || (value > 0 && N % value != 0))
            return fail(DGAMR_EINVAL, "slab rows must be 0 or a divisor of n_cell");
        f->slab_rows = int(value);
    } else {
        return fail(DGAMR_EINVAL, "unknown tuning knob");
    }
    return DGAMR_OK;
}

int dgamr_profile_enable(dgamr_forest *f, int enable)
{
    CHECK(check_ptr(f, "forest"));
    f->prof = enable != 0;
    return DGAMR_OK;
}

int dgamr_profile_read(dgamr_forest *f, double *stage_ms, int64_t *stage_launches)
{
    CHECK(check_ptr(f, "forest"));
    CHECK(check_ptr(stage_ms, "stage_ms"));
    CHECK(check_ptr(stage_launches, "stage_launches"));
    double total = 0.0;
    for (auto &pr : f->ev_rec) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        total += ms;
        f->ev_free.push_back(pr.first);
        f->ev_free.push_back(pr.second);
    }
    *stage_ms = total;
    *stage_launches = int64_t(f->ev_rec.size());
    f->ev_rec.clear();
    return DGAMR_OK;
}

} // extern "C"
