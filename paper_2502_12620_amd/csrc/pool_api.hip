// Pools: many forests of one class in one arena of leaf slots, stepped
// together by the same stage kernels (work list of leaf slots, per-member
// time step), plus HIP-graph capture of pool steps and the launch-shape
// autotuner.  See include/dgamr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "api_internal.hpp"
#include "kernels_small.hpp"
#include "launch.hpp"

using dgamr::FaceLink;
using dgamr::LeafGeo;
using namespace dgapi;

struct dgamr_pool {
    dgamr_forest_desc cls{};
    int dim = 2, degree = 1, N = 2, nb = 1, nv = 4, ncell = 4, nfc = 2;
    int64_t cap = 0;
    int maxm = 0;
    int device = 0;
    // device tables (capacity leaves / max members)
    LeafGeo *d_geo = nullptr;
    FaceLink *d_links = nullptr;
    int *d_member = nullptr;
    int *d_work = nullptr;
    dgk::MemberDesc *d_members = nullptr;
    // pinned host mirrors, written only after the previous upload finished
    LeafGeo *h_geo = nullptr;
    FaceLink *h_links = nullptr;
    int *h_member = nullptr;
    int *h_work = nullptr;
    dgk::MemberDesc *h_members = nullptr;
    hipEvent_t uploaded = nullptr;
    bool upload_pending = false;
    // host bookkeeping
    std::vector<char> used;   // per slot
    int nwork = 0;            // listed leaves
    int active = 0;           // active members
    long version = 0;         // bumped by every admit / release
    dgk::StageShape shape;    // stage kernel launch shape (variant 1: thread per cell)
};

namespace {

size_t leaf_elems(const dgamr_pool *p) { return size_t(p->nv) * p->nb * p->ncell; }
size_t guard_leaf_elems(const dgamr_pool *p) { return size_t(2 * p->dim) * p->nv * p->nb * p->nfc; }

// work layout: [U1 | U2 | guard | leaf maxima | member dt]
struct PoolWork {
    double *u1, *u2, *guard, *leafmax, *dt;
};
PoolWork carve(const dgamr_pool *p, void *work)
{
    PoolWork w;
    const size_t s = leaf_elems(p) * p->cap;
    w.u1 = static_cast<double *>(work);
    w.u2 = w.u1 + s;
    w.guard = w.u2 + s;
    w.leafmax = w.guard + guard_leaf_elems(p) * p->cap;
    w.dt = w.leafmax + p->cap;
    return w;
}
size_t pool_work_elems(const dgamr_pool *p)
{
    return 2 * leaf_elems(p) * p->cap + guard_leaf_elems(p) * p->cap + p->cap + p->maxm;
}

int wait_upload(dgamr_pool *p)
{
    if (p->upload_pending) {
        HIP_TRY(hipEventSynchronize(p->uploaded));
        p->upload_pending = false;
    }
    return DGAMR_OK;
}

// rebuild the work list (listed slots in slot order) and upload it with the
// member table
int upload_lists(dgamr_pool *p, hipStream_t s)
{
    int n = 0;
    for (int64_t i = 0; i < p->cap; ++i)
        if (p->used[i]) p->h_work[n++] = int(i);
    p->nwork = n;
    HIP_TRY(hipMemcpyAsync(p->d_members, p->h_members, sizeof(dgk::MemberDesc) * p->maxm, hipMemcpyHostToDevice, s));
    if (n) HIP_TRY(hipMemcpyAsync(p->d_work, p->h_work, sizeof(int) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(p->uploaded, s));
    p->upload_pending = true;
    return DGAMR_OK;
}

bool same_class(const dgamr_forest_desc &a, const dgamr_forest_desc &b)
{
    return a.dim == b.dim && a.degree == b.degree && a.n_cell == b.n_cell && a.gamma == b.gamma &&
           a.precision == b.precision && a.hanging == b.hanging && a.limiter == b.limiter;
}

int pool_dt(dgamr_pool *p, const double *u, const PoolWork &w, hipStream_t s)
{
    int block = 1;
    while (block < p->ncell && block < 256) block <<= 1;
    if (p->dim == 2)
        hipLaunchKernelGGL(dgk::k_rate<2>, dim3(p->nwork), dim3(block), 0, s, u, p->d_geo, p->N, p->nb,
                           p->cls.gamma, w.leafmax, p->d_work);
    else
        hipLaunchKernelGGL(dgk::k_rate<3>, dim3(p->nwork), dim3(block), 0, s, u, p->d_geo, p->N, p->nb,
                           p->cls.gamma, w.leafmax, p->d_work);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(dgk::k_dt_members, dim3(p->maxm), dim3(256), 0, s, w.leafmax, p->d_members, w.dt);
    HIP_TRY(hipGetLastError());
    return DGAMR_OK;
}

// one SSP-RK3 stage over the work list
int pool_stage(dgamr_pool *p, int stage, const double *us, const double *un, double *out, const PoolWork &w,
               const dgk::StageShape &sh, hipStream_t s)
{
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
    dgk::StageArgs a{};
    a.us = us;
    a.un = un;
    a.out64 = out;
    a.dt = w.dt;
    a.rk_a = A[stage];
    a.rk_b = B[stage];
    a.gamma = p->cls.gamma;
    a.nleaves = p->nwork;
    a.N = p->N;
    a.work = p->d_work;
    a.leaf_member = p->d_member;
    a.geo = p->d_geo;
    a.links = p->d_links;
    a.conservative = p->cls.hanging == DGAMR_HANG_CONSERVATIVE;
    const bool lim = p->cls.limiter == DGAMR_LIMITER_POSITIVITY;
    const bool fp32 = p->cls.precision == DGAMR_FP32;
    int gm = dgk::GUARD_INLINE;
    // the 3-D lane kernel reads guard traces of the listed leaves' faces
    if (dgk::stage_reads_traces(p->dim, sh, lim, fp32, a.conservative != 0, false, p->N)) {
        gm = dgk::GUARD_TRACE;
        a.guard = w.guard;
        dgk::FillArgs fa{us, w.guard, p->d_links, nullptr, p->d_work, p->nwork * 2 * p->dim, p->N, 1, 0};
        CHECK(dispatch(p->dim, p->degree, [&](auto D, auto P) -> int {
            HIP_TRY((dgk::launch_fill<D, P>(fa, p->nfc, s)));
            return DGAMR_OK;
        }));
    }
    return dispatch(p->dim, p->degree, [&](auto D, auto P) -> int {
        HIP_TRY((dgk::launch_stage<D, P>(a, gm, dgk::OUT_RK, lim, fp32, sh, s)));
        return DGAMR_OK;
    });
}

int pool_step(dgamr_pool *p, double *u, void *work, hipStream_t s)
{
    if (p->nwork == 0) return DGAMR_OK;
    PoolWork w = carve(p, work);
    CHECK(pool_dt(p, u, w, s));
    const double *us = u;
    double *outs[3] = {w.u1, w.u2, u};
    for (int st = 0; st < 3; ++st) {
        CHECK(pool_stage(p, st, us, u, outs[st], w, p->shape, s));
        us = outs[st];
    }
    return DGAMR_OK;
}

} // namespace

extern "C" {

// classes the lane-per-(cell, variable) kernel takes, and its slab heights
static bool lanes_class(const dgamr_pool *p)
{
    return p->cls.precision == DGAMR_FP64 && p->cls.limiter == DGAMR_LIMITER_NONE &&
           (p->dim == 2 || p->cls.hanging != DGAMR_HANG_CONSERVATIVE);
}

static bool lanes_rows_ok(const dgamr_pool *p, int r)
{
    return p->dim == 2 ? (r >= 1 && p->N % r == 0 && 4 * r * p->N <= 512) : dgk::rows_ok_3v(p->N, r);
}

int dgamr_pool_create(const dgamr_forest_desc *cls, int64_t capacity_leaves, int32_t max_members, dgamr_pool **out)
{
    GUARD_API({
        CHECK(check_ptr(cls, "cls"));
        CHECK(check_ptr(out, "out"));
        *out = nullptr;
        if (capacity_leaves <= 0 || capacity_leaves > (int64_t(1) << 28))
            return fail(DGAMR_EINVAL, "capacity_leaves must be in 1 .. 2^28");
        if (max_members <= 0 || max_members > (1 << 20)) return fail(DGAMR_EINVAL, "max_members must be in 1 .. 2^20");
        // validate the class with a one-root forest of it
        dgamr_forest_desc d = *cls;
        for (int a = 0; a < 3; ++a) {
            d.roots[a] = 1;
            d.lo[a] = 0.0;
            d.hi[a] = 1.0;
            d.bc[a] = DGAMR_BC_PERIODIC;
        }
        d.max_level = 1;
        std::string err;
        int rc = dgamr::Forest::validate(d, err);
        if (rc != DGAMR_OK) return fail(rc, err);
        if (cls->equation != DGAMR_EQ_EULER) return fail(DGAMR_EUNSUPPORTED, "pools hold Euler forests");
        auto *p = new dgamr_pool;
        p->cls = *cls;
        p->dim = cls->dim;
        p->degree = cls->degree;
        p->N = cls->n_cell;
        p->nb = dgk::num_modes(cls->dim, cls->degree);
        p->nv = cls->dim + 2;
        p->ncell = cls->dim == 2 ? p->N * p->N : p->N * p->N * p->N;
        p->nfc = cls->dim == 2 ? p->N : p->N * p->N;
        p->cap = capacity_leaves;
        // default stage kernel as for a single forest of the class: one lane
        // per (cell, variable) in 3-D at degree 3, one thread per cell else
        if (p->dim == 3 && p->degree >= 3 && lanes_class(p)) p->shape.variant = 0;
        p->maxm = max_members;
        p->used.assign(size_t(capacity_leaves), 0);
        auto cleanup = [&](int code, const char *what) {
            dgamr_pool_destroy(p);
            return fail(code, what);
        };
        if (hipGetDevice(&p->device) != hipSuccess) return cleanup(DGAMR_EHIP, "hipGetDevice failed");
        const size_t nl = size_t(capacity_leaves), nf = nl * 2 * cls->dim;
        if (hipMalloc(&p->d_geo, sizeof(LeafGeo) * nl) != hipSuccess ||
            hipMalloc(&p->d_links, sizeof(FaceLink) * nf) != hipSuccess ||
            hipMalloc(&p->d_member, sizeof(int) * nl) != hipSuccess ||
            hipMalloc(&p->d_work, sizeof(int) * nl) != hipSuccess ||
            hipMalloc(&p->d_members, sizeof(dgk::MemberDesc) * max_members) != hipSuccess)
            return cleanup(DGAMR_EHIP, "device table allocation failed");
        if (hipHostMalloc(&p->h_geo, sizeof(LeafGeo) * nl) != hipSuccess ||
            hipHostMalloc(&p->h_links, sizeof(FaceLink) * nf) != hipSuccess ||
            hipHostMalloc(&p->h_member, sizeof(int) * nl) != hipSuccess ||
            hipHostMalloc(&p->h_work, sizeof(int) * nl) != hipSuccess ||
            hipHostMalloc(&p->h_members, sizeof(dgk::MemberDesc) * max_members) != hipSuccess)
            return cleanup(DGAMR_EHIP, "pinned host table allocation failed");
        std::memset(p->h_members, 0, sizeof(dgk::MemberDesc) * max_members);
        if (hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming) != hipSuccess)
            return cleanup(DGAMR_EHIP, "event creation failed");
        if (hipMemcpy(p->d_members, p->h_members, sizeof(dgk::MemberDesc) * max_members, hipMemcpyHostToDevice) !=
            hipSuccess)
            return cleanup(DGAMR_EHIP, "member table upload failed");
        *out = p;
        return DGAMR_OK;
    })
}

int dgamr_pool_destroy(dgamr_pool *p)
{
    if (!p) return DGAMR_OK;
    if (p->uploaded) {
        (void)hipEventSynchronize(p->uploaded);
        (void)hipEventDestroy(p->uploaded);
    }
    (void)hipFree(p->d_geo);
    (void)hipFree(p->d_links);
    (void)hipFree(p->d_member);
    (void)hipFree(p->d_work);
    (void)hipFree(p->d_members);
    (void)hipHostFree(p->h_geo);
    (void)hipHostFree(p->h_links);
    (void)hipHostFree(p->h_member);
    (void)hipHostFree(p->h_work);
    (void)hipHostFree(p->h_members);
    delete p;
    return DGAMR_OK;
}

int dgamr_pool_bytes(const dgamr_pool *p, size_t *state_bytes, size_t *work_bytes)
{
    CHECK(check_ptr(p, "pool"));
    if (state_bytes) *state_bytes = sizeof(double) * leaf_elems(p) * p->cap;
    if (work_bytes) *work_bytes = sizeof(double) * pool_work_elems(p);
    return DGAMR_OK;
}

int dgamr_pool_admit(dgamr_pool *p, const dgamr_forest *f, double cfl, int32_t *member, int64_t *slot_first,
                     hipStream_t stream)
{
    GUARD_API({
        CHECK(check_ptr(p, "pool"));
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(member, "member"));
        CHECK(check_ptr(slot_first, "slot_first"));
        if (!same_class(p->cls, f->topo.desc())) return fail(DGAMR_EINVAL, "forest is not of the pool's class");
        if (f->topo.rotated()) return fail(DGAMR_EUNSUPPORTED, "pools hold forests whose roots share one frame");
        if (f->topo.mapped()) return fail(DGAMR_EUNSUPPORTED, "pools hold forests of box roots");
        if (!(cfl > 0.0)) return fail(DGAMR_EINVAL, "cfl must be positive");
        const int64_t n = f->topo.n();
        if (n == 0) return fail(DGAMR_EINVAL, "empty forest");
        int mid = -1;
        for (int m = 0; m < p->maxm; ++m)
            if (p->h_members[m].count == 0) {
                mid = m;
                break;
            }
        // first fit over the slot map
        int64_t first = -1, run = 0;
        for (int64_t i = 0; i < p->cap; ++i) {
            run = p->used[i] ? 0 : run + 1;
            if (run == n) {
                first = i - n + 1;
                break;
            }
        }
        if (mid < 0 || first < 0) return fail(DGAMR_EFULL, mid < 0 ? "no free member id" : "no free slot range");
        CHECK(wait_upload(p));
        const int nf = 2 * p->dim;
        std::vector<LeafGeo> geo = f->topo.geometry();
        const auto &links = f->topo.links();
        for (int64_t i = 0; i < n; ++i) {
            p->h_geo[first + i] = geo[i];
            p->h_member[first + i] = mid;
            p->used[first + i] = 1;
            for (int k = 0; k < nf; ++k) {
                FaceLink L = links[size_t(i) * nf + k];
                for (int q = 0; q < 4; ++q)
                    if (L.nbr[q] >= 0) L.nbr[q] += int(first);
                p->h_links[size_t(first + i) * nf + k] = L;
            }
        }
        p->h_members[mid] = dgk::MemberDesc{int(first), int(n), cfl};
        HIP_TRY(hipMemcpyAsync(p->d_geo + first, p->h_geo + first, sizeof(LeafGeo) * n, hipMemcpyHostToDevice,
                               stream));
        HIP_TRY(hipMemcpyAsync(p->d_links + first * nf, p->h_links + first * nf, sizeof(FaceLink) * n * nf,
                               hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(p->d_member + first, p->h_member + first, sizeof(int) * n, hipMemcpyHostToDevice,
                               stream));
        CHECK(upload_lists(p, stream));
        p->active += 1;
        p->version += 1;
        *member = mid;
        *slot_first = first;
        return DGAMR_OK;
    })
}

int dgamr_pool_release(dgamr_pool *p, int32_t member, hipStream_t stream)
{
    GUARD_API({
        CHECK(check_ptr(p, "pool"));
        if (member < 0 || member >= p->maxm || p->h_members[member].count == 0)
            return fail(DGAMR_EINVAL, "not an active member");
        CHECK(wait_upload(p));
        const dgk::MemberDesc M = p->h_members[member];
        for (int64_t i = 0; i < M.count; ++i) p->used[M.first + i] = 0;
        p->h_members[member] = dgk::MemberDesc{0, 0, 0.0};
        CHECK(upload_lists(p, stream));
        p->active -= 1;
        p->version += 1;
        return DGAMR_OK;
    })
}

int dgamr_pool_step(dgamr_pool *p, double *u_arena, void *work, hipStream_t stream)
{
    CHECK(check_ptr(p, "pool"));
    CHECK(check_ptr(u_arena, "u_arena"));
    CHECK(check_ptr(work, "work"));
    return pool_step(p, u_arena, work, stream);
}

int dgamr_pool_dt(const dgamr_pool *p, void *work, double **dt_dev)
{
    CHECK(check_ptr(p, "pool"));
    CHECK(check_ptr(work, "work"));
    CHECK(check_ptr(dt_dev, "dt_dev"));
    *dt_dev = carve(p, work).dt;
    return DGAMR_OK;
}

int dgamr_pool_stats(const dgamr_pool *p, int64_t *leaves_used, int32_t *members)
{
    CHECK(check_ptr(p, "pool"));
    if (leaves_used) *leaves_used = p->nwork;
    if (members) *members = p->active;
    return DGAMR_OK;
}

int dgamr_pool_set_shape(dgamr_pool *p, int32_t rows, int32_t grid)
{
    CHECK(check_ptr(p, "pool"));
    if (rows < 0 || grid < 0) return fail(DGAMR_EINVAL, "rows and grid must be >= 0");
    if (rows > 0) {
        int opts[16];
        int n = dispatch(p->dim, p->degree, [&](auto D, auto P) -> int {
            return dgk::stage_rows_options<D, P>(p->N, opts, 16, p->cls.precision == DGAMR_FP32);
        });
        if (std::find(opts, opts + n, rows) == opts + n) return fail(DGAMR_EINVAL, "rows not allowed for this class");
    }
    p->shape.variant = 1; // the thread-per-cell kernel
    p->shape.rows = rows;
    p->shape.grid = grid;
    return DGAMR_OK;
}

int dgamr_pool_set_lanes(dgamr_pool *p, int32_t rows)
{
    CHECK(check_ptr(p, "pool"));
    if (!lanes_class(p)) return fail(DGAMR_EINVAL, "the lane kernel takes FP64 classes without the limiter (3-D: without mortar faces)");
    if (rows < 0 || (rows > 0 && !lanes_rows_ok(p, rows))) return fail(DGAMR_EINVAL, "rows not allowed for the lane kernel");
    p->shape.variant = 0;
    p->shape.rows = rows;
    p->shape.grid = 0;
    return DGAMR_OK;
}

int dgamr_pool_autotune(dgamr_pool *p, double *u_arena, void *work, hipStream_t stream, int32_t *variant,
                        int32_t *rows, int32_t *grid, double *best_us)
{
    GUARD_API({
        CHECK(check_ptr(p, "pool"));
        CHECK(check_ptr(u_arena, "u_arena"));
        CHECK(check_ptr(work, "work"));
        if (p->nwork == 0) return fail(DGAMR_ESTATE, "pool has no members to tune on");
        int opts[16];
        const int nopt = dispatch(p->dim, p->degree, [&](auto D, auto P) -> int {
            return dgk::stage_rows_options<D, P>(p->N, opts, 16, p->cls.precision == DGAMR_FP32);
        });
        // FP64 without the limiter (3-D: and without mortar faces) also has
        // the lane-per-(cell, variable) kernel: 2-D slabs of r rows with
        // 4 r N <= 512 lanes, 3-D slabs of r layers as rows_ok_3v allows
        const bool try_lanes = lanes_class(p);
        PoolWork w = carve(p, work);
        CHECK(pool_dt(p, u_arena, w, stream));
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        double best = 1e300;
        dgk::StageShape best_sh = p->shape;
        const int reps = 3;
        int rc = DGAMR_OK;
        // candidates: the thread-per-cell kernel at every allowed slab
        // height, one workgroup per item or a persistent grid of 1, 2 or 4
        // workgroups per compute unit; the lane-per-variable kernel at every
        // slab height it allows
        struct Cand { int variant, rows, grid; };
        std::vector<Cand> cands;
        for (int oi = 0; oi < nopt; ++oi) {
            const long items = long(p->nwork) * (p->N / opts[oi]);
            for (int gsz : {0, 256, 512, 1024})
                if (gsz == 0 || gsz < items) cands.push_back({1, opts[oi], gsz});
        }
        if (try_lanes)
            for (int r = p->N; r >= 1; --r)
                if (lanes_rows_ok(p, r)) cands.push_back({0, r, 0});
        for (size_t ci = 0; ci < cands.size() && rc == DGAMR_OK; ++ci) {
            {
                dgk::StageShape sh;
                sh.variant = cands[ci].variant;
                sh.rows = cands[ci].rows;
                sh.grid = cands[ci].grid;
                rc = pool_stage(p, 0, u_arena, u_arena, w.u1, w, sh, stream); // warm-up
                if (rc != DGAMR_OK) break;
                if (hipEventRecord(e0, stream) != hipSuccess) { rc = fail(DGAMR_EHIP, "event record"); break; }
                for (int r = 0; r < reps && rc == DGAMR_OK; ++r)
                    rc = pool_stage(p, 0, u_arena, u_arena, w.u1, w, sh, stream);
                if (rc != DGAMR_OK) break;
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(DGAMR_EHIP, "event record");
                    break;
                }
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = fail(DGAMR_EHIP, "event time"); break; }
                const double us = 1e3 * ms / reps;
                if (us < best) {
                    best = us;
                    best_sh = sh;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != DGAMR_OK) return rc;
        p->shape = best_sh;
        if (variant) *variant = best_sh.variant;
        if (rows) *rows = best_sh.rows;
        if (grid) *grid = best_sh.grid;
        if (best_us) *best_us = best;
        return DGAMR_OK;
    })
}

int dgamr_pools_capture(dgamr_pool *const *pools, double *const *u_arenas, void *const *works, int32_t npools,
                        int32_t nsteps, dgamr_graph **out)
{
    GUARD_API({
        CHECK(check_ptr(pools, "pools"));
        CHECK(check_ptr(u_arenas, "u_arenas"));
        CHECK(check_ptr(works, "works"));
        CHECK(check_ptr(out, "out"));
        *out = nullptr;
        if (npools <= 0 || nsteps <= 0) return fail(DGAMR_EINVAL, "npools and nsteps must be positive");
        for (int i = 0; i < npools; ++i) {
            CHECK(check_ptr(pools[i], "pool"));
            CHECK(check_ptr(u_arenas[i], "u_arena"));
            CHECK(check_ptr(works[i], "work"));
            CHECK(wait_upload(pools[i]));
        }
        // One branch per pool: the pools share no memory, so their steps
        // run concurrently; each branch keeps its pool's steps in order.  The
        // branches fork from and join into the capturing stream through
        // events (no event nodes are left in the graph).
        hipStream_t s;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        std::vector<hipStream_t> br(npools, nullptr);
        std::vector<hipEvent_t> ev(npools + 1, nullptr);
        int rc = DGAMR_OK;
        for (int i = 0; i < npools && rc == DGAMR_OK; ++i)
            if (hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) rc = fail(DGAMR_EHIP, "stream");
        for (int i = 0; i <= npools && rc == DGAMR_OK; ++i)
            if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) rc = fail(DGAMR_EHIP, "event");
        auto *g = new dgamr_graph;
        if (rc != DGAMR_OK) {
        } else if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(DGAMR_EHIP, "hipStreamBeginCapture failed");
        } else {
            if (hipEventRecord(ev[npools], s) != hipSuccess) rc = fail(DGAMR_EHIP, "fork event");
            for (int i = 0; i < npools && rc == DGAMR_OK; ++i) {
                if (hipStreamWaitEvent(br[i], ev[npools], 0) != hipSuccess) rc = fail(DGAMR_EHIP, "fork wait");
                for (int st = 0; st < nsteps && rc == DGAMR_OK; ++st)
                    rc = pool_step(pools[i], u_arenas[i], works[i], br[i]);
                if (rc == DGAMR_OK && hipEventRecord(ev[i], br[i]) != hipSuccess) rc = fail(DGAMR_EHIP, "join event");
                if (rc == DGAMR_OK && hipStreamWaitEvent(s, ev[i], 0) != hipSuccess) rc = fail(DGAMR_EHIP, "join wait");
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc == DGAMR_OK && e != hipSuccess) rc = fail(DGAMR_EHIP, "hipStreamEndCapture failed");
            g->graph = graph;
            if (rc == DGAMR_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(DGAMR_EHIP, "hipGraphInstantiate failed");
        }
        (void)hipStreamDestroy(s);
        for (auto b : br)
            if (b) (void)hipStreamDestroy(b);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        if (rc != DGAMR_OK) {
            dgamr_graph_destroy(g);
            return rc;
        }
        for (int i = 0; i < npools; ++i) g->versions.emplace_back(&pools[i]->version, pools[i]->version);
        *out = g;
        return DGAMR_OK;
    })
}

int dgamr_graph_launch(dgamr_graph *g, hipStream_t stream)
{
    CHECK(check_ptr(g, "graph"));
    for (const auto &pv : g->versions)
        if (*pv.first != pv.second) return fail(DGAMR_ESTATE, "a forest or pool changed since the graph was captured");
    HIP_TRY(hipGraphLaunch(g->exec, stream));
    return DGAMR_OK;
}

int dgamr_graph_destroy(dgamr_graph *g)
{
    delete g;
    return DGAMR_OK;
}

} // extern "C"
