// dgamr_step_static: one SSP-RK3 step whose work area is a library-owned
// static device array, for callers that cannot allocate device memory.
// See include/dgamr.h.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_internal.hpp"

using namespace dgapi;

namespace {

// The work area: stage states U1 and U2, guard traces, leaf maxima and
// scalars, laid out as in the caller-owned work buffer of dgamr_step.  One
// copy per GPU, held until the process ends.
constexpr size_t kStaticWorkBytes = size_t(DGAMR_STATIC_WORK_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

// Device address of `scratch` per device, taken once per device with that
// device current.  In host code the name `scratch` is a host-side stand-in,
// never a device address; only these pointers reach kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_dev[kMaxDevices] = {};

int scratch_on(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(DGAMR_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[device]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != device) return fail(DGAMR_EINVAL, "the forest's device is not the current device");
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(DGAMR_EHIP, "hipGetSymbolAddress returned a null address");
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return DGAMR_OK;
}

} // namespace

extern "C" {

int dgamr_step_static(dgamr_forest *f, double cfl, double *u, double *dt_dev, hipStream_t stream)
{
    GUARD_API({
        CHECK(check_ptr(f, "forest"));
        CHECK(check_ptr(u, "u"));
        CHECK(check_ptr(dt_dev, "dt_dev"));
        const size_t need = work_bytes_of(f);
        if (need > kStaticWorkBytes)
            return fail(DGAMR_EUNSUPPORTED, "dgamr_step_static: the forest needs " + std::to_string(need) +
                                                " bytes of work area, more than the static " +
                                                std::to_string(kStaticWorkBytes) + " (use dgamr_step)");
        void *work = nullptr;
        CHECK(scratch_on(f->device, &work));
        return step_in_work(f, cfl, u, work, dt_dev, stream);
    })
}

} // extern "C"
