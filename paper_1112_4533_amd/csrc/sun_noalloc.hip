// sun_noalloc.hip -- the plaquette of a field in caller memory with no
// lattice handle and no allocation of any kind: the reduction partials live
// in a fixed device array of this library instead of a caller's scratch
// buffer.  For callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <mutex>

#include "sun.h"
#include "sun_host.hpp"

using namespace sun_host;

namespace {

// One copy per GPU, held until the process ends.  In host code the name is a
// host-side stand-in, not a device address: host code uses only the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = SUN_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
double* scratch_on[kMaxDevices] = {};
std::mutex scratch_mutex;

// The device address of `scratch` on the current device, looked up once per
// device (with that device current).
int device_scratch(double** out) {
    int dev = -1;
    if (int rc = hip_check(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SUN_EUNSUP, "device %d is beyond the %d devices this library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_on[dev]) {
        void* p = nullptr;
        if (int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
            return rc;
        scratch_on[dev] = static_cast<double*>(p);
    }
    *out = scratch_on[dev];
    return SUN_OK;
}

}  // namespace

extern "C" {

int sun_plaquette_static(int nc, const int L[4], int dtype, const void* links, double* dev_out3,
                         sun_stream_t stream) {
    if (int rc = check_lattice(nc, L, dtype)) return rc;
    if (!links) return fail(SUN_ESIZE, "links is null");
    if (!dev_out3) return fail(SUN_ESIZE, "dev_out3 is null");
    if ((uintptr_t)links & 255) return fail(SUN_EINVAL, "links must be 256-byte aligned");
    const sun::Geom g = make_geom(L);
    // the plaquette kernels write 2 doubles per workgroup: one per tile of
    // 256 sites and parity on the register path, one per site on the
    // workgroup-per-link path
    const size_t blocks = is_wide(nc, dtype) ? (size_t)g.V : (size_t)sun::plaquette_tiles(g);
    const size_t need = 2 * sizeof(double) * blocks;
    if (need > kStaticScratchBytes)
        return fail(SUN_ESIZE, "a %d-site lattice needs %zu bytes of partials, more than the %zu-byte static scratch",
                    g.V, need, kStaticScratchBytes);
    double* partial = nullptr;
    if (int rc = device_scratch(&partial)) return rc;
    const hipStream_t s = as_stream(stream);
    const sun::Ctx c{const_cast<void*>(links), g, s, {sun::Shape{}, sun::Shape{}}, nc, 0, 0};
    launch_plaquette(ops_for(nc, dtype), c, partial, dev_out3);
    return launch_check("plaquette (static scratch)");
}

}  // extern "C"
