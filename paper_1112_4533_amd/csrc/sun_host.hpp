// sun_host.hpp -- host-side helpers shared by the translation units of the C
// ABI: the thread's last error text, argument checks, the geometry of a
// lattice, the kernel table of an (Nc, storage) pair and the plaquette
// launch.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "sun.h"
#include "sun_ops.hpp"

namespace sun_host {

inline thread_local std::string last_error;

inline int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error = buf;
    return code;
}

inline int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return SUN_OK;
    return fail(SUN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Any launch error of the kernels just queued.
inline int launch_check(const char* what) { return hip_check(hipGetLastError(), what); }

inline hipStream_t as_stream(sun_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// dtype bit 0: FP64 storage; bit 1: SU(3) two-row storage; bit 2: the
// workgroup-per-link path (also taken by every Nc above the register path's).
inline int is_f64(int dtype) { return dtype & 1; }
inline int is_two_row(int dtype) { return (dtype >> 1) & 1; }
inline bool is_wide(int nc, int dtype) { return ((dtype >> 2) & 1) || nc > SUN_NC_MAX_REGISTER; }

inline const sun::Ops* ops_for(int nc, int dtype) {
    const int f64 = is_f64(dtype);
    if (is_wide(nc, dtype)) return sun::ops_wide(f64);
    if (is_two_row(dtype)) return nc == 3 ? sun::ops_nc3_two_row(f64) : nullptr;
    switch (nc) {
        case 2: return sun::ops_nc2(f64);
        case 3: return sun::ops_nc3(f64);
        case 4: return sun::ops_nc4(f64);
        default: return nullptr;
    }
}

inline int check_lattice(int nc, const int L[4], int dtype) {
    if (!L) return fail(SUN_EINVAL, "L is null");
    if (nc < 2 || nc > SUN_NC_MAX) return fail(SUN_EINVAL, "Nc = %d outside 2..%d", nc, SUN_NC_MAX);
    if (dtype < SUN_F32 || dtype > SUN_F64_WIDE) return fail(SUN_EINVAL, "dtype %d is not a SUN_F* code", dtype);
    if (is_two_row(dtype) && nc != 3) return fail(SUN_EUNSUP, "two-row storage exists for SU(3) only (Nc = %d)", nc);
    if (is_wide(nc, dtype)) {
        if (nc < 4) return fail(SUN_EUNSUP, "the workgroup-per-link path starts at Nc = 4 (Nc = %d)", nc);
        if (sun::wide_update_lds(nc, is_f64(dtype)) > sun::kWideLdsMax)
            return fail(SUN_EUNSUP, "Nc = %d in FP64 needs %zu bytes of LDS per workgroup (limit %zu)", nc,
                        sun::wide_update_lds(nc, 1), sun::kWideLdsMax);
    }
    if (L[0] < 2 || (L[0] & 1)) return fail(SUN_EINVAL, "L[0] = %d must be even and >= 2", L[0]);
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (!(L[mu] == 1 || (L[mu] >= 2 && !(L[mu] & 1))))
            return fail(SUN_EINVAL, "L[%d] = %d must be 1 or even >= 2 (checkerboard)", mu, L[mu]);
        V *= L[mu];
    }
    if (4 * V >= (1LL << 31)) return fail(SUN_EINVAL, "volume %lld too large (4V must fit in int32)", V);
    return SUN_OK;
}

inline sun::Geom make_geom(const int L[4]) {
    sun::Geom g{};
    int V = 1;
    g.present = 0;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.stride[mu] = V;
        V *= L[mu];
        if (L[mu] > 1) g.present |= 1 << mu;
    }
    g.V = V;
    g.Vh = V / 2;
    return g;
}

// The plaquette kernel and its final pass over partials in `partial`:
// {all planes, planes without direction 3, planes with it}.
inline void launch_plaquette(const sun::Ops* ops, const sun::Ctx& c, double* partial, double* dev_out3) {
    int n_sp = 0, n_tm = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu)
            if (((c.g.present >> mu) & 1) && ((c.g.present >> nu) & 1)) (nu == 3 ? n_tm : n_sp)++;
    const double norm = (double)c.nc * (double)c.g.V;
    const int nblk = ops->plaquette(c, partial);
    sun::launch_plaquette_final(partial, nblk, dev_out3, norm * n_sp, norm * n_tm, norm * (n_sp + n_tm), c.stream);
}

}  // namespace sun_host
