// ops_wide.hip -- launchers of the large-Nc kernels (one workgroup per link;
// Nc is a run-time argument, the LDS size follows it).
#include "sun_ops.hpp"
#include "sun_wide.hpp"

namespace sun {

template <typename T>
struct OpsWide {
    using P = T2<T>;
    static constexpr int f64 = sizeof(T) == 8;

    // Subgroup steps per slot (the same bits either way): the matrix-core and
    // register-accumulator forms exist only above Nc = 20, so only with four.
    template <bool MM, bool RA>
    static bool four_per_slot(int nc) {
        return MM || RA || wide::slot_steps(nc) == 4;
    }
    // The second of two wavefronts draws the heatbath batches where the ring
    // it hands them over in keeps the workgroups a CU holds (wide_handoff).
    template <int NT>
    static bool hand_off(int nc) {
        return NT > wide::kLanes && wide_handoff(nc, f64, wide::batch_ring_bytes<T>());
    }
    template <bool MM, bool RA, int NT>
    static void update_as(const Ctx& c, int kind, int mu, int par, double beta, uint32_t k0, uint32_t k1,
                          uint32_t step) {
        const bool ho = hand_off<NT>(c.nc);
        const size_t lds = wide_update_lds(c.nc, f64) + wide::handoff_lds<T>(ho);
        const int hb = kind == 0 ? 1 : 0;
        if (four_per_slot<MM, RA>(c.nc))
            wide::k_update<T, MM, RA, NT, 4><<<c.g.Vh, NT, lds, c.stream>>>((P*)c.links, c.g, c.nc, mu, par, hb,
                                                                            (T)beta, k0, k1, step, ho);
        else if constexpr (!MM && !RA)
            wide::k_update<T, MM, RA, NT, 2><<<c.g.Vh, NT, lds, c.stream>>>((P*)c.links, c.g, c.nc, mu, par, hb,
                                                                            (T)beta, k0, k1, step, ho);
    }
    // Threads per workgroup: a launch shape's block of 64 or 128 asks for one
    // or two wavefronts; any other block (the default 256) takes
    // wide_update_threads.  In the matrix-core form the second wavefront
    // shares the loads only: the products run on the first.
    static bool two_waves(const Shape& sh, int nc) {
        if (sh.block == wide::kLanes || sh.block == 2 * wide::kLanes) return sh.block > wide::kLanes;
        return wide_update_threads(nc, f64) > wide::kLanes;
    }
    static void update(const Ctx& c, int kind, int mu, int par, double beta, uint32_t k0, uint32_t k1, uint32_t step) {
        const bool ra = wide_update_regacc(c.nc, f64);
        const bool two = two_waves(c.shape[kind], c.nc);
        if constexpr (!f64) {
            if (c.nc > wide::kMfmaMinN) {
                if (ra) {
                    if (two)
                        update_as<true, true, 2 * wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
                    else
                        update_as<true, true, wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
                } else {
                    if (two)
                        update_as<true, false, 2 * wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
                    else
                        update_as<true, false, wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
                }
                return;
            }
        }
        if (ra) {
            if (two)
                update_as<false, true, 2 * wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
            else
                update_as<false, true, wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
        } else {
            if (two)
                update_as<false, false, 2 * wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
            else
                update_as<false, false, wide::kLanes>(c, kind, mu, par, beta, k0, k1, step);
        }
    }
    static void init(const Ctx& c, int hot, uint32_t k0, uint32_t k1) {
        wide::k_init<T><<<4 * c.g.V, wide::kLanes, wide::fp64_lds(c.nc, 2), c.stream>>>((P*)c.links, c.g, c.nc, hot, k0,
                                                                                        k1);
    }
    static int reunit(const Ctx& c, double* partial) {
        const size_t lds = wide::fp64_lds(c.nc, 1) + (size_t)c.nc * sizeof(double2);  // M and the projections
        if (partial)
            wide::k_reunit<T, true><<<4 * c.g.V, wide::kLanes, lds, c.stream>>>((P*)c.links, c.g, c.nc, partial);
        else
            wide::k_reunit<T, false><<<4 * c.g.V, wide::kLanes, lds, c.stream>>>((P*)c.links, c.g, c.nc, nullptr);
        return 4 * c.g.V;
    }
    static int unitarity(const Ctx& c, double* partial) {
        wide::k_unitarity<T><<<4 * c.g.V, wide::kLanes, wide::fp64_lds(c.nc, 1), c.stream>>>((const P*)c.links, c.g,
                                                                                             c.nc, partial);
        return 4 * c.g.V;
    }
    static int plaquette(const Ctx& c, double* partial) {
        wide::k_plaquette<T><<<c.g.V, wide::kLanes, wide::fp64_lds(c.nc, 3), c.stream>>>((const P*)c.links, c.g, c.nc,
                                                                                         partial);
        return c.g.V;
    }
    static int polyakov(const Ctx& c, double* partial) {
        const int Vs = c.g.V / c.g.L[3];
        wide::k_polyakov<T><<<Vs, wide::kLanes, wide::fp64_lds(c.nc, 3), c.stream>>>((const P*)c.links, c.g, c.nc,
                                                                                     partial);
        return Vs;
    }
    static int entry_blocks(const Ctx& c) {
        return (int)((4LL * c.g.V * c.nc * c.nc + 255) / 256);
    }
    static void export_field(const Ctx& c, double* out) {
        wide::k_export<T><<<entry_blocks(c), 256, 0, c.stream>>>((const P*)c.links, c.g, c.nc, out);
    }
    static void import_field(const Ctx& c, const double* in) {
        wide::k_import<T><<<entry_blocks(c), 256, 0, c.stream>>>((P*)c.links, c.g, c.nc, in);
    }

    // Batches: one launch per phase covers every chain of the group (same
    // Nc and precision), one workgroup per link.
    template <bool MM, bool RA, int NT>
    static void update_batch_as(const ChainDesc* d, int n, int tiles, int kind, int mu, int par, uint32_t off, int nc,
                                hipStream_t s) {
        const bool ho = hand_off<NT>(nc);
        const size_t lds = wide_update_lds(nc, f64) + wide::handoff_lds<T>(ho);
        const int hb = kind == 0 ? 1 : 0;
        if (four_per_slot<MM, RA>(nc))
            wide::k_update_batch<T, MM, RA, NT, 4><<<tiles, NT, lds, s>>>(d, n, nc, mu, par, hb, off, ho);
        else if constexpr (!MM && !RA)
            wide::k_update_batch<T, MM, RA, NT, 2><<<tiles, NT, lds, s>>>(d, n, nc, mu, par, hb, off, ho);
    }
    static void update_batch(const ChainDesc* d, int n, int tiles, int kind, int mu, int par, uint32_t off,
                             const Shape& shape, int nc, hipStream_t s) {
        const bool ra = wide_update_regacc(nc, f64);
        const bool two = two_waves(shape, nc);
        if constexpr (!f64) {
            if (nc > wide::kMfmaMinN) {
                if (ra) {
                    if (two)
                        update_batch_as<true, true, 2 * wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
                    else
                        update_batch_as<true, true, wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
                } else {
                    if (two)
                        update_batch_as<true, false, 2 * wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
                    else
                        update_batch_as<true, false, wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
                }
                return;
            }
        }
        if (ra) {
            if (two)
                update_batch_as<false, true, 2 * wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
            else
                update_batch_as<false, true, wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
        } else {
            if (two)
                update_batch_as<false, false, 2 * wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
            else
                update_batch_as<false, false, wide::kLanes>(d, n, tiles, kind, mu, par, off, nc, s);
        }
    }
    static void reunit_batch(const ChainDesc* d, int n, int tiles, int nc, hipStream_t s) {
        wide::k_reunit_batch<T><<<tiles, wide::kLanes, wide::fp64_lds(nc, 1) + (size_t)nc * sizeof(double2), s>>>(
            d, n, nc);
    }
    static void plaquette_batch(const ChainDesc* d, int n, int tiles, double* out, int nc, hipStream_t s) {
        wide::k_plaquette_batch<T><<<tiles, wide::kLanes, wide::fp64_lds(nc, 3), s>>>(d, n, nc);
        wide::k_plaquette_final_batch_wide<><<<n, kBlock, 0, s>>>(d, n, nc, out);
    }

    static const Ops* table() {
        static const Ops ops = {&update, &init, &reunit, &unitarity, &plaquette, &polyakov, &export_field,
                                &import_field, &update_batch, &reunit_batch, &plaquette_batch};
        return &ops;
    }
};

const Ops* ops_wide(int f64) { return f64 ? OpsWide<double>::table() : OpsWide<float>::table(); }

void launch_sample_su2_batched(int f64, const double* alpha, int n, uint32_t k0, uint32_t k1, uint32_t step,
                               uint32_t mu_sg, double* x, int* attempts, hipStream_t s) {
    const int sites = (n + wide::kSgBatch - 1) / wide::kSgBatch;
    if (f64)
        wide::k_sample_su2_batched<double><<<sites, wide::kLanes, 0, s>>>(alpha, n, k0, k1, step, mu_sg, x, attempts);
    else
        wide::k_sample_su2_batched<float><<<sites, wide::kLanes, 0, s>>>(alpha, n, k0, k1, step, mu_sg, x, attempts);
}

}  // namespace sun
