// sun_ops_impl.hpp -- launcher bodies; included once per Nc by ops_nc*.hip.
#pragma once

#include "sun_kernels.hpp"
#include "sun_ops.hpp"

namespace sun {

template <int N, typename T, int R>
struct OpsImpl {
    using P = T2<T>;

    template <bool HB, int MU, int BS>
    static void update_bs(const Ctx& c, int par, T beta, uint32_t k0, uint32_t k1, uint32_t step, int lds,
                          const Walk& w) {
        P* u = (P*)c.links;
        const int nblk = half_blocks(c.g, BS), grid = grid_for(nblk, w.spt);
        Walk wk = w;
        if (c.order) random_tile_order(c.order, nblk, wk);
        if (c.nt)
            k_update<N, T, R, HB, MU, BS, true><<<grid, BS, lds, c.stream>>>(u, c.g, par, beta, k0, k1, step, wk, nblk);
        else
            k_update<N, T, R, HB, MU, BS, false><<<grid, BS, lds, c.stream>>>(u, c.g, par, beta, k0, k1, step, wk, nblk);
    }

    template <bool HB, int MU>
    static void update_mu(const Ctx& c, int par, T beta, uint32_t k0, uint32_t k1, uint32_t step) {
        const Shape& sh = c.shape[HB ? 0 : 1];
        const int lds = lds_for_wave_cap(sh.waves, sh.block);
        Walk w = walk_for(c.g, sh);
        w.rev = c.rev;
        switch (sh.block) {
            case 64: update_bs<HB, MU, 64>(c, par, beta, k0, k1, step, lds, w); break;
            case 128: update_bs<HB, MU, 128>(c, par, beta, k0, k1, step, lds, w); break;
            default: update_bs<HB, MU, 256>(c, par, beta, k0, k1, step, lds, w); break;
        }
    }

    template <bool HB, int BS>
    static void update_batch_bs(const ChainDesc* d, int n, int tiles, int mu, int par, uint32_t off, int xcd,
                                int spt, int lds, hipStream_t s) {
        const int grid = grid_for(tiles, spt);
        switch (mu) {
            case 0: k_update_batch<N, T, R, HB, 0, BS><<<grid, BS, lds, s>>>(d, n, par, off, xcd, tiles, spt); break;
            case 1: k_update_batch<N, T, R, HB, 1, BS><<<grid, BS, lds, s>>>(d, n, par, off, xcd, tiles, spt); break;
            case 2: k_update_batch<N, T, R, HB, 2, BS><<<grid, BS, lds, s>>>(d, n, par, off, xcd, tiles, spt); break;
            default: k_update_batch<N, T, R, HB, 3, BS><<<grid, BS, lds, s>>>(d, n, par, off, xcd, tiles, spt); break;
        }
    }

    template <bool HB>
    static void update_batch_kind(const ChainDesc* d, int n, int tiles, int mu, int par, uint32_t off,
                                  const Shape& sh, int lds, hipStream_t s) {
        switch (sh.block) {
            case 64: update_batch_bs<HB, 64>(d, n, tiles, mu, par, off, sh.xcd, sh.spt, lds, s); break;
            case 128: update_batch_bs<HB, 128>(d, n, tiles, mu, par, off, sh.xcd, sh.spt, lds, s); break;
            default: update_batch_bs<HB, 256>(d, n, tiles, mu, par, off, sh.xcd, sh.spt, lds, s); break;
        }
    }

    static void update_batch(const ChainDesc* d, int n, int tiles, int kind, int mu, int par, uint32_t off,
                             const Shape& sh, int /*nc*/, hipStream_t s) {
        const int lds = lds_for_wave_cap(sh.waves, sh.block);
        if (kind == 0)
            update_batch_kind<true>(d, n, tiles, mu, par, off, sh, lds, s);
        else
            update_batch_kind<false>(d, n, tiles, mu, par, off, sh, lds, s);
    }

    static void reunit_batch(const ChainDesc* d, int n, int tiles, int /*nc*/, hipStream_t s) {
        k_reunit_batch<N, T, R><<<tiles, kBlock, 0, s>>>(d, n);
    }

    static void plaquette_batch(const ChainDesc* d, int n, int tiles, double* out, int /*nc*/, hipStream_t s) {
        // the chains of a batch are small, cache-resident lattices
        k_plaquette_batch<N, T, R><<<tiles, kBlock, lds_for_wave_cap(plaquette_wave_cap(0), kBlock), s>>>(d, n);
        k_plaquette_final_batch<N><<<n, kBlock, 0, s>>>(d, n, out);
    }

    template <bool HB>
    static void update_kind(const Ctx& c, int mu, int par, T beta, uint32_t k0, uint32_t k1, uint32_t step) {
        switch (mu) {
            case 0: update_mu<HB, 0>(c, par, beta, k0, k1, step); break;
            case 1: update_mu<HB, 1>(c, par, beta, k0, k1, step); break;
            case 2: update_mu<HB, 2>(c, par, beta, k0, k1, step); break;
            default: update_mu<HB, 3>(c, par, beta, k0, k1, step); break;
        }
    }

    static void update(const Ctx& c, int kind, int mu, int par, double beta, uint32_t k0, uint32_t k1,
                       uint32_t step) {
        if (kind == 0)
            update_kind<true>(c, mu, par, (T)beta, k0, k1, step);
        else
            update_kind<false>(c, mu, par, (T)beta, k0, k1, step);
    }

    static void init(const Ctx& c, int hot, uint32_t k0, uint32_t k1) {
        k_init<N, T, R><<<link_blocks(c.g), kBlock, 0, c.stream>>>((P*)c.links, c.g, hot, k0, k1);
    }
    static int reunit(const Ctx& c, double* partial) {
        if (partial)
            k_reunit<N, T, R, true><<<link_blocks(c.g), kBlock, 0, c.stream>>>((P*)c.links, c.g, partial, c.nt);
        else
            k_reunit<N, T, R, false><<<link_blocks(c.g), kBlock, 0, c.stream>>>((P*)c.links, c.g, nullptr, c.nt);
        return link_blocks(c.g);
    }
    static int unitarity(const Ctx& c, double* partial) {
        k_unitarity<N, T, R><<<link_blocks(c.g), kBlock, 0, c.stream>>>((const P*)c.links, c.g, partial);
        return link_blocks(c.g);
    }
    static int plaquette(const Ctx& c, double* partial) {
        const size_t field = sizeof(P) * (size_t)Planes<N, R>::E * 4 * (size_t)c.g.V;
        k_plaquette<N, T, R><<<plaquette_tiles(c.g), kBlock, lds_for_wave_cap(plaquette_wave_cap(field), kBlock),
                               c.stream>>>((const P*)c.links, c.g, partial);
        return plaquette_tiles(c.g);
    }
    static int polyakov(const Ctx& c, double* partial) {
        const int nblk = polyakov_blocks<N>(c.g);
        k_polyakov<N, T, R><<<nblk, kBlock, 0, c.stream>>>((const P*)c.links, c.g, partial);
        return nblk;
    }
    static void export_field(const Ctx& c, double* out) {
        k_export<N, T, R><<<link_blocks(c.g), kBlock, 0, c.stream>>>((const P*)c.links, c.g, out);
    }
    static void import_field(const Ctx& c, const double* in) {
        k_import<N, T, R><<<link_blocks(c.g), kBlock, 0, c.stream>>>((P*)c.links, c.g, in);
    }

    static const Ops* table() {
        static const Ops ops = {&update,       &init,         &reunit,       &unitarity,
                                &plaquette,    &polyakov,     &export_field, &import_field,
                                &update_batch, &reunit_batch, &plaquette_batch};
        return &ops;
    }
};

}  // namespace sun

#define SUN_DEFINE_OPS(NC)                                                     \
    namespace sun {                                                            \
    const Ops* ops_nc##NC(int f64) {                                           \
        return f64 ? OpsImpl<NC, double, NC>::table() : OpsImpl<NC, float, NC>::table(); \
    }                                                                          \
    }

// SU(3) with two stored rows (12 reals per link); row 2 = conj(row0 x row1).
#define SUN_DEFINE_OPS_TWO_ROW()                                                \
    namespace sun {                                                             \
    const Ops* ops_nc3_two_row(int f64) {                                       \
        return f64 ? OpsImpl<3, double, 2>::table() : OpsImpl<3, float, 2>::table(); \
    }                                                                           \
    }
