// sun_ops.hpp -- host-side launchers, one table per (Nc, storage type).
// Each ops_nc*.hip translation unit instantiates the kernels of one Nc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sun_device.hpp"

namespace sun {

// Launch shape of a phase kernel.
struct Shape {
    int block = 256;  // work-items per workgroup (64, 128 or 256)
    int xcd = 1;      // XCD-aware workgroup order
    int waves = 0;    // resident waves per CU (0 = no cap)
    int tblock = 0;   // time slices per block of the tile walk (0: linear)
    int spt = 1;      // sites per work-item (1, 2 or 4): tiles a workgroup takes in turn
};
inline bool valid_spt(int s) { return s == 1 || s == 2 || s == 4; }
inline int grid_for(int nblk, int spt) { return (nblk + spt - 1) / spt; }

// The walk of a single lattice's phase for a shape; falls back to the linear
// walk where the t-blocked one is not a permutation of the tiles.
inline Walk walk_for(const Geom& g, const Shape& sh) {
    Walk w{sh.xcd, 0, 1, 1, 0, sh.spt};
    const long long plane_h = (long long)g.L[0] * g.L[1] / 2;
    if (sh.tblock > 1 && plane_h % sh.block == 0 && g.L[3] % sh.tblock == 0) {
        w.tb = sh.tblock;
        w.tpp = (int)(plane_h / sh.block);
        w.lz = g.L[2];
    }
    return w;
}
inline bool valid_tblock(int t) { return t == 0 || t == 1 || t == 2 || t == 4 || t == 8; }

struct Ctx {
    void* links;
    Geom g;
    hipStream_t stream;
    Shape shape[2];   // per update kind: heatbath, overrelaxation
    int nc;
    int nt;           // nontemporal access to updated links (field well above the Infinity Cache)
    int rev;          // this phase walks its tiles in reverse order
    uint64_t order = 0;  // nonzero: a random tile order drawn from this value (race check)
};

// The affine permutation q -> (pa q + pc) mod n of a random tile order,
// drawn from `order` (splitmix64 steps); pa is coprime to n.
inline void random_tile_order(uint64_t order, int n, Walk& w) {
    auto mix = [](uint64_t& x) {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto gcd = [](uint64_t a, uint64_t b) {
        while (b) {
            const uint64_t t = a % b;
            a = b;
            b = t;
        }
        return a;
    };
    if (n <= 1) return;
    uint64_t x = order;
    uint64_t a = 1 + mix(x) % (uint64_t)(n - 1);
    while (gcd(a, (uint64_t)n) != 1) a = a % (uint64_t)(n - 1) + 1;
    w.pa = (uint32_t)a;
    w.pc = (uint32_t)(mix(x) % (uint64_t)n);
}

// Infinity Cache (MALL) of an MI355X is 256 MB.  Updated links keep plain
// (cached) access up to 1.25 x that size: measured on 32^4 SU(3), a 302 MB
// field ran 3.6% faster with plain access, 402 and 604 MB fields 1-2% faster
// with nontemporal access (with alternating walk directions).
constexpr size_t kPlainAccessMaxBytes = 320ull << 20;

// Dynamic LDS per workgroup that limits a CU to `waves` resident waves of
// `block`-item workgroups (0 = no cap).  LDS per CU: 160 KiB on gfx950; the
// size is kLdsPerCu / (blocks + 1/2) rounded down to 512 bytes, so that
// `blocks` workgroups fit with room to spare and one more does not.
constexpr int kLdsPerCu = 160 * 1024;
inline int lds_for_wave_cap(int waves, int block) {
    if (waves <= 0) return 0;
    const int per_block = block / 64;
    const int blocks = waves / per_block < 1 ? 1 : waves / per_block;
    return (int)(2.0 * kLdsPerCu / (2 * blocks + 1)) & ~511;
}
inline bool valid_wave_cap(int w) { return w == 0 || w == 8 || w == 12 || w == 16; }

// The plaquette kernel re-reads each link from up to six sites; with its
// register use alone a CU holds 16 of its waves, and their combined working
// set can thrash the L2.  The best cap depends on whether the field stays in
// the Infinity Cache (measured on SU(3) 32^4): the 201 MB two-row FP32 field
// runs best uncapped at 16 waves per CU (8 / 12 / 16: 115.7 / 107.3 /
// 104.6 us), the 302 MB 18-real field at 8 (150 / 152 / 165.5 us), and the
// 604 MB FP64 field at 12 (358 us against 369 uncapped).
constexpr size_t kInfinityCacheBytes = 256ull << 20;
inline int plaquette_wave_cap(size_t field_bytes) {
    if (field_bytes <= kInfinityCacheBytes) return 16;
    if (field_bytes <= kPlainAccessMaxBytes) return 8;
    return 12;
}

// Launch shapes the phase kernels are instantiated for.
constexpr int kPhaseBlocks[3] = {64, 128, 256};
inline bool valid_phase_block(int b) { return b == 64 || b == 128 || b == 256; }

struct Ops {
    // one checkerboard phase; kind 0 heatbath, 1 overrelaxation
    void (*update)(const Ctx&, int kind, int mu, int par, double beta, uint32_t k0, uint32_t k1, uint32_t step);
    void (*init)(const Ctx&, int hot, uint32_t k0, uint32_t k1);
    // reductions write 2 doubles per workgroup into partial and return the
    // workgroup count (reunit: partial may be null, then nothing is reported)
    int (*reunit)(const Ctx&, double* partial);
    int (*unitarity)(const Ctx&, double* partial);
    int (*plaquette)(const Ctx&, double* partial);
    // partial: 2 doubles per block; returns the block count
    int (*polyakov)(const Ctx&, double* partial);
    void (*export_field)(const Ctx&, double* out);
    void (*import_field)(const Ctx&, const double* in);
    // batches: d is a device table of n chains of this Nc (nc) and storage
    // type; tiles is the total tile count of the grid kind the call uses (on
    // the workgroup-per-link path: links, sites or links, one workgroup each)
    void (*update_batch)(const ChainDesc* d, int n, int tiles, int kind, int mu, int par, uint32_t step_offset,
                         const Shape& shape, int nc, hipStream_t s);
    void (*reunit_batch)(const ChainDesc* d, int n, int tiles, int nc, hipStream_t s);
    void (*plaquette_batch)(const ChainDesc* d, int n, int tiles, double* out, int nc, hipStream_t s);
};

constexpr int kLaunchBlock = 256;
inline int blocks_for(long long n) { return (int)((n + kLaunchBlock - 1) / kLaunchBlock); }
inline int link_blocks(const Geom& g) { return blocks_for(4LL * g.V); }
inline int half_blocks(const Geom& g) { return blocks_for(g.Vh); }
inline int half_blocks(const Geom& g, int bs) { return (g.Vh + bs - 1) / bs; }
inline int spatial_blocks(const Geom& g) { return blocks_for(g.V / g.L[3]); }

// f64 = 0: float storage, 1: double storage
const Ops* ops_nc2(int f64);
const Ops* ops_nc3(int f64);
const Ops* ops_nc4(int f64);
const Ops* ops_nc3_two_row(int f64);  // SU(3), rows 0 and 1 stored
const Ops* ops_wide(int f64);         // 4 <= Nc <= 32: one workgroup per link, link-major storage

// Dynamic LDS of the wide phase kernel, and whether it fits a workgroup.  The
// kernel keeps three Nc x Nc matrices in LDS, or two with the staple sum in
// registers; the latter where three would leave fewer than 8 workgroups per
// CU (FP32 from Nc = 30, FP64 from Nc = 21), since a phase at 8^4 is 2048
// workgroups and fewer than 8 per CU take it two or more rounds.
constexpr size_t kWideLdsMax = 64 * 1024;
inline bool wide_update_regacc(int nc, int f64) { return (size_t)3 * nc * nc * (f64 ? 16 : 8) > kLdsPerCu / 8; }
// Threads of a large-Nc update workgroup: two wavefronts (the loads and
// vector-unit products shared, the subgroup steps on the first, and the
// heatbath draws on the second where wide_handoff allows) where that
// measured faster on 8^4
// -- FP32 from Nc = 9 (5-9% per iteration up to Nc = 20; above, where the
// matrix-core products stay on the first wavefront and only the loads are
// shared, 2% -- the overrelaxation 6%; below Nc = 9 the second wavefront
// costs more than it saves), and FP64 where a phase takes two rounds anyway
// (two matrices of more than 10 KB, Nc >= 26; SU(32) 25.3 -> 20.8 ms) --
// one otherwise.
inline int wide_update_threads(int nc, int f64) {
    if (!f64) return nc >= 9 ? 128 : 64;
    return (size_t)2 * nc * nc * 16 > kLdsPerCu / 8 ? 128 : 64;
}
inline size_t wide_update_lds(int nc, int f64) {
    return (size_t)(wide_update_regacc(nc, f64) ? 2 : 3) * nc * nc * (f64 ? 16 : 8);
}
// Whether the second of two wavefronts draws the heatbath batches for the
// first (through a ring of ring_bytes in LDS): always in FP64, whose draws
// (FP64 logarithms and cosines) are costly; in FP32 where the ring still
// leaves the 8 workgroups per CU a phase at 8^4 needs for one round (the
// chain gains 2-4% from Nc = 9 to 24 and at 32; at Nc = 28 the ring would
// cost the second round: 5.6 -> 7.8 ms).
inline bool wide_handoff(int nc, int f64, size_t ring_bytes) {
    return f64 || wide_update_lds(nc, f64) + ring_bytes <= (size_t)kLdsPerCu / 8;
}

void launch_finalize_max2(const double* partial, int nblk, double* out, hipStream_t s);
void launch_finalize_sum2(const double* partial, int nblk, double* out, double scale, hipStream_t s);
void launch_plaquette_final(const double* partial, int nblk, double* out, double norm_sp, double norm_tm,
                            double norm_all, hipStream_t s);
void launch_advance_steps(ChainDesc* d, int n, int n_hb, hipStream_t s);
void launch_sample_su2(int f64, const double* alpha, int n, uint32_t k0, uint32_t k1, uint32_t step,
                       uint32_t mu_sg, double* x, int* attempts, hipStream_t s);
// the large-Nc path's batched draw (element i: subgroup mu_sg + i mod 8 of site i / 8)
void launch_sample_su2_batched(int f64, const double* alpha, int n, uint32_t k0, uint32_t k1, uint32_t step,
                               uint32_t mu_sg, double* x, int* attempts, hipStream_t s);

}  // namespace sun
