// sun_device.hpp -- device-side building blocks for the SU(Nc) sweep on
// gfx950: counter-based RNG, lattice geometry, the SoA link layout, and
// register-resident complex matrix / quaternion algebra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Loops over matrix indices are fully unrolled, so that register-array
// indices are compile-time constants (the register path runs Nc <= 4; larger
// Nc keeps its matrices in LDS, sun_wide.hpp).
#define SUN_MAT_UNROLL _Pragma("unroll")

namespace sun {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit multiplies, key bumped by the Weyl constants between rounds.
// Stateless: every draw is a pure function of (key, counter), so no generator
// state is read from or written to HBM.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t w[4];
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves in one instruction
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{{c0, c1, c2, c3}};
}

// 24-bit uniform in (0, 1]: exact in float and double, so both precisions see
// the same numbers.
template <typename T>
__device__ __forceinline__ T uniform(uint32_t w) {
    return T((w >> 8) + 1u) * T(5.9604644775390625e-08);  // 2^-24
}

// Purpose tags in the top byte of counter word 3.
enum : uint32_t { RNG_ATTEMPT = 0u, RNG_DIRECTION = 1u, RNG_HOTSTART = 2u };

// ---------------------------------------------------------------------------
// Geometry.  Logical site s = x + L0 (y + L1 (z + L2 t)); with L0 even,
// s and s^1 have opposite parity, so h = s >> 1 indexes the sites of one
// parity contiguously (the checkerboard index).
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];
    int stride[4];
    int V;
    int Vh;
    int present;  // bit mu set when L[mu] > 1
};

// One chain of a batch (device-resident table entry): its field, its own
// partials buffer, geometry, coupling, Philox key, RNG step counter, and the
// first tile it occupies in each batched grid.
struct ChainDesc {
    void* links;
    double* scratch;     // the chain's own partials buffer
    Geom g;
    double beta;
    uint32_t k0, k1;     // Philox key (seed)
    uint64_t step;       // RNG step counter
    int tile0[5];        // first tile of the chain in grids over V/2 (heatbath shape), V, 4V, Vs
                         // and V/2 (overrelaxation shape) items
    int out_index;       // position of the chain in the caller's list (result slots)
};

enum TileKind { TILE_HALF_HB = 0, TILE_SITE = 1, TILE_LINK = 2, TILE_SPATIAL = 3, TILE_HALF_OR = 4 };

struct Site {
    int x[4];
    int s;
};

// Site of checkerboard index h in the given parity.
__device__ __forceinline__ Site site_of(const Geom& g, int par, int h) {
    Site st;
    const int s0 = 2 * h;
    int r = s0 / g.L[0];
    const int x0 = s0 - r * g.L[0];
    const int q1 = r / g.L[1];
    st.x[1] = r - q1 * g.L[1];
    const int q2 = q1 / g.L[2];
    st.x[2] = q1 - q2 * g.L[2];
    st.x[3] = q2;
    const int fix = (st.x[1] + st.x[2] + st.x[3] + par) & 1;  // x0 is even
    st.x[0] = x0 + fix;
    st.s = s0 + fix;
    return st;
}

// Site shifted by +1 / -1 along nu (periodic).
__device__ __forceinline__ Site step_up(const Geom& g, Site a, int nu) {
    if (a.x[nu] == g.L[nu] - 1) {
        a.x[nu] = 0;
        a.s -= (g.L[nu] - 1) * g.stride[nu];
    } else {
        a.x[nu] += 1;
        a.s += g.stride[nu];
    }
    return a;
}

__device__ __forceinline__ Site step_down(const Geom& g, Site a, int nu) {
    if (a.x[nu] == 0) {
        a.x[nu] = g.L[nu] - 1;
        a.s += (g.L[nu] - 1) * g.stride[nu];
    } else {
        a.x[nu] -= 1;
        a.s -= g.stride[nu];
    }
    return a;
}

__device__ __forceinline__ int parity_of(const Site& a) {
    return (a.x[0] + a.x[1] + a.x[2] + a.x[3]) & 1;
}

// ---------------------------------------------------------------------------
// Workgroup -> tile mapping.  The dispatcher hands workgroups to the 8 XCDs
// round-robin (XCD = blockIdx % 8), each XCD with its own L2.  Giving each XCD
// one contiguous eighth of the tiles keeps the z-neighbour planes a phase
// re-reads (2 tiles apart at 32^4) in the same L2.  Bijective for any count.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    const int q = nblk / kXcds, r = nblk - q * kXcds;
    const int x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Order in which a phase walks its tiles.  With tb > 1 the tiles of one
// (z, t) plane (tpp of them) are taken for tb consecutive t first, then the
// next z, then the next block of tb time slices: the t-neighbour planes a
// phase re-reads are then 2 tiles apart instead of a whole time slice, so
// they are still in L2 when the neighbouring tile asks for them.  The host
// sets tb > 1 only where a plane holds a whole number of tiles and tb
// divides L_t, which makes the walk a permutation of the tiles.
struct Walk {
    int xcd;      // XCD-aware workgroup order
    int tb;       // time slices per block of the walk (0 or 1: linear walk)
    int tpp;      // tiles per (z, t) plane
    int lz;       // L_z
    int rev;      // walk the tiles in reverse order
    int spt = 1;  // tiles per workgroup (sites per work-item), taken in turn
    // Race check only: walk position q -> (pa q + pc) mod nblk, a random
    // permutation of the positions (pa coprime to nblk; 0: off).  Results
    // must not depend on which workgroup takes which tile, or when.
    uint32_t pa = 0, pc = 0;
};

// Tiles of the plaquette grid (256-item workgroups): both parities of every
// checkerboard tile.
__host__ __device__ __forceinline__ int plaquette_tiles(const Geom& g) { return 2 * ((g.Vh + 255) / 256); }

// Consecutive phases walk in opposite directions (rev): a phase then starts
// where the previous one ended, on the links most recently brought into the
// Infinity Cache, which matters once the field is larger than that cache.
__device__ __forceinline__ int walk_tile(int b, int nblk, const Walk& w) {
    const int q0 = w.xcd ? xcd_tile(b, nblk) : b;
    int q = w.rev ? nblk - 1 - q0 : q0;
    if (w.pa) q = (int)(((uint64_t)q * w.pa + w.pc) % (uint64_t)nblk);
    if (w.tb <= 1) return q;
    const int i = q % w.tpp;
    int rest = q / w.tpp;
    const int ti = rest % w.tb;
    rest /= w.tb;
    const int z = rest % w.lz;
    const int blk = rest / w.lz;
    return i + w.tpp * (z + w.lz * (blk * w.tb + ti));
}

// ---------------------------------------------------------------------------
// Register matrices.
// ---------------------------------------------------------------------------
template <int N, typename T>
struct Mat {
    T re[N][N];
    T im[N][N];
};

template <int N, typename T>
__device__ __forceinline__ void set_zero(Mat<N, T>& a) {
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) a.re[i][j] = a.im[i][j] = T(0);
}

template <int N, typename T>
__device__ __forceinline__ void set_identity(Mat<N, T>& a) {
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            a.re[i][j] = (i == j) ? T(1) : T(0);
            a.im[i][j] = T(0);
        }
}

// Fused multiply-add, one rounding.  The products below are written as
// chains of these so that a complex multiply-add costs four VALU operations.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// NaN -> +infinity, for maxima that must not lose a NaN (fmax returns the
// other operand).
__device__ __forceinline__ double nan_to_inf(double x) { return x == x ? x : __builtin_inf(); }

// (r, m) += (ar + i ai)(br + i bi)
template <typename T>
__device__ __forceinline__ void cmac(T& r, T& m, T ar, T ai, T br, T bi) {
    r = fmadd(ar, br, r);
    r = fmadd(-ai, bi, r);
    m = fmadd(ar, bi, m);
    m = fmadd(ai, br, m);
}

// c = a b
template <int N, typename T>
__device__ __forceinline__ Mat<N, T> mul_nn(const Mat<N, T>& a, const Mat<N, T>& b) {
    Mat<N, T> c;
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            T r = T(0), m = T(0);
SUN_MAT_UNROLL
            for (int k = 0; k < N; ++k) cmac(r, m, a.re[i][k], a.im[i][k], b.re[k][j], b.im[k][j]);
            c.re[i][j] = r;
            c.im[i][j] = m;
        }
    return c;
}

// c = a b^dag
template <int N, typename T>
__device__ __forceinline__ Mat<N, T> mul_nd(const Mat<N, T>& a, const Mat<N, T>& b) {
    Mat<N, T> c;
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            T r = T(0), m = T(0);
SUN_MAT_UNROLL
            for (int k = 0; k < N; ++k) cmac(r, m, a.re[i][k], a.im[i][k], b.re[j][k], -b.im[j][k]);
            c.re[i][j] = r;
            c.im[i][j] = m;
        }
    return c;
}

// acc += a^dag b
template <int N, typename T>
__device__ __forceinline__ void add_mul_dn(Mat<N, T>& acc, const Mat<N, T>& a, const Mat<N, T>& b) {
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            T r = acc.re[i][j], m = acc.im[i][j];
SUN_MAT_UNROLL
            for (int k = 0; k < N; ++k) cmac(r, m, a.re[k][i], -a.im[k][i], b.re[k][j], b.im[k][j]);
            acc.re[i][j] = r;
            acc.im[i][j] = m;
        }
}

// acc += a b^dag
template <int N, typename T>
__device__ __forceinline__ void add_mul_nd(Mat<N, T>& acc, const Mat<N, T>& a, const Mat<N, T>& b) {
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            T r = acc.re[i][j], m = acc.im[i][j];
SUN_MAT_UNROLL
            for (int k = 0; k < N; ++k) cmac(r, m, a.re[i][k], a.im[i][k], b.re[j][k], -b.im[j][k]);
            acc.re[i][j] = r;
            acc.im[i][j] = m;
        }
}

// Partial products for SU(3) staple terms (3x3; only the named rows or
// columns of the result are written).

// rows 0, 1 of a b^dag (reads rows 0, 1 of a)
template <typename T>
__device__ __forceinline__ Mat<3, T> mul_nd_rows2(const Mat<3, T>& a, const Mat<3, T>& b) {
    Mat<3, T> c;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T r = T(0), m = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(r, m, a.re[i][k], a.im[i][k], b.re[j][k], -b.im[j][k]);
            c.re[i][j] = r;
            c.im[i][j] = m;
        }
    return c;
}

// columns 0, 1 of a b (reads columns 0, 1 of b)
template <typename T>
__device__ __forceinline__ Mat<3, T> mul_nn_cols2(const Mat<3, T>& a, const Mat<3, T>& b) {
    Mat<3, T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            T r = T(0), m = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(r, m, a.re[i][k], a.im[i][k], b.re[k][j], b.im[k][j]);
            c.re[i][j] = r;
            c.im[i][j] = m;
        }
    return c;
}

// rows 0, 1 of a^dag b (reads columns 0, 1 of a)
template <typename T>
__device__ __forceinline__ Mat<3, T> mul_dn_rows2(const Mat<3, T>& a, const Mat<3, T>& b) {
    Mat<3, T> c;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T r = T(0), m = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(r, m, a.re[k][i], -a.im[k][i], b.re[k][j], b.im[k][j]);
            c.re[i][j] = r;
            c.im[i][j] = m;
        }
    return c;
}

template <int N, typename T>
__device__ __forceinline__ void add_to(Mat<N, T>& acc, const Mat<N, T>& a) {
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) {
            acc.re[i][j] += a.re[i][j];
            acc.im[i][j] += a.im[i][j];
        }
}

// ---------------------------------------------------------------------------
// Quaternions: q <-> [[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]]
// (paper Sec. 2, U = a0 + i a.sigma).  Product:
// (a0, a)(b0, b) = (a0 b0 - a.b, a0 b + b0 a - a x b); conjugate = dagger.
// ---------------------------------------------------------------------------
template <typename T>
struct Quat {
    T q[4];
};

template <typename T>
__device__ __forceinline__ Quat<T> qmul(const Quat<T>& a, const Quat<T>& b) {
    Quat<T> c;
    c.q[0] = fmadd(-a.q[3], b.q[3], fmadd(-a.q[2], b.q[2], fmadd(-a.q[1], b.q[1], a.q[0] * b.q[0])));
    c.q[1] = fmadd(a.q[3], b.q[2], fmadd(-a.q[2], b.q[3], fmadd(b.q[0], a.q[1], a.q[0] * b.q[1])));
    c.q[2] = fmadd(a.q[1], b.q[3], fmadd(-a.q[3], b.q[1], fmadd(b.q[0], a.q[2], a.q[0] * b.q[2])));
    c.q[3] = fmadd(a.q[2], b.q[1], fmadd(-a.q[1], b.q[2], fmadd(b.q[0], a.q[3], a.q[0] * b.q[3])));
    return c;
}

template <typename T>
__device__ __forceinline__ Quat<T> qconj(const Quat<T>& a) {
    return Quat<T>{{a.q[0], -a.q[1], -a.q[2], -a.q[3]}};
}

template <typename T>
__device__ __forceinline__ void qadd(Quat<T>& acc, const Quat<T>& a) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc.q[c] += a.q[c];
}

// Quaternion (SU(2)-proportional) part of the 2x2 block (i, j) of W:
// P(w) = (w + conj-adjugate) / 2, returned in quaternion components.
template <int N, typename T>
__device__ __forceinline__ Quat<T> block_quat(const Mat<N, T>& W, int i, int j) {
    Quat<T> p;
    p.q[0] = T(0.5) * (W.re[i][i] + W.re[j][j]);
    p.q[3] = T(0.5) * (W.im[i][i] - W.im[j][j]);
    p.q[2] = T(0.5) * (W.re[i][j] - W.re[j][i]);
    p.q[1] = T(0.5) * (W.im[i][j] + W.im[j][i]);
    return p;
}

// Rows i, j of M <- a (2x2 from quaternion a) times rows i, j.
template <int N, typename T>
__device__ __forceinline__ void rows_left_mul(Mat<N, T>& M, int i, int j, const Quat<T>& a) {
    // a11 = a0 + i a3, a12 = a2 + i a1, a21 = -a2 + i a1, a22 = a0 - i a3
SUN_MAT_UNROLL
    for (int c = 0; c < N; ++c) {
        const T xr = M.re[i][c], xi = M.im[i][c], yr = M.re[j][c], yi = M.im[j][c];
        M.re[i][c] = fmadd(-a.q[1], yi, fmadd(a.q[2], yr, fmadd(-a.q[3], xi, a.q[0] * xr)));
        M.im[i][c] = fmadd(a.q[1], yr, fmadd(a.q[2], yi, fmadd(a.q[3], xr, a.q[0] * xi)));
        M.re[j][c] = fmadd(a.q[3], yi, fmadd(a.q[0], yr, fmadd(-a.q[1], xi, -a.q[2] * xr)));
        M.im[j][c] = fmadd(-a.q[3], yr, fmadd(a.q[0], yi, fmadd(a.q[1], xr, -a.q[2] * xi)));
    }
}

// ---------------------------------------------------------------------------
// Link storage (SoA).  A link is E "pair planes" of T2 values: Nc^2 complex
// entries (row-major) for Nc >= 3, or (a0, a1), (a2, a3) for the SU(2)
// quaternion.  Plane p of link (mu, parity) lives at
//   base + (((mu * 2 + parity) * E + p) * Vh + h),
// so the V/2 links a phase updates, and each of their neighbour sets, are
// read with unit stride across a wavefront.
// ---------------------------------------------------------------------------
template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using type = float2;
};
template <>
struct Pair<double> {
    using type = double2;
};
template <typename T>
using T2 = typename Pair<T>::type;

// Stored rows R: R = N keeps the whole matrix; R = 2 with N = 3 keeps rows 0
// and 1 (12 reals, the paper's Sec. 3 SU(3) parameterization) and rebuilds
// row 2 = conj(row0 x row1) on every load (exact for SU(3)).
template <int N, int R = N>
struct Planes {
    static_assert(R == N || (N == 3 && R == 2), "only SU(3) has a two-row form");
    static constexpr int E = (N == 2) ? 2 : R * N;
};

template <int N, typename T, int R = N>
__device__ __forceinline__ const T2<T>* plane0(const T2<T>* base, int mu, int par, int Vh) {
    return base + (size_t)((mu * 2 + par) * Planes<N, R>::E) * (size_t)Vh;
}

// Row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1).
template <typename T>
__device__ __forceinline__ void third_row_entry(Mat<3, T>& m, int c) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    // (row0 x row1)_c = r0a r1b - r0b r1a, complex
    T xr = m.re[0][a] * m.re[1][b], xi = m.re[0][a] * m.im[1][b];
    xr = fmadd(-m.im[0][a], m.im[1][b], xr);
    xi = fmadd(m.im[0][a], m.re[1][b], xi);
    xr = fmadd(-m.re[0][b], m.re[1][a], xr);
    xi = fmadd(-m.re[0][b], m.im[1][a], xi);
    xr = fmadd(m.im[0][b], m.im[1][a], xr);
    xi = fmadd(-m.im[0][b], m.re[1][a], xi);
    m.re[2][c] = xr;
    m.im[2][c] = -xi;
}

template <int N, typename T>
__device__ __forceinline__ void third_row(Mat<N, T>& m) {
    if constexpr (N == 3) {
#pragma unroll
        for (int c = 0; c < 3; ++c) third_row_entry<T>(m, c);
    }
}

template <int N, typename T, int R = N>
__device__ __forceinline__ Mat<N, T> load_mat(const T2<T>* base, int mu, int par, int h, int Vh) {
    const T2<T>* p = plane0<N, T, R>(base, mu, par, Vh) + h;
    Mat<N, T> m;
SUN_MAT_UNROLL
    for (int e = 0; e < R * N; ++e) {
        const T2<T> v = p[(size_t)e * Vh];
        m.re[e / N][e % N] = v.x;
        m.im[e / N][e % N] = v.y;
    }
    if constexpr (R < N) third_row(m);
    return m;
}

// Rows 0 and 1 of an SU(3) link (row 2 left unset), either storage.
template <typename T, int R>
__device__ __forceinline__ Mat<3, T> load_rows01(const T2<T>* base, int mu, int par, int h, int Vh) {
    const T2<T>* p = plane0<3, T, R>(base, mu, par, Vh) + h;
    Mat<3, T> m;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const T2<T> v = p[(size_t)e * Vh];
        m.re[e / 3][e % 3] = v.x;
        m.im[e / 3][e % 3] = v.y;
    }
    return m;
}

// Columns 0 and 1 of an SU(3) link (entry (2, 2) left unset): the two-row
// form rebuilds only those two entries of row 2.
template <typename T, int R>
__device__ __forceinline__ Mat<3, T> load_cols01(const T2<T>* base, int mu, int par, int h, int Vh) {
    Mat<3, T> m = load_rows01<T, R>(base, mu, par, h, Vh);
    if constexpr (R == 3) {
        const T2<T>* p = plane0<3, T, 3>(base, mu, par, Vh) + h;
#pragma unroll
        for (int e = 6; e < 8; ++e) {
            const T2<T> v = p[(size_t)e * Vh];
            m.re[2][e - 6] = v.x;
            m.im[2][e - 6] = v.y;
        }
    } else {
        third_row_entry<T>(m, 0);
        third_row_entry<T>(m, 1);
    }
    return m;
}

template <int N, typename T, int R = N>
__device__ __forceinline__ void store_mat(T2<T>* base, int mu, int par, int h, int Vh, const Mat<N, T>& m) {
    T2<T>* p = const_cast<T2<T>*>(plane0<N, T, R>(base, mu, par, Vh)) + h;
SUN_MAT_UNROLL
    for (int e = 0; e < R * N; ++e) {
        T2<T> v;
        v.x = m.re[e / N][e % N];
        v.y = m.im[e / N][e % N];
        p[(size_t)e * Vh] = v;
    }
}

// Streaming (nontemporal) access for data a phase touches exactly once: the
// link being updated is read once and written once, while the neighbour
// planes are re-read and should keep the cache.
template <typename T>
struct NativePair;
template <>
struct NativePair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct NativePair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ __forceinline__ T2<T> load_stream(const T2<T>* p) {
    const typename NativePair<T>::type v =
        __builtin_nontemporal_load(reinterpret_cast<const typename NativePair<T>::type*>(p));
    T2<T> r;
    r.x = v.x;
    r.y = v.y;
    return r;
}

template <typename T>
__device__ __forceinline__ void store_stream(T2<T>* p, const T2<T>& a) {
    typename NativePair<T>::type v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<typename NativePair<T>::type*>(p));
}

template <int N, typename T, int R = N>
__device__ __forceinline__ Mat<N, T> load_mat_stream(const T2<T>* base, int mu, int par, int h, int Vh) {
    const T2<T>* p = plane0<N, T, R>(base, mu, par, Vh) + h;
    Mat<N, T> m;
SUN_MAT_UNROLL
    for (int e = 0; e < R * N; ++e) {
        const T2<T> v = load_stream<T>(p + (size_t)e * Vh);
        m.re[e / N][e % N] = v.x;
        m.im[e / N][e % N] = v.y;
    }
    if constexpr (R < N) third_row(m);
    return m;
}

template <int N, typename T, int R = N>
__device__ __forceinline__ void store_mat_stream(T2<T>* base, int mu, int par, int h, int Vh, const Mat<N, T>& m) {
    T2<T>* p = const_cast<T2<T>*>(plane0<N, T, R>(base, mu, par, Vh)) + h;
SUN_MAT_UNROLL
    for (int e = 0; e < R * N; ++e) {
        T2<T> v;
        v.x = m.re[e / N][e % N];
        v.y = m.im[e / N][e % N];
        store_stream<T>(p + (size_t)e * Vh, v);
    }
}

template <typename T>
__device__ __forceinline__ Quat<T> load_quat_stream(const T2<T>* base, int mu, int par, int h, int Vh) {
    const T2<T>* p = plane0<2, T>(base, mu, par, Vh) + h;
    const T2<T> a = load_stream<T>(p), b = load_stream<T>(p + Vh);
    return Quat<T>{{a.x, a.y, b.x, b.y}};
}

template <typename T>
__device__ __forceinline__ void store_quat_stream(T2<T>* base, int mu, int par, int h, int Vh, const Quat<T>& q) {
    T2<T>* p = const_cast<T2<T>*>(plane0<2, T>(base, mu, par, Vh)) + h;
    T2<T> a, b;
    a.x = q.q[0];
    a.y = q.q[1];
    b.x = q.q[2];
    b.y = q.q[3];
    store_stream<T>(p, a);
    store_stream<T>(p + Vh, b);
}

template <typename T>
__device__ __forceinline__ Quat<T> load_quat(const T2<T>* base, int mu, int par, int h, int Vh) {
    const T2<T>* p = plane0<2, T>(base, mu, par, Vh) + h;
    const T2<T> a = p[0], b = p[Vh];
    return Quat<T>{{a.x, a.y, b.x, b.y}};
}

template <typename T>
__device__ __forceinline__ void store_quat(T2<T>* base, int mu, int par, int h, int Vh, const Quat<T>& q) {
    T2<T>* p = const_cast<T2<T>*>(plane0<2, T>(base, mu, par, Vh)) + h;
    T2<T> a, b;
    a.x = q.q[0];
    a.y = q.q[1];
    b.x = q.q[2];
    b.y = q.q[3];
    p[0] = a;
    p[Vh] = b;
}

// ---------------------------------------------------------------------------
// Math wrappers that pick the float or double device routine.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float d_log(float x) { return logf(x); }
__device__ __forceinline__ double d_log(double x) { return log(x); }
__device__ __forceinline__ float d_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double d_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float d_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double d_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float d_cos(float x) { return cosf(x); }
__device__ __forceinline__ double d_cos(double x) { return cos(x); }
__device__ __forceinline__ float d_sin(float x) { return sinf(x); }
__device__ __forceinline__ double d_sin(double x) { return sin(x); }
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }

// FP32 square roots and reciprocals of the draw and of the subgroup
// normalisation use the hardware instructions (about 1 ulp, against half an
// ulp for the correctly rounded sequences of a dozen instructions each, far
// inside the FP32 tolerance of a link update); FP64, and FP32 zero and
// subnormal arguments, keep the correctly rounded forms.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

// 1 / a for a > 0, and 0 for a = 0.
template <typename T>
__device__ __forceinline__ T fast_inverse(T a) {
    if constexpr (sizeof(T) == 4) {
        if (a >= 1.17549435e-38f) return __builtin_amdgcn_rcpf(a);
    }
    return a > T(0) ? T(1) / a : T(0);
}

// The SU(2) draw in FP32 uses the hardware logarithm and cosine/sine
// (relative error ~1e-7, far inside the FP32 comparison tolerance); the FP64
// draw keeps the correctly rounded routines.
__device__ __forceinline__ float draw_log(float x) { return __logf(x); }
__device__ __forceinline__ double draw_log(double x) { return log(x); }
__device__ __forceinline__ float draw_cos(float x) { return __cosf(x); }
__device__ __forceinline__ double draw_cos(double x) { return cos(x); }
__device__ __forceinline__ float draw_sin(float x) { return __sinf(x); }
__device__ __forceinline__ double draw_sin(double x) { return sin(x); }

template <typename T>
struct Const {
    static constexpr T two_pi = T(6.283185307179586476925286766559);
    static constexpr T switch_alpha = T(1.7);  // Creutz below, Kennedy-Pendleton above
};

constexpr int kMaxAttempts = 64;

// ---------------------------------------------------------------------------
// SU(2) heatbath draw (paper Sec. 2): x0 with density sqrt(1-x0^2) e^{alpha x0},
// (x1,x2,x3) uniform on the sphere of radius sqrt(1-x0^2).  Creutz inversion
// for alpha < 1.7, Kennedy-Pendleton above.  Returns the attempt count, or 0
// when kMaxAttempts draws were rejected (the caller then skips the step).
// ---------------------------------------------------------------------------
// One attempt of the x0 draw from the four uniforms of counter word `hit`:
// returns whether it is accepted, with x0 and the radius sqrt(1 - x0^2).
// em = expm1(-2 alpha) and ia = 1 / alpha (0 for alpha = 0) are the draw's
// loop invariants, so an attempt divides by nothing.
template <typename T>
__device__ __forceinline__ bool su2_attempt(T alpha, T ia, bool creutz, T em, const U4& r, T& x0, T& rad) {
    const T r0 = uniform<T>(r.w[0]), r1 = uniform<T>(r.w[1]);
    const T r2 = uniform<T>(r.w[2]), r3 = uniform<T>(r.w[3]);
    if (creutz) {
        x0 = (alpha == T(0)) ? T(2) * r0 - T(1) : T(1) + d_log1p((T(1) - r0) * em) * ia;
        const T rhs = T(1) - x0 * x0;
        if (r1 * r1 <= rhs) {
            rad = fast_sqrt(rhs);
            return true;
        }
    } else {
        const T c = draw_cos(Const<T>::two_pi * r1);
        const T lam2 = -(draw_log(r0) + c * c * draw_log(r2)) * (T(0.5) * ia);
        const T rhs = T(1) - lam2;
        if (r3 * r3 <= rhs) {
            x0 = T(1) - T(2) * lam2;
            rad = T(2) * fast_sqrt(lam2) * fast_sqrt(rhs);
            return true;
        }
    }
    return false;
}

// (x1, x2, x3) uniform on the sphere of radius rad, from the direction
// draw's Philox words d.
template <typename T>
__device__ __forceinline__ Quat<T> su2_direction(T x0, T rad, const U4& d) {
    const T cos_t = T(1) - T(2) * uniform<T>(d.w[0]);
    const T sin_t = fast_sqrt(T(1) - cos_t * cos_t);
    const T phi = Const<T>::two_pi * uniform<T>(d.w[1]);
    Quat<T> x;
    x.q[0] = x0;
    x.q[1] = rad * sin_t * draw_cos(phi);
    x.q[2] = rad * sin_t * draw_sin(phi);
    x.q[3] = rad * cos_t;
    return x;
}

template <typename T>
__device__ __forceinline__ int sample_su2(T alpha, uint32_t k0, uint32_t k1, uint32_t site, uint32_t step,
                                          uint32_t mu_sg, Quat<T>& x) {
    T x0 = T(1), rad = T(0);
    const bool creutz = alpha < Const<T>::switch_alpha;
    const T em = creutz ? d_expm1(T(-2) * alpha) : T(0);  // loop invariants
    const T ia = fast_inverse(alpha);
    int hit = 0;
    bool ok = false;
    for (; hit < kMaxAttempts; ++hit) {
        const U4 r = philox(site, step, mu_sg, (RNG_ATTEMPT << 24) | (uint32_t)hit, k0, k1);
        if (su2_attempt(alpha, ia, creutz, em, r, x0, rad)) {
            ok = true;
            break;
        }
    }
    if (!ok) return 0;
    x = su2_direction(x0, rad, philox(site, step, mu_sg, RNG_DIRECTION << 24, k0, k1));
    return hit + 1;
}

}  // namespace sun
