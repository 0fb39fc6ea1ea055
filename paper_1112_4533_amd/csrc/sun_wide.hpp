// sun_wide.hpp -- SU(Nc) for large Nc (4 <= Nc <= 32): one 64-lane
// workgroup per link (paper Sec. 3, generic SU(Nc) code; Sec. 4, the
// large-Nc runs at 8^4).
//
// At large Nc a link no longer fits in one work-item's registers (Nc = 32 is
// 2048 reals), so a workgroup of one wavefront (or two) owns one link: the
// matrices of the update live in LDS, every product is spread over the lanes
// element by element, and the SU(2) subgroup steps (Nc(Nc-1)/2 of them)
// update two rows with one lane per column, several steps at a time.  Links are stored
// link-major (the Nc^2 complex entries of one link are contiguous), so the
// workgroup reads a link with unit stride.  Operands that enter a product
// daggered are transposed while they are copied into LDS, so that every
// product reads one operand by broadcast and the other with unit stride.
//
// The arithmetic is that of the register kernels: the same closing staple,
// W = U A, the lexicographic subgroup order (run several steps at a time
// where they share no index, which gives the same bits: sun_pairs.hpp), the
// quaternion projection, the same Philox counters, and an SU(2) draw whose
// 64 attempts are evaluated one per lane, the first accepted one winning
// (which is the sequential draw's result).  Reductions and re-unitarization
// are FP64.
#pragma once

#include <cfloat>

#include "sun_kernels.hpp"
#include "sun_pairs.hpp"

namespace sun {
namespace wide {

constexpr int kLanes = 64;
static_assert(kMaxAttempts == kLanes, "one SU(2) attempt per lane");
constexpr int kNcMin = 4, kNcMax = 32;

// Buffers (n x n complex) the phase kernel keeps in LDS.
constexpr int kUpdateBuffers = 4;

template <typename T>
__host__ __device__ inline size_t update_lds(int n) {
    return (size_t)kUpdateBuffers * n * n * sizeof(T2<T>);
}
__host__ __device__ inline size_t fp64_lds(int n, int buffers) { return (size_t)buffers * n * n * sizeof(double2); }

template <typename T>
__device__ __forceinline__ T2<T> cpx(T re, T im) {
    T2<T> v;
    v.x = re;
    v.y = im;
    return v;
}

// Link-major storage: link (mu, parity, h) is n^2 consecutive entries.
template <typename T>
__device__ __forceinline__ const T2<T>* link_at(const T2<T>* U, int n2, int mu, int par, int h, int Vh) {
    return U + ((size_t)(mu * 2 + par) * Vh + h) * n2;
}

// dst (LDS, type D) = src or src^dag (global, type S), converted.  Each
// lane issues the global loads of kLoadBatch entries before it stores any,
// so a link costs a few load latencies instead of one per entry.
constexpr int kLoadBatch = 8;

template <typename D, typename S, int NT = kLanes>
__device__ __forceinline__ void lds_load(T2<D>* dst, const T2<S>* src, int n, bool dag) {
    const int n2 = n * n;
    if (n2 <= NT) {  // one entry per lane
        const int e = threadIdx.x;
        if (e < n2) {
            const T2<S> v = src[e];
            if (dag) {
                const int i = e / n, j = e - i * n;
                dst[j * n + i] = cpx<D>((D)v.x, -(D)v.y);
            } else {
                dst[e] = cpx<D>((D)v.x, (D)v.y);
            }
        }
        return;
    }
    for (int e0 = threadIdx.x; e0 < n2; e0 += kLoadBatch * NT) {
        T2<S> v[kLoadBatch];
#pragma unroll
        for (int c = 0; c < kLoadBatch; ++c) {
            const int e = e0 + c * NT;
            if (e < n2) v[c] = src[e];
        }
#pragma unroll
        for (int c = 0; c < kLoadBatch; ++c) {
            const int e = e0 + c * NT;
            if (e >= n2) break;
            if (dag) {
                const int i = e / n, j = e - i * n;
                dst[j * n + i] = cpx<D>((D)v[c].x, -(D)v[c].y);
            } else {
                dst[e] = cpx<D>((D)v[c].x, (D)v[c].y);
            }
        }
    }
}

// C = A B, or C += A B (n <= 32; C distinct from B, and from A unless acc is
// false: then C may be A itself, because a lane reads its block of rows
// completely in the k loop before it stores any of it, the lanes of a row
// group run that loop together in the one wavefront of the workgroup, and no
// other lane touches those rows).  With g = 64 / n
// row groups, lane l < g n owns column j = l mod n and rows i0, i0 + g, ...
// (i0 = l / n), which it takes R at a time: each B_kj it reads serves R rows,
// and the n lanes of a row group read the same A_ik (an LDS broadcast).  A
// block that runs past the lane's last row repeats that row and does not
// store it, so the k loop has no lane-dependent branch.  Every entry is the
// sum over k = 0 .. n-1 in increasing k, with the same complex multiply-add
// as the plain triple loop.
template <typename T, int R>
__device__ __forceinline__ void lds_mm_rows(T2<T>* C, const T2<T>* A, const T2<T>* B, int n, bool acc, int g, int j,
                                            int i0, int cnt) {
    for (int t0 = 0; t0 < cnt; t0 += R) {
        int row[R];
        T r[R], m[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int tt = t0 + t < cnt ? t0 + t : cnt - 1;
            row[t] = (i0 + g * tt) * n;
            r[t] = T(0);
            m[t] = T(0);
            if (acc) {
                const T2<T> c = C[row[t] + j];
                r[t] = c.x;
                m[t] = c.y;
            }
        }
        // four k per pass, their LDS reads issued together
        int k = 0;
        for (; k + 4 <= n; k += 4) {
            T2<T> y[4], x[4][R];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                y[q] = B[(k + q) * n + j];
#pragma unroll
                for (int t = 0; t < R; ++t) x[q][t] = A[row[t] + k + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < R; ++t) cmac(r[t], m[t], x[q][t].x, x[q][t].y, y[q].x, y[q].y);
        }
        for (; k < n; ++k) {
            const T2<T> y = B[k * n + j];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const T2<T> x = A[row[t] + k];
                cmac(r[t], m[t], x.x, x.y, y.x, y.y);
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t0 + t < cnt) C[row[t] + j] = cpx<T>(r[t], m[t]);
    }
}

// The same product on the matrix cores for FP32 and kMfmaMinN < n <= 32:
// the complex product is four real 32 x 32 x 32 products (C_re += A_re B_re
// - A_im B_im, C_im += A_re B_im + A_im B_re), each 16 v_mfma_f32_32x32x2f32
// over k in pairs, with rows, columns and k beyond n read as zero.  Operand
// layout: lane l gives A[l mod 32][k0 + l / 32] and B[k0 + l / 32][l mod 32];
// result register r of lane l is entry (8 (r / 4) + 4 (l / 32) + r mod 4,
// l mod 32).  Every lane takes part (the matrix instructions need the whole
// wavefront), and all reads of A and B precede the stores, so C may be A
// when acc is false.  Below kMfmaMinN the padded tile wastes more than the
// VALU product costs.
constexpr int kMfmaMinN = 20;
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void lds_mm_mfma(T2<float>* C, const T2<float>* A, const T2<float>* B, int n, bool acc) {
    const int l = threadIdx.x;
    const int lo = l & 31, hi = l >> 5;
    f32x16 cr, ci;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r / 4) + 4 * hi + (r % 4);
        T2<float> c = cpx<float>(0.f, 0.f);
        if (acc && i < n && lo < n) c = C[i * n + lo];
        cr[r] = c.x;
        ci[r] = c.y;
    }
    // the real and imaginary accumulations alternate, so that consecutive
    // matrix instructions do not wait on each other's result
#pragma unroll 2
    for (int k0 = 0; k0 < n; k0 += 2) {
        const int k = k0 + hi;
        T2<float> a = cpx<float>(0.f, 0.f), b = cpx<float>(0.f, 0.f);
        if (k < n && lo < n) {
            a = A[lo * n + k];
            b = B[k * n + lo];
        }
        cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.y, b.y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, ci, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r / 4) + 4 * hi + (r % 4);
        if (i < n && lo < n) C[i * n + lo] = cpx<float>(cr[r], ci[r]);
    }
}

// Row groups of the vector-unit products on NT threads (NT / 64
// wavefronts): each wavefront holds 64 / n groups of n lanes, group i0 =
// (wavefront) * (64 / n) + lane / n taking column j = lane mod n and rows
// i0, i0 + g, ... (g groups in all).  A group never spans two wavefronts,
// and every entry is computed by one lane with the same operations in the
// same order whatever NT is, so the products give the same bits with one
// wavefront or two.
template <int NT>
struct RowMap {
    int g, j, i0, cnt, most;
    bool active;
    __device__ __forceinline__ explicit RowMap(int n) {
        const int gw = kLanes / n;
        const int w = (int)threadIdx.x / kLanes, l = (int)threadIdx.x % kLanes;
        g = gw * (NT / kLanes);
        active = l < gw * n;
        j = l % n;
        i0 = w * gw + l / n;
        cnt = (n - i0 + g - 1) / g;  // rows i0 + g t < n of this lane
        most = (n + g - 1) / g;      // rows of group 0, the most of any group
    }
};

// MM: the matrix-core form (FP32, kMfmaMinN < n), compiled into its own
// kernel variant so that the others keep their register budget.
// RMAX caps the rows a lane takes at a time (fewer registers).
template <typename T, bool MM = false, int RMAX = 4, int NT = kLanes>
__device__ __forceinline__ void lds_mm(T2<T>* C, const T2<T>* A, const T2<T>* B, int n, bool acc) {
    if constexpr (MM) {
        static_assert(sizeof(T) == 4, "the matrix-core product is FP32");
        if (threadIdx.x < kLanes) lds_mm_mfma(C, A, B, n, acc);  // the whole tile on the first wavefront
        return;
    }
    const RowMap<NT> m(n);
    if (!m.active) return;
    if (RMAX >= 4 && m.most >= 4)
        lds_mm_rows<T, 4>(C, A, B, n, acc, m.g, m.j, m.i0, m.cnt);
    else if (m.most >= 2)
        lds_mm_rows<T, 2>(C, A, B, n, acc, m.g, m.j, m.i0, m.cnt);
    else
        lds_mm_rows<T, 1>(C, A, B, n, acc, m.g, m.j, m.i0, m.cnt);
}

// ---------------------------------------------------------------------------
// A product accumulator in registers instead of LDS (the staple sum, and W =
// U A on its way into LDS), so that the update kernel holds two matrices in
// LDS instead of three where LDS limits the workgroups per CU.  Each lane
// keeps the entries it owns in the LDS products above: on the vector units
// column j = lane mod n, rows i0 + g t (at most kAccRows of them); on the
// matrix cores the 16 result registers of its 32 x 32 tile.  The products
// are the same operations in the same order as lds_mm with C in LDS, so the
// results are the same bits.
// ---------------------------------------------------------------------------
constexpr int kAccRows = 16;   // rows of the most loaded lane: ceil(n / (64 / n)) <= 16 for n <= 32

// NT threads: at most kAccRows * 64 / NT rows per lane.
template <typename T, bool MM, int NT = kLanes>
struct Acc {
    static constexpr int kRows = kAccRows * kLanes / NT;
    T2<T> e[kRows];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int t = 0; t < kRows; ++t) e[t] = cpx<T>(T(0), T(0));
    }
};
template <int NT>
struct Acc<float, true, NT> {
    f32x16 re, im;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int r = 0; r < 16; ++r) re[r] = im[r] = 0.f;
    }
};

// c += A B (A, B in LDS) on the vector units, R rows of the lane at a time.
template <typename T, int R, int NT>
__device__ __forceinline__ void acc_mm_rows(Acc<T, false, NT>& c, const T2<T>* A, const T2<T>* B, int n, int g,
                                            int j, int i0, int cnt, int most) {
#pragma unroll
    for (int t0 = 0; t0 < Acc<T, false, NT>::kRows; t0 += R) {
        if (t0 >= most) break;  // the same for every lane
        int row[R];
        T r[R], m[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int tt = t0 + t < cnt ? t0 + t : cnt - 1;
            row[t] = (i0 + g * tt) * n;
            r[t] = c.e[t0 + t].x;
            m[t] = c.e[t0 + t].y;
        }
        int k = 0;
        for (; k + 4 <= n; k += 4) {
            T2<T> y[4], x[4][R];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                y[q] = B[(k + q) * n + j];
#pragma unroll
                for (int t = 0; t < R; ++t) x[q][t] = A[row[t] + k + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < R; ++t) cmac(r[t], m[t], x[q][t].x, x[q][t].y, y[q].x, y[q].y);
        }
        for (; k < n; ++k) {
            const T2<T> y = B[k * n + j];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const T2<T> x = A[row[t] + k];
                cmac(r[t], m[t], x.x, x.y, y.x, y.y);
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t0 + t < cnt) c.e[t0 + t] = cpx<T>(r[t], m[t]);
    }
}

template <typename T, bool MM, int NT>
__device__ __forceinline__ void acc_mm(Acc<T, MM, NT>& c, const T2<T>* A, const T2<T>* B, int n) {
    if constexpr (MM) {
        const int l = threadIdx.x;
        if (l >= kLanes) return;  // the whole tile on the first wavefront
        const int lo = l & 31, hi = l >> 5;
#pragma unroll 2
        for (int k0 = 0; k0 < n; k0 += 2) {
            const int k = k0 + hi;
            T2<float> a = cpx<float>(0.f, 0.f), b = cpx<float>(0.f, 0.f);
            if (k < n && lo < n) {
                a = A[lo * n + k];
                b = B[k * n + lo];
            }
            c.re = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, c.re, 0, 0, 0);
            c.im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, c.im, 0, 0, 0);
            c.re = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.y, b.y, c.re, 0, 0, 0);
            c.im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, c.im, 0, 0, 0);
        }
    } else {
        const RowMap<NT> m(n);
        if (!m.active) return;
        // FP64 takes two rows at a time: with four, the kernel's registers
        // (the sum itself is 64 VGPRs at Nc = 32) left one wave per SIMD
        if (sizeof(T) == 4 && m.most >= 4)
            acc_mm_rows<T, 4, NT>(c, A, B, n, m.g, m.j, m.i0, m.cnt, m.most);
        else if (m.most >= 2)
            acc_mm_rows<T, 2, NT>(c, A, B, n, m.g, m.j, m.i0, m.cnt, m.most);
        else
            acc_mm_rows<T, 1, NT>(c, A, B, n, m.g, m.j, m.i0, m.cnt, m.most);
    }
}

// C (LDS) = the accumulator.
template <typename T, bool MM, int NT>
__device__ __forceinline__ void acc_store(T2<T>* C, const Acc<T, MM, NT>& c, int n) {
    if constexpr (MM) {
        const int l = threadIdx.x;
        if (l >= kLanes) return;
        const int lo = l & 31, hi = l >> 5;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r / 4) + 4 * hi + (r % 4);
            if (i < n && lo < n) C[i * n + lo] = cpx<float>(c.re[r], c.im[r]);
        }
    } else {
        const RowMap<NT> m(n);
        if (!m.active) return;
#pragma unroll
        for (int t = 0; t < Acc<T, MM, NT>::kRows; ++t)
            if (t < m.cnt) C[(m.i0 + m.g * t) * n + m.j] = c.e[t];
    }
}

// Cross-lane moves of a wavefront without the LDS: lane l receives the
// value of its partner lane, for five pairings that together join all 64
// lanes -- l xor 1 and l xor 2 (quad permutes), 7 - l and 15 - l within
// groups of 8 and 16 (row mirrors), l xor 16 (swizzle) -- and l xor 32
// (the swap of the two halves).
template <int STEP>
__device__ __forceinline__ int partner(int v) {
    if constexpr (STEP == 0) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad [1,0,3,2]
    if constexpr (STEP == 1) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad [2,3,0,1]
    if constexpr (STEP == 2) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row half mirror
    if constexpr (STEP == 3) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row mirror
    if constexpr (STEP == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);                     // xor 16
    if constexpr (STEP == 5) {                                                                   // xor 32
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return threadIdx.x < 32 ? (int)r[1] : (int)r[0];
    }
    return v;
}
template <int STEP>
__device__ __forceinline__ double partner(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)partner<STEP>((int)(u & 0xffffffffu));
    const unsigned hi = (unsigned)partner<STEP>((int)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Wave reductions over the six pairings above in a fixed order: every lane
// combines the same two partial results at each step (in one order or the
// other, which for + and max gives the same bits), so all lanes end with
// the same deterministic value.
template <typename F>
__device__ __forceinline__ double wave_reduce(double v, F op) {
    v = op(v, partner<0>(v));
    v = op(v, partner<1>(v));
    v = op(v, partner<2>(v));
    v = op(v, partner<3>(v));
    v = op(v, partner<4>(v));
    v = op(v, partner<5>(v));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    return wave_reduce(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_max(double v) {
    return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}

// Every kernel here runs one wavefront per workgroup, and a wavefront's LDS
// operations complete in the order it issues them: a read issued after a
// write sees it, whichever lane wrote, and a write issued after a read leaves
// that read's value alone.  Steps that hand LDS data between lanes therefore
// need only compiler ordering (a wavefront-scope fence), not a wait for the
// LDS round trip that a workgroup barrier implies.
__device__ __forceinline__ void wave_lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// v on lane `lane` (uniform across the wave), read with readlane.
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double lane_value(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffu), lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The scalar steps of the subgroup chain -- the block's norm and its
// inverse, 1 / alpha, the draw's square roots -- are computed by the lanes
// of a step for the whole link, one slot after another, so their latency is
// the chain's; the correctly rounded sequences take a dozen dependent
// instructions each.  FP32 takes the hardware forms shared with the
// register path (fast_sqrt, fast_inverse, unit_quat: about 1 ulp each); FP64
// here takes the hardware reciprocal and reciprocal square root refined by
// two Newton steps each (about 1 ulp) and the correctly rounded square root.
// The extra half ulp is far inside the tolerance of a link update.  Zero and
// subnormal arguments keep the correctly rounded forms.
__device__ __forceinline__ double newton_rsqrt(double x) {  // normal x > 0
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {  // r <- r + r (1 - x r^2) / 2
        const double e = fma(-x * r, r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    return r;
}
__device__ __forceinline__ double newton_rcp(double x) {  // normal x > 0
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {  // r <- r + r (1 - x r)
        const double e = fma(-x, r, 1.0);
        r = fma(r, e, r);
    }
    return r;
}

template <typename T>
__device__ __forceinline__ T chain_inverse(T alpha) {
    if constexpr (sizeof(T) == 8) {
        if (alpha >= DBL_MIN) return newton_rcp(alpha);
    }
    return fast_inverse(alpha);
}

// k = |p| and v = p / k (v = 1 for p = 0), as unit_quat.
template <typename T>
__device__ __forceinline__ T chain_unit_quat(const Quat<T>& p, Quat<T>& v) {
    if constexpr (sizeof(T) == 8) {
        const double k2 = p.q[0] * p.q[0] + p.q[1] * p.q[1] + p.q[2] * p.q[2] + p.q[3] * p.q[3];
        if (k2 >= DBL_MIN) {
            const double r = newton_rsqrt(k2);
#pragma unroll
            for (int c = 0; c < 4; ++c) v.q[c] = p.q[c] * r;
            return k2 * r;
        }
    }
    return unit_quat(p, v);
}

// SU(2) draws of the subgroup steps, eight subgroups per pair of Philox
// passes.  The hybrid sampler accepts an attempt with probability at least
// about 0.71, so the first few attempts almost always decide: lane l holds
// the words of attempt l mod 8 of subgroup sg0 + l / 8, and lanes l hold the
// direction words of subgroup sg0 + l mod 8.  A draw whose first eight
// attempts all reject (about 5e-5 of draws) runs attempts 8 .. 63 one per
// lane.  Either way the draw takes the lowest accepting attempt of the
// counter-based stream, as the sequential sampler does.
constexpr int kSgBatch = 8;                    // subgroups per batch
constexpr int kFirstHits = kLanes / kSgBatch;  // attempts per subgroup in a batch

// What a batch keeps per lane: the uniforms of its attempt that the two
// samplers test (r0, r1, r3) and the Kennedy-Pendleton log term
// -(log r0 + cos^2(2 pi r1) log r2), which does not depend on alpha; and the
// direction of subgroup sg0 + lane mod 8 as cos/sin of its polar angle and
// of its azimuth.  Only the alpha-dependent remainder of a draw is left on
// the sequential chain of subgroup steps.
template <typename T>
struct DrawBatch {
    T r0, r1, r3, kp;
    T cos_t, sin_t, cos_p, sin_p;
};

// Lane l's share of a batch whose lane group l / 8 draws the attempts of
// subgroup sg_att and whose lanes l mod 8 = g hold the direction of the
// subgroup of group g, sg_dir.
template <typename T>
__device__ __forceinline__ DrawBatch<T> draw_batch_of(uint32_t k0, uint32_t k1, uint32_t site, uint32_t step,
                                                      uint32_t mu_hi, uint32_t sg_att, uint32_t sg_dir, uint32_t l) {
    const U4 a = philox(site, step, mu_hi | sg_att, (RNG_ATTEMPT << 24) | (l % kFirstHits), k0, k1);
    const U4 d = philox(site, step, mu_hi | sg_dir, RNG_DIRECTION << 24, k0, k1);
    DrawBatch<T> b;
    b.r0 = uniform<T>(a.w[0]);
    b.r1 = uniform<T>(a.w[1]);
    const T r2 = uniform<T>(a.w[2]);
    b.r3 = uniform<T>(a.w[3]);
    const T c = draw_cos(Const<T>::two_pi * b.r1);
    b.kp = -(draw_log(b.r0) + c * c * draw_log(r2));
    b.cos_t = T(1) - T(2) * uniform<T>(d.w[0]);
    b.sin_t = d_sqrt(T(1) - b.cos_t * b.cos_t);
    const T phi = Const<T>::two_pi * uniform<T>(d.w[1]);
    b.cos_p = draw_cos(phi);
    b.sin_p = draw_sin(phi);
    return b;
}
// The batch of subgroups sg0 .. sg0 + 7.
template <typename T>
__device__ __forceinline__ DrawBatch<T> draw_batch(uint32_t k0, uint32_t k1, uint32_t site, uint32_t step,
                                                   uint32_t mu_hi, uint32_t sg0, uint32_t l) {
    return draw_batch_of<T>(k0, k1, site, step, mu_hi, sg0 + l / kFirstHits, sg0 + l % kSgBatch, l);
}

// ---------------------------------------------------------------------------
// The subgroup steps in slots of SW (the order of pairs::make_table, which
// gives the link of the fixed order bit for bit): in each slot the lanes
// 64 m / SW .. 64 (m + 1) / SW - 1 run place m, each lane owning columns of
// U and of W.  A batch covers the eight subgroups of 8 / SW slots, lane
// group g drawing for place g mod SW of slot g / SW; its eight steps are
// four table words.  Four steps per slot from Nc = 10 (SU(32): 139 slots
// instead of 257), where the shorter chain pays for four column updates
// per lane; two below, where it does not (Nc = 5: 7 slots either way).
// Every width gives the same bits.
// ---------------------------------------------------------------------------
constexpr int kSlot4MinN = 10;
__host__ __device__ constexpr int slot_steps(int n) { return n >= kSlot4MinN ? 4 : 2; }
template <int SW>
struct SlotShape {
    static constexpr int kStepLanes = kLanes / SW;                              // lanes per step
    static constexpr int kStepCols = (kNcMax + kStepLanes - 1) / kStepLanes;     // columns per lane
    static constexpr int kWords = SW / 2;                                        // table words per slot
    static constexpr int kPerBatch = kSgBatch / SW;                              // slots per batch
};
constexpr int kBatchWords = kSgBatch / 2;
static __constant__ pairs::Table<2> kPairTable2 = pairs::make_table<2>();
static __constant__ pairs::Table<4> kPairTable4 = pairs::make_table<4>();
constexpr pairs::Table<2> kPairTable2Host = pairs::make_table<2>();
constexpr pairs::Table<4> kPairTable4Host = pairs::make_table<4>();
// The table words of a link, 64 to a register across the wavefront (lane l
// holds word 64 w + l of window w), so that a slot reads its steps with
// readlane.
constexpr int max_words() {
    const int a = pairs::slots(kPairTable2Host, kNcMax), b = 2 * pairs::slots(kPairTable4Host, kNcMax);
    return a > b ? a : b;
}
constexpr int kPairWindows = (max_words() + kLanes - 1) / kLanes;
static_assert(kLanes % kBatchWords == 0, "a batch's words share a window");
static_assert(kBatchWords == 4, "draw_pair_batch selects among four words");
constexpr uint32_t kNoWord = 0xFFFFFFFFu;  // beyond the last slot: no steps

template <int SW>
__device__ __forceinline__ void pair_windows(int n, uint32_t (&win)[kPairWindows], int& nslot) {
    const uint16_t* first = SW == 2 ? kPairTable2.first : kPairTable4.first;
    const uint32_t* word = SW == 2 ? kPairTable2.word : kPairTable4.word;
    constexpr int kw = SlotShape<SW>::kWords;
    const int f = first[n] * kw;
    nslot = first[n + 1] - first[n];
    const int l = (int)(threadIdx.x & (kLanes - 1));
#pragma unroll
    for (int w = 0; w < kPairWindows; ++w) win[w] = kLanes * w + l < nslot * kw ? word[f + kLanes * w + l] : kNoWord;
}
// The next window to the front (after every 64 words).
__device__ __forceinline__ void pair_windows_shift(uint32_t (&win)[kPairWindows]) {
#pragma unroll
    for (int w = 0; w + 1 < kPairWindows; ++w) win[w] = win[w + 1];
    win[kPairWindows - 1] = kNoWord;
}
__device__ __forceinline__ uint32_t pair_at(uint32_t win0, int u) {
    return (uint32_t)__builtin_amdgcn_readlane((int)win0, u);
}
// Subgroup number (the Philox counter) of half m of a table word; 0 for an
// empty place, whose draws go unused.
__device__ __forceinline__ uint32_t pair_sg(uint32_t e, int m, int n) {
    const int i = (int)((e >> (16 * m)) & 0xFF), j = (int)((e >> (16 * m + 8)) & 0xFF);
    return i == pairs::kNone ? 0u : pairs::step_index(n, i, j);
}
// The batch of the four table words u0 .. u0 + 3 of window win0.
template <typename T>
__device__ __forceinline__ DrawBatch<T> draw_pair_batch(uint32_t k0, uint32_t k1, uint32_t site, uint32_t step,
                                                        uint32_t mu_hi, uint32_t win0, int u0, int n, uint32_t l) {
    uint32_t e[kBatchWords];
#pragma unroll
    for (int q = 0; q < kBatchWords; ++q) e[q] = pair_at(win0, u0 + q);
    auto sg_of = [&](uint32_t g) {
        const uint32_t q = g >> 1;
        const uint32_t es = q == 0 ? e[0] : q == 1 ? e[1] : q == 2 ? e[2] : e[3];
        return pair_sg(es, (int)(g & 1), n);
    };
    return draw_batch_of<T>(k0, k1, site, step, mu_hi, sg_of(l / kFirstHits), sg_of(l % kSgBatch), l);
}

// A ring of two batches in LDS (slot, field, lane), through which a second
// wavefront hands the first the draws of the next eight subgroups.
constexpr int kBatchFields = 8;
template <typename T>
__host__ __device__ inline size_t batch_ring_bytes() {
    return (size_t)2 * kBatchFields * kLanes * sizeof(T);
}
// Dynamic LDS of an update launch beyond its matrices: the ring, where the
// second of two wavefronts draws the heatbath batches (ho: hand-off on).
template <typename T>
__host__ __device__ inline size_t handoff_lds(bool ho) {
    return ho ? batch_ring_bytes<T>() : 0;
}
template <typename T>
__device__ __forceinline__ void ring_store(T* ring, int slot, int l, const DrawBatch<T>& b) {
    T* r = ring + (size_t)slot * kBatchFields * kLanes + l;
    r[0 * kLanes] = b.r0;
    r[1 * kLanes] = b.r1;
    r[2 * kLanes] = b.r3;
    r[3 * kLanes] = b.kp;
    r[4 * kLanes] = b.cos_t;
    r[5 * kLanes] = b.sin_t;
    r[6 * kLanes] = b.cos_p;
    r[7 * kLanes] = b.sin_p;
}
template <typename T>
__device__ __forceinline__ DrawBatch<T> ring_load(const T* ring, int slot, int l) {
    const T* r = ring + (size_t)slot * kBatchFields * kLanes + l;
    DrawBatch<T> b;
    b.r0 = r[0 * kLanes];
    b.r1 = r[1 * kLanes];
    b.r3 = r[2 * kLanes];
    b.kp = r[3 * kLanes];
    b.cos_t = r[4 * kLanes];
    b.sin_t = r[5 * kLanes];
    b.cos_p = r[6 * kLanes];
    b.sin_p = r[7 * kLanes];
    return b;
}

// One attempt from a batch's precomputed terms: the same tests and results
// as su2_attempt on the attempt's Philox words.
template <typename T>
__device__ __forceinline__ bool su2_attempt_batched(T alpha, T ia, bool creutz, T em, const DrawBatch<T>& b, T& x0,
                                                    T& rad) {
    if (creutz) {
        x0 = (alpha == T(0)) ? T(2) * b.r0 - T(1) : T(1) + d_log1p((T(1) - b.r0) * em) * ia;
        const T rhs = T(1) - x0 * x0;
        if (b.r1 * b.r1 <= rhs) {
            rad = fast_sqrt(rhs);
            return true;
        }
    } else {
        const T lam2 = b.kp * (T(0.5) * ia);
        const T rhs = T(1) - lam2;
        if (b.r3 * b.r3 <= rhs) {
            x0 = T(1) - T(2) * lam2;
            rad = T(2) * fast_sqrt(lam2) * fast_sqrt(rhs);
            return true;
        }
    }
    return false;
}

// The draw of subgroup mu_sg, slot s of batch b.  Returns the number of the
// accepted attempt (1-based), or 0 (skip the step) when all kMaxAttempts
// attempts are rejected.
template <typename T>
__device__ __forceinline__ int sample_su2_lanes(T alpha, const DrawBatch<T>& b, int s, uint32_t k0, uint32_t k1,
                                                uint32_t site, uint32_t step, uint32_t mu_sg, Quat<T>& x) {
    const bool creutz = alpha < Const<T>::switch_alpha;
    const T em = creutz ? d_expm1(T(-2) * alpha) : T(0);
    const T ia = chain_inverse(alpha);
    T x0 = T(1), rad = T(0);
    bool ok = su2_attempt_batched(alpha, ia, creutz, em, b, x0, rad);
    unsigned long long mask = __ballot(ok) & (0xFFull << (kFirstHits * s));
    int hit0 = -kFirstHits * s;  // attempt number of lane 0, 0-based
    if (mask == 0ull) {
        const uint32_t hit = threadIdx.x + kFirstHits;
        const U4 r = philox(site, step, mu_sg, (RNG_ATTEMPT << 24) | hit, k0, k1);
        ok = hit < (uint32_t)kMaxAttempts && su2_attempt(alpha, ia, creutz, em, r, x0, rad);
        mask = __ballot(ok);
        if (mask == 0ull) return 0;
        hit0 = kFirstHits;
    }
    const int first = __ffsll(mask) - 1;  // the same on every lane
    x0 = lane_value(x0, first);
    rad = lane_value(rad, first);
    const T cos_t = lane_value(b.cos_t, s), sin_t = lane_value(b.sin_t, s);
    const T cos_p = lane_value(b.cos_p, s), sin_p = lane_value(b.sin_p, s);
    x.q[0] = x0;
    x.q[1] = rad * sin_t * cos_p;
    x.q[2] = rad * sin_t * sin_p;
    x.q[3] = rad * cos_t;
    return hit0 + first + 1;
}

// The draws of the np subgroups of slot q of a batch (lane groups
// kSlotSteps q + m hold the attempts of place m), as sample_su2_lanes draws
// each: alpha is the lane's own step's (place lane / (64 / kSlotSteps)),
// mu_sg the places' counters.  Returns, for the lane's own step, the accepted
// attempt's number (0: skip the step), and its element in x.
template <typename T, int kSlotSteps>
__device__ __forceinline__ int sample_su2_slot(T alpha, const DrawBatch<T>& b, int q, int np, uint32_t k0,
                                               uint32_t k1, uint32_t site, uint32_t step,
                                               const uint32_t (&mu_sg)[kSlotSteps], Quat<T>& x) {
    constexpr int kStepLanes = SlotShape<kSlotSteps>::kStepLanes;
    const int l = (int)threadIdx.x;
    T alm[kSlotSteps];
#pragma unroll
    for (int m = 0; m < kSlotSteps; ++m) alm[m] = m < np ? lane_value(alpha, m * kStepLanes) : alm[0];
    // each lane tries its attempt with the alpha of the subgroup it draws for
    const int gm = (l / kFirstHits) % kSlotSteps;
    T al = alm[0];
#pragma unroll
    for (int m = 1; m < kSlotSteps; ++m)
        if (gm == m) al = alm[m];
    const bool creutz = al < Const<T>::switch_alpha;
    const T em = creutz ? d_expm1(T(-2) * al) : T(0);
    const T ia = chain_inverse(al);
    T x0 = T(1), rad = T(0);
    const bool ok = su2_attempt_batched(al, ia, creutz, em, b, x0, rad);
    const unsigned long long ball = __ballot(ok);
    T mx0[kSlotSteps], mrad[kSlotSteps];
    int hit[kSlotSteps];
#pragma unroll
    for (int m = 0; m < kSlotSteps; ++m) {
        mx0[m] = T(1);
        mrad[m] = T(0);
        hit[m] = 0;
        if (m >= np) continue;
        const int g = kSlotSteps * q + m;
        unsigned long long mask = ball & (0xFFull << (kFirstHits * g));
        int hit0 = -kFirstHits * g;
        T fx0 = x0, frad = rad;
        if (mask == 0ull) {  // the first eight attempts all rejected: attempts 8 .. 63, one per lane
            const T a = alm[m];
            const bool cr = a < Const<T>::switch_alpha;
            const T e2 = cr ? d_expm1(T(-2) * a) : T(0);
            const T i2 = chain_inverse(a);
            const uint32_t h = (uint32_t)l + kFirstHits;
            const U4 r = philox(site, step, mu_sg[m], (RNG_ATTEMPT << 24) | h, k0, k1);
            fx0 = T(1);
            frad = T(0);
            const bool ok2 = h < (uint32_t)kMaxAttempts && su2_attempt(a, i2, cr, e2, r, fx0, frad);
            mask = __ballot(ok2);
            hit0 = kFirstHits;
        }
        if (mask != 0ull) {
            const int first = __ffsll(mask) - 1;  // the same on every lane
            mx0[m] = lane_value(fx0, first);
            mrad[m] = lane_value(frad, first);
            hit[m] = hit0 + first + 1;
        }
    }
    // the lane's own step; the direction of lane group g sits in the lanes
    // l mod 8 = g (read at uniform lanes, then selected)
    const int mo = l / kStepLanes;
    T x0o = mx0[0], ro = mrad[0];
    int ho = hit[0];
    T ct = lane_value(b.cos_t, kSlotSteps * q), st = lane_value(b.sin_t, kSlotSteps * q);
    T cp = lane_value(b.cos_p, kSlotSteps * q), sp = lane_value(b.sin_p, kSlotSteps * q);
#pragma unroll
    for (int m = 1; m < kSlotSteps; ++m) {
        const T ctm = lane_value(b.cos_t, kSlotSteps * q + m), stm = lane_value(b.sin_t, kSlotSteps * q + m);
        const T cpm = lane_value(b.cos_p, kSlotSteps * q + m), spm = lane_value(b.sin_p, kSlotSteps * q + m);
        if (mo == m && m < np) {
            x0o = mx0[m];
            ro = mrad[m];
            ho = hit[m];
            ct = ctm;
            st = stm;
            cp = cpm;
            sp = spm;
        }
    }
    x.q[0] = x0o;
    x.q[1] = ro * st * cp;
    x.q[2] = ro * st * sp;
    x.q[3] = ro * ct;
    return ho;
}

// Rows i, j of M (LDS), column c, left-multiplied by the 2x2 form of a,
// given their current entries x = M_ic and y = M_jc.
template <typename T>
__device__ __forceinline__ void rows_left_mul_col(T2<T>* M, int n, int i, int j, int c, const Quat<T>& a,
                                                  const T2<T>& x, const T2<T>& y) {
    M[i * n + c] = cpx<T>(fmadd(-a.q[1], y.y, fmadd(a.q[2], y.x, fmadd(-a.q[3], x.y, a.q[0] * x.x))),
                          fmadd(a.q[1], y.x, fmadd(a.q[2], y.y, fmadd(a.q[3], x.x, a.q[0] * x.y))));
    M[j * n + c] = cpx<T>(fmadd(a.q[3], y.y, fmadd(a.q[0], y.x, fmadd(-a.q[1], x.y, -a.q[2] * x.x))),
                          fmadd(-a.q[3], y.x, fmadd(a.q[0], y.y, fmadd(a.q[1], x.x, -a.q[2] * x.y))));
}

// ---------------------------------------------------------------------------
// One checkerboard phase: workgroup h updates U_mu(x), x = site h of parity
// par.  LDS: A (staple), B0, B1 (neighbour links); the first product of each
// staple term overwrites its left factor (B0 <- B0 B1), and after the staple
// B1 holds U and B0 holds W = U A.
// ---------------------------------------------------------------------------
// RA: the staple sum (and W on its way into LDS) in registers (Acc), so that
// LDS holds two matrices instead of three: B0 and B1, and after the staple U
// (B1) and W (B0).  At least two waves per SIMD (at most 256 registers): the
// FP64 form with the sum in registers would otherwise take a few more and
// leave one.
// NT: threads per workgroup, one wavefront or two.  With two, the loads and
// the vector-unit products are shared by both wavefronts (RowMap: the same
// bits), the first wavefront runs the subgroup steps, and with ho the
// second draws their heatbath batches (below); LDS then also holds the ring
// of two batches after the matrices (handoff_lds).
template <typename T, bool MM, bool RA, int NT, int SW>
__device__ __forceinline__ void update_link_wide(T2<T>* __restrict__ U, const Geom& g, int n, int mu, int par,
                                                 int hb, T beta, uint32_t k0, uint32_t k1, uint32_t step, int h,
                                                 bool ho) {
    static_assert(NT == kLanes || NT == 2 * kLanes, "one wavefront or two");
    extern __shared__ double4 smem_update[];
    const int n2 = n * n;
    T2<T>* A = reinterpret_cast<T2<T>*>(smem_update);  // the staple sum (without RA)
    T2<T>* B0 = RA ? A : A + n2;
    T2<T>* B1 = B0 + n2;
    Acc<T, MM, NT> acc;  // the staple sum (with RA)
    constexpr int kRows = (RA && sizeof(T) == 8) ? 2 : 4;  // FP64 with the sum in registers: fewer at a time
    const int Vh = g.Vh;
    const Site x = site_of(g, par, h);
    const Site xp = step_up(g, x, mu);
    const int op = par ^ 1;

    if constexpr (RA)
        acc.zero();
    else
        for (int e = threadIdx.x; e < n2; e += NT) A[e] = cpx<T>(T(0), T(0));
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu || !((g.present >> nu) & 1)) continue;
        const Site xpn = step_up(g, x, nu), xmn = step_down(g, x, nu), xpmn = step_down(g, xp, nu);
        // upper staple U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        lds_load<T, T, NT>(B0, link_at<T>(U, n2, nu, op, xp.s >> 1, Vh), n, false);
        lds_load<T, T, NT>(B1, link_at<T>(U, n2, mu, op, xpn.s >> 1, Vh), n, true);
        __syncthreads();
        lds_mm<T, MM, kRows, NT>(B0, B0, B1, n, false);
        __syncthreads();
        lds_load<T, T, NT>(B1, link_at<T>(U, n2, nu, par, h, Vh), n, true);
        __syncthreads();
        if constexpr (RA)
            acc_mm<T, MM, NT>(acc, B0, B1, n);
        else
            lds_mm<T, MM, 4, NT>(A, B0, B1, n, true);
        __syncthreads();
        // lower staple U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        lds_load<T, T, NT>(B0, link_at<T>(U, n2, nu, par, xpmn.s >> 1, Vh), n, true);
        lds_load<T, T, NT>(B1, link_at<T>(U, n2, mu, op, xmn.s >> 1, Vh), n, true);
        __syncthreads();
        lds_mm<T, MM, kRows, NT>(B0, B0, B1, n, false);
        __syncthreads();
        lds_load<T, T, NT>(B1, link_at<T>(U, n2, nu, op, xmn.s >> 1, Vh), n, false);
        __syncthreads();
        if constexpr (RA)
            acc_mm<T, MM, NT>(acc, B0, B1, n);
        else
            lds_mm<T, MM, 4, NT>(A, B0, B1, n, true);
        __syncthreads();
    }
    T2<T>* Us = B1;
    lds_load<T, T, NT>(Us, link_at<T>(U, n2, mu, par, h, Vh), n, false);
    T2<T>* W = B0;  // W = U A
    if constexpr (RA) {
        acc_store<T, MM, NT>(B0, acc, n);  // A into B0, which the last staple product has finished reading
        __syncthreads();
        acc.zero();
        acc_mm<T, MM, NT>(acc, Us, B0, n);
        __syncthreads();                   // every lane has read A
        acc_store<T, MM, NT>(W, acc, n);
    } else {
        __syncthreads();
        lds_mm<T, MM, 4, NT>(W, Us, A, n, false);
    }
    __syncthreads();
    // With two wavefronts the subgroup steps are the first's.  With the
    // hand-off the second draws the heatbath batches (whose Philox passes,
    // logarithms and cosines would otherwise sit on the chain at the first
    // step slot of each batch): batch 0 before the chain, batch b + 1 after barrier b,
    // into slot (b + 1) mod 2 of a ring after the matrices, which the first
    // read (into registers) before barrier b.  The first takes barrier b at
    // step slot kSlotsPerBatch b, then reads ring slot b mod 2.  Both
    // wavefronts pass the same ceil(S / kSlotsPerBatch) barriers, S the
    // number of step slots.  Without it the first wavefront draws its own,
    // as with one wavefront.  FP64 always hands off with two wavefronts
    // (decided at compile time: keeping both draw paths in the FP64 kernel
    // costs it 3-4%); FP32 as ho says.
    const bool hand_off = NT > kLanes && (sizeof(T) == 8 || ho);
    T* const ring = reinterpret_cast<T*>(reinterpret_cast<char*>(smem_update) + (RA ? 2 : 3) * n2 * sizeof(T2<T>));
    constexpr int kSlotSteps = SW, kStepLanes = SlotShape<SW>::kStepLanes, kStepCols = SlotShape<SW>::kStepCols;
    constexpr int kSlotWords = SlotShape<SW>::kWords, kSlotsPerBatch = SlotShape<SW>::kPerBatch;
    uint32_t win[kPairWindows];
    int nslot = 0;
    pair_windows<SW>(n, win, nslot);
    const int nbatch = (nslot + kSlotsPerBatch - 1) / kSlotsPerBatch;
    if (NT > kLanes && threadIdx.x >= kLanes) {
        if (hand_off && hb) {
            const uint32_t l = threadIdx.x - kLanes;
            const uint32_t mh = (uint32_t)mu << 16;
            ring_store<T>(ring, 0, (int)l, draw_pair_batch<T>(k0, k1, (uint32_t)x.s, step, mh, win[0], 0, n, l));
            for (int b = 0; b < nbatch; ++b) {
                __syncthreads();
                const int wb = kBatchWords * (b + 1);  // the next batch's first table word
                if (b + 1 < nbatch) {
                    if ((wb & (kLanes - 1)) == 0) pair_windows_shift(win);
                    ring_store<T>(ring, (b + 1) & 1, (int)l,
                                  draw_pair_batch<T>(k0, k1, (uint32_t)x.s, step, mh, win[0], wb & (kLanes - 1), n, l));
                }
            }
        }
        __syncthreads();
        T2<T>* dst = const_cast<T2<T>*>(link_at<T>(U, n2, mu, par, h, Vh));
        for (int e = threadIdx.x; e < n2; e += NT) dst[e] = Us[e];
        return;
    }

    const int lane = threadIdx.x;
    const uint32_t mu_hi = (uint32_t)mu << 16;
    DrawBatch<T> batch{};
    const T cb = T(2) * beta / T(n);  // alpha = 2 beta k / n
    // The slots are ordered by wave_lds_order; in each, lane l runs place
    // l / kStepLanes, owning columns l mod kStepLanes + k kStepLanes of U and
    // of W and reading its entries of rows i and j together with the 2x2
    // block.  A slot's places are filled first, so place 0 always holds a
    // step; the lanes of an empty place read that step's rows and write
    // nothing.
    const int place = lane / kStepLanes;
    const int c0 = lane % kStepLanes;
    for (int t = 0; t < nslot; ++t) {
        const int u = (t * kSlotWords) & (kLanes - 1);
        if (u == 0 && t > 0) pair_windows_shift(win);
        uint32_t wd[kSlotWords], stp[kSlotSteps];
        int np = 0;
#pragma unroll
        for (int k = 0; k < kSlotWords; ++k) wd[k] = pair_at(win[0], u + k);
#pragma unroll
        for (int m = 0; m < kSlotSteps; ++m) {
            stp[m] = (wd[m / 2] >> (16 * (m % 2))) & 0xFFFFu;
            np += stp[m] != pairs::kNoStep;
        }
        uint32_t es = stp[0];
#pragma unroll
        for (int m = 1; m < kSlotSteps; ++m)
            if (place == m && m < np) es = stp[m];
        const bool mine = place < np;
        const int i = (int)(es & 0xFF), j = (int)((es >> 8) & 0xFF);
        const T2<T> wii = W[i * n + i], wij = W[i * n + j], wji = W[j * n + i], wjj = W[j * n + j];
        T2<T> ui[kStepCols], uj[kStepCols], xi[kStepCols], xj[kStepCols];
#pragma unroll
        for (int cc = 0; cc < kStepCols; ++cc) {
            const int ck = c0 + cc * kStepLanes;
            const int c = ck < n ? ck : 0;
            ui[cc] = Us[i * n + c];
            uj[cc] = Us[j * n + c];
            xi[cc] = W[i * n + c];
            xj[cc] = W[j * n + c];
        }
        Quat<T> p;
        p.q[0] = T(0.5) * (wii.x + wjj.x);
        p.q[3] = T(0.5) * (wii.y - wjj.y);
        p.q[2] = T(0.5) * (wij.x - wji.x);
        p.q[1] = T(0.5) * (wij.y + wji.y);
        Quat<T> v;
        const T k = chain_unit_quat(p, v);
        Quat<T> a;
        bool apply = true;
        if (hb) {
            const int q = t % kSlotsPerBatch;
            if (q == 0) {
                if (hand_off) {
                    __syncthreads();
                    batch = ring_load<T>(ring, (t / kSlotsPerBatch) & 1, lane);
                } else {
                    batch = draw_pair_batch<T>(k0, k1, (uint32_t)x.s, step, mu_hi, win[0], u, n, (uint32_t)lane);
                }
            }
            const T alpha = cb * k;
            uint32_t sgs[kSlotSteps];
#pragma unroll
            for (int m = 0; m < kSlotSteps; ++m) sgs[m] = mu_hi | pair_sg(wd[m / 2], m % 2, n);
            Quat<T> xs;
            apply = sample_su2_slot<T, SW>(alpha, batch, q, np, k0, k1, (uint32_t)x.s, step, sgs, xs) != 0;
            if (apply) a = qmul(xs, qconj(v));
        } else {
            const Quat<T> vc = qconj(v);
            a = qmul(vc, vc);
        }
        if (apply && mine) {
#pragma unroll
            for (int cc = 0; cc < kStepCols; ++cc) {
                const int ck = c0 + cc * kStepLanes;
                if (ck < n) {
                    rows_left_mul_col<T>(Us, n, i, j, ck, a, ui[cc], uj[cc]);
                    rows_left_mul_col<T>(W, n, i, j, ck, a, xi[cc], xj[cc]);
                }
            }
        }
        wave_lds_order();
    }
    __syncthreads();
    T2<T>* dst = const_cast<T2<T>*>(link_at<T>(U, n2, mu, par, h, Vh));
    for (int e = threadIdx.x; e < n2; e += NT) dst[e] = Us[e];
}

// One checkerboard phase of one lattice: workgroup h updates link h.
template <typename T, bool MM, bool RA, int NT, int SW>
__global__ __launch_bounds__(NT, 2) void k_update(T2<T>* __restrict__ U, Geom g, int n, int mu, int par, int hb,
                                               T beta, uint32_t k0, uint32_t k1, uint32_t step, int ho) {
    update_link_wide<T, MM, RA, NT, SW>(U, g, n, mu, par, hb, beta, k0, k1, step, (int)blockIdx.x, ho != 0);
}

// One phase of every chain of a batch group (same Nc and precision): one
// workgroup per updated link of each chain, the chain found by binary search
// over the first-link prefix of the descriptor table (TILE_HALF_HB counts
// links here); coupling, Philox key and RNG step come from the table.
template <typename T, bool MM, bool RA, int NT, int SW>
__global__ __launch_bounds__(NT, 2) void k_update_batch(const ChainDesc* __restrict__ d, int nchains, int n,
                                                     int mu, int par, int hb, uint32_t step_offset, int ho) {
    const int c = find_chain<TILE_HALF_HB>(d, nchains, (int)blockIdx.x);
    const Geom g = d[c].g;
    if (!((g.present >> mu) & 1)) return;
    update_link_wide<T, MM, RA, NT, SW>((T2<T>*)d[c].links, g, n, mu, par, hb, (T)d[c].beta, d[c].k0, d[c].k1,
                                (uint32_t)(d[c].step + step_offset), (int)blockIdx.x - d[c].tile0[TILE_HALF_HB],
                                ho != 0);
}

// ---------------------------------------------------------------------------
// FP64 helpers on an LDS matrix whose column c belongs to lane c (n <= 32).
// ---------------------------------------------------------------------------

// det by LU with partial pivoting (the first largest pivot), destroying D.
__device__ __forceinline__ void lds_det(double2* D, int n, double& dr, double& di) {
    const int c = threadIdx.x;
    dr = 1.0;
    di = 0.0;
    for (int col = 0; col < n; ++col) {
        wave_lds_order();
        // pivot: the largest |D[r][col]|^2 over r >= col, the lowest r among
        // equals -- a scan by lane 0 for small n, a wave argmax otherwise
        // (the same choice: the scan keeps the first strict maximum)
        int piv = col;
        double best = -1.0;
        if (n <= 8) {
            if (c == 0)
                for (int r = col; r < n; ++r) {
                    const double a = D[r * n + col].x * D[r * n + col].x + D[r * n + col].y * D[r * n + col].y;
                    if (a > best) {
                        best = a;
                        piv = r;
                    }
                }
            piv = __shfl(piv, 0, kLanes);
            best = __shfl(best, 0, kLanes);
        } else {
            piv = c;
            if (c >= col && c < n) best = D[c * n + col].x * D[c * n + col].x + D[c * n + col].y * D[c * n + col].y;
            // the largest, the lowest row among equals: an order-free choice,
            // so every lane ends with the same pair
            auto take = [&](double ob, int op) {
                if (ob > best || (ob == best && op < piv)) {
                    best = ob;
                    piv = op;
                }
            };
            take(partner<0>(best), partner<0>(piv));
            take(partner<1>(best), partner<1>(piv));
            take(partner<2>(best), partner<2>(piv));
            take(partner<3>(best), partner<3>(piv));
            take(partner<4>(best), partner<4>(piv));
            take(partner<5>(best), partner<5>(piv));
        }
        if (best == 0.0) {
            dr = di = 0.0;
            return;
        }
        if (piv != col) {
            if (c < n) {
                const double2 t = D[col * n + c];
                D[col * n + c] = D[piv * n + c];
                D[piv * n + c] = t;
            }
            dr = -dr;
            di = -di;
        }
        wave_lds_order();
        const double pr = D[col * n + col].x, pi = D[col * n + col].y;
        const double nr = dr * pr - di * pi, ni = dr * pi + di * pr;
        dr = nr;
        di = ni;
        const double pm = pr * pr + pi * pi;
        const double inv = pm >= DBL_MIN ? newton_rcp(pm) : 1.0 / pm;
        // rows below the pivot are independent: above n = 8 the lower half
        // of the wavefront eliminates rows col + 1, col + 3, ... and the upper
        // half rows col + 2, col + 4, ..., lane q taking column q (n <= 32);
        // every entry sees the same operations in the same order either way
        const bool split = n > 8;
        const int q = c & 31, half = c >> 5;
        const bool works = (split || half == 0) && q >= col && q < n;
        // the pivot row's entry of column q, read once: only rows below it
        // change in this column's elimination
        const double2 u = works ? D[col * n + q] : make_double2(0.0, 0.0);
        for (int r = col + 1 + (split ? half : 0); r < n; r += split ? 2 : 1) {
            const double2 m = D[r * n + col];
            const double fr = (m.x * pr + m.y * pi) * inv;
            const double fi = (m.y * pr - m.x * pi) * inv;
            if (works) {
                double2 w = D[r * n + q];
                w.x -= fr * u.x - fi * u.y;
                w.y -= fr * u.y + fi * u.x;
                D[r * n + q] = w;
            }
        }
    }
}

// max_ij |(M^dag M - 1)_ij| (M unchanged).
__device__ __forceinline__ double lds_unitarity_dev(const double2* M, int n) {
    const int n2 = n * n;
    double du2 = 0.0;
    for (int e = threadIdx.x; e < n2; e += kLanes) {
        const int i = e / n, j = e - i * n;
        if (j < i) continue;  // Hermitian: the upper triangle has every modulus
        double r = (i == j) ? -1.0 : 0.0, m = 0.0;
        for (int k = 0; k < n; ++k) {
            const double2 a = M[k * n + i], b = M[k * n + j];
            cmac(r, m, a.x, -a.y, b.x, b.y);
        }
        du2 = fmax(du2, nan_to_inf(fmadd(m, m, r * r)));  // a NaN entry counts as infinite
    }
    return sqrt(wave_max(du2));
}

// Gram-Schmidt on all rows, then the last row times conj(det)/|det| (paper
// Sec. 2, re-unitarization; Nc > 3).  Each row is orthogonalized against the
// earlier ones by classical Gram-Schmidt, with a second pass where the
// first removed more than half the row's squared norm (Daniel, Gragg,
// Kaufman and Stewart, Math. Comp. 30 (1976): twice is enough, as stable as
// the modified form): lane k forms <r_k, r_i> from LDS, then lane c
// subtracts every projection from column c of r_i, so a row costs two LDS
// hand-offs per pass instead of a chain of wave reductions per projection.  P (n entries)
// holds the projections.  (dr, di) is det M of the matrix before the
// projection: row Gram-Schmidt writes M = L Q with L lower triangular and
// real positive on its diagonal, so det Q = det M / prod L_ii has the phase
// of det M, and the fix needs no determinant of Q.
__device__ __forceinline__ void lds_reunit(double2* M, double2* P, int n, double dr, double di) {
    const int lane = threadIdx.x;
    const bool own = lane < n;
    // n <= 32.  Above n = 8 the two halves of the wavefront share each sum,
    // lane q and lane q + 32 taking half of its terms each (below, the
    // exchange costs more than it saves and the lower half does it all).
    const bool split = n > 8;
    const int q = lane & 31, half = lane >> 5;
    const int m0 = split ? n / 2 : n;                    // columns of the lower half
    const int cbeg = half ? m0 : 0, clen = half ? n - m0 : m0;
    // |r_i|^2, the same value on every lane
    auto row_norm2 = [&](int i) {
        double s = 0.0;
        if (own) s = fmadd(M[i * n + lane].y, M[i * n + lane].y, M[i * n + lane].x * M[i * n + lane].x);
        return wave_sum(s);
    };
    // one classical pass: r_i -= sum_{k < i} <r_k, r_i> r_k
    auto project = [&](int i) {
        // p_q = <r_q, r_i> for q < i; columns taken from a lane-dependent
        // start within the half's range, so lanes hit different banks
        double pr = 0.0, pi = 0.0;
        if (q < i && clen > 0) {
            int t = q % clen;
#pragma unroll 4
            for (int u = 0; u < clen; ++u) {
                const int c = cbeg + t;
                const double2 a = M[q * n + c], b = M[i * n + c];
                cmac(pr, pi, a.x, -a.y, b.x, b.y);
                t = (t + 1 == clen) ? 0 : t + 1;
            }
        }
        if (split) {
            pr += partner<5>(pr);
            pi += partner<5>(pi);
        }
        if (q < i && half == 0) P[q] = make_double2(pr, pi);
        wave_lds_order();
        // r_i -= sum_{k < i} p_k r_k, the k range split between the halves
        double sr = 0.0, si = 0.0;
        if (q < n) {
            const int kmid = split ? i / 2 : i;
            const int kb = half ? kmid : 0, ke = half ? i : kmid;
#pragma unroll 4
            for (int k = kb; k < ke; ++k) {
                const double2 p = P[k], a = M[k * n + q];
                cmac(sr, si, p.x, p.y, a.x, a.y);
            }
        }
        if (split) {
            sr += partner<5>(sr);
            si += partner<5>(si);
        }
        if (own) {
            const double2 b = M[i * n + lane];
            M[i * n + lane] = make_double2(b.x - sr, b.y - si);
        }
        wave_lds_order();
    };
    for (int i = 0; i < n; ++i) {
        double s2;
        if (i > 0) {
            // a second pass only where the first removed more than half of
            // the row's squared norm (the DGKS criterion, "twice is
            // enough"): a row of a nearly unitary link keeps almost all of
            // it, and its one pass is orthogonal to rounding already
            const double s0 = row_norm2(i);
            project(i);
            s2 = row_norm2(i);
            if (s2 < 0.5 * s0) {
                project(i);
                s2 = row_norm2(i);
            }
        } else {
            s2 = row_norm2(i);
        }
        const double inv = s2 >= DBL_MIN ? newton_rsqrt(s2) : rsqrt(s2);
        if (own) {
            M[i * n + lane].x *= inv;
            M[i * n + lane].y *= inv;
        }
        wave_lds_order();
    }
    const double mod = sqrt(dr * dr + di * di);
    const double cr = dr / mod, ci = -di / mod;
    if (own) {
        const double2 r = M[(n - 1) * n + lane];
        M[(n - 1) * n + lane] = make_double2(r.x * cr - r.y * ci, r.x * ci + r.y * cr);
    }
    __syncthreads();
}

// Link id in [0, 4V) -> (mu, parity, h), as the register kernels number them.
__device__ __forceinline__ void link_id(const Geom& g, int id, int& mu, int& par, int& h) {
    mu = id / g.V;
    const int rem = id - mu * g.V;
    par = rem >= g.Vh ? 1 : 0;
    h = rem - par * g.Vh;
}

// Re-unitarization of link blockIdx.x; with REPORT the deviation found before
// the projection goes to partial[2 id], [2 id + 1].  LDS: one FP64 matrix M
// and the n projections P.  The link is read twice: once for det M (the LU
// elimination destroys its copy), once for the Gram-Schmidt.
template <typename T, bool REPORT>
__device__ __forceinline__ void reunit_link_wide(T2<T>* __restrict__ U, const Geom& g, int n, int id,
                                                 double* __restrict__ partial) {
    extern __shared__ double4 smem_reunit[];
    const int n2 = n * n;
    double2* M = reinterpret_cast<double2*>(smem_reunit);
    double2* P = M + n2;
    int mu, par, h;
    link_id(g, id, mu, par, h);
    double du = 0.0, dd = 0.0;
    if ((g.present >> mu) & 1) {
        const T2<T>* src = link_at<T>(U, n2, mu, par, h, g.Vh);
        lds_load<double, T>(M, src, n, false);
        __syncthreads();
        if (REPORT) du = lds_unitarity_dev(M, n);
        __syncthreads();
        double dr, di;
        lds_det(M, n, dr, di);
        if (REPORT) dd = nan_to_inf(sqrt(fmadd(di, di, (dr - 1.0) * (dr - 1.0))));
        __syncthreads();
        lds_load<double, T>(M, src, n, false);
        __syncthreads();
        lds_reunit(M, P, n, dr, di);
        T2<T>* dst = const_cast<T2<T>*>(src);
        for (int e = threadIdx.x; e < n2; e += kLanes) dst[e] = cpx<T>((T)M[e].x, (T)M[e].y);
    }
    if (REPORT && threadIdx.x == 0) {
        partial[2 * (size_t)id] = du;
        partial[2 * (size_t)id + 1] = dd;
    }
}

template <typename T, bool REPORT>
__global__ __launch_bounds__(kLanes) void k_reunit(T2<T>* __restrict__ U, Geom g, int n,
                                                   double* __restrict__ partial) {
    reunit_link_wide<T, REPORT>(U, g, n, (int)blockIdx.x, partial);
}

// Re-unitarization of every chain of a batch group: one workgroup per link
// (TILE_LINK counts links here).
template <typename T>
__global__ __launch_bounds__(kLanes) void k_reunit_batch(const ChainDesc* __restrict__ d, int nchains, int n) {
    const int c = find_chain<TILE_LINK>(d, nchains, (int)blockIdx.x);
    reunit_link_wide<T, false>((T2<T>*)d[c].links, d[c].g, n, (int)blockIdx.x - d[c].tile0[TILE_LINK], nullptr);
}

template <typename T>
__global__ __launch_bounds__(kLanes) void k_unitarity(const T2<T>* __restrict__ U, Geom g, int n,
                                                      double* __restrict__ partial) {
    extern __shared__ double4 smem_unit[];
    const int n2 = n * n;
    double2* M = reinterpret_cast<double2*>(smem_unit);
    const int id = blockIdx.x;
    int mu, par, h;
    link_id(g, id, mu, par, h);
    double du = 0.0, dd = 0.0;
    if ((g.present >> mu) & 1) {
        lds_load<double, T>(M, link_at<T>(U, n2, mu, par, h, g.Vh), n, false);
        __syncthreads();
        du = lds_unitarity_dev(M, n);
        __syncthreads();
        double dr, di;
        lds_det(M, n, dr, di);
        dd = nan_to_inf(sqrt(fmadd(di, di, (dr - 1.0) * (dr - 1.0))));
    }
    if (threadIdx.x == 0) {
        partial[2 * (size_t)id] = du;
        partial[2 * (size_t)id + 1] = dd;
    }
}

// Start configuration of link blockIdx.x: identity, or a Haar draw (Gaussian
// entries from Box-Muller on the same Philox counters as the register
// kernels, then re-unitarization).  LDS: M, D (a copy for the determinant,
// then the projections).
template <typename T>
__global__ __launch_bounds__(kLanes) void k_init(T2<T>* __restrict__ U, Geom g, int n, int hot, uint32_t k0,
                                                 uint32_t k1) {
    extern __shared__ double4 smem_init[];
    const int n2 = n * n;
    double2* M = reinterpret_cast<double2*>(smem_init);
    double2* D = M + n2;
    const int id = blockIdx.x;
    int mu, par, h;
    link_id(g, id, mu, par, h);
    if (hot && ((g.present >> mu) & 1)) {
        const uint32_t s = (uint32_t)site_of(g, par, h).s;
        // call q gives the Gaussians of entries 2q and 2q + 1
        for (int q = threadIdx.x; 2 * q < n2; q += kLanes) {
            const U4 r = philox(s, 0xFFFFFFFFu, (uint32_t)mu << 16, (RNG_HOTSTART << 24) | (uint32_t)q, k0, k1);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const double rad = sqrt(-2.0 * log(uniform<double>(r.w[2 * p])));
                const double ang = Const<double>::two_pi * uniform<double>(r.w[2 * p + 1]);
                if (2 * q + p < n2) M[2 * q + p] = make_double2(rad * cos(ang), rad * sin(ang));
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n2; e += kLanes) D[e] = M[e];
        __syncthreads();
        double dr, di;
        lds_det(D, n, dr, di);
        __syncthreads();
        lds_reunit(M, D, n, dr, di);
    } else {
        for (int e = threadIdx.x; e < n2; e += kLanes) {
            const int i = e / n;
            M[e] = make_double2(i * n + i == e ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
    }
    T2<T>* dst = const_cast<T2<T>*>(link_at<T>(U, n2, mu, par, h, g.Vh));
    for (int e = threadIdx.x; e < n2; e += kLanes) dst[e] = cpx<T>((T)M[e].x, (T)M[e].y);
}

// Plaquettes of site blockIdx.x (logical order): partial[2 s] = sum over the
// planes without direction 3, partial[2 s + 1] = with direction 3, FP64.
// ReTr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag) = Re sum_ij A_ij conj(B_ij)
// with A = U_mu(x) U_nu(x+mu), B = U_nu(x) U_mu(x+nu).  LDS: A, X, Y.
template <typename T>
__device__ __forceinline__ void plaquette_site_wide(const T2<T>* __restrict__ U, const Geom& g, int n, int s,
                                                    double* __restrict__ partial) {
    extern __shared__ double4 smem_plaq[];
    const int n2 = n * n;
    double2* A = reinterpret_cast<double2*>(smem_plaq);
    double2* X = A + n2;
    double2* Y = X + n2;
    Site x;
    {
        int r = s;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = r / g.L[m];
            x.x[m] = r - q * g.L[m];
            r = q;
        }
        x.s = s;
    }
    const int par = parity_of(x), op = par ^ 1, h = s >> 1;
    double acc[2] = {0.0, 0.0};
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            if (!((g.present >> mu) & 1) || !((g.present >> nu) & 1)) continue;
            const Site xm = step_up(g, x, mu), xn = step_up(g, x, nu);
            lds_load<double, T>(X, link_at<T>(U, n2, mu, par, h, g.Vh), n, false);
            lds_load<double, T>(Y, link_at<T>(U, n2, nu, op, xm.s >> 1, g.Vh), n, false);
            __syncthreads();
            lds_mm<double>(A, X, Y, n, false);
            __syncthreads();
            lds_load<double, T>(X, link_at<T>(U, n2, nu, par, h, g.Vh), n, false);
            lds_load<double, T>(Y, link_at<T>(U, n2, mu, op, xn.s >> 1, g.Vh), n, false);
            __syncthreads();
            double t = 0.0;
            for (int e = threadIdx.x; e < n2; e += kLanes) {
                const int i = e / n, j = e - i * n;
                double br = 0.0, bi = 0.0;
                for (int k = 0; k < n; ++k) {
                    const double2 a = X[i * n + k], b = Y[k * n + j];
                    cmac(br, bi, a.x, a.y, b.x, b.y);
                }
                t = fmadd(A[e].y, bi, fmadd(A[e].x, br, t));
            }
            acc[nu == 3 ? 1 : 0] += wave_sum(t);
            __syncthreads();
        }
    if (threadIdx.x == 0) {
        partial[2 * (size_t)s] = acc[0];
        partial[2 * (size_t)s + 1] = acc[1];
    }
}

template <typename T>
__global__ __launch_bounds__(kLanes) void k_plaquette(const T2<T>* __restrict__ U, Geom g, int n,
                                                      double* __restrict__ partial) {
    plaquette_site_wide<T>(U, g, n, (int)blockIdx.x, partial);
}

// Plaquette sums of every chain of a batch group: one workgroup per site
// (TILE_SITE counts sites here), the partials in each chain's own scratch at
// the index the single-lattice kernel uses.
template <typename T>
__global__ __launch_bounds__(kLanes) void k_plaquette_batch(const ChainDesc* __restrict__ d, int nchains, int n) {
    const int c = find_chain<TILE_SITE>(d, nchains, (int)blockIdx.x);
    plaquette_site_wide<T>((const T2<T>*)d[c].links, d[c].g, n, (int)blockIdx.x - d[c].tile0[TILE_SITE],
                           d[c].scratch);
}

// One block per chain: out[3 c .. 3 c + 2] from its V site partials.
template <int Dummy = 0>
__global__ __launch_bounds__(kBlock) void k_plaquette_final_batch_wide(const ChainDesc* __restrict__ d, int nchains,
                                                                       int n, double* __restrict__ out) {
    const int c = blockIdx.x;
    if (c >= nchains) return;
    int n_sp = 0, n_tm = 0;
    for (int m = 0; m < 4; ++m)
        for (int k = m + 1; k < 4; ++k)
            if (((d[c].g.present >> m) & 1) && ((d[c].g.present >> k) & 1)) (k == 3 ? n_tm : n_sp)++;
    const double norm = (double)n * (double)d[c].g.V;
    plaquette_final<2>(d[c].scratch, d[c].g.V, out + 3 * (size_t)d[c].out_index, norm * n_sp, norm * n_tm,
                       norm * (n_sp + n_tm));
}

// Polyakov loop at spatial site blockIdx.x: Tr prod_t U_3(x, t), FP64.
// LDS: P, X, Tm.
template <typename T>
__global__ __launch_bounds__(kLanes) void k_polyakov(const T2<T>* __restrict__ U, Geom g, int n,
                                                     double* __restrict__ partial) {
    extern __shared__ double4 smem_poly[];
    const int n2 = n * n;
    double2* P = reinterpret_cast<double2*>(smem_poly);
    double2* X = P + n2;
    double2* Tm = X + n2;
    const int xs = blockIdx.x;
    const int Vs = g.V / g.L[3];
    for (int e = threadIdx.x; e < n2; e += kLanes) {
        const int i = e / n;
        P[e] = make_double2(i * n + i == e ? 1.0 : 0.0, 0.0);
    }
    for (int t = 0; t < g.L[3]; ++t) {
        const int s = xs + t * Vs;
        Site st;
        int r = s;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = r / g.L[m];
            st.x[m] = r - q * g.L[m];
            r = q;
        }
        st.s = s;
        lds_load<double, T>(X, link_at<T>(U, n2, 3, parity_of(st), s >> 1, g.Vh), n, false);
        __syncthreads();
        lds_mm<double>(Tm, P, X, n, false);
        __syncthreads();
        double2* tmp = P;
        P = Tm;
        Tm = tmp;
    }
    double tr = 0.0, ti = 0.0;
    for (int i = threadIdx.x; i < n; i += kLanes) {
        tr += P[i * n + i].x;
        ti += P[i * n + i].y;
    }
    tr = wave_sum(tr);
    ti = wave_sum(ti);
    if (threadIdx.x == 0) {
        partial[2 * (size_t)xs] = tr;
        partial[2 * (size_t)xs + 1] = ti;
    }
}

// Canonical FP64 field [mu][s][i][j] (re, im) <-> link-major storage; one
// work-item per complex entry.
template <typename T>
__global__ __launch_bounds__(256) void k_export(const T2<T>* __restrict__ U, Geom g, int n,
                                                double* __restrict__ out) {
    const int n2 = n * n;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= 4LL * g.V * n2) return;
    const int id = (int)(idx / n2), e = (int)(idx - (long long)id * n2);
    int mu, par, h;
    link_id(g, id, mu, par, h);
    const int s = site_of(g, par, h).s;
    const T2<T> v = link_at<T>(U, n2, mu, par, h, g.Vh)[e];
    double* o = out + (((size_t)mu * g.V + s) * n2 + e) * 2;
    o[0] = (double)v.x;
    o[1] = (double)v.y;
}

template <typename T>
__global__ __launch_bounds__(256) void k_import(T2<T>* __restrict__ U, Geom g, int n, const double* __restrict__ in) {
    const int n2 = n * n;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= 4LL * g.V * n2) return;
    const int id = (int)(idx / n2), e = (int)(idx - (long long)id * n2);
    int mu, par, h;
    link_id(g, id, mu, par, h);
    const int s = site_of(g, par, h).s;
    const double* p = in + (((size_t)mu * g.V + s) * n2 + e) * 2;
    T2<T>* dst = const_cast<T2<T>*>(link_at<T>(U, n2, mu, par, h, g.Vh));
    dst[e] = cpx<T>((T)p[0], (T)p[1]);
}

// ---------------------------------------------------------------------------
// The batched SU(2) draw alone, for parity tests: element i is subgroup
// mu_sg + (i mod 8) of site i / 8, drawn as the update draws it (one batch
// per site, the slots in order).  dev_x gets 4n doubles, attempts n ints
// (the accepted attempt's number, 0 when all were rejected).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kLanes) void k_sample_su2_batched(const double* __restrict__ alpha, int n, uint32_t k0,
                                                               uint32_t k1, uint32_t step, uint32_t mu_sg,
                                                               double* __restrict__ x, int* __restrict__ attempts) {
    const uint32_t site = blockIdx.x;
    const DrawBatch<T> b = draw_batch<T>(k0, k1, site, step, 0u, mu_sg, threadIdx.x);
    for (int s = 0; s < kSgBatch; ++s) {
        const int i = (int)site * kSgBatch + s;
        if (i >= n) break;
        Quat<T> q{{T(1), T(0), T(0), T(0)}};
        const int a = sample_su2_lanes<T>((T)alpha[i], b, s, k0, k1, site, step, mu_sg + (uint32_t)s, q);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[4 * (size_t)i + c] = q.q[c];
            attempts[i] = a;
        }
    }
}

}  // namespace wide
}  // namespace sun
