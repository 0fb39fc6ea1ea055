// sun_kernels.hpp -- the gfx950 kernels of the SU(Nc) checkerboard sweep.
//
// One work-item per updated link; a phase launch covers the V/2 links
// U_mu(x) of one parity.  Every kernel is templated on (Nc, storage type);
// the update kernel also on the update kind and on mu, so that all neighbour
// arithmetic and register-array indices are compile-time constants.
#pragma once

#include "sun_device.hpp"

namespace sun {

constexpr int kBlock = 256;  // 4 wave64 per workgroup
static_assert(kBlock == 256, "plaquette_tiles counts 256-item workgroups");
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed butterfly inside a wave64, then the
// waves in order).  Every thread of the block must call them.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out) {
    __shared__ double red[kWaves][K];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < K; ++c) red[wave][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < K; ++c) {
            double s = red[0][c];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) s += red[w][c];
            out[c] = s;
        }
}

template <int K>
__device__ __forceinline__ void block_max(double (&v)[K], double* out) {
    __shared__ double red[kWaves][K];
#pragma unroll
    for (int c = 0; c < K; ++c)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] = fmax(v[c], __shfl_xor(v[c], off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < K; ++c) red[wave][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < K; ++c) {
            double s = red[0][c];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) s = fmax(s, red[w][c]);
            out[c] = s;
        }
}

// Second pass: one block folds nblk partial records of K doubles, each
// thread a fixed strided subset in order, then the block tree.
template <int K, bool MAX>
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partial, int nblk,
                                                     double* __restrict__ out, double s0, double s1,
                                                     double s2) {
    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = 0.0;
    // unrolled so that the loads of several records are in flight at once;
    // the fold order (and so the result) is that of the plain loop
#pragma unroll 8
    for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] = MAX ? fmax(v[c], partial[(size_t)b * K + c]) : v[c] + partial[(size_t)b * K + c];
    __shared__ double res[K];
    if (MAX)
        block_max<K>(v, res);
    else
        block_sum<K>(v, res);
    if (threadIdx.x == 0) {
        const double sc[3] = {s0, s1, s2};
#pragma unroll
        for (int c = 0; c < K; ++c) out[c] = res[c] * sc[c < 3 ? c : 2];
    }
}

// Watchdog pass over nblk partial records {max |U^dag U - 1|, max |det U - 1|}
// (NaN entries already turned into infinities): when either maximum exceeds
// threshold the check counts as tripped, state[0] += 1 and state[1] keeps the
// largest deviation a tripped check saw; state[2] is this check's deviation.
template <int Dummy = 0>
__global__ __launch_bounds__(kBlock) void k_watchdog(const double* __restrict__ partial, int nblk, double threshold,
                                                     double* __restrict__ state) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += kBlock)
        v[0] = fmax(v[0], fmax(partial[2 * (size_t)b], partial[2 * (size_t)b + 1]));
    __shared__ double res[1];
    block_max<1>(v, res);
    if (threadIdx.x == 0) {
        const double d = res[0];
        state[2] = d;
        if (d > threshold) {
            state[0] += 1.0;
            state[1] = fmax(state[1], d);
        }
    }
}

// p[0 .. n) = v (a kernel rather than a memset, so that captured graphs hold
// no memset nodes).
template <int Dummy = 0>
__global__ void k_fill(double* __restrict__ p, int n, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Staple (paper Sec. 2), closing orientation: for nu != mu
//   U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
// so that ReTr(U_mu(x) A) is the sum of the plaquettes containing the link.
// ---------------------------------------------------------------------------
// One direction's two staples, added to A.  The direction is a template
// parameter so that the whole staple is straight-line code: neighbour
// coordinates and plane offsets are compile-time, and the scheduler can issue
// the loads of later directions ahead of the arithmetic of earlier ones.
//
// For SU(3) in FP64 each staple term is itself in SU(3), so only its rows 0
// and 1 are formed by products and row 2 is conj(row0 x row1); the leading
// factor then needs only its rows 0 and 1 (upper staple) or its columns 0 and
// 1 (lower staple), about a tenth of the update's arithmetic.  The identity
// holds only for unitary factors: for factors off SU(3) by a unitarity
// deviation delta the rebuilt row is off by 1.2 delta typically and 4 delta
// at most, which FP64 links (delta ~ 1e-15 between re-unitarizations) never
// notice.  FP32 links drift to delta ~ 1e-5 across a sweep, the size of the
// comparison tolerance itself, so FP32 forms every term by full products
// (2.8% of the two-row step, 9% of the 18-real one).
template <int N, typename T, int R, int MU, int NU>
__device__ __forceinline__ void staple_dir(Mat<N, T>& A, const T2<T>* __restrict__ U, const Geom& g, const Site& x,
                                           const Site& xp, int par, int h) {
    if constexpr (NU != MU) {
        if (!((g.present >> NU) & 1)) return;
        const int op = par ^ 1;
        const Site xpn = step_up(g, x, NU);
        const Site xmn = step_down(g, x, NU);
        const Site xpmn = step_down(g, xp, NU);
        if constexpr (N == 3 && sizeof(T) == 8) {
            // upper: rows 0, 1 of U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
            const Mat<3, T> t = mul_nd_rows2(load_rows01<T, R>(U, NU, op, xp.s >> 1, g.Vh),
                                             load_mat<3, T, R>(U, MU, op, xpn.s >> 1, g.Vh));
            Mat<3, T> su = mul_nd_rows2(t, load_mat<3, T, R>(U, NU, par, h, g.Vh));
            third_row(su);
            add_to(A, su);
            // lower: rows 0, 1 of (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu), from
            // columns 0, 1 of the product in parentheses
            const Mat<3, T> l = mul_nn_cols2(load_mat<3, T, R>(U, MU, op, xmn.s >> 1, g.Vh),
                                             load_cols01<T, R>(U, NU, par, xpmn.s >> 1, g.Vh));
            Mat<3, T> sd = mul_dn_rows2(l, load_mat<3, T, R>(U, NU, op, xmn.s >> 1, g.Vh));
            third_row(sd);
            add_to(A, sd);
        } else {
            const Mat<N, T> m = mul_nd(load_mat<N, T, R>(U, NU, op, xp.s >> 1, g.Vh),
                                       load_mat<N, T, R>(U, MU, op, xpn.s >> 1, g.Vh));
            add_mul_nd(A, m, load_mat<N, T, R>(U, NU, par, h, g.Vh));
            const Mat<N, T> l = mul_nn(load_mat<N, T, R>(U, MU, op, xmn.s >> 1, g.Vh),
                                       load_mat<N, T, R>(U, NU, par, xpmn.s >> 1, g.Vh));
            add_mul_dn(A, l, load_mat<N, T, R>(U, NU, op, xmn.s >> 1, g.Vh));
        }
    }
}

template <int N, typename T, int R, int MU>
__device__ __forceinline__ Mat<N, T> staple(const T2<T>* __restrict__ U, const Geom& g, const Site& x, int par,
                                            int h) {
    const Site xp = step_up(g, x, MU);
    Mat<N, T> A;
    set_zero(A);
    staple_dir<N, T, R, MU, 0>(A, U, g, x, xp, par, h);
    staple_dir<N, T, R, MU, 1>(A, U, g, x, xp, par, h);
    staple_dir<N, T, R, MU, 2>(A, U, g, x, xp, par, h);
    staple_dir<N, T, R, MU, 3>(A, U, g, x, xp, par, h);
    return A;
}

template <typename T, int MU, int NU>
__device__ __forceinline__ void staple_dir_su2(Quat<T>& A, const T2<T>* __restrict__ U, const Geom& g, const Site& x,
                                               const Site& xp, int par, int h) {
    if constexpr (NU != MU) {
        if (!((g.present >> NU) & 1)) return;
        const int op = par ^ 1;
        const Site xpn = step_up(g, x, NU);
        const Site xmn = step_down(g, x, NU);
        const Site xpmn = step_down(g, xp, NU);
        const Quat<T> m = qmul(load_quat<T>(U, NU, op, xp.s >> 1, g.Vh), qconj(load_quat<T>(U, MU, op, xpn.s >> 1, g.Vh)));
        qadd(A, qmul(m, qconj(load_quat<T>(U, NU, par, h, g.Vh))));
        const Quat<T> l = qmul(load_quat<T>(U, MU, op, xmn.s >> 1, g.Vh), load_quat<T>(U, NU, par, xpmn.s >> 1, g.Vh));
        qadd(A, qmul(qconj(l), load_quat<T>(U, NU, op, xmn.s >> 1, g.Vh)));
    }
}

template <typename T, int MU>
__device__ __forceinline__ Quat<T> staple_su2(const T2<T>* __restrict__ U, const Geom& g, const Site& x, int par,
                                              int h) {
    const Site xp = step_up(g, x, MU);
    Quat<T> A{{T(0), T(0), T(0), T(0)}};
    staple_dir_su2<T, MU, 0>(A, U, g, x, xp, par, h);
    staple_dir_su2<T, MU, 1>(A, U, g, x, xp, par, h);
    staple_dir_su2<T, MU, 2>(A, U, g, x, xp, par, h);
    staple_dir_su2<T, MU, 3>(A, U, g, x, xp, par, h);
    return A;
}

// Normalised subgroup direction V = P / |P| (identity when P = 0); returns k.
template <typename T>
__device__ __forceinline__ T unit_quat(const Quat<T>& p, Quat<T>& v) {
    const T k2 = p.q[0] * p.q[0] + p.q[1] * p.q[1] + p.q[2] * p.q[2] + p.q[3] * p.q[3];
    if constexpr (sizeof(T) == 4) {
        // FP32: the hardware reciprocal square root (about 1 ulp)
        if (k2 >= 1.17549435e-38f) {
            const float r = __builtin_amdgcn_rsqf(k2);
#pragma unroll
            for (int c = 0; c < 4; ++c) v.q[c] = p.q[c] * r;
            return k2 * r;
        }
    }
    const T k = k2 > T(0) ? d_sqrt(k2) : T(0);
    if (k > T(0)) {
        const T inv = T(1) / k;
#pragma unroll
        for (int c = 0; c < 4; ++c) v.q[c] = p.q[c] * inv;
    } else {
        v = Quat<T>{{T(1), T(0), T(0), T(0)}};
    }
    return k;
}

// ---------------------------------------------------------------------------
// Update of one link U_mu(x), x = site h of parity par, Nc >= 3 (paper Sec. 2,
// Cabibbo-Marinari steps 1-5, and the subgroup overrelaxation).  W = U A is
// kept in registers and updated with U.  Shared by the single-lattice and the
// batched kernels, so a chain gives the same bits either way.
// ---------------------------------------------------------------------------
template <int N, typename T, int R, bool HB, int MU, bool NT>
__device__ __forceinline__ void update_link(T2<T>* __restrict__ U, const Geom& g, int par, int h, T beta,
                                            uint32_t k0, uint32_t k1, uint32_t step) {
    const Site x = site_of(g, par, h);
    const Mat<N, T> A = staple<N, T, R, MU>(U, g, x, par, h);
    Mat<N, T> Ul = NT ? load_mat_stream<N, T, R>(U, MU, par, h, g.Vh) : load_mat<N, T, R>(U, MU, par, h, g.Vh);
    Mat<N, T> W = mul_nn(Ul, A);
    const T cb = T(2) * beta / T(N);  // alpha = 2 beta k / N
    int sg = 0;
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = i + 1; j < N; ++j, ++sg) {
            Quat<T> v;
            const T k = unit_quat(block_quat(W, i, j), v);
            Quat<T> a;
            if (HB) {
                const T alpha = cb * k;
                Quat<T> xs;
                if (!sample_su2<T>(alpha, k0, k1, (uint32_t)x.s, step, ((uint32_t)MU << 16) | (uint32_t)sg, xs))
                    continue;
                a = qmul(xs, qconj(v));
            } else {
                const Quat<T> vc = qconj(v);
                a = qmul(vc, vc);
            }
            rows_left_mul(Ul, i, j, a);
            rows_left_mul(W, i, j, a);
        }
    if constexpr (NT)
        store_mat_stream<N, T, R>(U, MU, par, h, g.Vh, Ul);
    else
        store_mat<N, T, R>(U, MU, par, h, g.Vh, Ul);
}

// The same for SU(2) in the 4-real parameterization (paper Sec. 2, Sec. 3).
template <typename T, bool HB, int MU, bool NT>
__device__ __forceinline__ void update_link_su2(T2<T>* __restrict__ U, const Geom& g, int par, int h, T beta,
                                                uint32_t k0, uint32_t k1, uint32_t step) {
    const Site x = site_of(g, par, h);
    const Quat<T> A = staple_su2<T, MU>(U, g, x, par, h);
    const Quat<T> u = NT ? load_quat_stream<T>(U, MU, par, h, g.Vh) : load_quat<T>(U, MU, par, h, g.Vh);
    Quat<T> v;
    const T k = unit_quat(qmul(u, A), v);
    Quat<T> a;
    if (HB) {
        Quat<T> xs;
        if (!sample_su2<T>(beta * k, k0, k1, (uint32_t)x.s, step, (uint32_t)MU << 16, xs)) return;
        a = qmul(xs, qconj(v));
    } else {
        const Quat<T> vc = qconj(v);
        a = qmul(vc, vc);
    }
    if constexpr (NT)
        store_quat_stream<T>(U, MU, par, h, g.Vh, qmul(a, u));
    else
        store_quat<T>(U, MU, par, h, g.Vh, qmul(a, u));
}

// NT: nontemporal access to the updated link, for a field larger than the
// Infinity Cache (the link is then not re-read soon enough to stay cached);
// a field that fits keeps it cached for the next phase, which reads it.  A
// compile-time choice: as a run-time branch it kept the plain loads from
// being scheduled early.
template <int N, typename T, int R, bool HB, int MU, bool NT>
__device__ __forceinline__ void update_any(T2<T>* __restrict__ U, const Geom& g, int par, int h, T beta, uint32_t k0,
                                           uint32_t k1, uint32_t step) {
    if constexpr (N == 2)
        update_link_su2<T, HB, MU, NT>(U, g, par, h, beta, k0, k1, step);
    else
        update_link<N, T, R, HB, MU, NT>(U, g, par, h, beta, k0, k1, step);
}

// One checkerboard phase of one lattice, BS work-items per workgroup; xcd
// selects the XCD-aware workgroup order (a tuning choice that never changes
// results: every link is computed by the same code whichever work-item runs it).
//
// Occupancy cap.  A phase touches far more data per XCD than its 4 MB L2
// holds; fewer resident waves shrink the in-flight footprint and raise the
// L2 hit rate (measured on 32^4 SU(3): 8 waves per CU beat 20).  The cap is
// set by the dynamic LDS size a launch requests, which the dispatcher
// reserves per workgroup; the kernels never touch it (a reference to a
// dynamic LDS array costs them a scratch spill).

// Grid: ceil(nblk / walk.spt) workgroups over nblk tiles of BS sites; a
// workgroup takes walk positions blockIdx.x + r gridDim.x, r < walk.spt, in
// turn (r apart by a multiple of 8 when the grid is, so they stay on one XCD).
template <int N, typename T, int R, bool HB, int MU, int BS, bool NT>
__global__ __launch_bounds__(BS) void k_update(T2<T>* __restrict__ U, Geom g, int par, T beta, uint32_t k0,
                                               uint32_t k1, uint32_t step, Walk walk, int nblk) {
    for (int r = 0; r < walk.spt; ++r) {
        const int b = (int)blockIdx.x + r * (int)gridDim.x;
        if (b >= nblk) break;
        const int h = walk_tile(b, nblk, walk) * BS + threadIdx.x;
        if (h < g.Vh) update_any<N, T, R, HB, MU, NT>(U, g, par, h, beta, k0, k1, step);
    }
}

// ---------------------------------------------------------------------------
// Batches of independent chains (same Nc and storage type, any extents,
// couplings and seeds).  One launch covers one phase of every chain: the
// grid is the concatenation of each chain's tiles, and the chain of a tile is
// found by binary search over the first-tile prefix of the descriptor table.
// The RNG step counter of each chain lives in the table, so a captured graph
// replays with fresh randomness.
// ---------------------------------------------------------------------------


template <int KIND>
__device__ __forceinline__ int find_chain(const ChainDesc* __restrict__ d, int n, int tile) {
    int lo = 0, hi = n - 1;  // last chain whose first tile <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0[KIND] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Batched phase: tile0[TILE_HALF_HB / _OR] counts tiles of BS work-items.
// Grid: ceil(tiles / spt) workgroups; workgroup b takes tiles b + r gridDim.x,
// r < spt, in turn.
template <int N, typename T, int R, bool HB, int MU, int BS>
__global__ __launch_bounds__(BS) void k_update_batch(const ChainDesc* __restrict__ d, int n, int par,
                                                     uint32_t step_offset, int xcd, int tiles, int spt) {
    constexpr int KIND = HB ? TILE_HALF_HB : TILE_HALF_OR;
    for (int r = 0; r < spt; ++r) {
        const int b = (int)blockIdx.x + r * (int)gridDim.x;
        if (b >= tiles) break;
        const int tile = xcd ? xcd_tile(b, tiles) : b;
        const int c = find_chain<KIND>(d, n, tile);
        const Geom g = d[c].g;
        const int h = (tile - d[c].tile0[KIND]) * BS + threadIdx.x;
        if (h < g.Vh && ((g.present >> MU) & 1))
            update_any<N, T, R, HB, MU, false>((T2<T>*)d[c].links, g, par, h, (T)d[c].beta, d[c].k0, d[c].k1,
                                               (uint32_t)(d[c].step + step_offset));
    }
}

// Advances every chain's RNG step counter after a sweep of n_hb heatbath steps.
template <int Dummy = 0>
__global__ void k_advance_steps(ChainDesc* __restrict__ d, int n, int n_hb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) d[c].step += (uint64_t)n_hb;
}

// ---------------------------------------------------------------------------
// FP64 helpers for re-unitarization and diagnostics.
// ---------------------------------------------------------------------------
// STREAM selects nontemporal accesses (for kernels that touch each link once).
template <int N, typename T, int R, bool STREAM = false>
__device__ __forceinline__ Mat<N, double> load_link_f64(const T2<T>* __restrict__ U, int mu, int par, int h,
                                                        int Vh) {
    Mat<N, double> m;
    if constexpr (N == 2) {
        const Quat<T> q = STREAM ? load_quat_stream<T>(U, mu, par, h, Vh) : load_quat<T>(U, mu, par, h, Vh);
        m.re[0][0] = q.q[0];
        m.im[0][0] = q.q[3];
        m.re[0][1] = q.q[2];
        m.im[0][1] = q.q[1];
        m.re[1][0] = -(double)q.q[2];
        m.im[1][0] = q.q[1];
        m.re[1][1] = q.q[0];
        m.im[1][1] = -(double)q.q[3];
    } else {
        const Mat<N, T> t = STREAM ? load_mat_stream<N, T, R>(U, mu, par, h, Vh) : load_mat<N, T, R>(U, mu, par, h, Vh);
SUN_MAT_UNROLL
        for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
            for (int j = 0; j < N; ++j) {
                m.re[i][j] = t.re[i][j];
                m.im[i][j] = t.im[i][j];
            }
    }
    return m;
}

template <int N, typename T, int R, bool STREAM = false>
__device__ __forceinline__ void store_link_from_f64(T2<T>* __restrict__ U, int mu, int par, int h, int Vh,
                                                    const Mat<N, double>& m) {
    if constexpr (N == 2) {
        const Quat<T> q{{(T)m.re[0][0], (T)m.im[0][1], (T)m.re[0][1], (T)m.im[0][0]}};
        if (STREAM)
            store_quat_stream<T>(U, mu, par, h, Vh, q);
        else
            store_quat<T>(U, mu, par, h, Vh, q);
    } else {
        Mat<N, T> t;
SUN_MAT_UNROLL
        for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
            for (int j = 0; j < N; ++j) {
                t.re[i][j] = (T)m.re[i][j];
                t.im[i][j] = (T)m.im[i][j];
            }
        if (STREAM)
            store_mat_stream<N, T, R>(U, mu, par, h, Vh, t);
        else
            store_mat<N, T, R>(U, mu, par, h, Vh, t);
    }
}

// Determinant by Gaussian elimination with partial pivoting (row swaps done
// with selects so that every register index stays compile-time).
template <int N>
__device__ __forceinline__ void det_lu(Mat<N, double> m, double& dr, double& di) {
    dr = 1.0;
    di = 0.0;
SUN_MAT_UNROLL
    for (int col = 0; col < N; ++col) {
        int piv = col;
        double best = m.re[col][col] * m.re[col][col] + m.im[col][col] * m.im[col][col];
SUN_MAT_UNROLL
        for (int r = col + 1; r < N; ++r) {
            const double a = m.re[r][col] * m.re[r][col] + m.im[r][col] * m.im[r][col];
            if (a > best) {
                best = a;
                piv = r;
            }
        }
        if (best == 0.0) {
            dr = di = 0.0;
            return;
        }
SUN_MAT_UNROLL
        for (int r = col + 1; r < N; ++r) {
            const bool sw = (r == piv);
SUN_MAT_UNROLL
            for (int c = 0; c < N; ++c) {
                const double ar = m.re[col][c], ai = m.im[col][c], br = m.re[r][c], bi = m.im[r][c];
                m.re[col][c] = sw ? br : ar;
                m.im[col][c] = sw ? bi : ai;
                m.re[r][c] = sw ? ar : br;
                m.im[r][c] = sw ? ai : bi;
            }
        }
        if (piv != col) {
            dr = -dr;
            di = -di;
        }
        const double pr = m.re[col][col], pi = m.im[col][col];
        const double nr = dr * pr - di * pi, ni = dr * pi + di * pr;
        dr = nr;
        di = ni;
        const double inv = 1.0 / (pr * pr + pi * pi);
SUN_MAT_UNROLL
        for (int r = col + 1; r < N; ++r) {
            // f = m[r][col] / m[col][col]
            const double fr = (m.re[r][col] * pr + m.im[r][col] * pi) * inv;
            const double fi = (m.im[r][col] * pr - m.re[r][col] * pi) * inv;
SUN_MAT_UNROLL
            for (int c = col; c < N; ++c) {
                m.re[r][c] -= fr * m.re[col][c] - fi * m.im[col][c];
                m.im[r][c] -= fr * m.im[col][c] + fi * m.re[col][c];
            }
        }
    }
}

template <int N>
__device__ __forceinline__ void normalize_row(Mat<N, double>& M, int i) {
    double s = 0.0;
SUN_MAT_UNROLL
    for (int c = 0; c < N; ++c) s = fmadd(M.im[i][c], M.im[i][c], fmadd(M.re[i][c], M.re[i][c], s));
    const double inv = rsqrt(s);
SUN_MAT_UNROLL
    for (int c = 0; c < N; ++c) {
        M.re[i][c] *= inv;
        M.im[i][c] *= inv;
    }
}

// Re-unitarization (paper Sec. 2, last paragraph), FP64.
template <int N>
__device__ __forceinline__ void reunit(Mat<N, double>& M) {
    if constexpr (N == 2) {
        normalize_row<2>(M, 0);
        M.re[1][0] = -M.re[0][1];
        M.im[1][0] = M.im[0][1];
        M.re[1][1] = M.re[0][0];
        M.im[1][1] = -M.im[0][0];
        return;
    } else {
        constexpr int gs_rows = (N == 3) ? 2 : N;
SUN_MAT_UNROLL
        for (int i = 0; i < gs_rows; ++i) {
SUN_MAT_UNROLL
            for (int k = 0; k < i; ++k) {
                double pr = 0.0, pi = 0.0;  // <r_k, r_i> = sum conj(r_k) r_i
SUN_MAT_UNROLL
                for (int c = 0; c < N; ++c) cmac(pr, pi, M.re[k][c], -M.im[k][c], M.re[i][c], M.im[i][c]);
                // r_i -= <r_k, r_i> r_k
SUN_MAT_UNROLL
                for (int c = 0; c < N; ++c) cmac(M.re[i][c], M.im[i][c], -pr, -pi, M.re[k][c], M.im[k][c]);
            }
            normalize_row<N>(M, i);
        }
        if constexpr (N == 3) {
            third_row(M);  // row 2 = conj(row0 x row1)
        } else {
            double dr, di;
            det_lu<N>(M, dr, di);
            const double mod = sqrt(dr * dr + di * di);
            const double cr = dr / mod, ci = -di / mod;  // conj(det)/|det|
SUN_MAT_UNROLL
            for (int c = 0; c < N; ++c) {
                const double r = M.re[N - 1][c], i = M.im[N - 1][c];
                M.re[N - 1][c] = r * cr - i * ci;
                M.im[N - 1][c] = r * ci + i * cr;
            }
        }
    }
}

// det of a 3x3 matrix by cofactors of row 2.
__device__ __forceinline__ void det3(const Mat<3, double>& m, double& dr, double& di) {
    Mat<3, double> c = m;
    third_row(c);  // row 2 of c = conj(row0 x row1); det = sum_c m[2][c] (row0 x row1)_c
    dr = 0.0;
    di = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) cmac(dr, di, m.re[2][k], m.im[2][k], c.re[2][k], -c.im[2][k]);
}

// {max_ij |(U^dag U - 1)_ij|, |det U - 1|}.  U^dag U - 1 is Hermitian, so
// its upper triangle holds every modulus; the maximum is taken over squared
// moduli and rooted once.  A NaN entry makes both deviations infinite (fmax
// alone would drop it), so that every maximum over links reports it.
template <int N>
__device__ __forceinline__ void unitarity_dev(const Mat<N, double>& M, double& du, double& dd) {
    double du2 = 0.0;
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = i; j < N; ++j) {
            double r = (i == j) ? -1.0 : 0.0, m = 0.0;
SUN_MAT_UNROLL
            for (int k = 0; k < N; ++k) cmac(r, m, M.re[k][i], -M.im[k][i], M.re[k][j], M.im[k][j]);
            du2 = fmax(du2, nan_to_inf(fmadd(m, m, r * r)));
        }
    du = sqrt(du2);
    double dr, di;
    if constexpr (N == 3)
        det3(M, dr, di);
    else
        det_lu<N>(M, dr, di);
    dd = nan_to_inf(sqrt(fmadd(di, di, (dr - 1.0) * (dr - 1.0))));
}

// Link id in [0, 4V): mu-major, then parity, then checkerboard index.
struct LinkId {
    int mu, par, h;
};
__device__ __forceinline__ LinkId link_of(const Geom& g, int id) {
    LinkId l;
    l.mu = id / g.V;
    const int rem = id - l.mu * g.V;
    l.par = rem >= g.Vh ? 1 : 0;
    l.h = rem - l.par * g.Vh;
    return l;
}

// ---------------------------------------------------------------------------
// Re-unitarization of every link, optionally reporting the deviation found
// before the projection.
// ---------------------------------------------------------------------------
// REPORT is a template flag (not a runtime one) so that the projection
// compiles to the same instructions in every kernel that runs it: a chain in
// a batch must get the same bits as the chain alone.
template <int N, typename T, int R, bool REPORT>
__device__ __forceinline__ void reunit_link(T2<T>* __restrict__ U, const Geom& g, int id, double (&dev)[2],
                                            bool nt) {
    if (id >= 4 * g.V) return;
    const LinkId l = link_of(g, id);
    if (!((g.present >> l.mu) & 1)) return;
    Mat<N, double> M;
    if (nt)
        M = load_link_f64<N, T, R, true>(U, l.mu, l.par, l.h, g.Vh);
    else
        M = load_link_f64<N, T, R, false>(U, l.mu, l.par, l.h, g.Vh);
    if (REPORT) unitarity_dev<N>(M, dev[0], dev[1]);
    reunit<N>(M);
    if (nt)
        store_link_from_f64<N, T, R, true>(U, l.mu, l.par, l.h, g.Vh, M);
    else
        store_link_from_f64<N, T, R, false>(U, l.mu, l.par, l.h, g.Vh, M);
}

// nt as for the phase kernels.
template <int N, typename T, int R, bool REPORT>
__global__ __launch_bounds__(kBlock) void k_reunit(T2<T>* __restrict__ U, Geom g, double* __restrict__ partial,
                                                   int nt) {
    double dev[2] = {0.0, 0.0};
    reunit_link<N, T, R, REPORT>(U, g, blockIdx.x * kBlock + threadIdx.x, dev, nt != 0);
    if (REPORT) block_max<2>(dev, partial + 2 * (size_t)blockIdx.x);
}

template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_reunit_batch(const ChainDesc* __restrict__ d, int n) {
    const int tile = blockIdx.x;
    const int c = find_chain<TILE_LINK>(d, n, tile);
    double dev[2] = {0.0, 0.0};
    reunit_link<N, T, R, false>((T2<T>*)d[c].links, d[c].g, (tile - d[c].tile0[TILE_LINK]) * kBlock + threadIdx.x, dev,
                                false);
}

template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_unitarity(const T2<T>* __restrict__ U, Geom g,
                                                      double* __restrict__ partial) {
    const int id = blockIdx.x * kBlock + threadIdx.x;
    double dev[2] = {0.0, 0.0};
    if (id < 4 * g.V) {
        const LinkId l = link_of(g, id);
        if ((g.present >> l.mu) & 1) {
            const Mat<N, double> M = load_link_f64<N, T, R>(U, l.mu, l.par, l.h, g.Vh);
            unitarity_dev<N>(M, dev[0], dev[1]);
        }
    }
    block_max<2>(dev, partial + 2 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Plaquette (paper Sec. 2): P_mu_nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
// evaluated in FP64 from the stored links; per-block partial sums
// {spatial planes, planes with direction 3}.
// ---------------------------------------------------------------------------
template <int N, typename T, int R, int MU, int NU>
__device__ __forceinline__ double re_tr_plaq(const T2<T>* __restrict__ U, const Geom& g, const Site& x, int par,
                                             int h) {
    const Site xm = step_up(g, x, MU), xn = step_up(g, x, NU);
    const int op = par ^ 1;
    // ReTr(U_mu(x) U_nu(x+mu) [U_nu(x) U_mu(x+nu)]^dag): two independent
    // products, then sum_ij Re(a_ij conj(c_ij))
    const Mat<N, double> a = mul_nn(load_link_f64<N, T, R>(U, MU, par, h, g.Vh),
                                    load_link_f64<N, T, R>(U, NU, op, xm.s >> 1, g.Vh));
    const Mat<N, double> c = mul_nn(load_link_f64<N, T, R>(U, NU, par, h, g.Vh),
                                    load_link_f64<N, T, R>(U, MU, op, xn.s >> 1, g.Vh));
    double t = 0.0;
SUN_MAT_UNROLL
    for (int i = 0; i < N; ++i)
SUN_MAT_UNROLL
        for (int j = 0; j < N; ++j) t = fmadd(a.im[i][j], c.im[i][j], fmadd(a.re[i][j], c.re[i][j], t));
    return t;
}

// Tile q of the plaquette grid covers parity q & 1 of checkerboard tile
// walk(q >> 1): the two parities of one stretch of sites share their
// neighbour links, and the t-blocked walk (4 time slices, where a plane holds
// whole tiles) keeps the t-neighbours of a tile in L2.  The walk depends on
// the geometry alone, so a chain's plaquette has the same bits alone and in a
// batch.
__device__ __forceinline__ void plaquette_tile(const Geom& g, int q, int& par, int& h) {
    Walk w{0, 0, 1, 1, 0};
    const int plane_h = g.L[0] * g.L[1] / 2;
    if (plane_h % kBlock == 0 && g.L[3] % 4 == 0) {
        w.tb = 4;
        w.tpp = plane_h / kBlock;
        w.lz = g.L[2];
    }
    par = q & 1;
    h = walk_tile(q >> 1, plaquette_tiles(g) >> 1, w) * kBlock + (int)threadIdx.x;
}

// Sums ReTr P over the planes of site (par, h) into acc = {planes without
// direction 3, planes with direction 3}.
template <int N, typename T, int R>
__device__ __forceinline__ void plaquette_site(const T2<T>* __restrict__ U, const Geom& g, int par, int h,
                                               double (&acc)[2]) {
    if (h >= g.Vh) return;
    const Site x = site_of(g, par, h);
    const int p = g.present;
#define SUN_PLAQ(m, n, slot) \
    if (((p >> m) & 1) && ((p >> n) & 1)) acc[slot] += re_tr_plaq<N, T, R, m, n>(U, g, x, par, h);
    SUN_PLAQ(0, 1, 0)
    SUN_PLAQ(0, 2, 0)
    SUN_PLAQ(1, 2, 0)
    SUN_PLAQ(0, 3, 1)
    SUN_PLAQ(1, 3, 1)
    SUN_PLAQ(2, 3, 1)
#undef SUN_PLAQ
}

// Grid: plaquette_tiles(g) workgroups; partial[2 q .. 2 q + 1] per tile q.
template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_plaquette(const T2<T>* __restrict__ U, Geom g,
                                                      double* __restrict__ partial) {
    const int q = xcd_tile(blockIdx.x, gridDim.x);
    int par, h;
    plaquette_tile(g, q, par, h);
    double acc[2] = {0.0, 0.0};
    plaquette_site<N, T, R>(U, g, par, h, acc);
    block_sum<2>(acc, partial + 2 * (size_t)q);
}

// Batched plaquette: each chain's per-tile partials go to that chain's own
// scratch at the same index the single-lattice kernel uses.
template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_plaquette_batch(const ChainDesc* __restrict__ d, int n) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int c = find_chain<TILE_SITE>(d, n, tile);
    const int local = tile - d[c].tile0[TILE_SITE];
    int par, h;
    plaquette_tile(d[c].g, local, par, h);
    double acc[2] = {0.0, 0.0};
    plaquette_site<N, T, R>((const T2<T>*)d[c].links, d[c].g, par, h, acc);
    block_sum<2>(acc, d[c].scratch + 2 * (size_t)local);
}

// Second pass for the plaquette: {total, spatial, temporal} means.
template <int K = 2>
__device__ __forceinline__ void plaquette_final(const double* __restrict__ partial, int nblk, double* __restrict__ out,
                                                double norm_sp, double norm_tm, double norm_all) {
    double v[K] = {};
#pragma unroll 8
    for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] += partial[K * (size_t)b + c];
    __shared__ double res[K];
    block_sum<K>(v, res);
    if (threadIdx.x == 0) {
        out[0] = norm_all > 0.0 ? (res[0] + res[1]) / norm_all : 0.0;
        out[1] = norm_sp > 0.0 ? res[0] / norm_sp : 0.0;
        out[2] = norm_tm > 0.0 ? res[1] / norm_tm : 0.0;
    }
}

template <int K = 2>
__global__ __launch_bounds__(kBlock) void k_plaquette_final(const double* __restrict__ partial, int nblk,
                                                            double* __restrict__ out, double norm_sp,
                                                            double norm_tm, double norm_all) {
    plaquette_final<K>(partial, nblk, out, norm_sp, norm_tm, norm_all);
}

// Normalisations {spatial, temporal, all}: Nc V times the number of planes.
template <int N>
__device__ __forceinline__ void plaquette_norms(const Geom& g, double& sp, double& tm, double& all) {
    int n_sp = 0, n_tm = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m + 1; n < 4; ++n)
            if (((g.present >> m) & 1) && ((g.present >> n) & 1)) {
                if (n == 3)
                    ++n_tm;
                else
                    ++n_sp;
            }
    const double norm = (double)N * (double)g.V;
    sp = norm * n_sp;
    tm = norm * n_tm;
    all = norm * (n_sp + n_tm);
}

// One block per chain: out[3 c .. 3 c + 2].
template <int N>
__global__ __launch_bounds__(kBlock) void k_plaquette_final_batch(const ChainDesc* __restrict__ d, int n,
                                                                  double* __restrict__ out) {
    const int c = blockIdx.x;
    if (c >= n) return;
    double sp, tm, all;
    plaquette_norms<N>(d[c].g, sp, tm, all);
    plaquette_final<2>(d[c].scratch, plaquette_tiles(d[c].g), out + 3 * (size_t)d[c].out_index, sp, tm, all);
}

// ---------------------------------------------------------------------------
// Polyakov loop along direction 3, FP64.
// ---------------------------------------------------------------------------
// Time segments per spatial site: the product along t is split into S
// consecutive stretches multiplied by S work-items, whose S partial products
// are then multiplied in order through LDS (FP64, 2 N^2 doubles per item).
template <int N>
constexpr int polyakov_segments() {
    return N <= 3 ? 8 : (N == 4 ? 4 : 1);
}
template <int N>
__host__ __device__ inline int polyakov_blocks(const Geom& g) {
    constexpr int sites = kBlock / polyakov_segments<N>();
    return (g.V / g.L[3] + sites - 1) / sites;
}

// Work-item (seg, j) of a workgroup multiplies U_3 along its time stretch at
// spatial site blockIdx.x * (kBlock / S) + j; lanes of one segment take
// consecutive spatial sites, so each load instruction reads consecutive links.
template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_polyakov(const T2<T>* __restrict__ U, Geom g,
                                                     double* __restrict__ partial) {
    constexpr int S = polyakov_segments<N>();
    constexpr int SITES = kBlock / S;
    const int seg = threadIdx.x / SITES, j = threadIdx.x - seg * SITES;
    const int xs = blockIdx.x * SITES + j;
    const int Vs = g.V / g.L[3];
    const bool live = xs < Vs;
    Mat<N, double> P;
    set_identity(P);
    const int t0 = seg * g.L[3] / S, t1 = (seg + 1) * g.L[3] / S;
    // link U_3 at time t of this spatial site
    auto time_link = [&](int t) {
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
        return load_link_f64<N, T, R>(U, 3, parity_of(st), s >> 1, g.Vh);
    };
    if (live && t1 > t0) {
        // the stretch's product, starting from its first link
        P = time_link(t0);
        for (int t = t0 + 1; t < t1; ++t) P = mul_nn(P, time_link(t));
    }
    double tr[2] = {0.0, 0.0};
    if constexpr (S > 1) {
        // ordered product of the S stretches as a tree: at level w, stretch
        // seg (a multiple of 2w) takes the product of seg + w on its right
        __shared__ double part[S][2 * N * N][SITES];
SUN_MAT_UNROLL
        for (int e = 0; e < N * N; ++e) {
            part[seg][2 * e][j] = P.re[e / N][e % N];
            part[seg][2 * e + 1][j] = P.im[e / N][e % N];
        }
        __syncthreads();
#pragma unroll
        for (int w = 1; w < S; w *= 2) {
            if (seg % (2 * w) == 0 && live) {
                Mat<N, double> Q;
SUN_MAT_UNROLL
                for (int e = 0; e < N * N; ++e) {
                    Q.re[e / N][e % N] = part[seg + w][2 * e][j];
                    Q.im[e / N][e % N] = part[seg + w][2 * e + 1][j];
                }
                P = mul_nn(P, Q);
SUN_MAT_UNROLL
                for (int e = 0; e < N * N; ++e) {
                    part[seg][2 * e][j] = P.re[e / N][e % N];
                    part[seg][2 * e + 1][j] = P.im[e / N][e % N];
                }
            }
            __syncthreads();
        }
    }
    if (seg == 0 && live) {
SUN_MAT_UNROLL
        for (int i = 0; i < N; ++i) {
            tr[0] += P.re[i][i];
            tr[1] += P.im[i][i];
        }
    }
    block_sum<2>(tr, partial + 2 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Start configuration (paper Sec. 3): identity, or Haar links from a complex
// Gaussian matrix (Box-Muller on Philox uniforms) re-unitarized in FP64.
// ---------------------------------------------------------------------------
template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_init(T2<T>* __restrict__ U, Geom g, int hot, uint32_t k0,
                                                 uint32_t k1) {
    const int id = blockIdx.x * kBlock + threadIdx.x;
    if (id >= 4 * g.V) return;
    const LinkId l = link_of(g, id);
    Mat<N, double> M;
    set_identity(M);
    if (hot && ((g.present >> l.mu) & 1)) {
        const int s = site_of(g, l.par, l.h).s;
        constexpr int rows_needed = (N == 2) ? 1 : N;  // SU(2): row 0 fixes the matrix
        constexpr int ncalls = (2 * N * rows_needed + 3) / 4;
        double gs[4 * ncalls];
#pragma unroll
        for (int call = 0; call < ncalls; ++call) {
            const U4 r = philox((uint32_t)s, 0xFFFFFFFFu, (uint32_t)l.mu << 16,
                                (RNG_HOTSTART << 24) | (uint32_t)call, k0, k1);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const double rad = sqrt(-2.0 * log(uniform<double>(r.w[2 * p])));
                const double ang = Const<double>::two_pi * uniform<double>(r.w[2 * p + 1]);
                gs[4 * call + 2 * p] = rad * cos(ang);
                gs[4 * call + 2 * p + 1] = rad * sin(ang);
            }
        }
SUN_MAT_UNROLL
        for (int e = 0; e < N * rows_needed; ++e) {
            M.re[e / N][e % N] = gs[2 * e];
            M.im[e / N][e % N] = gs[2 * e + 1];
        }
        reunit<N>(M);
    }
    store_link_from_f64<N, T, R>(U, l.mu, l.par, l.h, g.Vh, M);
}

// ---------------------------------------------------------------------------
// Canonical FP64 field <-> SoA storage.
// ---------------------------------------------------------------------------
template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_export(const T2<T>* __restrict__ U, Geom g, double* __restrict__ out) {
    const int id = blockIdx.x * kBlock + threadIdx.x;
    if (id >= 4 * g.V) return;
    const LinkId l = link_of(g, id);
    const int s = site_of(g, l.par, l.h).s;
    const Mat<N, double> M = load_link_f64<N, T, R>(U, l.mu, l.par, l.h, g.Vh);
    double* o = out + ((size_t)l.mu * g.V + s) * (2 * N * N);
SUN_MAT_UNROLL
    for (int e = 0; e < N * N; ++e) {
        o[2 * e] = M.re[e / N][e % N];
        o[2 * e + 1] = M.im[e / N][e % N];
    }
}

template <int N, typename T, int R>
__global__ __launch_bounds__(kBlock) void k_import(T2<T>* __restrict__ U, Geom g, const double* __restrict__ in) {
    const int id = blockIdx.x * kBlock + threadIdx.x;
    if (id >= 4 * g.V) return;
    const LinkId l = link_of(g, id);
    const int s = site_of(g, l.par, l.h).s;
    const double* p = in + ((size_t)l.mu * g.V + s) * (2 * N * N);
    Mat<N, double> M;
SUN_MAT_UNROLL
    for (int e = 0; e < N * N; ++e) {
        M.re[e / N][e % N] = p[2 * e];
        M.im[e / N][e % N] = p[2 * e + 1];
    }
    store_link_from_f64<N, T, R>(U, l.mu, l.par, l.h, g.Vh, M);
}

// ---------------------------------------------------------------------------
// The SU(2) draw alone, for distribution and parity tests.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sample_su2(const double* __restrict__ alpha, int n, uint32_t k0,
                                                       uint32_t k1, uint32_t step, uint32_t mu_sg,
                                                       double* __restrict__ x, int* __restrict__ attempts) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    Quat<T> q{{T(1), T(0), T(0), T(0)}};
    const int a = sample_su2<T>((T)alpha[i], k0, k1, (uint32_t)i, step, mu_sg, q);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[4 * (size_t)i + c] = q.q[c];
    attempts[i] = a;
}

}  // namespace sun
