/*
 * sun_oracle.c -- FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, obviously correct reference for the pure-gauge SU(Nc) sweep of
 * Cardoso & Bicudo (arXiv:1112.4533).  Every function names the passage of the
 * paper it follows.  Only tests, the smoke check and the benchmark's CPU
 * baseline may use this file; the HIP library never includes or links it.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - Staple orientation: the staple is the "closing" path, so that
 *    ReTr(U_mu(x) A_mu(x)) is the sum of the real traces of the 2(d-1)
 *    plaquettes that contain the link; the local weight is
 *    exp[(beta/Nc) ReTr(U A)] (Sec. 2, Wilson action and SU(2) heatbath
 *    distribution).  The product U A is what the Cabibbo-Marinari list calls
 *    "U Sigma^dagger".
 *  - SU(2) subgroup coupling: for subgroup (i,j) the 2x2 block w of W = U A is
 *    projected onto the quaternion (SU(2)-proportional) part P(w) = k V,
 *    k = sqrt(det P(w)); the subgroup element is drawn with weight
 *    exp(alpha x0), alpha = 2 beta k / Nc (for Nc = 2 this is beta k, Sec. 2).
 *  - a0 sampler: Creutz inversion for alpha < 1.7, Kennedy-Pendleton above;
 *    direction uniform on the 2-sphere via (cos theta, phi); after 64 rejected
 *    attempts the subgroup step is skipped (the link keeps its value).
 *  - Subgroups are visited in lexicographic (i,j) order for every Nc.
 *  - Re-unitarization (Sec. 2, last paragraph): Nc = 2 normalizes row 0 and
 *    rebuilds row 1; Nc = 3 Gram-Schmidt on rows 0,1 and row 2 =
 *    conj(r0 x r1); Nc > 3 Gram-Schmidt on all rows, then the last row is
 *    multiplied by conj(det)/|det|.
 *  - Hot start: a complex Gaussian matrix (Box-Muller on Philox uniforms)
 *    passed through the re-unitarization above (Haar on SU(Nc)).
 *  - Sweep order (Sec. 3 kernel list and Sec. 4 protocol): n_hb heatbath
 *    steps, then n_or overrelaxation steps, then re-unitarization; each step
 *    runs, for mu = 0..3, the even then the odd sites.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include "sun_oracle.h"

#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define NC_MAX 32
#define SAMPLER_MAX_ATTEMPTS 64
#define CREUTZ_KP_SWITCH 1.7
#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies, with a  */
/* Weyl-sequence key schedule.                                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

int orc_num_threads(void)
{
    return omp_get_max_threads();
}

/* Threads of later lattice-wide calls (n >= 1); results do not depend on it. */
int orc_set_num_threads(int n)
{
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}

/* 24-bit uniform in (0, 1]; exactly representable in float and double. */
double orc_uniform(uint32_t w)
{
    return (double)((w >> 8) + 1u) * (1.0 / 16777216.0);
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double u[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = orc_uniform(w[i]);
}

/* ------------------------------------------------------------------------ */
/* Geometry: 4D periodic hypercubic lattice (Sec. 2), logical site index    */
/* s = x + Lx (y + Ly (z + Lz t)), parity (x+y+z+t) mod 2 (Sec. 3           */
/* chessboard).                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nc;
    int L[4];
    int64_t V;
    int64_t stride[4];
    int present[4];
    int d;
} geom;

int orc_check(int nc, const int L[4])
{
    if (nc < 2 || nc > NC_MAX) return -1;
    if (L[0] < 2 || (L[0] & 1)) return -1;
    for (int mu = 1; mu < 4; ++mu)
        if (!(L[mu] == 1 || (L[mu] >= 2 && !(L[mu] & 1)))) return -1;
    return 0;
}

static void make_geom(int nc, const int L[4], geom *g)
{
    g->nc = nc;
    g->V = 1;
    g->d = 0;
    for (int mu = 0; mu < 4; ++mu) {
        g->L[mu] = L[mu];
        g->stride[mu] = g->V;
        g->V *= L[mu];
        g->present[mu] = L[mu] > 1;
        g->d += g->present[mu];
    }
}

static void coords(const geom *g, int64_t s, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

static int64_t index_of(const geom *g, const int x[4])
{
    int64_t s = 0;
    for (int mu = 3; mu >= 0; --mu) s = s * g->L[mu] + x[mu];
    return s;
}

static int parity_of(const geom *g, int64_t s)
{
    int x[4];
    coords(g, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* s shifted by dir (+1 or -1) steps along direction mu, periodic. */
static int64_t shift(const geom *g, int64_t s, int mu, int dir)
{
    int x[4];
    coords(g, s, x);
    x[mu] = (x[mu] + dir + g->L[mu]) % g->L[mu];
    return index_of(g, x);
}

/* ------------------------------------------------------------------------ */
/* Access log (race check; test infrastructure of its own): while a phase   */
/* runs serially under orc_phase_access_check, every link an update reads   */
/* (clink) or takes for writing (link) is noted with the site of the update */
/* that touched it.  Per link: -1 untouched, the site of its only toucher,  */
/* or -2 when several updates touched it.                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t owner;
    int64_t *reader;
    int64_t *writer;
} access_log;
static access_log *alog = NULL;

static void note_access(int64_t *tab, int64_t l, int64_t owner)
{
    if (tab[l] == -1)
        tab[l] = owner;
    else if (tab[l] != owner)
        tab[l] = -2;
}

static cplx *link(const geom *g, cplx *U, int mu, int64_t s)
{
    if (alog) note_access(alog->writer, (int64_t)mu * g->V + s, alog->owner);
    return U + ((int64_t)mu * g->V + s) * g->nc * g->nc;
}

static const cplx *clink(const geom *g, const cplx *U, int mu, int64_t s)
{
    if (alog) note_access(alog->reader, (int64_t)mu * g->V + s, alog->owner);
    return U + ((int64_t)mu * g->V + s) * g->nc * g->nc;
}

/* ------------------------------------------------------------------------ */
/* Dense complex matrix algebra (n x n, row-major).                         */
/* ------------------------------------------------------------------------ */
static void mat_mul(int n, const cplx *a, const cplx *b, cplx *c)
{
    cplx tmp[NC_MAX * NC_MAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx acc = 0;
            for (int k = 0; k < n; ++k) acc += a[i * n + k] * b[k * n + j];
            tmp[i * n + j] = acc;
        }
    memcpy(c, tmp, sizeof(cplx) * n * n);
}

static void mat_dag(int n, const cplx *a, cplx *c)
{
    cplx tmp[NC_MAX * NC_MAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) tmp[i * n + j] = conj(a[j * n + i]);
    memcpy(c, tmp, sizeof(cplx) * n * n);
}

static void mat_add(int n, cplx *acc, const cplx *a)
{
    for (int i = 0; i < n * n; ++i) acc[i] += a[i];
}

static void mat_identity(int n, cplx *a)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[i * n + j] = (i == j) ? 1.0 : 0.0;
}

static double re_trace(int n, const cplx *a)
{
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += creal(a[i * n + i]);
    return t;
}

/* Determinant by Gaussian elimination with partial pivoting. */
static cplx mat_det(int n, const cplx *a)
{
    cplx m[NC_MAX * NC_MAX];
    memcpy(m, a, sizeof(cplx) * n * n);
    cplx det = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (cabs(m[r * n + col]) > cabs(m[piv * n + col])) piv = r;
        if (cabs(m[piv * n + col]) == 0.0) return 0.0;
        if (piv != col) {
            for (int j = 0; j < n; ++j) {
                cplx t = m[col * n + j];
                m[col * n + j] = m[piv * n + j];
                m[piv * n + j] = t;
            }
            det = -det;
        }
        det *= m[col * n + col];
        for (int r = col + 1; r < n; ++r) {
            cplx f = m[r * n + col] / m[col * n + col];
            for (int j = col; j < n; ++j) m[r * n + j] -= f * m[col * n + j];
        }
    }
    return det;
}

/* SU(2) element from its four real parameters, U = a0 1 + i a.sigma
 * (Sec. 2): [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]]. */
static void su2_from_params(const double a[4], cplx m[4])
{
    m[0] = a[0] + I * a[3];
    m[1] = a[2] + I * a[1];
    m[2] = -a[2] + I * a[1];
    m[3] = a[0] - I * a[3];
}

static void mat2_mul(const cplx a[4], const cplx b[4], cplx c[4])
{
    cplx t[4];
    t[0] = a[0] * b[0] + a[1] * b[2];
    t[1] = a[0] * b[1] + a[1] * b[3];
    t[2] = a[2] * b[0] + a[3] * b[2];
    t[3] = a[2] * b[1] + a[3] * b[3];
    memcpy(c, t, sizeof t);
}

static void mat2_dag(const cplx a[4], cplx c[4])
{
    cplx t[4] = {conj(a[0]), conj(a[2]), conj(a[1]), conj(a[3])};
    memcpy(c, t, sizeof t);
}

/* Left-multiply rows i and j of the n x n matrix M by the 2x2 matrix a
 * (the subgroup embedding S_ij of Sec. 2, acting as U^k = A_k U^{k-1}). */
static void rows_left_mul(int n, cplx *M, int i, int j, const cplx a[4])
{
    for (int c = 0; c < n; ++c) {
        cplx ri = M[i * n + c], rj = M[j * n + c];
        M[i * n + c] = a[0] * ri + a[1] * rj;
        M[j * n + c] = a[2] * ri + a[3] * rj;
    }
}

/* ------------------------------------------------------------------------ */
/* Re-unitarization (Sec. 2, last paragraph).                               */
/* ------------------------------------------------------------------------ */
static void normalize_row(int n, cplx *r)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += creal(r[j]) * creal(r[j]) + cimag(r[j]) * cimag(r[j]);
    double inv = 1.0 / sqrt(s);
    for (int j = 0; j < n; ++j) r[j] *= inv;
}

/* r_i -= <r_k, r_i> r_k with <u, v> = sum_j conj(u_j) v_j */
static void remove_projection(int n, const cplx *rk, cplx *ri)
{
    cplx p = 0;
    for (int j = 0; j < n; ++j) p += conj(rk[j]) * ri[j];
    for (int j = 0; j < n; ++j) ri[j] -= p * rk[j];
}

static void reunit(int n, cplx *M)
{
    if (n == 2) {
        normalize_row(2, M);
        M[2] = -conj(M[1]);
        M[3] = conj(M[0]);
        return;
    }
    int gs_rows = (n == 3) ? 2 : n;
    for (int i = 0; i < gs_rows; ++i) {
        for (int k = 0; k < i; ++k) remove_projection(n, M + k * n, M + i * n);
        normalize_row(n, M + i * n);
    }
    if (n == 3) {
        const cplx *a = M, *b = M + 3;
        M[6] = conj(a[1] * b[2] - a[2] * b[1]);
        M[7] = conj(a[2] * b[0] - a[0] * b[2]);
        M[8] = conj(a[0] * b[1] - a[1] * b[0]);
    } else {
        cplx det = mat_det(n, M);
        cplx phase = conj(det) / cabs(det);
        for (int j = 0; j < n; ++j) M[(n - 1) * n + j] *= phase;
    }
}

int orc_reunit_matrix(int nc, double *Md)
{
    if (nc < 2 || nc > NC_MAX) return -1;
    reunit(nc, (cplx *)Md);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Staple (Sec. 2): the sum over nu != mu of the two paths that close the   */
/* plaquettes containing U_mu(x):                                           */
/*   U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag                                  */
/* + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu).                           */
/* ------------------------------------------------------------------------ */
static void staple(const geom *g, const cplx *U, int64_t s, int mu, cplx *A)
{
    const int n = g->nc;
    cplx t1[NC_MAX * NC_MAX], t2[NC_MAX * NC_MAX], t3[NC_MAX * NC_MAX];
    for (int i = 0; i < n * n; ++i) A[i] = 0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu || !g->present[nu]) continue;
        int64_t x_pmu = shift(g, s, mu, +1);
        int64_t x_pnu = shift(g, s, nu, +1);
        int64_t x_mnu = shift(g, s, nu, -1);
        int64_t x_pmu_mnu = shift(g, x_pmu, nu, -1);
        /* upper */
        mat_dag(n, clink(g, U, mu, x_pnu), t2);
        mat_mul(n, clink(g, U, nu, x_pmu), t2, t1);
        mat_dag(n, clink(g, U, nu, s), t3);
        mat_mul(n, t1, t3, t1);
        mat_add(n, A, t1);
        /* lower */
        mat_dag(n, clink(g, U, nu, x_pmu_mnu), t1);
        mat_dag(n, clink(g, U, mu, x_mnu), t2);
        mat_mul(n, t1, t2, t1);
        mat_mul(n, t1, clink(g, U, nu, x_mnu), t1);
        mat_add(n, A, t1);
    }
}

/* ------------------------------------------------------------------------ */
/* SU(2) heatbath draw (Sec. 2): x0 in [-1, 1] with density                 */
/* sqrt(1 - x0^2) exp(alpha x0), then (x1, x2, x3) on the sphere of radius  */
/* sqrt(1 - x0^2).                                                          */
/* Returns the number of attempts, or 0 when the cap was reached (the       */
/* caller then leaves the link unchanged).  *margin is lowered to the       */
/* distance of every decision from its threshold.                          */
/* ------------------------------------------------------------------------ */
static int sample_su2(double alpha, uint64_t seed, uint32_t site, uint32_t step,
                      uint32_t mu_sg, double x[4], double *margin)
{
    double m = fabs(alpha - CREUTZ_KP_SWITCH);
    double x0 = 0.0, radius = 0.0;
    int hit, accepted = 0;
    for (hit = 0; hit < SAMPLER_MAX_ATTEMPTS; ++hit) {
        double r[4];
        draw(seed, site, step, mu_sg, (0u << 24) | (uint32_t)hit, r);
        if (alpha < CREUTZ_KP_SWITCH) {
            /* Creutz: invert the CDF of exp(alpha x0) on [-1, 1], then accept
             * with probability sqrt(1 - x0^2). */
            if (alpha == 0.0)
                x0 = 2.0 * r[0] - 1.0;
            else
                x0 = 1.0 + log1p((1.0 - r[0]) * expm1(-2.0 * alpha)) / alpha;
            double lhs = r[1] * r[1], rhs = 1.0 - x0 * x0;
            if (fabs(lhs - rhs) < m) m = fabs(lhs - rhs);
            if (lhs <= rhs) {
                radius = sqrt(rhs);
                accepted = 1;
                break;
            }
        } else {
            /* Kennedy-Pendleton: lambda^2 from a 3D Gaussian with variance
             * 1/(4 alpha), accept with probability sqrt(1 - lambda^2),
             * x0 = 1 - 2 lambda^2. */
            double c = cos(TWO_PI * r[1]);
            double lam2 = -(log(r[0]) + c * c * log(r[2])) / (2.0 * alpha);
            double lhs = r[3] * r[3], rhs = 1.0 - lam2;
            if (fabs(lhs - rhs) < m) m = fabs(lhs - rhs);
            if (lhs <= rhs) {
                x0 = 1.0 - 2.0 * lam2;
                radius = 2.0 * sqrt(lam2) * sqrt(1.0 - lam2);
                accepted = 1;
                break;
            }
        }
    }
    if (margin && m < *margin) *margin = m;
    if (!accepted) return 0;
    double u[4];
    draw(seed, site, step, mu_sg, (1u << 24), u);
    double cos_t = 1.0 - 2.0 * u[0];
    double sin_t = sqrt(1.0 - cos_t * cos_t);
    double phi = TWO_PI * u[1];
    x[0] = x0;
    x[1] = radius * sin_t * cos(phi);
    x[2] = radius * sin_t * sin(phi);
    x[3] = radius * cos_t;
    return hit + 1;
}

int orc_sample_su2(const double *alpha, int n, uint64_t seed, uint32_t step,
                   uint32_t mu_sg, double *x, int *attempts, double *margin)
{
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i) {
        double m = INFINITY;
        double xi[4] = {1.0, 0.0, 0.0, 0.0};
        int a = sample_su2(alpha[i], seed, (uint32_t)i, step, mu_sg, xi, &m);
        for (int c = 0; c < 4; ++c) x[4 * i + c] = xi[c];
        attempts[i] = a;
        if (margin) margin[i] = m;
    }
    return 0;
}

/* Quaternion projection of the 2x2 block (i, j) of W (Sec. 2: a sum of SU(2)
 * elements is proportional to an SU(2) element):
 *   P(w) = (w + adj-conj) / 2 = [[w11 + conj(w22), w12 - conj(w21)],
 *                                [w21 - conj(w12), w22 + conj(w11)]] / 2,
 * k = sqrt(det P(w)), V = P(w) / k.  Returns k. */
static double subgroup_projection(int n, const cplx *W, int i, int j, cplx V[4])
{
    cplx w11 = W[i * n + i], w12 = W[i * n + j], w21 = W[j * n + i], w22 = W[j * n + j];
    cplx P[4];
    P[0] = 0.5 * (w11 + conj(w22));
    P[1] = 0.5 * (w12 - conj(w21));
    P[2] = 0.5 * (w21 - conj(w12));
    P[3] = 0.5 * (w22 + conj(w11));
    double det = creal(P[0] * P[3] - P[1] * P[2]);
    double k = det > 0.0 ? sqrt(det) : 0.0;
    if (k > 0.0) {
        for (int c = 0; c < 4; ++c) V[c] = P[c] / k;
    } else {
        V[0] = 1.0; V[1] = 0.0; V[2] = 0.0; V[3] = 1.0;
    }
    return k;
}

/* Cabibbo-Marinari pseudo-heatbath of one link (Sec. 2, steps 1-5):
 * staple, W = U A, then for every subgroup draw x ~ exp(alpha x0) and
 * left-multiply U (and W) by a = x V^dag. */
static double frobenius(int n, const cplx *a)
{
    double s = 0.0;
    for (int i = 0; i < n * n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(s);
}

/* Conditioning of a link update: |A|_F / min_k, the staple norm over the
 * smallest subgroup projection norm (V = P / k divides rounding by k). */
static double conditioning(double a_norm, double kmin)
{
    return kmin > 0.0 ? a_norm / kmin : INFINITY;
}

static double heatbath_link(const geom *g, cplx *U, int64_t s, int mu, double beta,
                            uint64_t seed, uint64_t step, int *attempts_out, double *cond_out)
{
    const int n = g->nc;
    cplx A[NC_MAX * NC_MAX], W[NC_MAX * NC_MAX];
    cplx *Ul = link(g, U, mu, s);
    staple(g, U, s, mu, A);
    mat_mul(n, Ul, A, W);
    double margin = INFINITY, kmin = INFINITY;
    int attempts = 0, sg = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j, ++sg) {
            cplx V[4], Vd[4], X[4], a[4];
            double k = subgroup_projection(n, W, i, j, V);
            if (k < kmin) kmin = k;
            double alpha = 2.0 * beta * k / n;
            double x[4];
            uint32_t mu_sg = ((uint32_t)mu << 16) | (uint32_t)sg;
            int got = sample_su2(alpha, seed, (uint32_t)s, (uint32_t)step, mu_sg, x, &margin);
            attempts += got;
            if (!got) continue;
            su2_from_params(x, X);
            mat2_dag(V, Vd);
            mat2_mul(X, Vd, a);
            rows_left_mul(n, Ul, i, j, a);
            rows_left_mul(n, W, i, j, a);
        }
    if (attempts_out) *attempts_out = attempts;
    if (cond_out) *cond_out = conditioning(frobenius(n, A), kmin);
    return margin;
}

/* Overrelaxation of one link (Sec. 2): per subgroup a = V^dag V^dag, the
 * SU(2) reflection applied inside each subgroup of SU(Nc). */
static double overrelax_link(const geom *g, cplx *U, int64_t s, int mu, int reverse)
{
    const int n = g->nc;
    cplx A[NC_MAX * NC_MAX], W[NC_MAX * NC_MAX];
    cplx *Ul = link(g, U, mu, s);
    staple(g, U, s, mu, A);
    mat_mul(n, Ul, A, W);
    int npairs = n * (n - 1) / 2;
    int pi[NC_MAX * NC_MAX / 2], pj[NC_MAX * NC_MAX / 2], np = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            pi[np] = i;
            pj[np] = j;
            ++np;
        }
    double kmin = INFINITY;
    for (int q = 0; q < npairs; ++q) {
        int p = reverse ? npairs - 1 - q : q;
        cplx V[4], Vd[4], a[4];
        double k = subgroup_projection(n, W, pi[p], pj[p], V);
        if (k < kmin) kmin = k;
        mat2_dag(V, Vd);
        mat2_mul(Vd, Vd, a);
        rows_left_mul(n, Ul, pi[p], pj[p], a);
        rows_left_mul(n, W, pi[p], pj[p], a);
    }
    return conditioning(frobenius(n, A), kmin);
}

/* ------------------------------------------------------------------------ */
/* Lattice-wide steps.                                                      */
/* ------------------------------------------------------------------------ */
int orc_init(int nc, const int L[4], double *Ud, int hot, uint64_t seed)
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    cplx *U = (cplx *)Ud;
    const int n = nc;
    const int nreal = 2 * n * n;
    const int ncalls = (nreal + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        for (int mu = 0; mu < 4; ++mu) {
            cplx *Ul = link(&g, U, mu, s);
            if (!hot || !g.present[mu]) {
                mat_identity(n, Ul);
                continue;
            }
            double gauss[NC_MAX * NC_MAX * 2 + 4];
            for (int call = 0; call < ncalls; ++call) {
                double u[4];
                draw(seed, (uint32_t)s, 0xFFFFFFFFu, (uint32_t)mu << 16, (2u << 24) | (uint32_t)call, u);
                /* Box-Muller: two normal deviates from each pair of uniforms */
                for (int p = 0; p < 2; ++p) {
                    double rad = sqrt(-2.0 * log(u[2 * p]));
                    double ang = TWO_PI * u[2 * p + 1];
                    gauss[4 * call + 2 * p] = rad * cos(ang);
                    gauss[4 * call + 2 * p + 1] = rad * sin(ang);
                }
            }
            for (int e = 0; e < n * n; ++e) Ul[e] = gauss[2 * e] + I * gauss[2 * e + 1];
            reunit(n, Ul);
        }
    }
    return 0;
}

int orc_phase(int nc, const int L[4], double *Ud, int kind, int mu, int parity,
              double beta, uint64_t seed, uint64_t step, double *margin, int *attempts,
              double *cond)
{
    if (orc_check(nc, L) || mu < 0 || mu > 3 || (kind != 0 && kind != 1)) return -1;
    geom g;
    make_geom(nc, L, &g);
    cplx *U = (cplx *)Ud;
    if (!g.present[mu]) return 0;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        if (parity_of(&g, s) != (parity & 1)) {
            if (margin) margin[s] = -1.0;
            if (attempts) attempts[s] = 0;
            if (cond) cond[s] = -1.0;
            continue;
        }
        if (kind == 0) {
            int a = 0;
            double c = INFINITY;
            double m = heatbath_link(&g, U, s, mu, beta, seed, step, &a, &c);
            if (margin) margin[s] = m;
            if (attempts) attempts[s] = a;
            if (cond) cond[s] = c;
        } else {
            double c = overrelax_link(&g, U, s, mu, 0);
            if (margin) margin[s] = INFINITY;
            if (attempts) attempts[s] = 0;
            if (cond) cond[s] = c;
        }
    }
    return 0;
}

/* The chessboard's promise (Sec. 3: the update kernels run on the even and
 * then the odd sites of one direction so that the updates of one call are
 * independent): no link a phase writes is read by any update of that phase
 * other than its own, and no link is written twice.  Runs the phase serially
 * with the access log on and counts out[0] links written by more than one
 * update, out[1] links written by one update and read by another, out[2]
 * links written.  parity 2 updates both parities in one pass (a broken
 * schedule, for testing this check). */
int orc_phase_access_check(int nc, const int L[4], double *Ud, int kind, int mu, int parity,
                           double beta, uint64_t seed, uint64_t step, int64_t out[3])
{
    if (orc_check(nc, L) || mu < 0 || mu > 3 || (kind != 0 && kind != 1) || parity < 0 || parity > 2)
        return -1;
    geom g;
    make_geom(nc, L, &g);
    cplx *U = (cplx *)Ud;
    const int64_t nl = 4 * g.V;
    access_log log;
    log.reader = (int64_t *)malloc(sizeof(int64_t) * nl);
    log.writer = (int64_t *)malloc(sizeof(int64_t) * nl);
    if (!log.reader || !log.writer) {
        free(log.reader);
        free(log.writer);
        return -2;
    }
    for (int64_t l = 0; l < nl; ++l) log.reader[l] = log.writer[l] = -1;
    alog = &log;
    if (g.present[mu])
        for (int64_t s = 0; s < g.V; ++s) {
            if (parity != 2 && parity_of(&g, s) != parity) continue;
            log.owner = s;
            if (kind == 0)
                heatbath_link(&g, U, s, mu, beta, seed, step, NULL, NULL);
            else
                overrelax_link(&g, U, s, mu, 0);
        }
    alog = NULL;
    out[0] = out[1] = out[2] = 0;
    for (int64_t l = 0; l < nl; ++l) {
        if (log.writer[l] == -1) continue;
        out[2] += 1;
        if (log.writer[l] == -2) out[0] += 1;
        else if (log.reader[l] != -1 && log.reader[l] != log.writer[l]) out[1] += 1;
    }
    free(log.reader);
    free(log.writer);
    return 0;
}

int orc_reunitarize(int nc, const int L[4], double *Ud)
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    cplx *U = (cplx *)Ud;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            if (g.present[mu]) reunit(nc, link(&g, U, mu, s));
    return 0;
}

int orc_sweep(int nc, const int L[4], double *Ud, double beta, int n_hb, int n_or,
              uint64_t seed, uint64_t step0, int reunitarize)
{
    if (orc_check(nc, L) || n_hb < 0 || n_or < 0) return -1;
    for (int h = 0; h < n_hb; ++h)
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                orc_phase(nc, L, Ud, 0, mu, p, beta, seed, step0 + (uint64_t)h, NULL, NULL, NULL);
    for (int o = 0; o < n_or; ++o)
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                orc_phase(nc, L, Ud, 1, mu, p, beta, seed, 0, NULL, NULL, NULL);
    if (reunitarize) orc_reunitarize(nc, L, Ud);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables, in FP64 with fixed-order sums (per-site values first, then  */
/* a sequential sum over sites).                                            */
/* ------------------------------------------------------------------------ */

/* Plaquette P_mu_nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 * (Sec. 2); reported as the mean of ReTr P / Nc over sites and planes. */
static double re_tr_plaquette(const geom *g, const cplx *U, int64_t s, int mu, int nu)
{
    const int n = g->nc;
    cplx t1[NC_MAX * NC_MAX], t2[NC_MAX * NC_MAX];
    mat_mul(n, clink(g, U, mu, s), clink(g, U, nu, shift(g, s, mu, +1)), t1);
    mat_dag(n, clink(g, U, mu, shift(g, s, nu, +1)), t2);
    mat_mul(n, t1, t2, t1);
    mat_dag(n, clink(g, U, nu, s), t2);
    mat_mul(n, t1, t2, t1);
    return re_trace(n, t1);
}

int orc_plaquette(int nc, const int L[4], const double *Ud, double out[3])
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    const cplx *U = (const cplx *)Ud;
    double *site_sp = (double *)malloc(sizeof(double) * g.V);
    double *site_tm = (double *)malloc(sizeof(double) * g.V);
    if (!site_sp || !site_tm) {
        free(site_sp);
        free(site_tm);
        return -1;
    }
    int n_sp = 0, n_tm = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu)
            if (g.present[mu] && g.present[nu]) {
                if (nu == 3) ++n_tm;
                else ++n_sp;
            }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        double sp = 0.0, tm = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                if (!g.present[mu] || !g.present[nu]) continue;
                double p = re_tr_plaquette(&g, U, s, mu, nu);
                if (nu == 3) tm += p;
                else sp += p;
            }
        site_sp[s] = sp;
        site_tm[s] = tm;
    }
    double sum_sp = 0.0, sum_tm = 0.0;
    for (int64_t s = 0; s < g.V; ++s) {
        sum_sp += site_sp[s];
        sum_tm += site_tm[s];
    }
    free(site_sp);
    free(site_tm);
    double norm = (double)nc * (double)g.V;
    out[0] = (n_sp + n_tm) ? (sum_sp + sum_tm) / (norm * (n_sp + n_tm)) : 0.0;
    out[1] = n_sp ? sum_sp / (norm * n_sp) : 0.0;
    out[2] = n_tm ? sum_tm / (norm * n_tm) : 0.0;
    return 0;
}

int orc_action(int nc, const int L[4], const double *Ud, double beta, double *out)
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    double p[3];
    orc_plaquette(nc, L, Ud, p);
    double nplanes = (double)g.V * g.d * (g.d - 1) / 2.0;
    /* S = (beta/Nc) sum ReTr(1 - P) = beta * nplanes * (1 - mean(ReTr P / Nc)) */
    *out = beta * nplanes * (1.0 - p[0]);
    return 0;
}

/* Polyakov loop (1/(Nc Vs)) sum_xvec Tr prod_{t=0}^{Nt-1} U_3(xvec, t). */
int orc_polyakov(int nc, const int L[4], const double *Ud, double out[2])
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    const cplx *U = (const cplx *)Ud;
    const int n = nc;
    int64_t Vs = g.V / L[3];
    cplx *tr = (cplx *)malloc(sizeof(cplx) * Vs);
    if (!tr) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t xs = 0; xs < Vs; ++xs) {
        cplx P[NC_MAX * NC_MAX];
        mat_identity(n, P);
        for (int t = 0; t < L[3]; ++t) mat_mul(n, P, clink(&g, U, 3, xs + (int64_t)t * Vs), P);
        cplx acc = 0;
        for (int i = 0; i < n; ++i) acc += P[i * n + i];
        tr[xs] = acc;
    }
    cplx sum = 0;
    for (int64_t xs = 0; xs < Vs; ++xs) sum += tr[xs];
    free(tr);
    sum /= (double)n * (double)Vs;
    out[0] = creal(sum);
    out[1] = cimag(sum);
    return 0;
}

int orc_unitarity(int nc, const int L[4], const double *Ud, double out[2])
{
    if (orc_check(nc, L)) return -1;
    geom g;
    make_geom(nc, L, &g);
    const cplx *U = (const cplx *)Ud;
    const int n = nc;
    double *dev_u = (double *)malloc(sizeof(double) * g.V);
    double *dev_d = (double *)malloc(sizeof(double) * g.V);
    if (!dev_u || !dev_d) {
        free(dev_u);
        free(dev_d);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < g.V; ++s) {
        double mu_max = 0.0, md_max = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            if (!g.present[mu]) continue;
            cplx Ud_[NC_MAX * NC_MAX], P[NC_MAX * NC_MAX];
            const cplx *Ul = clink(&g, U, mu, s);
            mat_dag(n, Ul, Ud_);
            mat_mul(n, Ud_, Ul, P);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double e = cabs(P[i * n + j] - ((i == j) ? 1.0 : 0.0));
                    if (e > mu_max) mu_max = e;
                }
            double e = cabs(mat_det(n, Ul) - 1.0);
            if (e > md_max) md_max = e;
        }
        dev_u[s] = mu_max;
        dev_d[s] = md_max;
    }
    double a = 0.0, b = 0.0;
    for (int64_t s = 0; s < g.V; ++s) {
        if (dev_u[s] > a) a = dev_u[s];
        if (dev_d[s] > b) b = dev_d[s];
    }
    free(dev_u);
    free(dev_d);
    out[0] = a;
    out[1] = b;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-link entry points for the pins.                                   */
/* ------------------------------------------------------------------------ */
int orc_staple(int nc, const int L[4], const double *Ud, int64_t s, int mu, double *Ad)
{
    if (orc_check(nc, L) || mu < 0 || mu > 3) return -1;
    geom g;
    make_geom(nc, L, &g);
    if (s < 0 || s >= g.V) return -1;
    staple(&g, (const cplx *)Ud, s, mu, (cplx *)Ad);
    return 0;
}

int orc_heatbath_link(int nc, const int L[4], double *Ud, int64_t s, int mu, double beta,
                      uint64_t seed, uint64_t step)
{
    if (orc_check(nc, L) || mu < 0 || mu > 3) return -1;
    geom g;
    make_geom(nc, L, &g);
    if (s < 0 || s >= g.V) return -1;
    heatbath_link(&g, (cplx *)Ud, s, mu, beta, seed, step, NULL, NULL);
    return 0;
}

int orc_overrelax_link(int nc, const int L[4], double *Ud, int64_t s, int mu, int reverse)
{
    if (orc_check(nc, L) || mu < 0 || mu > 3) return -1;
    geom g;
    make_geom(nc, L, &g);
    if (s < 0 || s >= g.V) return -1;
    overrelax_link(&g, (cplx *)Ud, s, mu, reverse);
    return 0;
}
