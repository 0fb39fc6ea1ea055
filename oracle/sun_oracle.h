/*
 * sun_oracle.h -- FP64 CPU oracle for the SU(Nc) Wilson-action checkerboard
 * sweep of Cardoso & Bicudo, "Generating SU(Nc) pure gauge lattice QCD
 * configurations on GPUs with CUDA" (arXiv:1112.4533).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the HIP library: its own Philox, its own algebra, its own reductions.
 *
 * Field layout (canonical, also the HIP library's export format):
 *   U[mu][s][i][j] as double complex, mu = 0..3, s = logical site index
 *   s = x + Lx*(y + Ly*(z + Lz*t)), i,j = 0..Nc-1 (row-major matrix).
 * Extents: L[0] even >= 2; L[1..3] even >= 2, or 1 (direction absent, which
 * gives 2D/3D lattices).  Links of absent directions are the identity and are
 * never updated or measured.
 *
 * Counter-based randomness (the method's draws are fixed by this contract):
 *   Philox4x32-10, key = (lo32(seed), hi32(seed)),
 *   counter = (site, lo32(step), (mu << 16) | subgroup, (purpose << 24) | hit)
 *   purpose 0 = SU(2) a0 attempt, 1 = S^2 direction, 2 = hot-start Gaussians
 *   (hot start uses counter (site, 0xFFFFFFFF, mu << 16, (2 << 24) | call)).
 *   Uniform from a 32-bit word w: u = ((w >> 8) + 1) * 2^-24, in (0, 1].
 */
#ifndef SUN_ORACLE_H
#define SUN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OpenMP threads the lattice-wide calls use, and a setter for them (n >= 1;
 * results do not depend on the thread count). */
int orc_num_threads(void);
int orc_set_num_threads(int n);

/* Raw generator, for known-answer tests. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t w);

/* Lattice-wide operations.  U points to 4*V*Nc*Nc double complex values
 * stored as interleaved (re, im) doubles.  All return 0, or -1 on bad
 * arguments. */
int orc_check(int nc, const int L[4]);
int orc_init(int nc, const int L[4], double *U, int hot, uint64_t seed);
/* One checkerboard phase: kind 0 = heatbath, 1 = overrelaxation; updates
 * U_mu(x) for every site x of the given parity.  margin (length V, may be
 * NULL) receives, for each updated site, the smallest distance of any
 * floating-point decision (branch switch or accept test) from its threshold;
 * other sites get -1.  attempts (length V, may be NULL) receives the number
 * of a0 attempts summed over subgroups; cond (length V, may be NULL) the
 * conditioning |A|_F / k_min of the update (staple norm over the smallest
 * subgroup projection norm, since V = P / k divides rounding by k), -1 for
 * sites not updated. */
int orc_phase(int nc, const int L[4], double *U, int kind, int mu, int parity,
              double beta, uint64_t seed, uint64_t step, double *margin, int *attempts,
              double *cond);
/* n_hb heatbath steps (steps step0 .. step0+n_hb-1), then n_or
 * overrelaxation steps, then re-unitarization if reunit != 0. */
int orc_sweep(int nc, const int L[4], double *U, double beta, int n_hb, int n_or,
              uint64_t seed, uint64_t step0, int reunit);
int orc_reunitarize(int nc, const int L[4], double *U);
/* Race check of one phase (chessboard independence); see the source. */
int orc_phase_access_check(int nc, const int L[4], double *U, int kind, int mu, int parity,
                           double beta, uint64_t seed, uint64_t step, int64_t out[3]);
/* out = {mean plaquette, spatial-plane mean, planes-with-direction-3 mean} */
int orc_plaquette(int nc, const int L[4], const double *U, double out[3]);
/* out = {Re, Im} of the Polyakov loop along direction 3 */
int orc_polyakov(int nc, const int L[4], const double *U, double out[2]);
/* out = {max_ij |(U^dag U - 1)_ij|, max |det U - 1|} over present links */
int orc_unitarity(int nc, const int L[4], const double *U, double out[2]);
/* Wilson action (beta/Nc) sum_x sum_{mu<nu} ReTr(1 - P_mu_nu(x)) */
int orc_action(int nc, const int L[4], const double *U, double beta, double *out);

/* Single-link and single-matrix entry points, for pins. */
int orc_staple(int nc, const int L[4], const double *U, int64_t s, int mu, double *A);
int orc_heatbath_link(int nc, const int L[4], double *U, int64_t s, int mu, double beta,
                      uint64_t seed, uint64_t step);
/* reverse != 0 walks the subgroups in the opposite order */
int orc_overrelax_link(int nc, const int L[4], double *U, int64_t s, int mu, int reverse);
int orc_reunit_matrix(int nc, double *M);
/* Samples x in SU(2) with density ~ exp(alpha x0) dHaar, for n values of
 * alpha, using counters (i, step, (mu << 16) | sg, ...).  x: 4n doubles,
 * attempts: n ints (0 when the attempt cap was hit and the step skipped),
 * margin: n doubles (may be NULL). */
int orc_sample_su2(const double *alpha, int n, uint64_t seed, uint32_t step,
                   uint32_t mu_sg, double *x, int *attempts, double *margin);

#ifdef __cplusplus
}
#endif
#endif
