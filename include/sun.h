/*
 * sun.h -- C ABI of libsun, the MI355X (gfx950) implementation of the
 * pure-gauge SU(Nc) Wilson-action checkerboard sweep of Cardoso & Bicudo,
 * "Generating SU(Nc) pure gauge lattice QCD configurations on GPUs with CUDA"
 * (arXiv:1112.4533).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns SUN_OK (0) or a negative SUN_E* code; the text of
 *    the last error of the calling thread is returned by sun_last_error().
 *  - Device memory is owned by the caller.  The library allocates no device
 *    memory; the link field and a scratch buffer are handed in at creation
 *    and must outlive the handle.  Sizes come from sun_lattice_bytes().
 *  - Every call that takes a stream is asynchronous on that stream (a
 *    hipStream_t passed as void*; NULL is the null stream).  Output pointers
 *    named dev_* are device pointers written by kernels on that stream.
 *  - A handle is used by one host thread at a time.  Calls on one handle that
 *    overlap on different streams race on its scratch buffer.
 *  - Lattice: extents L[0..3] (directions x, y, z, t).  L[0] is even >= 2;
 *    every other extent is even >= 2, or 1 for an absent direction (2D and 3D
 *    lattices).  Links of absent directions are the identity and are never
 *    updated.  Site index s = x + L0*(y + L1*(z + L2*t)), parity
 *    (x+y+z+t) mod 2.  Periodic boundaries (paper Sec. 2).
 *  - Randomness: Philox4x32-10 (Salmon et al., SC'11) with key
 *    (lo32(seed), hi32(seed)) and counter
 *    (site, lo32(step), (mu << 16) | subgroup, (purpose << 24) | attempt);
 *    uniforms u = ((w >> 8) + 1) * 2^-24.  Heatbath step h of a sweep uses
 *    step = (current step counter) + h; the counter advances by n_hb per sweep
 *    and is part of the chain state (sun_get_step / sun_set_step).
 */
#ifndef SUN_H
#define SUN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sun_lattice_s *sun_lattice_t;
typedef void *sun_stream_t; /* hipStream_t */

enum {
    SUN_OK = 0,
    SUN_EINVAL = -1, /* bad Nc, extent, dtype, direction, parity or count */
    SUN_ESIZE = -2,  /* null or undersized buffer */
    SUN_EHIP = -3,   /* a HIP runtime error (text in sun_last_error) */
    SUN_EUNSUP = -4, /* valid request this build does not implement */
    SUN_ENUMERIC = -5 /* the watchdog found a non-finite or non-unitary field */
};

/* Link storage.  Reductions, re-unitarization and the start configuration
 * are always computed in FP64.  The TWO_ROW forms (SU(3) only, paper Sec. 3:
 * 12 reals instead of 18) store rows 0 and 1 and rebuild row 2 as
 * conj(row0 x row1) on every load, which cuts link traffic by a third.
 *
 * Nc <= SUN_NC_MAX_REGISTER runs one link per work-item with the link
 * matrices in registers and the field split into planes by (direction,
 * parity, matrix entry).  Larger Nc (the paper's generic SU(Nc) code, Sec. 4:
 * up to 32 in single and 16 in double precision at 8^4) runs one workgroup
 * of one or two wavefronts per link, matrices in LDS and the entries of each
 * link contiguous in memory; SUN_F32 and SUN_F64 select it by themselves
 * there, and the WIDE codes select it at Nc = 4 too (for comparisons with
 * the register path).  Its update keeps three or, at large Nc, two Nc^2
 * complex matrices in LDS (32 KiB at Nc = 32 in FP64), plus a ring of
 * heatbath draws when two wavefronts share it.  Of a launch shape only the
 * block size applies to it: 64 runs each link's update on one wavefront,
 * 128 on two (the link loads and the vector-unit products shared, the
 * subgroup steps on the first and, where LDS allows, the heatbath draws on
 * the second; the same bits either way; in the FP32 matrix-core form above
 * Nc = 20 the products stay on the first), and any other block, the default
 * 256 included, picks by Nc and precision. */
enum {
    SUN_F32 = 0,
    SUN_F64 = 1,
    SUN_F32_TWO_ROW = 2,
    SUN_F64_TWO_ROW = 3,
    SUN_F32_WIDE = 4,
    SUN_F64_WIDE = 5
};

/* Update kinds of one checkerboard phase (paper Sec. 3 kernel list). */
enum { SUN_HEATBATH = 0, SUN_OVERRELAX = 1 };

/* Largest Nc of the register path, and of the build. */
#define SUN_NC_MAX_REGISTER 4
#define SUN_NC_MAX 32

/* Bytes of device memory a lattice needs: the link field (SoA planes split by
 * direction, parity and matrix element) and the scratch buffer used by the
 * reductions.  Either output pointer may be NULL. */
int sun_lattice_bytes(int nc, const int L[4], int dtype, size_t *link_bytes,
                      size_t *scratch_bytes);

/* Creates a handle over caller-owned device buffers (links: link_bytes,
 * scratch: scratch_bytes, both 256-byte aligned).  Nc in 2..SUN_NC_MAX;
 * SUN_EUNSUP for a TWO_ROW dtype with Nc != 3 or a WIDE dtype with Nc < 4.
 * The field content is undefined until sun_init or sun_import. */
int sun_lattice_create(int nc, const int L[4], int dtype, void *links, size_t link_bytes,
                       void *scratch, size_t scratch_bytes, sun_lattice_t *out);
void sun_lattice_destroy(sun_lattice_t h);

/* Start configuration (paper Sec. 3, "Initialization of the lattice
 * array"): cold (hot = 0) sets every link to the identity; hot draws each
 * link Haar-distributed (complex Gaussian matrix from Box-Muller on Philox
 * uniforms, then the re-unitarization below).  Resets the step counter to 0. */
int sun_init(sun_lattice_t h, int hot, uint64_t seed, sun_stream_t stream);

/* One checkerboard phase (paper Sec. 3: the update kernels run by direction
 * and by even/odd sites): updates U_mu(x) for every site x of the given
 * parity by the Cabibbo-Marinari pseudo-heatbath (kind SUN_HEATBATH, paper
 * Sec. 2, using RNG step `step`) or by subgroup overrelaxation (kind
 * SUN_OVERRELAX, paper Sec. 2).  Does not touch the step counter. */
int sun_phase(sun_lattice_t h, int kind, int mu, int parity, double beta, uint64_t seed,
              uint64_t step, sun_stream_t stream);

/* One sweep (paper Sec. 4 protocol): n_hb heatbath steps, then n_or
 * overrelaxation steps, each step running for mu = 0..3 the even then the
 * odd phase; then, if reunit != 0, re-unitarization of every link.  The
 * heatbath steps use RNG steps counter .. counter + n_hb - 1; the counter
 * then advances by n_hb. */
int sun_sweep(sun_lattice_t h, double beta, int n_hb, int n_or, uint64_t seed, int reunit,
              sun_stream_t stream);

/* Re-unitarization (paper Sec. 2, last paragraph), in FP64: Nc = 2 normalizes
 * the quaternion; Nc = 3 Gram-Schmidt on rows 0, 1 and row 2 =
 * conj(row0 x row1); Nc > 3 Gram-Schmidt on all rows, then the last row times
 * conj(det)/|det|.  If dev_out2 is not NULL it receives the deviation of the
 * field BEFORE projection: {max_ij |(U^dag U - 1)_ij|, max |det U - 1|}. */
int sun_reunitarize(sun_lattice_t h, double *dev_out2, sun_stream_t stream);

/* Mean plaquette (paper Sec. 2, plaquette; Sec. 3, plaquette kernel with a
 * reduction over sites), in FP64 with a deterministic reduction order:
 * dev_out3 = {mean of ReTr P/Nc over all planes, over planes without
 * direction 3, over planes with direction 3}. */
int sun_plaquette(sun_lattice_t h, double *dev_out3, sun_stream_t stream);

/* Polyakov loop along direction 3, (1/(Nc Vs)) sum_x Tr prod_t U_3(x, t),
 * FP64: dev_out2 = {Re, Im}. */
int sun_polyakov(sun_lattice_t h, double *dev_out2, sun_stream_t stream);

/* Unitarity diagnostics, FP64: dev_out2 = {max_ij |(U^dag U - 1)_ij|,
 * max |det U - 1|} over present links. */
int sun_unitarity(sun_lattice_t h, double *dev_out2, sun_stream_t stream);

/* Watchdog (failure detection; not in the paper, whose runs assume a healthy
 * field).  threshold > 0 arms a check in every later re-unitarization on this
 * handle (sun_reunitarize, and sun_sweep with reunit != 0): from the field
 * before the projection it takes max_ij |(U^dag U - 1)_ij| and
 * max |det U - 1| over the present links in FP64 -- the numbers the
 * re-unitarization's drift report gives -- and counts the check as tripped
 * when either exceeds threshold; a NaN or infinite entry counts as an
 * infinite deviation.  No extra pass over the field is made.  The state lives
 * in the scratch buffer, on the device, and nothing synchronizes until
 * sun_check.  threshold = 0 disarms the check.  Every call clears the state
 * (a kernel on stream).  SUN_EINVAL for a negative, infinite or NaN
 * threshold.  Typical thresholds: ~1e-4 for FP32 storage, whose drift between
 * re-unitarizations is ~1e-6..1e-5; ~1e-10 for FP64.  Batch sweeps do not run
 * the check. */
int sun_watchdog(sun_lattice_t h, double threshold, sun_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the mean plaquette of
 * sun_plaquette, of a field in caller memory given by its geometry, with no
 * lattice handle and no allocation of any kind -- no hipMalloc or hipFree,
 * no host allocation.  The reduction partials live in a fixed device array
 * of SUN_STATIC_SCRATCH_BYTES inside the library (one per GPU it runs on,
 * held until the process ends; its address on the current device is looked
 * up once, on the first call there).  Calls that overlap on one GPU, on any
 * streams, race on that array; calls in sequence on one stream are safe
 * (every call overwrites the partials it reads).  links: the field in the
 * SoA layout of a lattice of this (nc, L, dtype), 256-byte aligned, read
 * only.  dev_out3 as for sun_plaquette; the result has the same bits as
 * sun_plaquette on a handle over the same field.  SUN_EINVAL / SUN_EUNSUP as
 * sun_lattice_bytes; SUN_ESIZE for a null pointer or a lattice whose
 * partials (16 bytes per 256 sites on the register path, per site on the
 * workgroup-per-link path: up to 33.5M and 131072 sites) exceed the array.
 * Asynchronous on stream. */
#define SUN_STATIC_SCRATCH_BYTES (2u << 20)
int sun_plaquette_static(int nc, const int L[4], int dtype, const void *links, double *dev_out3,
                         sun_stream_t stream);

/* Waits for the work queued on stream and reads the watchdog state:
 * SUN_ENUMERIC if any check since sun_watchdog tripped (the message gives
 * the number of tripped checks and the largest deviation), SUN_OK otherwise;
 * *deviation (if not NULL) receives the largest deviation a tripped check saw
 * (0 if none).  SUN_EINVAL if sun_watchdog was never called on the handle.
 * Synchronous. */
int sun_check(sun_lattice_t h, double *deviation, sun_stream_t stream);

/* Field in the canonical layout: 4*V*Nc*Nc complex FP64 values, indexed
 * [mu][s][i][j], (re, im) interleaved, on the device.  Import of Nc = 2 reads
 * row 0 of each matrix (an SU(2) matrix is fixed by it). */
int sun_export(sun_lattice_t h, double *dev_canonical, sun_stream_t stream);
int sun_import(sun_lattice_t h, const double *dev_canonical, sun_stream_t stream);

/* RNG step counter (chain state for checkpoint / resume). */
int sun_get_step(sun_lattice_t h, uint64_t *step);
int sun_set_step(sun_lattice_t h, uint64_t step);

/* Launch shape of the phase kernels of one update kind (SUN_HEATBATH,
 * SUN_OVERRELAX, or -1 for both): block work-items per workgroup (64, 128 or
 * 256), the XCD-aware workgroup order (1) or the plain order (0), a cap on
 * resident waves per CU (8, 12, 16, or 0 for none) enforced through the
 * workgroups' LDS allocation (a phase's per-XCD working set exceeds the L2,
 * so fewer resident waves raise the L2 hit rate), and the depth of the
 * t-blocked tile walk (2, 4 or 8 time slices; 0 or 1 for the linear walk):
 * the tiles of tblock consecutive time slices are walked together so that a
 * phase re-reads its t-neighbours from L2.  The t-blocked walk applies where
 * L_t is a multiple of tblock and an (x, y) plane holds a whole number of
 * workgroups (L_x L_y / 2 a multiple of block); elsewhere the linear walk
 * runs, and sun_get_launch reports the walk in effect (0 for linear).
 * Defaults: heatbath (256, 1, 16, 4); overrelaxation (256, 1, 12, 4) for
 * links of at most 48 bytes, (256, 1, 8, 4) for larger ones.  A tuning
 * choice only: results are bitwise the same for every shape. */
int sun_set_launch(sun_lattice_t h, int kind, int block, int xcd, int waves, int tblock);
int sun_get_launch(sun_lattice_t h, int kind, int *block, int *xcd, int *waves, int *tblock);

/* Sites per work-item of the phase kernels of one update kind (SUN_HEATBATH,
 * SUN_OVERRELAX, or -1 for both): 1, 2 or 4 (default 1; 2 for the heatbath
 * on lattices of at least 2048 tiles of 256 sites per parity, e.g. 32^4).  A workgroup then
 * updates that many tiles of its walk in turn and the grid is that many
 * times smaller.  Kept by sun_set_launch.  A tuning choice only: results are
 * bitwise the same. */
int sun_set_sites_per_item(sun_lattice_t h, int kind, int spt);
int sun_get_sites_per_item(sun_lattice_t h, int kind, int *spt);

/* Race check, not a tuning choice: seed != 0 makes every later phase of this
 * handle (register path, Nc <= SUN_NC_MAX_REGISTER) take the tiles of its
 * walk in a random order of its own -- a random affine permutation of the
 * walk positions, drawn from seed and the handle's phase count -- so that
 * which workgroup updates which sites, and in what order the workgroups run,
 * changes from phase to phase.  A phase's updates are independent of one
 * another (the chessboard, paper Sec. 3), so results are bitwise those of
 * the default order; a dependence between workgroups would show as a
 * difference.  seed = 0 restores the default order.  Slower (the walk no
 * longer keeps neighbour planes in L2). */
int sun_set_tile_order(sun_lattice_t h, uint64_t seed);

/* Per-kernel timing with HIP events recorded around launches on the launch
 * stream.  kernel: 0 heatbath phase, 1 overrelaxation phase,
 * 2 re-unitarization, 3 plaquette, 4 Polyakov loop.  sun_profile(h, every)
 * clears the totals and, for every > 0, brackets one launch in `every` of
 * each kernel kind with an event pair (1: every launch; a period coprime to
 * the 8 phases of an update step samples all directions and parities);
 * every = 0 stops recording.  An event pair costs a few microseconds of
 * stream time, so sampling keeps timed runs close to unprofiled ones.
 * every = -1 brackets runs instead: the heatbath phases of a sun_sweep, and
 * its overrelaxation phases, are each one run of back-to-back launches timed
 * by one event pair (the time includes the gaps between those launches, and
 * no bracket slows a launch); every other call is a run of one launch.
 * sun_profile_read synchronizes the recorded events and returns the summed
 * milliseconds and the number of launches recorded. */
int sun_profile(sun_lattice_t h, int every);
int sun_profile_read(sun_lattice_t h, int kernel, double *total_ms, int64_t *launches);

/* The SU(2) heatbath draw alone (paper Sec. 2, SU(2) heatbath), for tests:
 * for i < n draws x in SU(2) with density ~ exp(alpha[i] x0) dHaar using the
 * counter (i, step, mu_sg, ...), computing in the given dtype.  dev_x gets 4n
 * doubles, dev_attempts n ints (the accepted attempt's number, 0 = attempt
 * cap reached).  With SUN_F32_WIDE / SUN_F64_WIDE the draw is the large-Nc
 * path's, batched over eight subgroups: element i uses the counter of site
 * i / 8 and subgroup mu_sg + (i mod 8), which is the sequential draw's
 * result for that counter. */
int sun_sample_su2(int dtype, const double *dev_alpha, int n, uint64_t seed, uint32_t step,
                   uint32_t mu_sg, double *dev_x, int *dev_attempts, sun_stream_t stream);

/* ------------------------------------------------------------------------
 * Batches of independent chains (many small lattices in one launch per
 * phase).  A batch groups n lattices of any Nc, precision and extents; each
 * chain has its own coupling beta[i] and seed[i].  One launch per phase and
 * per (Nc, storage) group covers every chain of the group (register path:
 * one group per dtype; workgroup-per-link path: one per precision, a
 * workgroup per link of every chain in the group); the chains'
 * RNG step counters live in the device table, so a captured graph replays
 * with fresh random numbers.  A chain run in a batch gives bitwise the same
 * field as the same chain run alone with sun_sweep.
 * While the batch exists, drive its lattices only through it; sun_batch_sync
 * hands the advanced step counters back to the lattice handles.
 * ------------------------------------------------------------------------ */
typedef struct sun_batch_s *sun_batch_t;

/* Device bytes of the descriptor table of an n-chain batch. */
int sun_batch_bytes(int n, size_t *table_bytes);

/* Creates a batch over n existing lattice handles (which must outlive it);
 * SUN_EINVAL if two of them share link or scratch memory.  betas, seeds: host arrays of n values.  table: caller-owned device memory
 * of sun_batch_bytes() bytes, 256-byte aligned; it is written once here with
 * a synchronous copy. */
int sun_batch_create(int n, const sun_lattice_t *chains, const double *betas, const uint64_t *seeds,
                     void *table, size_t table_bytes, sun_batch_t *out);

/* One sweep of every chain (same schedule as sun_sweep).  dev_beta: NULL, or
 * a device array of n couplings in the caller's chain order, which a kernel
 * on stream copies into the table ahead of the sweep (the couplings then
 * stay in force for later sweeps given NULL, until another array or a
 * launch-shape change, which restores the couplings given at creation). */
int sun_batch_sweep(sun_batch_t b, int n_hb, int n_or, int reunit, const double *dev_beta,
                    sun_stream_t stream);

/* Mean plaquettes, FP64: dev_out[3 i .. 3 i + 2] = {total, spatial, temporal}
 * of chain i (caller's order). */
int sun_batch_plaquette(sun_batch_t b, double *dev_out, sun_stream_t stream);

/* Captures n_sweeps sweeps (each followed by the plaquettes into dev_plaq if
 * not NULL) as one HIP graph owned by the batch, replacing any earlier one.
 * With dev_beta (as for sun_batch_sweep) every captured sweep first copies
 * the couplings from that array, so each replay reads its contents at that
 * time: a coupling scan rewrites the array between replays.  stream must not
 * be the null stream.  Nothing runs until sun_batch_replay. */
int sun_batch_capture(sun_batch_t b, int n_sweeps, int n_hb, int n_or, int reunit, const double *dev_beta,
                      double *dev_plaq, sun_stream_t stream);
int sun_batch_replay(sun_batch_t b, sun_stream_t stream);

/* Launch shape of the batch's register-path phase kernels (as
 * sun_set_launch, always with the linear tile walk; default (256, 1, 0) for
 * both kinds; the workgroup-per-link groups take only its block size, as a
 * single lattice does).  Waits for the
 * device, rewrites the table, and drops any captured graph. */
int sun_batch_set_launch(sun_batch_t b, int kind, int block, int xcd, int waves);
/* Sites per work-item of the batch's phase kernels (as
 * sun_set_sites_per_item; same waiting, table rewrite and graph drop as
 * sun_batch_set_launch). */
int sun_batch_set_sites_per_item(sun_batch_t b, int kind, int spt);

/* Writes the chains' advanced RNG step counters back to their handles. */
int sun_batch_sync(sun_batch_t b);
void sun_batch_destroy(sun_batch_t b);

const char *sun_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SUN_H */
