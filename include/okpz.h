/*
 * okpz.h - C ABI of the MI355X (gfx950) octahedron-model KPZ simulator.
 *
 * The library runs random-sequential (RS) updates of the 2+1-dimensional
 * octahedron model (Kelling, Odor, Gemming, arXiv:1705.01022, Sec. 2.1) on a
 * GPU-resident, bit-packed slope lattice, parallelised by double tiling with
 * a random origin every Monte Carlo step (DTr, Sec. 3) across workgroups and
 * single-hit DT, DB (delayed borders) or DTr updates of thread cells inside
 * each workgroup (Sec. 3.1).  It also measures the roughness W^2 (Sec. 2.1)
 * and the height autocorrelation C_h(t,s) (Sec. 2.1) with exact integer
 * reductions.
 *
 * Conventions
 *   - Sites (x, y) in [0, L)^2, periodic, x fast.  Slope bits per site:
 *     sx = 1 iff h(x,y) - h(x-1,y) = +1, sy = 1 iff h(x,y) - h(x,y-1) = +1
 *     (each site keeps its slopes towards the left and lower neighbours,
 *     Sec. 3, DB scheme).
 *   - Host site arrays ("sites") are L*L bytes, index y*L + x,
 *     bit 0 = sx, bit 1 = sy, other bits zero.
 *   - Packed device layout ("words", 2 bits per site as in the paper's
 *     bit-coded lattice, Sec. 3.1, arranged as row bit-planes): the lattice
 *     is cut into blocks of 32 x 4 sites; block (x/32, y/4) has index
 *     (y/4)*(L/32) + x/32 and owns 8 consecutive uint32 words: word y%4 holds
 *     the sx bits of row y, word 4 + y%4 the sy bits, bit x%32.  L*L/4 bytes.
 *   - One MCS is L*L update attempts (Sec. 2.1, time unit).
 *   - Heights use the gauge h(0,0) = 0; every reported observable is
 *     invariant under the gauge.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by
 *     (seed, stream), counters built from (MCS, step, tile, cell, round), so
 *     results depend only on the parameters and the sequence of run calls:
 *     never on launch shape, batch composition or stream.
 *
 * Errors: every call returns OKPZ_OK (0) or a negative status; on OKPZ_EHIP
 * okpz_last_error() holds the HIP error text of the calling thread.  A
 * failed call leaves the lattice unchanged unless it says otherwise.
 *
 * Threading: one handle must not be used by two threads at once; different
 * handles are independent.  All work of a handle runs on its HIP stream, in
 * order; calls that return host data synchronise that stream.
 *
 * Ownership: the library owns every device buffer it allocates and frees it
 * in okpz_destroy.  Buffers passed by the caller stay the caller's.
 */
#ifndef OKPZ_H
#define OKPZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define OKPZ_OK 0
#define OKPZ_EINVAL (-1)    /* invalid argument or parameter combination     */
#define OKPZ_ENOMEM (-2)    /* device or host allocation failed               */
#define OKPZ_EHIP (-3)      /* HIP runtime error, see okpz_last_error()        */
#define OKPZ_EOVERFLOW (-4) /* a counter or an exact reduction would overflow  */
#define OKPZ_ESTATE (-5)    /* call not valid in the current state             */
#define OKPZ_EWAIT (-6)     /* a batch kernel's dependency wait timed out      */

/* block-level (thread-cell) decomposition schemes, Sec. 3.1 */
#define OKPZ_BLOCK_DT 0  /* single-hit double tiling: random quadrant per round  */
#define OKPZ_BLOCK_DB 1  /* single-hit dead border, delayed borders, random cell origin per round */
#define OKPZ_BLOCK_DTR 2 /* single-hit DT with the cell origin re-drawn per round */

/* device-level origin of the decomposition */
#define OKPZ_ORIGIN_RANDOM 0 /* DTr: uniform over all sites every MCS (Sec. 3, DTr)     */
#define OKPZ_ORIGIN_FIXED 1  /* plain DT: origin stays at (0,0) (negative control)      */
#define OKPZ_ORIGIN_COARSE 2 /* origin on the 4x4-site word grid (cDB with _DEVICE_DB)  */

/* device-level decomposition (Sec. 3) */
#define OKPZ_DEVICE_DT 0 /* double tiling: four domain sets, four steps per MCS (DTr) */
#define OKPZ_DEVICE_DB 1 /* dead border: every dom_x x dom_y tile in one step per MCS,
                            its last column and last row inactive (negative control) */

/*
 * Simulation parameters.  Physics parameters (Sec. 3.1 notation DTrDT etc.
 * and TC=log2(cell_x/4),log2(cell_y/4)):
 *   L             lateral size, power of two, 64 <= L <= 2^17
 *   dom_x, dom_y  device domain (sub-tile) size in sites; tiles are
 *                 2*dom_x x 2*dom_y (dead border: dom_x x dom_y, the whole
 *                 tile active but for its last column and row).  Powers of
 *                 two, >= 4, 2*dom <= L; the
 *                 staged window, two bit planes of (dom_y + 4) rows by
 *                 (dom_x/32 + 3) words (plus 8 bytes per cell for DB), must
 *                 fit 160 KiB of LDS (dom_x <= 7936).
 *   cell_x,cell_y thread-cell size in sites, powers of two, 2 .. 64,
 *                 cell <= dom, at most 4096 cells per domain.
 *                 (TC=1,1 is 8 x 8 sites.)
 *   block_scheme  OKPZ_BLOCK_DT / _DB / _DTR
 *   seed, stream  Philox key; one stream per independent realization
 *   origin_mode   OKPZ_ORIGIN_RANDOM (the method) or a negative control
 *   device_layer  OKPZ_DEVICE_DT (the method) or OKPZ_DEVICE_DB, the dead
 *                 border control (with OKPZ_ORIGIN_COARSE the paper's cDB,
 *                 Sec. 4.1): one step per MCS over all tiles, counter
 *                 c3 = 4 MCS; an attempt drawn on a tile's last column or
 *                 row is not carried out.  Single lattices only (batches and
 *                 the server reject it).
 */
typedef struct okpz_params {
    uint32_t L;
    uint32_t dom_x, dom_y;
    uint32_t cell_x, cell_y;
    int32_t block_scheme;
    uint32_t seed;
    uint32_t stream;
    int32_t origin_mode;
    uint32_t device_layer; /* OKPZ_DEVICE_DT or OKPZ_DEVICE_DB */
} okpz_params;

/* 128-bit two's-complement integer: value = hi * 2^64 + lo */
typedef struct okpz_i128 {
    uint64_t lo;
    int64_t hi;
} okpz_i128;

/*
 * Exact height moments split by sublattice parity ((x+y) even / odd):
 * n = number of sites, s1 = sum of h, s2 = sum of h^2 (gauge h(0,0) = 0).
 *   w2     = (N*S2 - S1^2) / N^2 with N = L^2, S = even + odd: the roughness
 *            of Sec. 2.1 taken literally (1/4 on the flat zig-zag surface).
 *   w2_sub = mean of the two within-parity variances (0 on every flat
 *            surface; 0 <= w2 - w2_sub <= 1/4).
 * Both doubles are the exact rational values rounded once to nearest.
 */
typedef struct okpz_moments {
    uint64_t mcs;
    int64_t n_even, n_odd;
    okpz_i128 s1_even, s1_odd, s2_even, s2_odd;
    double w2, w2_sub;
} okpz_moments;

/*
 * Autocorrelations between the current state (time t) and the snapshot
 * (time s), Sec. 2.1:
 *   heights: C_h(t,s) = <h_t h_s> - <h_t><h_s> over sites (C_h(s,s) = W^2(s)).
 *     s_ts = sum h_t h_s, s1_t = sum h_t, s1_s = sum h_s;
 *     c_h = (N s_ts - s1_t s1_s) / N^2 rounded once to nearest.
 *   slopes (the lattice gas): C_s(t,s) = <n_t n_s> - <n_t><n_s> over the
 *     2 L^2 slope variables (sx and sy of every site), where particle
 *     conservation fixes <n> = 1/2 in every state.  overlap = number of slope
 *     variables equal to 1 in both states; c_s = overlap / (2 L^2) - 1/4
 *     (exact).
 */
typedef struct okpz_correlation {
    uint64_t t, s;
    okpz_i128 s_ts, s1_t, s1_s;
    double c_h;
    int64_t overlap;
    double c_s;
} okpz_correlation;

typedef struct okpz_lattice okpz_lattice;

/* Status text for a code (static string, never NULL). */
const char *okpz_strerror(int status);

/* Last HIP error text of the calling thread ("" if none). */
const char *okpz_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int okpz_version(void);

/*
 * Check parameters without allocating anything.  Returns OKPZ_OK or
 * OKPZ_EINVAL.  Writes the packed lattice size in bytes to *nbytes if
 * nbytes is not NULL.
 */
int okpz_validate(const okpz_params *params, size_t *nbytes);

/*
 * Create a lattice in the flat zig-zag state h = (x+y) mod 2 at MCS 0 on
 * the HIP stream `hip_stream` (a hipStream_t; NULL = the default stream).
 * Allocates the packed lattice (L*L/4 bytes) and small measurement buffers
 * (about 28*L bytes) on the current device.  *out receives the handle.
 */
int okpz_create(const okpz_params *params, void *hip_stream, okpz_lattice **out);

/*
 * As okpz_create, but the packed lattice lives in caller-owned device memory
 * `dev_words` of `nbytes` >= L*L/4 bytes (e.g. a torch tensor), 256-byte
 * aligned.  The caller keeps it alive until okpz_destroy.  The contents are
 * overwritten with the flat state.
 */
int okpz_create_external(const okpz_params *params, void *hip_stream, void *dev_words,
                         size_t nbytes, okpz_lattice **out);

/* Free the handle and every buffer the library allocated for it. */
int okpz_destroy(okpz_lattice *lat);

/* Reset to the flat zig-zag state at MCS 0; drops any snapshot. */
int okpz_init_flat(okpz_lattice *lat);

/*
 * Load a state from host `sites` (L*L bytes, see Conventions) and set the
 * MCS counter to `mcs` (< 2^30).  Rejects (OKPZ_EINVAL, lattice unchanged)
 * any array with bits other than 0-1 set or that is not a valid periodic
 * surface: every row needs L/2 set sx bits, every column L/2 set sy bits,
 * and sx[x,y-1] + sy[x,y] = sy[x-1,y] + sx[x,y] on every plaquette.
 * Drops any snapshot.  Synchronous.
 */
int okpz_init_from_host(okpz_lattice *lat, const uint8_t *sites, uint64_t mcs);

/*
 * Advance n_mcs Monte Carlo steps at deposition probability p and removal
 * probability q (0 <= p, q <= 1; Sec. 2.1 rule).  Each MCS draws a fresh
 * random tiling origin and an order of the four domain sets and sweeps them
 * (Sec. 3, DTr); with device_layer OKPZ_DEVICE_DB it sweeps every tile in one
 * step instead, their rims inactive (Sec. 3 DB).  Asynchronous on the
 * handle's stream.  OKPZ_EOVERFLOW if the MCS counter would reach 2^30.
 */
int okpz_run(okpz_lattice *lat, uint64_t n_mcs, double p, double q);

/* Exact height moments of the current state.  Synchronous. */
int okpz_measure(okpz_lattice *lat, okpz_moments *out);

/*
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid allocation): the exact
 * height moments of okpz_measure for a packed lattice in caller-owned device
 * memory, without a handle and without allocating anything.
 *   dev_words   device pointer to the L*L/4-byte packed lattice (layout of
 *               Conventions), caller-owned, read only.
 *   L           lattice size, power of two, 64 <= L <= 2^17 (the limit of the
 *               library's fixed 2 MiB device scratch array; larger: EINVAL).
 *   hip_stream  stream the kernels run on (a hipStream_t; NULL = null stream).
 *   dev_totals  device pointer, caller-owned, 8-byte aligned, 96 bytes:
 *               receives the exact totals as 6 (lo, hi) int64 pairs of
 *               128-bit integers: S1 even, S1 odd, S2 even, S2 odd, then two
 *               zero pairs.
 *   out         NULL: the call only enqueues three kernels on hip_stream and
 *               returns (asynchronous).  Otherwise a host struct: the call
 *               synchronises the stream and fills it as okpz_measure does,
 *               with mcs = 0 (there is no handle to count MCS).
 * The intermediate buffers live in the library's file-scope device array,
 * one per device for the life of the process (its address is looked up on
 * the first call on each device).  Every call on a device shares it: calls
 * that overlap on one device (two streams or two threads) race; calls on one
 * stream are ordered.  EINVAL for NULL or misaligned pointers or an L out of
 * range (okpz_last_error says which).
 */
int okpz_measure_noalloc(const void *dev_words, uint32_t L, void *hip_stream, int64_t *dev_totals,
                         okpz_moments *out);

/* Store the current state as the reference time s for okpz_autocorr. */
int okpz_snapshot(okpz_lattice *lat);

/* C_h(t, s) against the snapshot (OKPZ_ESTATE if none).  Synchronous. */
int okpz_autocorr(okpz_lattice *lat, okpz_correlation *out);

/*
 * Both observables from one pass over the lattice: the exact height moments
 * (as okpz_measure) into *moments and, if corr is not NULL, C_h(t, s)
 * against the snapshot (as okpz_autocorr; OKPZ_ESTATE without a snapshot).
 * Synchronous.
 */
int okpz_observe(okpz_lattice *lat, okpz_moments *moments, okpz_correlation *corr);

/*
 * Checkpoint and resume.  okpz_save writes the lattice state (and, if
 * with_snapshot, the snapshot of okpz_snapshot with its time s) to host_buf
 * as a self-describing blob of okpz_checkpoint_size bytes: a 128-byte header
 * (magic, format version, the lattice parameters, MCS count, word count and
 * a 64-bit checksum) followed by the words in the device layout.  The caller
 * owns the buffer.  okpz_load restores such a blob into a lattice created
 * with the same parameters (all okpz_params fields equal, seed and stream
 * included, so that the resumed run draws the same random numbers as an
 * uninterrupted one): the state, the MCS count and, when saved, the snapshot.
 * EINVAL for a short buffer, another format or version, other parameters, a
 * checksum mismatch or a state that is not a height configuration (a slope
 * plaquette that does not close, or nonzero slope sums along row 0 or
 * column 0); the lattice is unchanged then.  ESTATE: with_snapshot without a
 * snapshot.  Both synchronous.
 */
int okpz_checkpoint_size(const okpz_lattice *lat, int with_snapshot, size_t *nbytes);
int okpz_save(okpz_lattice *lat, int with_snapshot, void *host_buf, size_t nbytes);
int okpz_load(okpz_lattice *lat, const void *host_buf, size_t nbytes);

/* Copy the state to host `sites` (L*L bytes).  Synchronous. */
int okpz_get_sites(okpz_lattice *lat, uint8_t *sites);

/*
 * Copy the w x h window with corner (x0, y0) (periodic) to host `sites`
 * (w*h bytes, index j*w + i is site (x0+i, y0+j) mod L).  Synchronous.
 */
int okpz_get_window(okpz_lattice *lat, uint32_t x0, uint32_t y0, uint32_t w, uint32_t h,
                    uint8_t *sites);

/*
 * Overwrite the w x h window at (x0, y0) from host `sites` (same layout as
 * okpz_get_window).  The whole resulting state is NOT re-validated (this is
 * meant for small, known perturbations of large lattices); the caller is
 * responsible for keeping it a valid surface.  A snapshot taken earlier is
 * kept (it describes the earlier state).  Synchronous.
 */
int okpz_set_window(okpz_lattice *lat, uint32_t x0, uint32_t y0, uint32_t w, uint32_t h,
                    const uint8_t *sites);

/* Heights (gauge h(0,0) = 0) to host `heights` (L*L int32).  Synchronous. */
int okpz_get_heights(okpz_lattice *lat, int32_t *heights);

/* Packed lattice words to / from host (L*L/16 uint32).  Synchronous. */
int okpz_get_words(okpz_lattice *lat, uint32_t *words);

/* Device pointer and size of the packed lattice (owned by the handle). */
int okpz_device_words(okpz_lattice *lat, void **dev_words, size_t *nbytes);

/* MCS counter (number of MCS applied since the flat start). */
int okpz_get_mcs(const okpz_lattice *lat, uint64_t *mcs);

/*
 * Workgroup size of the device-step kernel: 64, 128, 256 or 512 threads, or
 * 0 for the default (512 when a device step has fewer tiles than four per
 * compute unit, else 256; at most ncell / 2 when the domain has 256 thread
 * cells or more, so that each thread holds two or more).  Each thread then
 * updates ncell / threads thread
 * cells (at most 16, else OKPZ_EINVAL).  A physical mapping only: the simulated
 * lattice does not depend on it (every random draw is keyed by cell, not by
 * thread).  Chosen by an autotuner per domain shape.
 */
int okpz_set_threads(okpz_lattice *lat, uint32_t threads);

/* Copy the parameters the handle was created with. */
int okpz_get_params(const okpz_lattice *lat, okpz_params *out);

/* Wait for all queued work of the handle. */
int okpz_sync(okpz_lattice *lat);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around
 * every launch of the device-step kernel (four per MCS) and of the
 * measurement kernels.  okpz_timing(lat, 1) enables and zeroes the
 * counters; okpz_timing(lat, 0) disables.  okpz_get_timing synchronises and
 * returns total milliseconds and launch counts.
 */
int okpz_timing(okpz_lattice *lat, int enable);
int okpz_get_timing(okpz_lattice *lat, double *step_ms, uint64_t *step_launches,
                    double *measure_ms, uint64_t *measure_launches);

/*
 * Device Philox4x32-10 (SC'11) on n counters: ctr and out are host arrays of
 * 4*n uint32 (counter words c0..c3 / output words per block), key = (k0, k1).
 * For testing the generator the step kernel uses.  Synchronous.
 */
int okpz_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, size_t n);

/* ------------------------------------------------------------------------
 * Batches: many independent lattices (realisations, each with its own
 * size, decomposition, seed/stream and rates) advanced together by ONE
 * persistent kernel launch per okpz_batch_run call.  The launch hands out
 * work items (lattice, MCS, device step, tile) in MCS-major order from a
 * device-wide queue; an item starts once its lattice's previous device step
 * has finished on every tile, i.e. each lattice keeps the step order of
 * Sec. 3 / Sec. 3.1 (DTr at device level) while the steps of different
 * lattices overlap.  Every member's result is bit-identical to running it
 * alone with okpz_run (random draws are keyed by lattice, MCS, step, tile,
 * cell and round only).
 *
 * Members are ordinary okpz_lattice handles created on the batch's stream;
 * the batch does not own them.  All members share one block scheme.  Every
 * okpz_* call on a member (measure, snapshot, get_sites, run, ...) stays
 * valid and is ordered with the batch's work on the shared stream.  Remove
 * a member before destroying it.
 *
 * Launches are captured once into a HIP graph and replayed while the
 * membership, the per-member MCS counts and rates, and the launch shape stay
 * the same (not available on the null stream).
 * ------------------------------------------------------------------------ */
typedef struct okpz_batch okpz_batch;

/* New empty batch whose work runs on hip_stream (a hipStream_t, or NULL:
 * the null stream, then without graph capture). */
int okpz_batch_create(void *hip_stream, okpz_batch **out);

/* Synchronise and free the batch (not its members). */
int okpz_batch_destroy(okpz_batch *batch);

/* Add a lattice; *slot receives its index (the lowest free one).  EINVAL if
 * the lattice is already a member, uses another stream or another block
 * scheme than the current members. */
int okpz_batch_add(okpz_batch *batch, okpz_lattice *lat, int32_t *slot);

/* Remove the member at slot (synchronises the stream first). */
int okpz_batch_remove(okpz_batch *batch, int32_t slot);

/* Number of slot indices in use (highest member index + 1); the arrays of
 * okpz_batch_run have this length. */
int okpz_batch_size(const okpz_batch *batch, uint32_t *nslots);

/*
 * Launch shape (physical mapping only; results do not depend on it):
 * threads per workgroup (64, 128, 256, 512, or 0: enough lanes for the
 * largest domain's cells, at most 256, or 512 when the launch has fewer
 * tiles per step than four per compute unit, and at most half the cells of
 * a domain of 256 cells or more), persistent workgroups
 * (0 = as many as fit on the device at once, but no more than the members'
 * tiles in one step), use_graph (capture and replay the launch).  Chosen by
 * the autotuner of the Python layer.
 */
int okpz_batch_config(okpz_batch *batch, uint32_t threads, uint32_t grid, int use_graph);

/*
 * Advance member s by n_mcs[s] MCS at rates p[s], q[s] (Sec. 2.1 rule),
 * for every slot s < okpz_batch_size (n_mcs[s] = 0: member idle; free
 * slots must have n_mcs = 0).  Asynchronous on the batch's stream; the host
 * arrays may be reused on return.  Everything is validated before anything
 * runs (EINVAL, EOVERFLOW past 2^30 MCS).  Runs longer than 2^31 / (4 x
 * tiles) MCS of any member are split into several launches.
 * EWAIT if an earlier launch of this batch failed (see okpz_batch_sync).
 */
int okpz_batch_run(okpz_batch *batch, const uint64_t *n_mcs, const double *p, const double *q);

/* Wait for the batch's work; OKPZ_EWAIT if a launch stopped on a timed-out
 * dependency wait (the members' lattices are then undefined and the batch
 * refuses further runs). */
int okpz_batch_sync(okpz_batch *batch);

/* HIP-event timing of the batch launches (as okpz_timing); get_timing
 * returns total milliseconds, launches and update attempts since enabled. */
int okpz_batch_timing(okpz_batch *batch, int enable);
int okpz_batch_get_timing(okpz_batch *batch, double *ms, uint64_t *launches, uint64_t *attempts);

/*
 * Observables of every member at once: the exact height moments W^2 and
 * W^2_sub (Eq. `eq:Wdef`, as okpz_measure) into moments[s] and, if corr is
 * not NULL, C_h(t, s) (Eq. `eq:kpz_ac_C`) and C_s against each member's snapshot
 * into corr[s], for every slot s < okpz_batch_size (free slots are zeroed).
 * Three launches for the whole batch (anchors, band moments, exact totals),
 * whatever the number of members; values are identical to okpz_observe on
 * each member.  Synchronous.  OKPZ_ESTATE if corr is given and a member has
 * no snapshot; OKPZ_EWAIT after a failed batch launch.
 */
int okpz_batch_observe(okpz_batch *batch, okpz_moments *moments, okpz_correlation *corr);

/* Snapshot of every member (as okpz_snapshot on each: the reference time s
 * of C_h(t, s)), in one copy launch plus the measurement launches.
 * Synchronous. */
int okpz_batch_snapshot(okpz_batch *batch);

/*
 * A measured series: for i = 0 .. n_times-1, advance every member to
 * times[i] MCS past its count at the call (times non-decreasing; rates
 * p[s], q[s] as in okpz_batch_run) and observe all members there:
 * moments[i * nslots + s] and, if corr is not NULL, corr[i * nslots + s]
 * (nslots = okpz_batch_size).  The log-spaced measurement times of the
 * roughness and autocorrelation curves (Sec. 2.1, Sec. 4.2) for a whole
 * ensemble of realisations.  Validates everything first (EINVAL, EOVERFLOW,
 * ESTATE without snapshots when corr is given).  Synchronous.
 */
int okpz_batch_series(okpz_batch *batch, const uint64_t *times, size_t n_times, const double *p, const double *q,
                      okpz_moments *moments, okpz_correlation *corr);

/* Dependency neighbourhood of a batch work item, the same function the batch
 * kernel evaluates on the device (exposed so that it can be checked on the
 * host).  The item is tile `tile` (row-major, L/(2 dom_x) tiles per row) of
 * one device step of a lattice of size L with domains dom_x x dom_y (Sec. 3
 * DTr: the step's domains are sub-tiles of the MCS's 2 dom_x x 2 dom_y
 * tiling); new_tiling != 0 says the step is the first of an MCS with origin
 * (ox, oy) whose previous MCS had origin (oxp, oyp) (otherwise the origins are
 * ignored but must be < L).  out[0..3] = first tile column, number of
 * columns, first tile row, number of rows (modulo the tiles per row / column)
 * of the previous step's tiles the item waits for, besides its own tile:
 * every tile of the previous step's tiling whose memory words can meet the
 * item's.  EINVAL for invalid sizes or a tile / origin out of range.  Host
 * only; touches no device.
 */
int okpz_batch_wait_set(uint32_t L, uint32_t dom_x, uint32_t dom_y, uint32_t tile, int32_t new_tiling, uint32_t ox,
                        uint32_t oy, uint32_t oxp, uint32_t oyp, uint32_t *out);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching (the system pattern that
 * keeps many independent realisations of Sec. 4's studies resident at once).  Requests (lattice
 * parameters, MCS count, rates) are queued from any thread; a native worker
 * thread admits them in arrival order while their device footprint fits the
 * HBM budget and a member slot is free (flat initial lattice, resident on
 * the GPU until the request retires), advances every admitted request by up
 * to chunk_mcs MCS per tick -- one persistent batch launch per block scheme
 * present among the admitted requests (a batch holds one scheme), queued
 * back to back on the server's stream -- and retires
 * finished requests: final moments (as okpz_measure), optionally the final
 * sites, timestamps.  Requests arriving while others run join at the next
 * tick.  Each result equals running the request alone (okpz_create +
 * okpz_run) bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct okpz_server okpz_server;

typedef struct okpz_server_config {
    uint64_t hbm_budget;  /* device bytes admitted requests may hold (> 0)          */
    uint32_t max_members; /* requests on the GPU at once (> 0)                      */
    uint32_t chunk_mcs;   /* MCS per request per tick (> 0)                         */
    uint32_t threads;     /* batch launch shape, see okpz_batch_config (0 = default) */
    uint32_t grid;
    int32_t use_graph;    /* capture/replay ticks (ignored on the null stream)     */
    uint32_t reserved;    /* 0 */
} okpz_server_config;

/* Result of one request.  Times are seconds on the server's steady clock
 * (0 at okpz_server_create): submitted, admitted to the GPU, finished. */
typedef struct okpz_result {
    uint64_t id;
    int32_t status; /* OKPZ_OK or the error that ended the request */
    uint32_t L;
    uint64_t n_mcs;
    okpz_moments moments; /* at the end of the run */
    double t_submit, t_start, t_finish;
} okpz_result;

typedef struct okpz_server_stats {
    uint64_t submitted, finished, queued, admitted;
    uint64_t ticks;       /* batch launches                               */
    uint64_t attempts;    /* update attempts done                         */
    uint64_t max_members; /* most requests on the GPU at once             */
    double busy_seconds;  /* wall time inside ticks (launch to sync)      */
    double clock;         /* server clock now                             */
} okpz_server_stats;

/* Start a server whose GPU work runs on hip_stream (NULL: null stream) of
 * the calling thread's current device. */
int okpz_server_create(const okpz_server_config *cfg, void *hip_stream, okpz_server **out);

/* Queue a request (validated as okpz_create / okpz_run; ENOMEM if it can
 * never fit the budget).  sites_out: NULL or an L*L host buffer (layout of
 * okpz_get_sites) that receives the final state and must stay valid until
 * the result has been polled.  *id numbers requests from 0. */
int okpz_server_submit(okpz_server *srv, const okpz_params *params, uint64_t n_mcs, double p, double q,
                       uint8_t *sites_out, uint64_t *id);

/* Move up to max finished results into out (completion order); *n = count.
 * Never blocks. */
int okpz_server_poll(okpz_server *srv, okpz_result *out, uint32_t max, uint32_t *n);

/* Block until every submitted request has finished (OKPZ_ESTATE on
 * timeout); returns the first error the worker met, else OKPZ_OK. */
int okpz_server_drain(okpz_server *srv, double timeout_seconds);

int okpz_server_get_stats(okpz_server *srv, okpz_server_stats *out);

/* Drop queued requests, finish the admitted ones, stop the worker, free. */
int okpz_server_destroy(okpz_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* OKPZ_H */
