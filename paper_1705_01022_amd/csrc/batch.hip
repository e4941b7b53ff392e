// Batched execution: many independent lattices (realisations of any size)
// advanced by one persistent kernel launch.
//
// Work items are (lattice, generation g = 4 * MCS-in-launch + step, tile).
// They are numbered generation-major and handed out in that order through a
// global ticket counter.  An item of lattice r, generation g and tile t may
// start once generation g - 1 has finished on every tile of r whose items can
// touch a memory word that (g, t) touches: a tile's items stay inside its
// "extended region", its 2D x 2D sites and the +1 halo widened to whole
// 32-site words and 4-row bands, and the neighbourhood is every tile of the
// previous generation's tiling whose extended region meets t's (the 3 x 3
// tiles around t for D >= 32 in the same tiling; around the old tile holding
// t's corner, one wider, after a new random origin).  It also waits for
// generation g - 1 of tile t itself, so every tile finishes its generations in
// order and one counter per tile ("stamp": generations finished) describes
// it.  By induction over g, every earlier item touching a word of t's extended
// region has finished when (g, t) starts (a site there lies in the extended
// region of one of the neighbourhood tiles of generation g - 1, which waited
// for the same in its own), and two items running at once never share a word.
// So the result is that of the device-wide step order of Sec. 3.1, while
// steps overlap across tiles of one lattice and across lattices.  An item only ever waits for
// items with smaller tickets, which are held by running workgroups, so the
// queue always drains; every wait is also bounded in time and a timed-out
// wait stops the whole launch with an error flag.
//
// Lattices are ordered by their MCS count of the launch (descending), so the
// lattices taking part in generation g are always a prefix of that order; the
// item numbering is described by a few "phases" of constant prefix length.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <new>

#include "internal.hpp"
#include "neighbourhood.hpp"

using namespace okpz;
using namespace okpz_host;

namespace {

struct BatchSlot {
    StepArgs a;            // lattice constants; ox, oy, set, c3 are filled per item
    uint32_t accept;       // lane draws carry acceptance variates
    uint32_t ntiles;       // tiles per device step
    uint32_t origin_mode;  // OKPZ_ORIGIN_*
    uint32_t n_mcs;        // MCS of this launch
};

struct BatchPhase {
    uint64_t first_item;     // ticket of the phase's first item
    uint32_t gen_begin;      // first generation of the phase
    uint32_t nslots;         // lattices taking part: the first nslots of the table
    uint32_t items_per_gen;  // tiles of those lattices
    uint32_t pad;
};

struct BatchArgs {
    const BatchSlot *slots;
    const uint32_t *tile_prefix;  // tile_prefix[i] = tiles of lattices 0 .. i-1
    const BatchPhase *phases;     // nphase phases, then a sentinel with first_item = total
    uint32_t nphase;
    uint64_t total_items;
    const uint64_t *mcs_base;  // MCS count of each lattice at the launch
    uint32_t *stamp;           // per tile (tile_prefix order): generations finished in this launch
    unsigned long long *ticket;
    uint32_t *error;      // sticky: set when a dependency wait timed out
    uint64_t wait_ticks;  // wait limit in wall-clock ticks
};

// Element k of permutation number `pick` (lexicographic order) of {0,1,2,3}.
__device__ __forceinline__ uint32_t perm_element(uint32_t pick, uint32_t k)
{
    uint32_t avail = 0x3210u;  // remaining elements, 4 bits each, ascending
    const uint32_t digit[4] = {pick / 6u, (pick % 6u) / 2u, pick % 2u, 0u};
    uint32_t e = 0;
    for (uint32_t i = 0; i <= k; ++i) {
        const uint32_t sh = 4u * digit[i];
        e = (avail >> sh) & 0xFu;
        const uint32_t low = avail & ((1u << sh) - 1u);
        avail = low | ((avail >> (sh + 4u)) << sh);
    }
    return e;
}

// Tiling origin of MCS m of a lattice (as the host draws it) and the word w
// whose third element picks the order of the domain sets.
__device__ __forceinline__ u32x4 mcs_origin(const BatchSlot &S, uint64_t m, uint32_t &ox, uint32_t &oy)
{
    const u32x4 w = philox4x32_10(S.a.key0, S.a.key1, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu, (uint32_t)(m << 2));
    ox = w.x & S.a.L_mask;
    oy = w.y & S.a.L_mask;
    if (S.origin_mode == OKPZ_ORIGIN_FIXED) ox = oy = 0u;
    if (S.origin_mode == OKPZ_ORIGIN_COARSE) {
        ox &= ~3u;
        oy &= ~3u;
    }
    return w;
}

// COLS: every lattice of the launch is DB with lanes x CPT cells per domain
// and at most 64 cells per row, so the column-mapped sweep serves them all.
// FL > 0 (with COLS): every lattice also draws 2^FL-bit lane fields, with
// acceptance draws iff FL = 4 and a whole number of Philox blocks of rounds,
// so the sweep with the rounds of one block unrolled serves them all.
//
// LD > 0 (with COLS and FL > 0): every lattice also has square 2^LD-site
// domains of 8 x 8-site cells, so the row-paired DB sweep serves them all.
// LD > 0 with DT or DTr: every lattice has square 128- or 256-site domains of
// 8 x 8-site cells, and each item runs the row-paired DT sweep for its
// lattice's domain size and rates.
//
// DT and DTr with at most 4 cells per lane: six waves per SIMD (80 VGPRs;
// the generic sweep spills 40 bytes to scratch for it and ran the
// 512-realisation batch 5 % faster than the five waves its unconstrained 93
// VGPRs allow; the row-paired DT sweep fits).  The row-paired DB sweep runs
// two cells per lane (63 VGPRs): with four, the batch kernel's own state on
// top of the sweep's needs 117 VGPRs (four waves), or spills at five.
template <int SCHEME, int CPT, bool COLS, int FL, int LD>
__global__ void __launch_bounds__(kMaxStepThreads)
__attribute__((amdgpu_waves_per_eu((SCHEME != kDB && CPT <= 4) || LD > 0 ? 6 : 1)))
batch_kernel(BatchArgs B)
{
    extern __shared__ uint32_t smem[];
    // lattice, tile, generation, stop; the neighbourhood to wait for: first
    // column, columns, first row, rows
    __shared__ uint32_t cmd[8];
    const uint32_t tid = threadIdx.x;
    uint32_t my_stamp = 0;
    for (;;) {
        if (tid < 64u) {
            if (tid == 0) {
                uint32_t r = 0, t = 0, g = 0, stop = 0;
                uint32_t cx0 = 0, ncol = 0, cy0 = 0, nrow = 0;
                const unsigned long long i = atomicAdd(B.ticket, 1ull);
                if (i >= B.total_items || __hip_atomic_load(B.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    stop = 1;
                } else {
                    uint32_t lo = 0, hi = B.nphase;
                    while (hi - lo > 1u) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (B.phases[mid].first_item <= i) lo = mid; else hi = mid;
                    }
                    const BatchPhase ph = B.phases[lo];
                    const uint64_t rel = i - ph.first_item;
                    g = ph.gen_begin + (uint32_t)(rel / ph.items_per_gen);
                    const uint32_t off = (uint32_t)(rel % ph.items_per_gen);
                    lo = 0;
                    hi = ph.nslots;
                    while (hi - lo > 1u) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (B.tile_prefix[mid] <= off) lo = mid; else hi = mid;
                    }
                    r = lo;
                    t = off - B.tile_prefix[r];
                    if (g > 0u) {
                        // the tiles of generation g - 1 whose words this item can share
                        const BatchSlot &S = B.slots[r];
                        const bool new_tiling = (g & 3u) == 0u;
                        uint32_t ox = 0, oy = 0, oxp = 0, oyp = 0;
                        if (new_tiling) {
                            const uint64_t m = B.mcs_base[r] + (g >> 2);
                            (void)mcs_origin(S, m, ox, oy);
                            (void)mcs_origin(S, m - 1u, oxp, oyp);
                        }
                        const WaitSet ws = wait_set(S.a.Dx, S.a.Dy, S.a.L_mask, S.a.log2ntx, S.ntiles, t,
                                                    new_tiling, ox, oy, oxp, oyp);
                        cx0 = ws.cx0;
                        ncol = ws.ncol;
                        cy0 = ws.cy0;
                        nrow = ws.nrow;
                    }
                }
                cmd[0] = r;
                cmd[1] = t;
                cmd[2] = g;
                cmd[3] = stop;
                cmd[4] = cx0;
                cmd[5] = ncol;
                cmd[6] = cy0;
                cmd[7] = nrow;
                my_stamp = stop ? 0u : B.tile_prefix[r] + t;
            }
            wave_order();
            // The first wave waits for the neighbourhood, one stamp per lane (and
            // for tile t itself, so that each tile finishes its generations in
            // order and its stamp counts them), every wait bounded in time.
            const uint32_t g = cmd[2];
            if (!cmd[3] && g > 0u) {
                const uint32_t r = cmd[0], t = cmd[1], cx0 = cmd[4], ncol = cmd[5], cy0 = cmd[6], nrow = cmd[7];
                const BatchSlot &S = B.slots[r];
                const uint32_t lx = S.a.log2ntx, ntx = 1u << lx, nty = S.ntiles >> lx;
                const uint32_t *st = B.stamp + B.tile_prefix[r];
                const uint32_t nwait = ncol * nrow + 1u;
                const uint64_t t0 = wall_clock64();
                bool bad = false;
                for (uint32_t nb = tid; nb < nwait; nb += 64u) {
                    const uint32_t nx = (cx0 + nb % ncol) & (ntx - 1u);
                    const uint32_t ny = (cy0 + nb / ncol) & (nty - 1u);
                    const uint32_t *sp = nb + 1u < nwait ? st + ((ny << lx) | nx) : st + t;
                    while (!bad && __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < g) {
                        if (__hip_atomic_load(B.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            bad = true;
                        } else if (wall_clock64() - t0 > B.wait_ticks) {
                            atomicOr(B.error, 1u);
                            bad = true;
                        } else {
                            __builtin_amdgcn_s_sleep(2);
                        }
                    }
                }
                const uint64_t any_bad = __ballot(bad);  // every lane of the wave takes part
                // the earlier steps' words, written by other workgroups, become visible
                // (the cache invalidation covers the whole workgroup's caches)
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (tid == 0 && any_bad) cmd[3] = 1u;
            }
        }
        __syncthreads();
        if (cmd[3]) break;
        const uint32_t r = __builtin_amdgcn_readfirstlane(cmd[0]);
        const uint32_t tile = __builtin_amdgcn_readfirstlane(cmd[1]);
        const uint32_t g = __builtin_amdgcn_readfirstlane(cmd[2]);
        const BatchSlot &S = B.slots[r];
        StepArgs A = S.a;
        // MCS draw of the lattice's MCS m (as on the host): origin and set order
        const uint64_t m = B.mcs_base[r] + (g >> 2);
        const uint32_t k = g & 3u;
        uint32_t ox, oy;
        const u32x4 w = mcs_origin(S, m, ox, oy);
        const uint32_t set = perm_element((uint32_t)(((uint64_t)w.z * 24u) >> 32), k);
        A.ox = ox;
        A.oy = oy;
        A.set_a = set & 1u;
        A.set_b = set >> 1;
        A.c3 = (uint32_t)(m << 2) | k;
        // Visibility of the earlier steps' words, written by other workgroups:
        // the first wave took the agent-scope acquire after its waits, before
        // the barrier above (it invalidates the caches this workgroup reads
        // through, which all its waves share).
        if constexpr (LD > 0 && SCHEME != kDB) {
            if (A.Dx == 256u) {
                if (S.accept)
                    sweep_dt_rows<SCHEME, true, CPT, 8, 3>(A, smem, tile);
                else
                    sweep_dt_rows<SCHEME, false, CPT, 8, 3>(A, smem, tile);
            } else {
                if (S.accept)
                    sweep_dt_rows<SCHEME, true, CPT, 7, 3>(A, smem, tile);
                else
                    sweep_dt_rows<SCHEME, false, CPT, 7, 3>(A, smem, tile);
            }
        } else if constexpr (LD > 0) {
            sweep_db_rows<FL == 4, CPT, LD, 3>(A, smem, tile);
        } else if constexpr (COLS && FL > 0) {
            sweep_db_columns<FL == 4, CPT, FL>(A, smem, tile);
        } else if constexpr (COLS) {
            if (S.accept)
                sweep_db_columns<true, CPT, 0>(A, smem, tile);
            else
                sweep_db_columns<false, CPT, 0>(A, smem, tile);
        } else {
            if (S.accept)
                sweep_tile<SCHEME, true, CPT, false>(A, smem, tile);
            else
                sweep_tile<SCHEME, false, CPT, false>(A, smem, tile);
        }
        // Publish this tile's words before stamping the tile with generation
        // g done: every lane waits until its own stores are acknowledged, the
        // barrier orders them before thread 0, whose agent-scope release store
        // writes them back for the other dies (once per item, not once per wave).
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) __hip_atomic_store(&B.stamp[my_stamp], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void batch_reset_kernel(uint32_t *stamp, uint32_t n, unsigned long long *ticket)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) stamp[i] = 0u;
    if (threadIdx.x == 0) *ticket = 0ull;
}

__global__ void batch_advance_kernel(uint64_t *mcs, const BatchSlot *slots, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) mcs[i] += slots[i].n_mcs;
}

constexpr uint64_t kWaitSeconds = 20;  // far above any single tile's sweep
constexpr uint32_t kStaticLds = 64;    // batch_kernel's static LDS, rounded up

// ---------------------------------------------------------------- batched measurement
// The measurement of every member in three launches: column-0 anchors (one
// workgroup per member), band moments (one wave per band of any member, bands
// numbered member-major through band_prefix) and the exact 128-bit totals
// (one workgroup per member).  Same arithmetic as the single-lattice
// measurement, only the band-to-lattice mapping differs.
struct MeasureSlot {
    const uint32_t *src;       // words measured
    int32_t *h0;               // column-0 heights of src (written)
    const uint32_t *snap;      // snapshot words (cross only)
    const int32_t *h0s;        // column-0 heights of the snapshot
    const uint32_t *copy_src;  // lattice words copied to the snapshot
    uint32_t *copy_dst;        // snapshot buffer written by the copy kernel
    uint64_t nwords;           // L^2 / 16
    uint32_t L, nbx_log2;
};

__global__ void __launch_bounds__(1024) batch_anchors_kernel(const MeasureSlot *ms)
{
    __shared__ int32_t part[1024];
    const MeasureSlot &m = ms[blockIdx.x];
    anchors_body(m.src, m.L, m.nbx_log2, m.h0, part);
}

__device__ __forceinline__ uint32_t member_of(const uint32_t *prefix, uint32_t n, uint32_t i)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

template <bool CROSS>
__global__ void __launch_bounds__(kMeasureThreads) batch_rows_kernel(const MeasureSlot *ms,
                                                                     const uint32_t *band_prefix, uint32_t n,
                                                                     int64_t *__restrict__ partial)
{
    __shared__ __align__(8) uint32_t lut[kLutWords];
    build_tables(lut);
    __syncthreads();
    const uint32_t gb = blockIdx.x * (kMeasureThreads / 64) + (threadIdx.x >> 6);
    if (gb >= band_prefix[n]) return;
    const uint32_t r = member_of(band_prefix, n, gb);
    const MeasureSlot &m = ms[r];
    rows_band<CROSS>(lut, m.src, m.h0, m.snap, m.h0s, gb - band_prefix[r], m.nbx_log2,
                     partial + static_cast<uint64_t>(gb) * kMomentFields);
}

__global__ void __launch_bounds__(256) batch_reduce_kernel(const uint32_t *band_prefix,
                                                           const int64_t *__restrict__ partial,
                                                           int64_t *__restrict__ out)
{
    __shared__ uint64_t lo_s[kMomentFields][kReduceMaxWaves];
    __shared__ int64_t hi_s[kMomentFields][kReduceMaxWaves];
    const uint32_t r = blockIdx.x;
    reduce_body(partial + static_cast<uint64_t>(band_prefix[r]) * kMomentFields, band_prefix[r + 1] - band_prefix[r],
                out + 2 * kMomentFields * r, lo_s, hi_s);
}

// Snapshot copies: chunk c of the concatenated lattices (up to 16 KiB, one
// workgroup of 256 lanes moving up to 4 x 16 B each; a lattice's last chunk
// may be partial, L^2/16 words being a multiple of 4 for L >= 64).
constexpr uint32_t kCopyChunkWords = 4096;

__global__ void __launch_bounds__(256) batch_copy_kernel(const MeasureSlot *ms, const uint32_t *chunk_prefix,
                                                         uint32_t n)
{
    const uint32_t c = blockIdx.x;
    const uint32_t r = member_of(chunk_prefix, n, c);
    const uint64_t base = static_cast<uint64_t>(c - chunk_prefix[r]) * kCopyChunkWords;
    const uint4 *src = reinterpret_cast<const uint4 *>(ms[r].copy_src + base);
    uint4 *dst = reinterpret_cast<uint4 *>(ms[r].copy_dst + base);
    const uint64_t nvec = (ms[r].nwords - base) / 4;  // > 0: chunk c lies inside lattice r
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t i = threadIdx.x + 256u * k;
        if (i < nvec) dst[i] = src[i];
    }
}

}  // namespace

struct okpz_batch {
    hipStream_t stream = nullptr;
    std::vector<okpz_lattice *> slots;  // nullptr: free slot
    int32_t scheme = -1;                // block scheme shared by all members
    // configuration (physical mapping only)
    uint32_t threads = 0;  // 0: 256
    uint32_t grid = 0;     // 0: as many workgroups as fit on the device at once
    bool use_graph = true;
    // device tables
    BatchSlot *d_slots = nullptr;
    uint32_t *d_prefix = nullptr;
    BatchPhase *d_phases = nullptr;
    uint64_t *d_mcs = nullptr;
    uint32_t *d_stamp = nullptr;
    unsigned long long *d_ticket = nullptr;
    uint32_t *d_error = nullptr;
    size_t cap_slots = 0, cap_phases = 0, cap_tiles = 0;
    // pinned staging for the tables (rewritten only after a stream sync)
    uint8_t *h_stage = nullptr;
    size_t stage_cap = 0;
    uint32_t *h_error = nullptr;
    // what the device tables hold
    std::vector<uint8_t> key;        // tables + launch shape of the captured graph
    std::vector<int32_t> table_slot; // table index -> slot
    std::vector<uint64_t> dev_mcs;   // per table index: MCS count the device holds
    hipGraphExec_t gexec = nullptr;
    bool failed = false;
    // timing
    bool timing = false;
    std::vector<TimedPair> pairs;
    uint64_t launches = 0;
    uint64_t attempts = 0;
    // batched measurement: tables, per-band partials, totals (device and pinned)
    MeasureSlot *d_meas = nullptr;
    uint32_t *d_mprefix = nullptr;  // band prefix, then chunk prefix
    int64_t *d_mpartial = nullptr;
    int64_t *d_mout = nullptr;
    uint8_t *h_mstage = nullptr;
    int64_t *h_mout = nullptr;
    size_t cap_meas = 0, cap_bands = 0;
};

namespace {

void batch_release(okpz_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (auto &tp : b->pairs) {
        (void)hipEventDestroy(tp.start);
        (void)hipEventDestroy(tp.stop);
    }
    (void)hipFree(b->d_slots);
    (void)hipFree(b->d_prefix);
    (void)hipFree(b->d_phases);
    (void)hipFree(b->d_mcs);
    (void)hipFree(b->d_stamp);
    (void)hipFree(b->d_ticket);
    (void)hipFree(b->d_error);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_error) (void)hipHostFree(b->h_error);
    (void)hipFree(b->d_meas);
    (void)hipFree(b->d_mprefix);
    (void)hipFree(b->d_mpartial);
    (void)hipFree(b->d_mout);
    if (b->h_mstage) (void)hipHostFree(b->h_mstage);
    if (b->h_mout) (void)hipHostFree(b->h_mout);
    delete b;
}

int grow_tables(okpz_batch *b, size_t nslots, size_t nphases, size_t ntiles)
{
    if (nslots > b->cap_slots) {
        const size_t cap = std::max<size_t>(nslots, 2 * b->cap_slots);
        (void)hipFree(b->d_slots);
        (void)hipFree(b->d_prefix);
        (void)hipFree(b->d_mcs);
        b->d_slots = nullptr;
        b->d_prefix = nullptr;
        b->d_mcs = nullptr;
        b->cap_slots = 0;
        if (hipMalloc(&b->d_slots, cap * sizeof(BatchSlot)) != hipSuccess ||
            hipMalloc(&b->d_prefix, (cap + 1) * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&b->d_mcs, cap * sizeof(uint64_t)) != hipSuccess)
            return OKPZ_ENOMEM;
        b->cap_slots = cap;
    }
    if (ntiles > b->cap_tiles) {
        const size_t cap = std::max<size_t>(ntiles, 2 * b->cap_tiles);
        (void)hipFree(b->d_stamp);
        b->d_stamp = nullptr;
        b->cap_tiles = 0;
        if (hipMalloc(&b->d_stamp, cap * sizeof(uint32_t)) != hipSuccess) return OKPZ_ENOMEM;
        b->cap_tiles = cap;
    }
    if (nphases + 1 > b->cap_phases) {
        const size_t cap = std::max<size_t>(nphases + 1, 2 * b->cap_phases);
        (void)hipFree(b->d_phases);
        b->d_phases = nullptr;
        b->cap_phases = 0;
        if (hipMalloc(&b->d_phases, cap * sizeof(BatchPhase)) != hipSuccess) return OKPZ_ENOMEM;
        b->cap_phases = cap;
    }
    const size_t need = b->cap_slots * (sizeof(BatchSlot) + sizeof(uint32_t) + sizeof(uint64_t)) + sizeof(uint32_t) +
                        8 + b->cap_phases * sizeof(BatchPhase);
    if (need > b->stage_cap) {
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        b->h_stage = nullptr;
        b->stage_cap = 0;
        if (hipHostMalloc(&b->h_stage, need, hipHostMallocDefault) != hipSuccess) return OKPZ_ENOMEM;
        b->stage_cap = need;
    }
    return OKPZ_OK;
}

template <int SCHEME, int CPT, bool COLS, int FL = 0, int LD = 0>
const void *batch_fn()
{
    return reinterpret_cast<const void *>(&batch_kernel<SCHEME, CPT, COLS, FL, LD>);
}

const void *batch_kernel_for(int scheme, uint32_t cpt, bool cols, int fl, int ld)
{
    if (scheme != kDB && ld) {
        switch (cpt * 4 + (uint32_t)(scheme == kDTR ? 1 : 0)) {
        case 4: return batch_fn<kDT, 1, false, 0, 8>();
        case 5: return batch_fn<kDTR, 1, false, 0, 8>();
        case 8: return batch_fn<kDT, 2, false, 0, 8>();
        case 9: return batch_fn<kDTR, 2, false, 0, 8>();
        case 16: return batch_fn<kDT, 4, false, 0, 8>();
        case 17: return batch_fn<kDTR, 4, false, 0, 8>();
        default: return nullptr;
        }
    }
    if (cpt == 2 && ld == 8) return fl == 4 ? batch_fn<kDB, 2, true, 4, 8>() : batch_fn<kDB, 2, true, 3, 8>();
    if (cpt == 2 && ld == 7) return fl == 4 ? batch_fn<kDB, 2, true, 4, 7>() : batch_fn<kDB, 2, true, 3, 7>();
#define OKPZ_BATCH_CASES(S)                          \
    switch (cpt) {                                   \
    case 1: return batch_fn<S, 1, false>();          \
    case 2: return batch_fn<S, 2, false>();          \
    case 4: return batch_fn<S, 4, false>();          \
    case 8: return batch_fn<S, 8, false>();          \
    case 16: return batch_fn<S, 16, false>();        \
    default: return nullptr;                         \
    }
    if (cols && scheme == kDB && fl == 4) {
        switch (cpt) {
        case 2: return batch_fn<kDB, 2, true, 4>();
        case 4: return batch_fn<kDB, 4, true, 4>();
        case 8: return batch_fn<kDB, 8, true, 4>();
        default: break;
        }
    }
    if (cols && scheme == kDB && fl == 3) {
        switch (cpt) {
        case 2: return batch_fn<kDB, 2, true, 3>();
        case 4: return batch_fn<kDB, 4, true, 3>();
        case 8: return batch_fn<kDB, 8, true, 3>();
        default: break;
        }
    }
    if (cols && scheme == kDB) {
        switch (cpt) {
        case 2: return batch_fn<kDB, 2, true>();
        case 4: return batch_fn<kDB, 4, true>();
        case 8: return batch_fn<kDB, 8, true>();
        case 16: return batch_fn<kDB, 16, true>();
        default: break;
        }
    }
    switch (scheme) {
    case kDT: OKPZ_BATCH_CASES(kDT)
    case kDB: OKPZ_BATCH_CASES(kDB)
    case kDTR: OKPZ_BATCH_CASES(kDTR)
    default: return nullptr;
    }
#undef OKPZ_BATCH_CASES
}

// The launches of one batch run, in stream order: reset counters, the
// persistent kernel, advance the per-lattice MCS counts.
struct LaunchPlan {
    const void *fn;
    uint32_t threads, grid, nslots, ntiles;
    size_t lds;
    BatchArgs args;
};

int enqueue(okpz_batch *b, const LaunchPlan &lp)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1024), 0, b->stream, b->d_stamp, lp.ntiles, b->d_ticket);
    void *kargs[] = {const_cast<BatchArgs *>(&lp.args)};
    HIP_TRY(hipLaunchKernel(lp.fn, dim3(lp.grid), dim3(lp.threads), kargs, lp.lds, b->stream));
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(256), 0, b->stream, b->d_mcs, b->d_slots, lp.nslots);
    HIP_TRY(hipGetLastError());
    return OKPZ_OK;
}

int batch_check_error(okpz_batch *b)
{
    HIP_TRY(hipMemcpyAsync(b->h_error, b->d_error, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (*b->h_error) b->failed = true;
    return b->failed ? OKPZ_EWAIT : OKPZ_OK;
}

}  // namespace

extern "C" {

int okpz_batch_create(void *hip_stream, okpz_batch **out)
{
    if (!out) return OKPZ_EINVAL;
    *out = nullptr;
    okpz_batch *b = new (std::nothrow) okpz_batch();
    if (!b) return OKPZ_ENOMEM;
    b->stream = (hipStream_t)hip_stream;
    b->use_graph = hip_stream != nullptr;  // the null stream cannot be captured
    if (hipMalloc(&b->d_ticket, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&b->d_error, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&b->h_error, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        batch_release(b);
        return OKPZ_ENOMEM;
    }
    *b->h_error = 0;
    if (hipMemcpyAsync(b->d_error, b->h_error, sizeof(uint32_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        batch_release(b);
        return OKPZ_EHIP;
    }
    *out = b;
    return OKPZ_OK;
}

int okpz_batch_destroy(okpz_batch *b)
{
    if (!b) return OKPZ_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    return OKPZ_OK;
}

int okpz_batch_add(okpz_batch *b, okpz_lattice *lat, int32_t *slot)
{
    if (!b || !lat || !slot) return OKPZ_EINVAL;
    if (lat->stream != b->stream) return OKPZ_EINVAL;
    if (b->scheme >= 0 && lat->prm.block_scheme != b->scheme) return OKPZ_EINVAL;
    if (lat->prm.device_layer != OKPZ_DEVICE_DT)
        return fail_with(OKPZ_EINVAL, "okpz_batch_add: the dead-border control runs on single lattices only");
    for (okpz_lattice *m : b->slots)
        if (m == lat) return OKPZ_EINVAL;
    int32_t s = -1;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (!b->slots[i]) {
            s = (int32_t)i;
            break;
        }
    if (s < 0) {
        s = (int32_t)b->slots.size();
        b->slots.push_back(nullptr);
    }
    b->slots[s] = lat;
    b->scheme = lat->prm.block_scheme;
    *slot = s;
    return OKPZ_OK;
}

int okpz_batch_remove(okpz_batch *b, int32_t slot)
{
    if (!b || slot < 0 || (size_t)slot >= b->slots.size() || !b->slots[slot]) return OKPZ_EINVAL;
    // the lattice may be destroyed right after: finish what uses it
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->slots[slot] = nullptr;
    bool any = false;
    for (okpz_lattice *m : b->slots) any |= m != nullptr;
    if (!any) b->scheme = -1;
    while (!b->slots.empty() && !b->slots.back()) b->slots.pop_back();
    b->key.clear();  // tables refer to the removed lattice
    return OKPZ_OK;
}

int okpz_batch_size(const okpz_batch *b, uint32_t *nslots)
{
    if (!b || !nslots) return OKPZ_EINVAL;
    *nslots = (uint32_t)b->slots.size();
    return OKPZ_OK;
}

int okpz_batch_wait_set(uint32_t L, uint32_t dom_x, uint32_t dom_y, uint32_t tile, int32_t new_tiling, uint32_t ox,
                        uint32_t oy, uint32_t oxp, uint32_t oyp, uint32_t *out)
{
    if (!out || !is_pow2(L) || !is_pow2(dom_x) || !is_pow2(dom_y) || 2ull * dom_x > L || 2ull * dom_y > L)
        return OKPZ_EINVAL;
    const uint32_t log2ntx = ilog2(L / (2u * dom_x));
    const uint32_t ntiles = (L / (2u * dom_x)) * (L / (2u * dom_y));
    if (tile >= ntiles || ox >= L || oy >= L || oxp >= L || oyp >= L) return OKPZ_EINVAL;
    const okpz::WaitSet w = okpz::wait_set(dom_x, dom_y, L - 1u, log2ntx, ntiles, tile, new_tiling != 0, ox, oy, oxp, oyp);
    out[0] = w.cx0;
    out[1] = w.ncol;
    out[2] = w.cy0;
    out[3] = w.nrow;
    return OKPZ_OK;
}

int okpz_batch_config(okpz_batch *b, uint32_t threads, uint32_t grid, int use_graph)
{
    if (!b) return OKPZ_EINVAL;
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512) return OKPZ_EINVAL;
    if (use_graph && !b->stream) return OKPZ_EINVAL;
    b->threads = threads;
    b->grid = grid;
    b->use_graph = use_graph != 0;
    b->key.clear();
    return OKPZ_OK;
}

}  // extern "C"

namespace {

// One persistent launch (reset, batch kernel, advance) for the members with
// n_mcs[s] > 0, already validated; 4 * n_mcs * tiles < 2^31 for each.
uint64_t tiles_of(const okpz_params &prm) { return (uint64_t)(prm.L / (2 * prm.dom_x)) * (prm.L / (2 * prm.dom_y)); }

int batch_run_once(okpz_batch *b, const uint64_t *n_mcs, const double *p, const double *q)
{
    const size_t ns = b->slots.size();
    std::vector<int32_t> order;
    for (size_t s = 0; s < ns; ++s)
        if (n_mcs[s] > 0) order.push_back((int32_t)s);
    if (order.empty()) return OKPZ_OK;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return n_mcs[a] > n_mcs[c]; });
    const uint32_t n = (uint32_t)order.size();

    // launch shape: lanes per workgroup (default: enough for the largest
    // domain's cells, 64 .. 256, at most half of them from 256 cells on),
    // cells per lane
    uint32_t max_cells = 1;
    for (int32_t s : order) max_cells = std::max(max_cells, cells_of(b->slots[s]->prm));
    uint32_t nt = b->threads;
    if (nt == 0) {
        uint64_t tiles = 0;
        for (int32_t s : order) tiles += tiles_of(b->slots[s]->prm);
        int dev = 0, cus = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const uint32_t cap = default_threads(tiles, (uint32_t)std::max(cus, 1), max_cells);
        nt = 64;
        while (nt < cap && nt < max_cells) nt *= 2;
    }
    uint32_t cpt = 1;
    while (cpt * nt < max_cells) cpt *= 2;
    if (cpt > 16) return OKPZ_EINVAL;
    // DB lattices that all fill the workgroup exactly take the column-mapped sweep
    bool cols = b->scheme == kDB && cpt >= 2;
    for (int32_t s : order) {
        const okpz_params &prm = b->slots[s]->prm;
        cols = cols && cells_of(prm) == nt * cpt && prm.dom_x / prm.cell_x <= 64u;
    }

    // tables
    std::vector<BatchSlot> slots(n);
    std::vector<uint32_t> prefix(n + 1, 0);
    size_t lds = 0;
    uint64_t attempts = 0;
    for (uint32_t i = 0; i < n; ++i) {
        okpz_lattice *lat = b->slots[order[i]];
        const okpz_params &prm = lat->prm;
        const double pd = p[order[i]], qr = q[order[i]];
        const LaneShape ls = lane_shape(prm, pd, qr);
        BatchSlot &S = slots[i];
        std::memset(&S, 0, sizeof(S));
        S.a = base_args(lat, ls, pd, qr);
        S.accept = ls.accept ? 1u : 0u;
        S.ntiles = (prm.L / (2 * prm.dom_x)) * (prm.L / (2 * prm.dom_y));
        S.origin_mode = (uint32_t)prm.origin_mode;
        S.n_mcs = (uint32_t)n_mcs[order[i]];
        prefix[i + 1] = prefix[i] + S.ntiles;
        lds = std::max<size_t>(lds, step_lds_bytes(prm, cols ? nt : nt * cpt));  // columns: one slot per lane
        attempts += (uint64_t)prm.L * prm.L * S.n_mcs;
    }
    // the kernel's own 16 bytes of static LDS come on top
    if (lds > kMaxLds - kStaticLds) return OKPZ_EINVAL;
    std::vector<BatchPhase> phases;
    uint64_t total = 0;
    {
        uint32_t gen = 0;
        uint32_t count = n;
        while (count > 0) {
            const uint32_t gen_end = 4u * slots[count - 1].n_mcs;
            if (gen_end > gen) {
                BatchPhase ph;
                ph.first_item = total;
                ph.gen_begin = gen;
                ph.nslots = count;
                ph.items_per_gen = prefix[count];
                ph.pad = 0;
                phases.push_back(ph);
                total += (uint64_t)(gen_end - gen) * prefix[count];
                gen = gen_end;
            }
            --count;
        }
        BatchPhase end;
        std::memset(&end, 0, sizeof(end));
        end.first_item = total;
        phases.push_back(end);
    }
    const uint32_t nphase = (uint32_t)phases.size() - 1;

    // one lane-field width for every member: the sweep with unrolled rounds
    int fl = 0;
    if (cols && cpt <= 8) {
        fl = slots[0].accept ? 4 : 3;
        for (uint32_t i = 0; i < n; ++i)
            if ((int)slots[i].a.F_log2 != fl || (slots[i].accept != 0) != (fl == 4) ||
                slots[i].a.rounds % (128u >> fl) != 0u)
                fl = 0;
    }
    // square 128- or 256-site domains of 8 x 8-site cells throughout: the
    // row-paired sweep (its own LDS size), two cells per lane: four per lane
    // take twice the lanes
    int ld = 0;
    if (fl > 0 && (cpt == 2 || (cpt == 4 && 2 * nt <= (uint32_t)kMaxStepThreads))) {
        const uint32_t d0 = slots[0].a.Dx;
        ld = d0 == 256u ? 8 : d0 == 128u ? 7 : 0;
        for (uint32_t i = 0; i < n && ld; ++i) {
            const StepArgs &a = slots[i].a;
            if (a.Dx != d0 || a.Dy != d0 || a.log2Cx != 3u || a.log2Cy != 3u || a.s_bits != 6u) ld = 0;
        }
        if (ld && cpt == 4) {
            nt *= 2;
            cpt = 2;
        }
        if (ld == 8) lds = 4u * rowpair_lds_words<8, 3>(nt);
        if (ld == 7) lds = 4u * rowpair_lds_words<7, 3>(nt);
    }
    // DT / DTr with square 128- or 256-site domains of 8 x 8-site cells
    // throughout, at most four cells per lane: the row-paired DT sweep (the
    // window alone in LDS)
    if (b->scheme != kDB && cpt <= 4) {
        bool rows = true, any256 = false;
        for (uint32_t i = 0; i < n && rows; ++i) {
            const StepArgs &a = slots[i].a;
            rows = a.Dx == a.Dy && (a.Dx == 256u || a.Dx == 128u) && a.log2Cx == 3u && a.log2Cy == 3u &&
                   a.s_bits == 4u && !a.shared_edges && a.F_log2 == (slots[i].accept ? 4u : 2u);
            any256 = any256 || a.Dx == 256u;
        }
        if (rows) {
            ld = 8;
            lds = 4u * (any256 ? rowpair_dt_lds_words<8, 3>() : rowpair_dt_lds_words<7, 3>());
        }
    }
    const void *fn = batch_kernel_for(b->scheme, cpt, cols, fl, ld);
    if (!fn) return OKPZ_EINVAL;
    if (lds > 64u * 1024u)
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLds - kStaticLds)));
    uint32_t grid = b->grid;
    if (grid == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)nt, lds));
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        grid = (uint32_t)std::max(1, per_cu * cus);
        // no more workgroups than tiles in one step of all members: a workgroup
        // beyond them would only wait for the next step's dependencies while
        // sharing its compute unit with a working one
        grid = std::min(grid, prefix[n]);
    }
    grid = (uint32_t)std::min<uint64_t>(grid, total);

    // identity of the tables and the launch shape: an unchanged key replays the graph
    std::vector<uint8_t> key(sizeof(BatchSlot) * n + sizeof(uint32_t) * (n + 1) + sizeof(BatchPhase) * phases.size() +
                             4 * sizeof(uint32_t));
    {
        uint8_t *k = key.data();
        std::memcpy(k, slots.data(), sizeof(BatchSlot) * n);
        k += sizeof(BatchSlot) * n;
        std::memcpy(k, prefix.data(), sizeof(uint32_t) * (n + 1));
        k += sizeof(uint32_t) * (n + 1);
        std::memcpy(k, phases.data(), sizeof(BatchPhase) * phases.size());
        k += sizeof(BatchPhase) * phases.size();
        const uint32_t shape[4] = {nt, cpt | (cols ? 0x100u : 0u) | ((uint32_t)fl << 16) | ((uint32_t)ld << 24), grid,
                                   b->use_graph ? 1u : 0u};
        std::memcpy(k, shape, sizeof(shape));
    }
    std::vector<int32_t> table_slot(order.begin(), order.end());
    const bool same_tables = key == b->key && table_slot == b->table_slot;
    bool mcs_current = same_tables;
    if (same_tables)
        for (uint32_t i = 0; i < n; ++i) mcs_current &= b->dev_mcs[i] == b->slots[order[i]]->mcs;

    if (!same_tables || !mcs_current) {
        HIP_TRY(hipStreamSynchronize(b->stream));  // the staging buffer may still be read
        const int rc = grow_tables(b, n, phases.size(), prefix[n]);
        if (rc != OKPZ_OK) return rc;
        uint8_t *st = b->h_stage;
        BatchSlot *hs = reinterpret_cast<BatchSlot *>(st);
        std::memcpy(hs, slots.data(), sizeof(BatchSlot) * n);
        uint64_t *hm = reinterpret_cast<uint64_t *>(hs + n);
        for (uint32_t i = 0; i < n; ++i) hm[i] = b->slots[order[i]]->mcs;
        uint32_t *hp = reinterpret_cast<uint32_t *>(hm + n);
        std::memcpy(hp, prefix.data(), sizeof(uint32_t) * (n + 1));
        BatchPhase *hph = reinterpret_cast<BatchPhase *>(
            reinterpret_cast<uint8_t *>(hp) + ((sizeof(uint32_t) * (n + 1) + 7) & ~size_t(7)));
        std::memcpy(hph, phases.data(), sizeof(BatchPhase) * phases.size());
        HIP_TRY(hipMemcpyAsync(b->d_slots, hs, sizeof(BatchSlot) * n, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->d_mcs, hm, sizeof(uint64_t) * n, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->d_prefix, hp, sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->d_phases, hph, sizeof(BatchPhase) * phases.size(), hipMemcpyHostToDevice,
                               b->stream));
        b->dev_mcs.assign(n, 0);
        for (uint32_t i = 0; i < n; ++i) b->dev_mcs[i] = b->slots[order[i]]->mcs;
    }

    LaunchPlan lp;
    lp.fn = fn;
    lp.threads = nt;
    lp.grid = grid;
    lp.nslots = n;
    lp.ntiles = prefix[n];
    lp.lds = lds;
    lp.args.slots = b->d_slots;
    lp.args.tile_prefix = b->d_prefix;
    lp.args.phases = b->d_phases;
    lp.args.nphase = nphase;
    lp.args.total_items = total;
    lp.args.mcs_base = b->d_mcs;
    lp.args.stamp = b->d_stamp;
    lp.args.ticket = b->d_ticket;
    lp.args.error = b->d_error;
    {
        int dev = 0, khz = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        lp.args.wait_ticks = (uint64_t)std::max(khz, 1) * 1000ull * kWaitSeconds;
    }

    TimedPair tp;
    tp.kind = 0;
    if (b->timing) {
        HIP_TRY(hipEventCreate(&tp.start));
        HIP_TRY(hipEventCreate(&tp.stop));
        HIP_TRY(hipEventRecord(tp.start, b->stream));
    }
    if (b->use_graph) {
        if (!same_tables || !b->gexec) {
            if (b->gexec) {
                (void)hipGraphExecDestroy(b->gexec);
                b->gexec = nullptr;
            }
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue(b, lp);
            const hipError_t ec = hipStreamEndCapture(b->stream, &graph);
            if (rc != OKPZ_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
            const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                b->gexec = nullptr;
                return hip_fail(ei, "hipGraphInstantiate");
            }
        }
        HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
    } else {
        const int rc = enqueue(b, lp);
        if (rc != OKPZ_OK) return rc;
    }
    if (b->timing) {
        HIP_TRY(hipEventRecord(tp.stop, b->stream));
        b->pairs.push_back(tp);
    }
    b->key.swap(key);
    b->table_slot.swap(table_slot);
    for (uint32_t i = 0; i < n; ++i) {
        okpz_lattice *lat = b->slots[order[i]];
        lat->mcs += slots[i].n_mcs;
        b->dev_mcs[i] = lat->mcs;
    }
    b->launches += 1;
    b->attempts += attempts;
    return OKPZ_OK;
}


}  // namespace

extern "C" {

int okpz_batch_run(okpz_batch *b, const uint64_t *n_mcs, const double *p, const double *q)
{
    if (!b || !n_mcs || !p || !q) return OKPZ_EINVAL;
    if (b->failed) return OKPZ_EWAIT;
    const size_t ns = b->slots.size();
    // validate everything before anything is launched
    uint64_t max_n = 0;
    for (size_t s = 0; s < ns; ++s) {
        if (n_mcs[s] == 0) continue;
        okpz_lattice *lat = b->slots[s];
        if (!lat) return OKPZ_EINVAL;
        if (!(p[s] >= 0.0 && p[s] <= 1.0 && q[s] >= 0.0 && q[s] <= 1.0)) return OKPZ_EINVAL;
        if (n_mcs[s] > kMcsLimit || lat->mcs + n_mcs[s] > kMcsLimit) return OKPZ_EOVERFLOW;
        max_n = std::max(max_n, n_mcs[s]);
    }
    // launches of at most `chunk` MCS per lattice keep the per-lattice item
    // counters below 2^31
    uint64_t chunk = max_n;
    for (size_t s = 0; s < ns; ++s)
        if (n_mcs[s] > 0) chunk = std::min<uint64_t>(chunk, ((uint64_t(1) << 31) - 1) / (4 * tiles_of(b->slots[s]->prm)));
    std::vector<uint64_t> left(n_mcs, n_mcs + ns), part(ns);
    while (max_n > 0) {
        for (size_t s = 0; s < ns; ++s) part[s] = std::min(left[s], chunk);
        const int rc = batch_run_once(b, part.data(), p, q);
        if (rc != OKPZ_OK) return rc;
        max_n = 0;
        for (size_t s = 0; s < ns; ++s) {
            left[s] -= part[s];
            max_n = std::max(max_n, left[s]);
        }
    }
    return OKPZ_OK;
}

int okpz_batch_sync(okpz_batch *b)
{
    if (!b) return OKPZ_EINVAL;
    return batch_check_error(b);
}

int okpz_batch_timing(okpz_batch *b, int enable)
{
    if (!b) return OKPZ_EINVAL;
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (auto &tp : b->pairs) {
        (void)hipEventDestroy(tp.start);
        (void)hipEventDestroy(tp.stop);
    }
    b->pairs.clear();
    b->timing = enable != 0;
    b->launches = 0;
    b->attempts = 0;
    return OKPZ_OK;
}

int okpz_batch_get_timing(okpz_batch *b, double *ms, uint64_t *launches, uint64_t *attempts)
{
    if (!b) return OKPZ_EINVAL;
    HIP_TRY(hipStreamSynchronize(b->stream));
    double total = 0;
    for (auto &tp : b->pairs) {
        float e = 0;
        HIP_TRY(hipEventElapsedTime(&e, tp.start, tp.stop));
        total += e;
    }
    if (ms) *ms = total;
    if (launches) *launches = b->launches;
    if (attempts) *attempts = b->attempts;
    return OKPZ_OK;
}

}  // extern "C"

namespace {

int grow_measure(okpz_batch *b, size_t n, size_t bands)
{
    if (n > b->cap_meas) {
        const size_t cap = std::max<size_t>(n, 2 * b->cap_meas);
        (void)hipFree(b->d_meas);
        (void)hipFree(b->d_mprefix);
        (void)hipFree(b->d_mout);
        if (b->h_mstage) (void)hipHostFree(b->h_mstage);
        if (b->h_mout) (void)hipHostFree(b->h_mout);
        b->d_meas = nullptr;
        b->d_mprefix = nullptr;
        b->d_mout = nullptr;
        b->h_mstage = nullptr;
        b->h_mout = nullptr;
        b->cap_meas = 0;
        if (hipMalloc(&b->d_meas, cap * sizeof(MeasureSlot)) != hipSuccess ||
            hipMalloc(&b->d_mprefix, 2 * (cap + 1) * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&b->d_mout, cap * 2 * kMomentFields * sizeof(int64_t)) != hipSuccess ||
            hipHostMalloc(&b->h_mstage, cap * sizeof(MeasureSlot) + 2 * (cap + 1) * sizeof(uint32_t),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&b->h_mout, cap * 2 * kMomentFields * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
            return OKPZ_ENOMEM;
        b->cap_meas = cap;
    }
    if (bands > b->cap_bands) {
        const size_t cap = std::max<size_t>(bands, 2 * b->cap_bands);
        (void)hipFree(b->d_mpartial);
        b->d_mpartial = nullptr;
        b->cap_bands = 0;
        if (hipMalloc(&b->d_mpartial, cap * kMomentFields * sizeof(int64_t)) != hipSuccess) return OKPZ_ENOMEM;
        b->cap_bands = cap;
    }
    return OKPZ_OK;
}

// Measures every member (slot order) and leaves each member's 128-bit totals
// in its host_out.  of_snapshot: copy the words to the snapshot first and
// measure the snapshot (its anchors go to h0s); cross: also the sums against
// the snapshot.  Synchronises the stream; a failed earlier batch launch is
// reported as OKPZ_EWAIT.
int batch_measure(okpz_batch *b, const std::vector<okpz_lattice *> &mem, bool of_snapshot, bool cross)
{
    const size_t n = mem.size();
    if (n == 0) return OKPZ_OK;
    if (n > 0xFFFFFFFFull / 2) return OKPZ_EINVAL;
    std::vector<MeasureSlot> ms(n);
    std::vector<uint32_t> bp(n + 1, 0), cp(n + 1, 0);
    for (size_t i = 0; i < n; ++i) {
        okpz_lattice *lat = mem[i];
        const uint32_t L = lat->prm.L;
        MeasureSlot &m = ms[i];
        m.src = of_snapshot ? lat->snap : lat->words;
        m.h0 = of_snapshot ? lat->h0s : lat->h0;
        m.snap = cross ? lat->snap : nullptr;
        m.h0s = cross ? lat->h0s : nullptr;
        m.copy_src = of_snapshot ? lat->words : nullptr;
        m.copy_dst = of_snapshot ? lat->snap : nullptr;
        m.nwords = (uint64_t)L * L / 16;
        m.L = L;
        m.nbx_log2 = ilog2(L / 32);
        const uint64_t bands = (uint64_t)bp[i] + L / 4;
        const uint64_t chunks = (uint64_t)cp[i] + (m.nwords + kCopyChunkWords - 1) / kCopyChunkWords;
        if (bands > 0xFFFFFFFFull || chunks > 0xFFFFFFFFull) return OKPZ_EINVAL;
        bp[i + 1] = (uint32_t)bands;
        cp[i + 1] = (uint32_t)chunks;
    }
    // the staging buffer and the tables may still be in use by a previous
    // measurement only if it failed half-way: wait for the stream first
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int rc = grow_measure(b, n, bp[n]);
    if (rc != OKPZ_OK) return rc;
    MeasureSlot *hs = reinterpret_cast<MeasureSlot *>(b->h_mstage);
    std::memcpy(hs, ms.data(), n * sizeof(MeasureSlot));
    uint32_t *hp = reinterpret_cast<uint32_t *>(hs + n);
    std::memcpy(hp, bp.data(), (n + 1) * sizeof(uint32_t));
    std::memcpy(hp + n + 1, cp.data(), (n + 1) * sizeof(uint32_t));
    HIP_TRY(hipMemcpyAsync(b->d_meas, hs, n * sizeof(MeasureSlot), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_mprefix, hp, 2 * (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, b->stream));
    const uint32_t *d_bp = b->d_mprefix, *d_cp = b->d_mprefix + n + 1;
    if (of_snapshot)
        hipLaunchKernelGGL(batch_copy_kernel, dim3(cp[n]), dim3(256), 0, b->stream, b->d_meas, d_cp, (uint32_t)n);
    hipLaunchKernelGGL(batch_anchors_kernel, dim3((uint32_t)n), dim3(1024), 0, b->stream, b->d_meas);
    const uint32_t per_block = kMeasureThreads / 64;
    const uint32_t blocks = (bp[n] + per_block - 1) / per_block;
    if (cross)
        hipLaunchKernelGGL((batch_rows_kernel<true>), dim3(blocks), dim3(kMeasureThreads), 0, b->stream, b->d_meas,
                           d_bp, (uint32_t)n, b->d_mpartial);
    else
        hipLaunchKernelGGL((batch_rows_kernel<false>), dim3(blocks), dim3(kMeasureThreads), 0, b->stream, b->d_meas,
                           d_bp, (uint32_t)n, b->d_mpartial);
    hipLaunchKernelGGL(batch_reduce_kernel, dim3((uint32_t)n), dim3(256), 0, b->stream, d_bp, b->d_mpartial,
                       b->d_mout);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(b->h_mout, b->d_mout, n * 2 * kMomentFields * sizeof(int64_t), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->h_error, b->d_error, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (*b->h_error) b->failed = true;
    if (b->failed) return OKPZ_EWAIT;
    for (size_t i = 0; i < n; ++i)
        std::memcpy(mem[i]->host_out, b->h_mout + 2 * kMomentFields * i, 2 * kMomentFields * sizeof(int64_t));
    return OKPZ_OK;
}

std::vector<okpz_lattice *> members_of(const okpz_batch *b)
{
    std::vector<okpz_lattice *> mem;
    for (okpz_lattice *m : b->slots)
        if (m) mem.push_back(m);
    return mem;
}

int batch_snapshot(okpz_batch *b)
{
    const std::vector<okpz_lattice *> mem = members_of(b);
    for (okpz_lattice *lat : mem) {
        const uint32_t L = lat->prm.L;
        if (!lat->snap && hipMalloc(&lat->snap, (size_t)L * L / 4) != hipSuccess) {
            lat->snap = nullptr;
            return OKPZ_ENOMEM;
        }
        if (!lat->h0s && hipMalloc(&lat->h0s, L * sizeof(int32_t)) != hipSuccess) {
            lat->h0s = nullptr;
            return OKPZ_ENOMEM;
        }
        lat->has_snap = false;
    }
    const int rc = batch_measure(b, mem, true, false);
    if (rc != OKPZ_OK) return rc;
    for (okpz_lattice *lat : mem) {
        lat->snap_s1 = pair_to_i128(lat->host_out + 0) + pair_to_i128(lat->host_out + 2);
        lat->snap_mcs = lat->mcs;
        lat->has_snap = true;
    }
    return OKPZ_OK;
}

int batch_observe(okpz_batch *b, okpz_moments *moments, okpz_correlation *corr)
{
    const std::vector<okpz_lattice *> mem = members_of(b);
    if (corr)
        for (okpz_lattice *lat : mem)
            if (!lat->has_snap) return OKPZ_ESTATE;
    const int rc = batch_measure(b, mem, false, corr != nullptr);
    if (rc != OKPZ_OK) return rc;
    for (size_t s = 0; s < b->slots.size(); ++s) {
        okpz_lattice *lat = b->slots[s];
        if (!lat) {
            std::memset(&moments[s], 0, sizeof(okpz_moments));
            if (corr) std::memset(&corr[s], 0, sizeof(okpz_correlation));
            continue;
        }
        fill_moments(lat, &moments[s]);
        if (corr) fill_correlation(lat, &corr[s]);
    }
    return OKPZ_OK;
}

}  // namespace

extern "C" {

int okpz_batch_snapshot(okpz_batch *b)
{
    if (!b) return OKPZ_EINVAL;
    if (b->failed) return OKPZ_EWAIT;
    return batch_snapshot(b);
}

int okpz_batch_observe(okpz_batch *b, okpz_moments *moments, okpz_correlation *corr)
{
    if (!b || !moments) return OKPZ_EINVAL;
    if (b->failed) return OKPZ_EWAIT;
    return batch_observe(b, moments, corr);
}

int okpz_batch_series(okpz_batch *b, const uint64_t *times, size_t n_times, const double *p, const double *q,
                      okpz_moments *moments, okpz_correlation *corr)
{
    if (!b || (n_times > 0 && (!times || !moments)) || !p || !q) return OKPZ_EINVAL;
    if (b->failed) return OKPZ_EWAIT;
    const size_t ns = b->slots.size();
    for (size_t i = 1; i < n_times; ++i)
        if (times[i] < times[i - 1]) return OKPZ_EINVAL;
    if (n_times > 0 && times[n_times - 1] > kMcsLimit) return OKPZ_EOVERFLOW;
    for (size_t s = 0; s < ns; ++s) {
        okpz_lattice *lat = b->slots[s];
        if (!lat) continue;
        if (!(p[s] >= 0.0 && p[s] <= 1.0 && q[s] >= 0.0 && q[s] <= 1.0)) return OKPZ_EINVAL;
        if (n_times > 0 && lat->mcs + times[n_times - 1] > kMcsLimit) return OKPZ_EOVERFLOW;
        if (corr && !lat->has_snap) return OKPZ_ESTATE;
    }
    std::vector<uint64_t> step(ns);
    uint64_t t = 0;
    for (size_t i = 0; i < n_times; ++i) {
        for (size_t s = 0; s < ns; ++s) step[s] = b->slots[s] ? times[i] - t : 0;
        t = times[i];
        int rc = okpz_batch_run(b, step.data(), p, q);
        if (rc != OKPZ_OK) return rc;
        rc = batch_observe(b, moments + i * ns, corr ? corr + i * ns : nullptr);
        if (rc != OKPZ_OK) return rc;
    }
    return OKPZ_OK;
}

}  // extern "C"
