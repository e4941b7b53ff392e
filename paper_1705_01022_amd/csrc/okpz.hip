// C ABI of the MI355X octahedron-model simulator: host side.
//
// Each Monte Carlo step (MCS) draws a fresh random origin and a random
// order of the four domain sets of the double tiling (Sec. 3, DTr) and
// launches the device-step kernel once per set; the kernel boundary is the
// device-wide synchronisation between sets (Sec. 3.1).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdio>
#include <new>

#include "internal.hpp"

using namespace okpz;
using namespace okpz_host;

namespace okpz_host {

namespace {
thread_local std::string g_last_error;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return OKPZ_EHIP;
}

int fail_with(int status, const char *what)
{
    g_last_error = what;
    return status;
}

}  // namespace okpz_host

namespace {

// Launch one device-step kernel instance (LDS above 64 KiB needs the
// attribute raised once per instance and process).
template <typename Kernel>
int launch_instance(Kernel *fn, uint32_t nt, uint32_t ntiles, size_t lds, hipStream_t st, const StepArgs &a)
{
    if (lds > 64u * 1024u) {
        static bool raised = false;
        if (!raised) {
            HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds));
            raised = true;
        }
    }
    hipLaunchKernelGGL(fn, dim3(ntiles), dim3(nt), lds, st, a);
    return OKPZ_OK;
}

// The row-paired DB kernel for its shapes: square 128- or 256-site domains
// of 8 x 8-site cells (lane draws of 6 site bits in 16-bit fields with
// acceptance prefixes, 8-bit without), two or four cells per lane.
template <bool ACCEPT, int CPT>
bool launch_db_rows(uint32_t nt, uint32_t ntiles, hipStream_t st, const StepArgs &a, int &rc)
{
    if constexpr (CPT == 2 || CPT == 4) {
        constexpr uint32_t FL = ACCEPT ? 4u : 3u;
        if (a.Dx != a.Dy || a.log2Cx != 3u || a.log2Cy != 3u || a.s_bits != 6u || a.F_log2 != FL ||
            a.shared_edges)
            return false;
        if (a.Dx == 256u) {
            rc = launch_instance(&step_db_rows_kernel<ACCEPT, CPT, 8, 3>, nt, ntiles,
                                 4u * rowpair_lds_words<8, 3>(nt), st, a);
            return true;
        }
        if (a.Dx == 128u) {
            rc = launch_instance(&step_db_rows_kernel<ACCEPT, CPT, 7, 3>, nt, ntiles,
                                 4u * rowpair_lds_words<7, 3>(nt), st, a);
            return true;
        }
    }
    return false;
}

// The row-paired DT / DTr kernel for square 128- or 256-site domains of
// 8 x 8-site cells (4 site bits per lane draw, in 16-bit fields with
// acceptance prefixes, 4-bit fields without), one to four cells per lane.
template <int SCHEME, bool ACCEPT, int CPT>
bool launch_dt_rows(uint32_t nt, uint32_t ntiles, hipStream_t st, const StepArgs &a, int &rc)
{
    if constexpr ((SCHEME == kDT || SCHEME == kDTR) && (CPT == 1 || CPT == 2 || CPT == 4)) {
        constexpr uint32_t FL = ACCEPT ? 4u : 2u;
        if (a.Dx != a.Dy || a.log2Cx != 3u || a.log2Cy != 3u || a.s_bits != 4u || a.F_log2 != FL ||
            a.shared_edges)
            return false;
        if (a.Dx == 256u) {
            rc = launch_instance(&step_dt_rows_kernel<SCHEME, ACCEPT, CPT, 8, 3>, nt, ntiles,
                                 4u * rowpair_dt_lds_words<8, 3>(), st, a);
            return true;
        }
        if (a.Dx == 128u) {
            rc = launch_instance(&step_dt_rows_kernel<SCHEME, ACCEPT, CPT, 7, 3>, nt, ntiles,
                                 4u * rowpair_dt_lds_words<7, 3>(), st, a);
            return true;
        }
    }
    return false;
}

// DB runs the row-paired kernel where it applies, else, with at least two
// cells per lane and at most 64 cells per domain row, the column-mapped
// kernel (same results, less bookkeeping than the generic one).
template <int SCHEME, bool ACCEPT, int CPT>
int launch_step_inst(uint32_t nt, uint32_t ntiles, size_t lds, hipStream_t st, const StepArgs &a)
{
    // the dead-border control runs the generic kernel (the only one that
    // masks the tiles' rims and XORs back the words they share)
    if (a.dev_db) return launch_instance(&step_kernel<SCHEME, ACCEPT, CPT>, nt, ntiles, lds, st, a);
    if constexpr (SCHEME != kDB) {
        int rc = OKPZ_OK;
        if (launch_dt_rows<SCHEME, ACCEPT, CPT>(nt, ntiles, st, a, rc)) return rc;
    }
    if constexpr (SCHEME == kDB && CPT >= 2) {
        int rc = OKPZ_OK;
        if (launch_db_rows<ACCEPT, CPT>(nt, ntiles, st, a, rc)) return rc;
        if ((1u << a.log2ncx) <= 64u) {
            // the column kernel publishes one top-cell site per lane, not one per cell
            lds -= 8u * nt * (CPT - 1);
            // the common field widths (16 bits with acceptance draws, 8 without)
            // with whole Philox blocks per domain sweep take the unrolled variant
            constexpr int FL = ACCEPT ? 4 : 3;
            if constexpr (CPT <= 8) {
                if (a.F_log2 == (uint32_t)FL && a.rounds % (128u >> FL) == 0u)
                    return launch_instance(&step_db_columns_kernel<ACCEPT, CPT, FL>, nt, ntiles, lds, st, a);
            }
            return launch_instance(&step_db_columns_kernel<ACCEPT, CPT, 0>, nt, ntiles, lds, st, a);
        }
    }
    return launch_instance(&step_kernel<SCHEME, ACCEPT, CPT>, nt, ntiles, lds, st, a);
}

template <int SCHEME, bool ACCEPT>
int launch_step_cpt(uint32_t cpt, uint32_t nt, uint32_t ntiles, size_t lds, hipStream_t st, const StepArgs &a)
{
    switch (cpt) {
    case 1: return launch_step_inst<SCHEME, ACCEPT, 1>(nt, ntiles, lds, st, a);
    case 2: return launch_step_inst<SCHEME, ACCEPT, 2>(nt, ntiles, lds, st, a);
    case 4: return launch_step_inst<SCHEME, ACCEPT, 4>(nt, ntiles, lds, st, a);
    case 8: return launch_step_inst<SCHEME, ACCEPT, 8>(nt, ntiles, lds, st, a);
    case 16: return launch_step_inst<SCHEME, ACCEPT, 16>(nt, ntiles, lds, st, a);
    default: return OKPZ_EINVAL;
    }
}

int launch_step(okpz_lattice *lat, const StepArgs &a, bool accept)
{
    const okpz_params &p = lat->prm;
    const uint32_t ncell = a.ncell;
    const uint32_t span = a.dev_db ? 1u : 2u;  // dead border: every dom_x x dom_y tile in one step
    const uint32_t ntiles = (p.L / (span * p.dom_x)) * (p.L / (span * p.dom_y));
    uint32_t cpt, nt;
    step_shape(ncell, lat->threads ? lat->threads : default_threads(ntiles, lat->cus, ncell), cpt, nt);
    if (cpt > 16) return OKPZ_EINVAL;
    const size_t lds = step_lds_bytes(p, nt * cpt);
    int rc;
    switch (p.block_scheme * 2 + (accept ? 1 : 0)) {
    case 0: rc = launch_step_cpt<kDT, false>(cpt, nt, ntiles, lds, lat->stream, a); break;
    case 1: rc = launch_step_cpt<kDT, true>(cpt, nt, ntiles, lds, lat->stream, a); break;
    case 2: rc = launch_step_cpt<kDB, false>(cpt, nt, ntiles, lds, lat->stream, a); break;
    case 3: rc = launch_step_cpt<kDB, true>(cpt, nt, ntiles, lds, lat->stream, a); break;
    case 4: rc = launch_step_cpt<kDTR, false>(cpt, nt, ntiles, lds, lat->stream, a); break;
    default: rc = launch_step_cpt<kDTR, true>(cpt, nt, ntiles, lds, lat->stream, a); break;
    }
    if (rc != OKPZ_OK) return rc;
    HIP_TRY(hipGetLastError());
    return OKPZ_OK;
}

int fill_flat(okpz_lattice *lat)
{
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(4096, (lat->nwords + 255) / 256);
    hipLaunchKernelGGL(fill_flat_kernel, dim3(blocks), dim3(256), 0, lat->stream, lat->words, lat->nwords);
    HIP_TRY(hipGetLastError());
    lat->mcs = 0;
    lat->has_snap = false;
    return OKPZ_OK;
}

// Heights of the current words into h0 (anchors) and per-row partials, then
// the exact totals into lat->host_out (10 or 5x2 int64).  cross: also sum
// h_t h_s against the snapshot.
int run_measure(okpz_lattice *lat, bool cross, const uint32_t *src, int32_t *h0_dst)
{
    const okpz_params &p = lat->prm;
    const uint32_t nbx_log2 = ilog2(p.L / 32);
    TimedPair tp;
    begin_timed(lat, 1, tp);
    // the partials buffer (48 bytes per band) first holds the column-0 bytes (one per band)
    uint8_t *col0 = reinterpret_cast<uint8_t *>(lat->partial);
    hipLaunchKernelGGL(col0_kernel, dim3((p.L / 4 + 255) / 256), dim3(256), 0, lat->stream, src, p.L, nbx_log2, col0);
    hipLaunchKernelGGL(anchors_kernel, dim3(1), dim3(1024), 0, lat->stream, col0, p.L, h0_dst);
    const uint32_t rows_per_block = kMeasureThreads / 64;
    const uint32_t blocks = (p.L / 4 + rows_per_block - 1) / rows_per_block;
    if (cross)
        hipLaunchKernelGGL((rows_kernel<true>), dim3(blocks), dim3(kMeasureThreads), 0, lat->stream, src, h0_dst,
                           lat->snap, lat->h0s, p.L, nbx_log2, lat->partial);
    else
        hipLaunchKernelGGL((rows_kernel<false>), dim3(blocks), dim3(kMeasureThreads), 0, lat->stream, src, h0_dst,
                           nullptr, nullptr, p.L, nbx_log2, lat->partial);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kReduceThreads), 0, lat->stream, lat->partial, p.L / 4, lat->reduced);
    end_timed(lat, tp);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(lat->host_out, lat->reduced, 2 * kMomentFields * sizeof(int64_t),
                           hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

}  // namespace

void okpz_host::fill_moments(const okpz_lattice *lat, okpz_moments *out)
{
    moments_from_totals(lat->prm.L, lat->mcs, lat->host_out, out);
}

void okpz_host::moments_from_totals(uint64_t L, uint64_t mcs, const int64_t *r, okpz_moments *out)
{
    const __int128 s1e = pair_to_i128(r + 0), s1o = pair_to_i128(r + 2);
    const __int128 s2e = pair_to_i128(r + 4), s2o = pair_to_i128(r + 6);
    const __int128 n = (__int128)L * L, ne = n / 2, no = n / 2;
    out->mcs = mcs;
    out->n_even = (int64_t)ne;
    out->n_odd = (int64_t)no;
    out->s1_even = to_abi(s1e);
    out->s1_odd = to_abi(s1o);
    out->s2_even = to_abi(s2e);
    out->s2_odd = to_abi(s2o);
    const int sh = 4 * (int)ilog2(L);  // N^2 = 2^(4 log2 L)
    const __int128 s1 = s1e + s1o, s2 = s2e + s2o;
    out->w2 = std::ldexp(i128_to_double(n * s2 - s1 * s1), -sh);
    // (var_e + var_o)/2 = 2 [(ne s2e - s1e^2) + (no s2o - s1o^2)] / L^4
    out->w2_sub = std::ldexp(i128_to_double(2 * ((ne * s2e - s1e * s1e) + (no * s2o - s1o * s1o))), -sh);
}

namespace {

// host packing / unpacking: site (x, y) lives in block (x/32, y/4), word
// 8 * block + y%4 (sx) or 8 * block + 4 + y%4 (sy), bit x%32
inline uint64_t sx_word(uint32_t L, uint32_t x, uint32_t y)
{
    return (((uint64_t)(y >> 2) * (L / 32) + (x >> 5)) << 3) + (y & 3);
}

void pack_sites(const uint8_t *sites, uint32_t L, uint32_t *words)
{
    std::memset(words, 0, sizeof(uint32_t) * (size_t)L * L / 16);
    for (uint32_t y = 0; y < L; ++y)
        for (uint32_t x = 0; x < L; ++x) {
            const uint8_t v = sites[(size_t)y * L + x];
            const uint64_t w = sx_word(L, x, y);
            words[w] |= (uint32_t)(v & 1) << (x & 31);
            words[w + 4] |= (uint32_t)((v >> 1) & 1) << (x & 31);
        }
}

bool valid_surface(const uint8_t *s, uint32_t L)
{
    for (size_t i = 0; i < (size_t)L * L; ++i)
        if (s[i] & ~3u) return false;
    std::vector<uint32_t> col(L, 0);
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t row = 0;
        for (uint32_t x = 0; x < L; ++x) {
            row += s[(size_t)y * L + x] & 1;
            col[x] += (s[(size_t)y * L + x] >> 1) & 1;
        }
        if (2 * row != L) return false;
    }
    for (uint32_t x = 0; x < L; ++x)
        if (2 * col[x] != L) return false;
    for (uint32_t y = 0; y < L; ++y) {
        const uint32_t ym = (y + L - 1) & (L - 1);
        for (uint32_t x = 0; x < L; ++x) {
            const uint32_t xm = (x + L - 1) & (L - 1);
            const int lhs = (s[(size_t)ym * L + x] & 1) + ((s[(size_t)y * L + x] >> 1) & 1);
            const int rhs = ((s[(size_t)y * L + xm] >> 1) & 1) + (s[(size_t)y * L + x] & 1);
            if (lhs != rhs) return false;
        }
    }
    return true;
}

// The blocks covering a site window: bands by0 .. by0+nby-1 and blocks
// bx0 .. bx0+nbx-1 of each band (periodic), 8 words each, as
// buf[(band * nbx + block) * 8 + word].
struct BlockRect {
    uint32_t bx0, by0, nbx, nby;
};

BlockRect rect_of(uint32_t L, uint32_t x0, uint32_t y0, uint32_t w, uint32_t h)
{
    BlockRect r;
    r.bx0 = x0 >> 5;
    r.by0 = y0 >> 2;
    r.nbx = std::min(L / 32, ((x0 & 31) + w + 31) / 32);
    r.nby = std::min(L / 4, ((y0 & 3) + h + 3) / 4);
    return r;
}

int read_blocks(okpz_lattice *lat, const BlockRect &r, std::vector<uint32_t> &buf)
{
    const uint32_t nbx_all = lat->prm.L / 32, nby_all = lat->prm.L / 4;
    buf.assign((size_t)r.nbx * r.nby * 8, 0);
    for (uint32_t b = 0; b < r.nby; ++b) {
        const uint64_t band = (uint64_t)((r.by0 + b) % nby_all) * nbx_all;
        uint32_t done = 0;
        while (done < r.nbx) {
            const uint32_t gx = (r.bx0 + done) % nbx_all;
            const uint32_t run = std::min(r.nbx - done, nbx_all - gx);
            HIP_TRY(hipMemcpyAsync(&buf[((size_t)b * r.nbx + done) * 8], lat->words + (band + gx) * 8,
                                   run * 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, lat->stream));
            done += run;
        }
    }
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

int write_blocks(okpz_lattice *lat, const BlockRect &r, const std::vector<uint32_t> &buf)
{
    const uint32_t nbx_all = lat->prm.L / 32, nby_all = lat->prm.L / 4;
    for (uint32_t b = 0; b < r.nby; ++b) {
        const uint64_t band = (uint64_t)((r.by0 + b) % nby_all) * nbx_all;
        uint32_t done = 0;
        while (done < r.nbx) {
            const uint32_t gx = (r.bx0 + done) % nbx_all;
            const uint32_t run = std::min(r.nbx - done, nbx_all - gx);
            HIP_TRY(hipMemcpyAsync(lat->words + (band + gx) * 8, &buf[((size_t)b * r.nbx + done) * 8],
                                   run * 8 * sizeof(uint32_t), hipMemcpyHostToDevice, lat->stream));
            done += run;
        }
    }
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

// word of buf holding row gy of (global) column gx, relative to the rectangle
inline size_t rect_word(uint32_t L, const BlockRect &r, uint32_t gx, uint32_t gy)
{
    const uint32_t bx = ((gx >> 5) + L / 32 - r.bx0) % (L / 32);
    const uint32_t by = ((gy >> 2) + L / 4 - r.by0) % (L / 4);
    return ((size_t)by * r.nbx + bx) * 8 + (gy & 3);
}

void release(okpz_lattice *lat)
{
    if (!lat) return;
    for (auto &tp : lat->pairs) {
        (void)hipEventDestroy(tp.start);
        (void)hipEventDestroy(tp.stop);
    }
    if (!lat->external && lat->words) (void)hipFree(lat->words);
    if (lat->h0) (void)hipFree(lat->h0);
    if (lat->h0s) (void)hipFree(lat->h0s);
    if (lat->snap) (void)hipFree(lat->snap);
    if (lat->partial) (void)hipFree(lat->partial);
    if (lat->reduced) (void)hipFree(lat->reduced);
    if (lat->host_out) (void)hipHostFree(lat->host_out);
    delete lat;
}

int create_common(const okpz_params *params, void *hip_stream, void *dev_words, size_t nbytes,
                  okpz_lattice **out)
{
    if (!out) return OKPZ_EINVAL;
    *out = nullptr;
    const int rc = check_params(params);
    if (rc != OKPZ_OK) return rc;
    const uint64_t need = (uint64_t)params->L * params->L / 4;
    okpz_lattice *lat = new (std::nothrow) okpz_lattice();
    if (!lat) return OKPZ_ENOMEM;
    lat->prm = *params;
    lat->stream = (hipStream_t)hip_stream;
    lat->nwords = need / 4;
    if (dev_words) {
        if (nbytes < need || ((uintptr_t)dev_words & 255u)) {
            delete lat;
            return OKPZ_EINVAL;
        }
        lat->words = (uint32_t *)dev_words;
        lat->external = true;
    } else if (hipMalloc(&lat->words, need) != hipSuccess) {
        lat->words = nullptr;
        release(lat);
        return OKPZ_ENOMEM;
    }
    const uint32_t L = params->L;
    if (hipMalloc(&lat->h0, L * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&lat->partial, (size_t)(L / 4) * kMomentFields * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&lat->reduced, 2 * kMomentFields * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc(&lat->host_out, 2 * kMomentFields * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        release(lat);
        return OKPZ_ENOMEM;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        release(lat);
        return OKPZ_EHIP;
    }
    lat->cus = (uint32_t)std::max(cus, 1);
    const int frc = fill_flat(lat);
    if (frc != OKPZ_OK) {
        release(lat);
        return frc;
    }
    *out = lat;
    return OKPZ_OK;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

const char *okpz_strerror(int status)
{
    switch (status) {
    case OKPZ_OK: return "ok";
    case OKPZ_EINVAL: return "invalid argument";
    case OKPZ_ENOMEM: return "out of memory";
    case OKPZ_EHIP: return "HIP runtime error";
    case OKPZ_EOVERFLOW: return "counter or reduction overflow";
    case OKPZ_ESTATE: return "invalid state for this call";
    case OKPZ_EWAIT: return "a batch kernel's dependency wait timed out; the batch's lattices are undefined";
    default: return "unknown status";
    }
}

const char *okpz_last_error(void) { return g_last_error.c_str(); }

int okpz_version(void) { return 100; }

int okpz_validate(const okpz_params *params, size_t *nbytes)
{
    const int rc = check_params(params);
    if (rc == OKPZ_OK && nbytes) *nbytes = (size_t)params->L * params->L / 4;
    return rc;
}

int okpz_create(const okpz_params *params, void *hip_stream, okpz_lattice **out)
{
    return create_common(params, hip_stream, nullptr, 0, out);
}

int okpz_create_external(const okpz_params *params, void *hip_stream, void *dev_words, size_t nbytes,
                         okpz_lattice **out)
{
    if (!dev_words) return OKPZ_EINVAL;
    return create_common(params, hip_stream, dev_words, nbytes, out);
}

int okpz_destroy(okpz_lattice *lat)
{
    if (!lat) return OKPZ_EINVAL;
    (void)hipStreamSynchronize(lat->stream);
    release(lat);
    return OKPZ_OK;
}

int okpz_init_flat(okpz_lattice *lat)
{
    if (!lat) return OKPZ_EINVAL;
    return fill_flat(lat);
}

int okpz_init_from_host(okpz_lattice *lat, const uint8_t *sites, uint64_t mcs)
{
    if (!lat || !sites || mcs >= kMcsLimit) return OKPZ_EINVAL;
    const uint32_t L = lat->prm.L;
    if (!valid_surface(sites, L)) return OKPZ_EINVAL;
    std::vector<uint32_t> w((size_t)L * L / 16);
    pack_sites(sites, L, w.data());
    HIP_TRY(hipMemcpyAsync(lat->words, w.data(), w.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->mcs = mcs;
    lat->has_snap = false;
    return OKPZ_OK;
}

int okpz_run(okpz_lattice *lat, uint64_t n_mcs, double p, double q)
{
    if (!lat) return OKPZ_EINVAL;
    if (!(p >= 0.0 && p <= 1.0 && q >= 0.0 && q <= 1.0)) return OKPZ_EINVAL;
    if (n_mcs > kMcsLimit || lat->mcs + n_mcs > kMcsLimit) return OKPZ_EOVERFLOW;
    const LaneShape ls = lane_shape(lat->prm, p, q);
    StepArgs a = base_args(lat, ls, p, q);
    for (uint64_t i = 0; i < n_mcs; ++i) {
        const uint64_t m = lat->mcs;
        const McsDraw d = mcs_draw(lat->prm, m);
        a.ox = d.ox;
        a.oy = d.oy;
        // double tiling: the four domain sets in the drawn order; dead border:
        // one step over all tiles (counter 4 MCS + 0)
        const uint32_t nsteps = a.dev_db ? 1u : 4u;
        for (uint32_t k = 0; k < nsteps; ++k) {
            a.set_a = a.dev_db ? 0u : (uint32_t)d.perm[k] & 1u;
            a.set_b = a.dev_db ? 0u : (uint32_t)d.perm[k] >> 1;
            a.c3 = (uint32_t)(m << 2) | k;
            TimedPair tp;
            begin_timed(lat, 0, tp);
            const int rc = launch_step(lat, a, ls.accept);
            end_timed(lat, tp);
            if (rc != OKPZ_OK) return rc;
        }
        lat->mcs = m + 1;
    }
    return OKPZ_OK;
}

int okpz_measure(okpz_lattice *lat, okpz_moments *out)
{
    if (!lat || !out) return OKPZ_EINVAL;
    const int rc = run_measure(lat, false, lat->words, lat->h0);
    if (rc != OKPZ_OK) return rc;
    fill_moments(lat, out);
    return OKPZ_OK;
}

int okpz_snapshot(okpz_lattice *lat)
{
    if (!lat) return OKPZ_EINVAL;
    const uint32_t L = lat->prm.L;
    // each buffer under its own check: a failed second allocation leaves the
    // first in place for the next call, which then allocates only the missing one
    if (!lat->snap && hipMalloc(&lat->snap, (size_t)L * L / 4) != hipSuccess) {
        lat->snap = nullptr;
        return OKPZ_ENOMEM;
    }
    if (!lat->h0s && hipMalloc(&lat->h0s, L * sizeof(int32_t)) != hipSuccess) {
        lat->h0s = nullptr;
        return OKPZ_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(lat->snap, lat->words, (size_t)L * L / 4, hipMemcpyDeviceToDevice, lat->stream));
    const int rc = run_measure(lat, false, lat->snap, lat->h0s);
    if (rc != OKPZ_OK) return rc;
    lat->snap_s1 = pair_to_i128(lat->host_out + 0) + pair_to_i128(lat->host_out + 2);
    lat->snap_mcs = lat->mcs;
    lat->has_snap = true;
    return OKPZ_OK;
}

int okpz_observe(okpz_lattice *lat, okpz_moments *moments, okpz_correlation *corr)
{
    if (!lat || !moments) return OKPZ_EINVAL;
    if (corr && !lat->has_snap) return OKPZ_ESTATE;
    const int rc = run_measure(lat, corr != nullptr, lat->words, lat->h0);
    if (rc != OKPZ_OK) return rc;
    fill_moments(lat, moments);
    if (corr) fill_correlation(lat, corr);
    return OKPZ_OK;
}

int okpz_autocorr(okpz_lattice *lat, okpz_correlation *out)
{
    if (!lat || !out) return OKPZ_EINVAL;
    if (!lat->has_snap) return OKPZ_ESTATE;
    const int rc = run_measure(lat, true, lat->words, lat->h0);
    if (rc != OKPZ_OK) return rc;
    fill_correlation(lat, out);
    return OKPZ_OK;
}

}  // extern "C"

void okpz_host::fill_correlation(const okpz_lattice *lat, okpz_correlation *out)
{
    const uint64_t L = lat->prm.L;
    const __int128 n = (__int128)L * L;
    const __int128 s1t = pair_to_i128(lat->host_out + 0) + pair_to_i128(lat->host_out + 2);
    const __int128 sts = pair_to_i128(lat->host_out + 8);
    out->t = lat->mcs;
    out->s = lat->snap_mcs;
    out->s_ts = to_abi(sts);
    out->s1_t = to_abi(s1t);
    out->s1_s = to_abi(lat->snap_s1);
    out->c_h = std::ldexp(i128_to_double(n * sts - s1t * lat->snap_s1), -4 * (int)ilog2(L));
    // C_s = overlap / (2 L^2) - 1/4 = (2 overlap - L^2) / (4 L^2)
    const __int128 ov = pair_to_i128(lat->host_out + 10);
    out->overlap = (int64_t)ov;
    out->c_s = std::ldexp(i128_to_double(2 * ov - n), -2 - 2 * (int)ilog2(L));
}

extern "C" {

int okpz_get_window(okpz_lattice *lat, uint32_t x0, uint32_t y0, uint32_t w, uint32_t h, uint8_t *sites)
{
    if (!lat || !sites) return OKPZ_EINVAL;
    const uint32_t L = lat->prm.L;
    if (w == 0 || h == 0 || w > L || h > L) return OKPZ_EINVAL;
    x0 &= L - 1;
    y0 &= L - 1;
    const BlockRect r = rect_of(L, x0, y0, w, h);
    std::vector<uint32_t> buf;
    const int rc = read_blocks(lat, r, buf);
    if (rc != OKPZ_OK) return rc;
    for (uint32_t j = 0; j < h; ++j)
        for (uint32_t i = 0; i < w; ++i) {
            const uint32_t gx = (x0 + i) & (L - 1), gy = (y0 + j) & (L - 1);
            const size_t wi = rect_word(L, r, gx, gy);
            sites[(size_t)j * w + i] = (uint8_t)(((buf[wi] >> (gx & 31)) & 1) | (((buf[wi + 4] >> (gx & 31)) & 1) << 1));
        }
    return OKPZ_OK;
}

int okpz_set_window(okpz_lattice *lat, uint32_t x0, uint32_t y0, uint32_t w, uint32_t h, const uint8_t *sites)
{
    if (!lat || !sites) return OKPZ_EINVAL;
    const uint32_t L = lat->prm.L;
    if (w == 0 || h == 0 || w > L || h > L) return OKPZ_EINVAL;
    for (size_t i = 0; i < (size_t)w * h; ++i)
        if (sites[i] & ~3u) return OKPZ_EINVAL;
    x0 &= L - 1;
    y0 &= L - 1;
    const BlockRect r = rect_of(L, x0, y0, w, h);
    std::vector<uint32_t> buf;
    const int rc = read_blocks(lat, r, buf);
    if (rc != OKPZ_OK) return rc;
    for (uint32_t j = 0; j < h; ++j)
        for (uint32_t i = 0; i < w; ++i) {
            const uint32_t gx = (x0 + i) & (L - 1), gy = (y0 + j) & (L - 1);
            const size_t wi = rect_word(L, r, gx, gy);
            const uint32_t bit = 1u << (gx & 31);
            const uint8_t v = sites[(size_t)j * w + i];
            buf[wi] = (buf[wi] & ~bit) | ((v & 1) ? bit : 0u);
            buf[wi + 4] = (buf[wi + 4] & ~bit) | ((v & 2) ? bit : 0u);
        }
    return write_blocks(lat, r, buf);
}

int okpz_get_sites(okpz_lattice *lat, uint8_t *sites)
{
    if (!lat) return OKPZ_EINVAL;
    return okpz_get_window(lat, 0, 0, lat->prm.L, lat->prm.L, sites);
}

int okpz_get_heights(okpz_lattice *lat, int32_t *heights)
{
    if (!lat || !heights) return OKPZ_EINVAL;
    const uint32_t L = lat->prm.L;
    std::vector<uint8_t> s((size_t)L * L);
    const int rc = okpz_get_sites(lat, s.data());
    if (rc != OKPZ_OK) return rc;
    for (uint32_t y = 0; y < L; ++y) {
        int32_t h = y == 0 ? 0 : heights[(size_t)(y - 1) * L] + 2 * ((s[(size_t)y * L] >> 1) & 1) - 1;
        heights[(size_t)y * L] = h;
        for (uint32_t x = 1; x < L; ++x) {
            h += 2 * (s[(size_t)y * L + x] & 1) - 1;
            heights[(size_t)y * L + x] = h;
        }
    }
    return OKPZ_OK;
}

int okpz_get_words(okpz_lattice *lat, uint32_t *words)
{
    if (!lat || !words) return OKPZ_EINVAL;
    HIP_TRY(hipMemcpyAsync(words, lat->words, lat->nwords * sizeof(uint32_t), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

// ---------------------------------------------------------------- checkpoints
// Blob: a 128-byte header (magic, version, flags, parameters, MCS counts,
// word count, checksum) followed by the lattice words and, if the snapshot
// is saved, the snapshot words, all in the device layout.

}  // extern "C"

namespace {

constexpr char kCkpMagic[8] = {'O', 'K', 'P', 'Z', 'C', 'K', 'P', 0};
constexpr uint32_t kCkpVersion = 1;
constexpr size_t kCkpHeader = 128;

struct CkpHeader {
    char magic[8];
    uint32_t version;
    uint32_t flags;  // bit 0: snapshot words follow the lattice words
    okpz_params prm;
    uint64_t mcs, snap_mcs, nwords;
    uint64_t checksum;  // over the header (this field zero) and the payload
};
static_assert(sizeof(CkpHeader) <= kCkpHeader, "checkpoint header");

// Multiply-xor checksum over 8-byte units (n a multiple of 8).
uint64_t ckp_mix(uint64_t h, const uint8_t *p, size_t n)
{
    for (size_t i = 0; i < n; i += 8) {
        uint64_t v;
        std::memcpy(&v, p + i, 8);
        h = (h ^ v) * 0x100000001B3ull;
        h ^= h >> 29;
    }
    return h;
}

size_t ckp_bytes(const okpz_lattice *lat, bool snap)
{
    return kCkpHeader + (snap ? 2 : 1) * lat->nwords * sizeof(uint32_t);
}

// Word-level check of a height state (as valid_surface, on the packed words):
// every plaquette closes, sx(x, y-1) + sy(x, y) = sy(x-1, y) + sx(x, y), and
// the slopes of row 0 and of column 0 sum to zero.  On the torus a closed
// slope field has the same sum along every row (every column), so these two
// loops suffice.
bool valid_words(const uint32_t *w, uint32_t L)
{
    const uint32_t nbx = L / 32, nrow = L;
    auto sx = [&](uint32_t bx, uint32_t y) { return w[(((uint64_t)(y >> 2) * nbx + bx) << 3) + (y & 3)]; };
    auto sy = [&](uint32_t bx, uint32_t y) { return w[(((uint64_t)(y >> 2) * nbx + bx) << 3) + 4 + (y & 3)]; };
    for (uint32_t y = 0; y < nrow; ++y) {
        const uint32_t ym = (y + L - 1) & (L - 1);
        for (uint32_t bx = 0; bx < nbx; ++bx) {
            const uint32_t a = sx(bx, ym), b = sy(bx, y), d = sx(bx, y);
            const uint32_t prev = sy((bx + nbx - 1) % nbx, y);
            const uint32_t c = (b << 1) | (prev >> 31);  // sy(x-1, y) at bit x
            if ((a ^ b) != (c ^ d) || (a & b) != (c & d)) return false;
        }
    }
    uint64_t row0 = 0, col0 = 0;
    for (uint32_t bx = 0; bx < nbx; ++bx) row0 += (uint64_t)__builtin_popcount(sx(bx, 0));
    for (uint32_t y = 0; y < nrow; ++y) col0 += sy(0, y) & 1u;
    return 2 * row0 == L && 2 * col0 == L;
}

}  // namespace

extern "C" {

int okpz_checkpoint_size(const okpz_lattice *lat, int with_snapshot, size_t *nbytes)
{
    if (!lat || !nbytes) return OKPZ_EINVAL;
    if (with_snapshot && !lat->has_snap) return OKPZ_ESTATE;
    *nbytes = ckp_bytes(lat, with_snapshot != 0);
    return OKPZ_OK;
}

int okpz_save(okpz_lattice *lat, int with_snapshot, void *host_buf, size_t nbytes)
{
    if (!lat || !host_buf) return OKPZ_EINVAL;
    const bool snap = with_snapshot != 0;
    if (snap && !lat->has_snap) return OKPZ_ESTATE;
    if (nbytes < ckp_bytes(lat, snap)) return OKPZ_EINVAL;
    uint8_t *out = static_cast<uint8_t *>(host_buf);
    const size_t wb = lat->nwords * sizeof(uint32_t);
    HIP_TRY(hipMemcpyAsync(out + kCkpHeader, lat->words, wb, hipMemcpyDeviceToHost, lat->stream));
    if (snap) HIP_TRY(hipMemcpyAsync(out + kCkpHeader + wb, lat->snap, wb, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    CkpHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kCkpMagic, sizeof(h.magic));
    h.version = kCkpVersion;
    h.flags = snap ? 1u : 0u;
    h.prm = lat->prm;
    h.mcs = lat->mcs;
    h.snap_mcs = snap ? lat->snap_mcs : 0;
    h.nwords = lat->nwords;
    std::memset(out, 0, kCkpHeader);
    std::memcpy(out, &h, sizeof(h));
    h.checksum = ckp_mix(ckp_mix(0xCBF29CE484222325ull, out, kCkpHeader), out + kCkpHeader, (snap ? 2 : 1) * wb);
    std::memcpy(out, &h, sizeof(h));
    return OKPZ_OK;
}

int okpz_load(okpz_lattice *lat, const void *host_buf, size_t nbytes)
{
    if (!lat || !host_buf || nbytes < kCkpHeader) return OKPZ_EINVAL;
    const uint8_t *in = static_cast<const uint8_t *>(host_buf);
    CkpHeader h;
    std::memcpy(&h, in, sizeof(h));
    if (std::memcmp(h.magic, kCkpMagic, sizeof(h.magic)) != 0 || h.version != kCkpVersion || (h.flags & ~1u))
        return OKPZ_EINVAL;
    if (std::memcmp(&h.prm, &lat->prm, sizeof(okpz_params)) != 0 || h.nwords != lat->nwords) return OKPZ_EINVAL;
    const bool snap = (h.flags & 1u) != 0;
    if (h.mcs >= kMcsLimit || (snap && h.snap_mcs > h.mcs)) return OKPZ_EINVAL;
    const size_t wb = lat->nwords * sizeof(uint32_t);
    if (nbytes < ckp_bytes(lat, snap)) return OKPZ_EINVAL;
    std::vector<uint8_t> head(in, in + kCkpHeader);
    std::memset(head.data() + offsetof(CkpHeader, checksum), 0, sizeof(uint64_t));
    if (ckp_mix(ckp_mix(0xCBF29CE484222325ull, head.data(), kCkpHeader), in + kCkpHeader, (snap ? 2 : 1) * wb) !=
        h.checksum)
        return OKPZ_EINVAL;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(in + kCkpHeader);
    if (!valid_words(words, lat->prm.L) || (snap && !valid_words(words + lat->nwords, lat->prm.L)))
        return OKPZ_EINVAL;
    if (snap && !lat->snap) {
        const uint32_t L = lat->prm.L;
        if (hipMalloc(&lat->snap, (size_t)L * L / 4) != hipSuccess) {
            lat->snap = nullptr;
            return OKPZ_ENOMEM;
        }
    }
    if (snap && !lat->h0s && hipMalloc(&lat->h0s, lat->prm.L * sizeof(int32_t)) != hipSuccess) {
        lat->h0s = nullptr;
        return OKPZ_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(lat->words, words, wb, hipMemcpyHostToDevice, lat->stream));
    lat->mcs = h.mcs;
    lat->has_snap = false;
    if (snap) {
        HIP_TRY(hipMemcpyAsync(lat->snap, words + lat->nwords, wb, hipMemcpyHostToDevice, lat->stream));
        const int rc = run_measure(lat, false, lat->snap, lat->h0s);
        if (rc != OKPZ_OK) return rc;
        lat->snap_s1 = pair_to_i128(lat->host_out + 0) + pair_to_i128(lat->host_out + 2);
        lat->snap_mcs = h.snap_mcs;
        lat->has_snap = true;
    }
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

int okpz_device_words(okpz_lattice *lat, void **dev_words, size_t *nbytes)
{
    if (!lat) return OKPZ_EINVAL;
    if (dev_words) *dev_words = lat->words;
    if (nbytes) *nbytes = lat->nwords * sizeof(uint32_t);
    return OKPZ_OK;
}

int okpz_get_mcs(const okpz_lattice *lat, uint64_t *mcs)
{
    if (!lat || !mcs) return OKPZ_EINVAL;
    *mcs = lat->mcs;
    return OKPZ_OK;
}

int okpz_set_threads(okpz_lattice *lat, uint32_t threads)
{
    if (!lat) return OKPZ_EINVAL;
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512) return OKPZ_EINVAL;
    const uint32_t ncell = (lat->prm.dom_x / lat->prm.cell_x) * (lat->prm.dom_y / lat->prm.cell_y);
    uint32_t cpt, nt;
    step_shape(ncell, threads, cpt, nt);
    if (cpt > 16) return OKPZ_EINVAL;
    lat->threads = threads;
    return OKPZ_OK;
}

int okpz_get_params(const okpz_lattice *lat, okpz_params *out)
{
    if (!lat || !out) return OKPZ_EINVAL;
    *out = lat->prm;
    return OKPZ_OK;
}

int okpz_sync(okpz_lattice *lat)
{
    if (!lat) return OKPZ_EINVAL;
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return OKPZ_OK;
}

int okpz_timing(okpz_lattice *lat, int enable)
{
    if (!lat) return OKPZ_EINVAL;
    HIP_TRY(hipStreamSynchronize(lat->stream));
    for (auto &tp : lat->pairs) {
        (void)hipEventDestroy(tp.start);
        (void)hipEventDestroy(tp.stop);
    }
    lat->pairs.clear();
    lat->timing = enable != 0;
    return OKPZ_OK;
}

int okpz_get_timing(okpz_lattice *lat, double *step_ms, uint64_t *step_launches, double *measure_ms,
                    uint64_t *measure_launches)
{
    if (!lat) return OKPZ_EINVAL;
    HIP_TRY(hipStreamSynchronize(lat->stream));
    double ms[2] = {0, 0};
    uint64_t cnt[2] = {0, 0};
    for (auto &tp : lat->pairs) {
        float e = 0;
        HIP_TRY(hipEventElapsedTime(&e, tp.start, tp.stop));
        ms[tp.kind] += e;
        cnt[tp.kind] += 1;
    }
    if (step_ms) *step_ms = ms[0];
    if (step_launches) *step_launches = cnt[0];
    if (measure_ms) *measure_ms = ms[1];
    if (measure_launches) *measure_launches = cnt[1];
    return OKPZ_OK;
}

int okpz_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, size_t n)
{
    if (!ctr || !out) return OKPZ_EINVAL;
    if (n == 0) return OKPZ_OK;
    uint32_t *dctr = nullptr, *dout = nullptr;
    HIP_TRY(hipMalloc(&dctr, n * 4 * sizeof(uint32_t)));
    if (hipMalloc(&dout, n * 4 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(dctr);
        return OKPZ_ENOMEM;
    }
    int rc = OKPZ_OK;
    hipError_t e = hipMemcpy(dctr, ctr, n * 4 * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, k0, k1, dctr,
                           dout, (uint64_t)n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, n * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "okpz_philox");
    (void)hipFree(dctr);
    (void)hipFree(dout);
    return rc;
}

}  // extern "C"
