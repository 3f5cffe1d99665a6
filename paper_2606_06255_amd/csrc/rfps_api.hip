// C ABI of librfps (declared in include/rfps.h): argument validation,
// workspace layout, device checks and the launch sequence of each call.
// Host code only; the kernels live in index_build.hip, sample_rfps.hip and
// sample_plain.hip.
#include <math.h>
#include <cmath>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "rfps_internal.h"

using namespace rfps;

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kKnownFlags =
    RFPS_F_NO_PRUNE | RFPS_F_NO_POINT_SKIP | RFPS_F_TELEMETRY | RFPS_F_TRACE | RFPS_F_SINGLE_PICK | RFPS_F_SQRT | RFPS_F_UNFUSED |
    RFPS_F_CLOCKS;
constexpr int kDefaultLookahead = 2;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct DeviceInfo {
    bool probed = false;
    bool ok = false;       // a gfx950 device with cooperative launch
    int cus = 0;
    int max_lds = 0;       // bytes of LDS one workgroup may use
    double wall_hz = 0.0;  // rate of the device wall clock
};

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

// Probes the current device once.  Returns nullptr when there is no device.
const DeviceInfo *device_info()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceInfo &d = g_dev[dev];
    if (!d.probed) {
        d.probed = true;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return nullptr;
        int coop = 0, lds = 0, lds_optin = 0, clk = 0;
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
        hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, dev);  // kHz
        d.cus = prop.multiProcessorCount;
        // gfx950 lets one workgroup opt in to the whole 160 KB LDS of a CU
        d.max_lds = std::max(lds, lds_optin);
        d.wall_hz = (double)clk * 1000.0;
        d.ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0 && coop != 0 && d.cus > 0;
    }
    return &d;
}

// Index workspace layout.  Every segment is 256-byte aligned.  A batched
// workspace appends the per-cloud arrays to the index of all its points.
struct IndexLayout {
    size_t hdr, keyA, keyB, valA, valB, xs, ys, zs, inv, flags, hscan, vstart, tcount, tbase, tstart, tcnt, tcx,
        tcy, tcz, trad, partials, hist, board, trace, total;
    size_t cl_pmin, cl_L, cl_bb, cl_nvox, cl_base, cl_out, tile_first, order, bstate;
    int radix_passes, nblk, batch;
};

int bit_length(uint64_t v)
{
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Sort passes for keys below `cells` (8 bits per pass, at least one).
int passes_for(uint64_t cells) { return std::max(1, (bit_length(cells - 1) + 7) / 8); }

IndexLayout layout_common(int n, int passes, int batch)
{
    IndexLayout L;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = align_up(cur);
        cur = o + bytes;
        return o;
    };
    const size_t N = (size_t)n;
    L.nblk = (n + kRadixTile - 1) / kRadixTile;
    L.radix_passes = passes;
    L.batch = batch;
    const size_t scan_elems = std::max(N, (size_t)256 * L.nblk);
    L.hdr = take(sizeof(IndexHeader));
    L.keyA = take(4 * N);
    L.keyB = take(4 * N);
    L.valA = take(4 * N);
    L.valB = take(4 * N);
    L.xs = take(4 * N);
    L.ys = take(4 * N);
    L.zs = take(4 * N);
    L.inv = take(4 * N);
    L.flags = take(4 * N);
    L.hscan = take(4 * N);
    L.vstart = take(4 * (N + 1));
    L.tcount = take(4 * N);
    L.tbase = take(4 * N);
    L.tstart = take(4 * N);
    L.tcnt = take(4 * N);
    L.tcx = take(4 * N);
    L.tcy = take(4 * N);
    L.tcz = take(4 * N);
    L.trad = take(4 * N);
    L.partials = take(4 * ((scan_elems + kScanChunk - 1) / kScanChunk + 1));
    L.hist = take(4 * (size_t)256 * L.nblk);
    L.board = take(8 * (size_t)kBoardWords);
    L.trace = take(8 * (size_t)2 * kTraceCap);
    const size_t B = (size_t)batch;
    L.cl_pmin = take(24 * B);
    L.cl_L = take(8 * B);
    L.cl_bb = take(24 * B);
    L.cl_nvox = take(4 * B);
    L.cl_base = take(4 * (B + 1));
    L.cl_out = take(4 * (B + 1));
    L.tile_first = take(4 * (B + 1));
    L.order = take(4 * B);
    L.bstate = take(sizeof(BatchState));
    L.total = align_up(cur);
    return L;
}

IndexLayout layout_index(int n, int n_vox, int shells)
{
    return layout_common(n, passes_for((uint64_t)n_vox * n_vox * n_vox * (uint64_t)shells), 0);
}

// A batch sorts by cloud-prefixed keys: with a fixed n_vox the key range is
// known here; with the per-cloud rule it is only known on the device, so the
// sort takes all four passes.
IndexLayout layout_batch(int n, int batch, int fixed_n_vox, bool shells)
{
    const uint64_t n3 = (uint64_t)fixed_n_vox * fixed_n_vox * fixed_n_vox;
    const int passes = fixed_n_vox ? passes_for((uint64_t)batch * n3 * shell_cap_for(fixed_n_vox, shells)) : 4;
    return layout_common(n, std::min(passes, 4), batch);
}

IndexView make_view_l(void *ws, const IndexLayout &L, int n, int n_vox, int tile)
{
    unsigned char *b = static_cast<unsigned char *>(ws);
    IndexView v;
    v.hdr = reinterpret_cast<IndexHeader *>(b + L.hdr);
    v.keyA = reinterpret_cast<uint32_t *>(b + L.keyA);
    v.keyB = reinterpret_cast<uint32_t *>(b + L.keyB);
    v.valA = reinterpret_cast<uint32_t *>(b + L.valA);
    v.valB = reinterpret_cast<uint32_t *>(b + L.valB);
    const bool in_b = (L.radix_passes % 2) == 1;
    v.skey = in_b ? v.keyB : v.keyA;
    v.orig = in_b ? v.valB : v.valA;
    v.xs = reinterpret_cast<float *>(b + L.xs);
    v.ys = reinterpret_cast<float *>(b + L.ys);
    v.zs = reinterpret_cast<float *>(b + L.zs);
    v.inv = reinterpret_cast<uint32_t *>(b + L.inv);
    v.flags = reinterpret_cast<uint32_t *>(b + L.flags);
    v.hscan = reinterpret_cast<uint32_t *>(b + L.hscan);
    v.vstart = reinterpret_cast<uint32_t *>(b + L.vstart);
    v.tcount = reinterpret_cast<uint32_t *>(b + L.tcount);
    v.tbase = reinterpret_cast<uint32_t *>(b + L.tbase);
    v.tstart = reinterpret_cast<uint32_t *>(b + L.tstart);
    v.tcnt = reinterpret_cast<uint32_t *>(b + L.tcnt);
    v.tcx = reinterpret_cast<float *>(b + L.tcx);
    v.tcy = reinterpret_cast<float *>(b + L.tcy);
    v.tcz = reinterpret_cast<float *>(b + L.tcz);
    v.trad = reinterpret_cast<float *>(b + L.trad);
    v.partials = reinterpret_cast<uint32_t *>(b + L.partials);
    v.hist = reinterpret_cast<uint32_t *>(b + L.hist);
    v.board = reinterpret_cast<unsigned long long *>(b + L.board);
    v.trace = reinterpret_cast<unsigned long long *>(b + L.trace);
    v.n = n;
    v.n_vox = n_vox;
    v.tile = tile;
    v.radix_passes = L.radix_passes;
    v.shell_inv = 0.0;
    v.shell_cap = 1;
    v.batch = L.batch;
    v.bc = BatchCtl{};
    v.cl_pmin = reinterpret_cast<double *>(b + L.cl_pmin);
    v.cl_L = reinterpret_cast<double *>(b + L.cl_L);
    v.cl_bb = reinterpret_cast<uint32_t *>(b + L.cl_bb);
    v.cl_nvox = reinterpret_cast<uint32_t *>(b + L.cl_nvox);
    v.cl_base = reinterpret_cast<uint32_t *>(b + L.cl_base);
    v.bc.out_offsets = reinterpret_cast<uint32_t *>(b + L.cl_out);
    v.tile_first = reinterpret_cast<uint32_t *>(b + L.tile_first);
    v.order = reinterpret_cast<int32_t *>(b + L.order);
    v.bstate = reinterpret_cast<BatchState *>(b + L.bstate);
    return v;
}

IndexView make_view(void *ws, int n, int n_vox, int tile, int shells)
{
    IndexView v = make_view_l(ws, layout_index(n, n_vox, shells), n, n_vox, tile);
    v.shell_cap = (uint32_t)shells;
    return v;
}

bool params_valid(const rfps_params *p)
{
    if (!p)
        return true;
    return p->n_vox >= 0 && p->n_vox <= kMaxNVox && p->tile >= 0 && p->tile <= kWave && p->groups >= 0 &&
           p->groups <= kMaxGroups && (p->flags & ~kKnownFlags) == 0 &&
           (p->lookahead == 0 || (p->lookahead >= 2 && p->lookahead <= 4) || p->lookahead == 8) &&
           p->shell_spacing >= 0.0f;  // also rejects NaN
}

bool use_shells(const rfps_params *p) { return p && p->shell_spacing > 0.0f && std::isfinite(p->shell_spacing); }
double shell_inv_of(const rfps_params *p) { return use_shells(p) ? 1.0 / (double)p->shell_spacing : 0.0; }
int resolve_shells(int n_vox, const rfps_params *p) { return (int)shell_cap_for((uint32_t)n_vox, use_shells(p)); }

int resolve_n_vox(int n, const rfps_params *p) { return (p && p->n_vox) ? p->n_vox : rfps_default_n_vox(n); }
int resolve_tile(const rfps_params *p) { return (p && p->tile) ? p->tile : kWave; }

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

// Plain-FPS workspace: status word, exchange board, distance array.
struct PlainLayout {
    size_t status, board, dist, total;
};
PlainLayout layout_plain(int n)
{
    PlainLayout L;
    L.status = 0;
    L.board = align_up(16);
    L.dist = align_up(L.board + 8 * (size_t)kBoardWords);
    L.total = align_up(L.dist + 4 * (size_t)n);
    return L;
}

}  // namespace

extern "C" {

int32_t rfps_default_n_vox(int32_t n)
{
    static const int cand[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    const double target = sqrt((double)(n > 0 ? n : 1) / 40.0);
    int best = cand[0];
    for (int c : cand)
        if (fabs(log((double)c / target)) < fabs(log((double)best / target)))
            best = c;
    return best;
}

const char *rfps_status_str(rfps_status s)
{
    switch (s) {
    case RFPS_OK: return "ok";
    case RFPS_ERR_INVALID_ARG: return "invalid argument";
    case RFPS_ERR_NONFINITE: return "non-finite input coordinate";
    case RFPS_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case RFPS_ERR_DEVICE: return "HIP runtime error";
    case RFPS_ERR_UNSUPPORTED: return "unsupported device or launch shape";
    case RFPS_ERR_CAPACITY: return "cloud share per workgroup exceeds the on-chip budget";
    case RFPS_ERR_TIMEOUT: return "bounded wait in a persistent kernel expired";
    case RFPS_ERR_INTERNAL: return "internal consistency check failed";
    case RFPS_ERR_SCRATCH_LIMIT: return "input exceeds the library's fixed scratch array (no-allocation entry point)";
    }
    return "unknown status";
}

size_t rfps_index_workspace_size(int32_t n, const rfps_params *params)
{
    if (n < 1 || n > kMaxPoints || !params_valid(params))
        return 0;
    const int n_vox = resolve_n_vox(n, params);
    return layout_index(n, n_vox, resolve_shells(n_vox, params)).total;
}

rfps_status rfps_build_index(const float *xyz, int32_t n, const rfps_params *params, void *ws, size_t ws_bytes,
                             void *stream, rfps_index *out)
{
    if (!xyz || !out || n < 1 || n > kMaxPoints || !params_valid(params))
        return RFPS_ERR_INVALID_ARG;
    const int n_vox = resolve_n_vox(n, params);
    const int tile = resolve_tile(params);
    const int shells = resolve_shells(n_vox, params);
    if (!ws || !aligned(ws) || ws_bytes < layout_index(n, n_vox, shells).total)
        return RFPS_ERR_WORKSPACE;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok)
        return RFPS_ERR_UNSUPPORTED;
    IndexView v = make_view(ws, n, n_vox, tile, shells);
    v.shell_inv = shell_inv_of(params);
    if (launch_build_index(v, xyz, static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    out->n = n;
    out->n_vox = n_vox;
    out->tile = tile;
    out->shells = shells;
    out->ws = ws;
    out->ws_bytes = ws_bytes;
    return RFPS_OK;
}

static rfps_status check_index(const rfps_index *index)
{
    if (!index || index->n < 1 || index->n > kMaxPoints || index->n_vox < 1 || index->n_vox > kMaxNVox ||
        index->tile < 1 || index->tile > kWave || index->shells < 1 || index->shells > kMaxShells ||
        (uint64_t)index->n_vox * index->n_vox * index->n_vox * (uint64_t)index->shells > (1ull << 32))
        return RFPS_ERR_INVALID_ARG;
    if (!index->ws || !aligned(index->ws) ||
        index->ws_bytes < layout_index(index->n, index->n_vox, index->shells).total)
        return RFPS_ERR_WORKSPACE;
    return RFPS_OK;
}

rfps_status rfps_sample(const rfps_index *index, int32_t m, int32_t start, const rfps_params *params,
                        int32_t *out_idx, float *out_d2, void *stream)
{
    rfps_status st = check_index(index);
    if (st != RFPS_OK)
        return st;
    if (m < 1 || m > index->n || start < 0 || start >= index->n || !out_idx || !params_valid(params))
        return RFPS_ERR_INVALID_ARG;
    if (params && (params->flags & RFPS_F_UNFUSED) &&
        (params->flags & (RFPS_F_TELEMETRY | RFPS_F_TRACE | RFPS_F_CLOCKS)))
        return RFPS_ERR_UNSUPPORTED;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok)
        return RFPS_ERR_UNSUPPORTED;
    SampleLaunch L;
    L.flags = params ? params->flags : 0u;
    // default workgroups: every compute unit; clouds below 64k points take
    // half of them for the multi-pick sampler (a round then exchanges and
    // merges half the candidates, and each workgroup still owns a few hundred
    // points: measured 5-10 % faster on 4k-30k point clouds)
    const int all = std::min(d->cus, kMaxGroups);
    const bool small = index->n < (1 << 16) && !(L.flags & (RFPS_F_SINGLE_PICK | RFPS_F_NO_PRUNE));
    L.G = (params && params->groups) ? params->groups : (small ? std::max(1, all / 2) : all);
    // the multi-pick sampler is the default; plain (unpruned) sampling and an
    // explicit request use one selection per exchange
    const bool single = (L.flags & (RFPS_F_SINGLE_PICK | RFPS_F_NO_PRUNE)) != 0;
    L.R = single ? 0 : ((params && params->lookahead) ? params->lookahead : kDefaultLookahead);
    const size_t stat = rfps_sampler_static_lds(L.R);
    if (stat == 0 || (size_t)d->max_lds <= stat + 1024)
        return RFPS_ERR_UNSUPPORTED;
    L.lds_budget = (uint32_t)((d->max_lds - stat - 256) & ~(size_t)255);
    if (L.G > d->cus)
        return RFPS_ERR_UNSUPPORTED;
    const IndexView v = make_view(index->ws, index->n, index->n_vox, index->tile, index->shells);
    hipError_t e = launch_rfps_sample(v, m, start, L, out_idx, out_d2, static_cast<hipStream_t>(stream));
    if (e == hipSuccess && out_d2 && (L.flags & RFPS_F_SQRT))
        e = launch_sqrt_out(out_d2, m, static_cast<hipStream_t>(stream));
    if (e == hipErrorCooperativeLaunchTooLarge)
        return RFPS_ERR_UNSUPPORTED;
    return e == hipSuccess ? RFPS_OK : RFPS_ERR_DEVICE;
}

rfps_status rfps_read_status(const rfps_index *index, void *stream)
{
    rfps_status st = check_index(index);
    if (st != RFPS_OK)
        return st;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    uint32_t w[2];
    if (hipMemcpy(w, index->ws, sizeof w, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    return (rfps_status)(w[0] ? w[0] : w[1]);
}

rfps_status rfps_read_index_info(const rfps_index *index, void *stream, rfps_index_info *out)
{
    rfps_status st = check_index(index);
    if (st != RFPS_OK)
        return st;
    if (!out)
        return RFPS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    IndexHeader h;
    if (hipMemcpy(&h, index->ws, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    out->n_voxels = h.n_voxels;
    out->n_tiles = h.n_tiles;
    for (int a = 0; a < 3; ++a)
        out->pmin[a] = h.pmin[a];
    out->voxel_edge = h.L;
    return RFPS_OK;
}

rfps_status rfps_read_telemetry(const rfps_index *index, void *stream, rfps_telemetry *out)
{
    rfps_status st = check_index(index);
    if (st != RFPS_OK)
        return st;
    if (!out)
        return RFPS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    IndexHeader h;
    if (hipMemcpy(&h, index->ws, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    static_assert(sizeof(rfps_telemetry) == kTeleFields * sizeof(unsigned long long), "telemetry layout");
    memcpy(out, h.tele, sizeof *out);
    const DeviceInfo *d = device_info();
    out->tick_hz = d ? (int64_t)d->wall_hz : 0;
    return RFPS_OK;
}

rfps_status rfps_probe_exchange(const rfps_index *index, int32_t groups, int32_t words, int32_t rounds,
                                void *stream, double *us_per_round)
{
    rfps_status st = check_index(index);
    if (st != RFPS_OK)
        return st;
    if (!us_per_round || words < 1 || words > kMaxSlotWords || rounds < 1 || rounds > (1 << 20) || groups < 0)
        return RFPS_ERR_INVALID_ARG;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok)
        return RFPS_ERR_UNSUPPORTED;
    const int G = groups ? groups : std::min(d->cus, kMaxGroups);
    if (G > d->cus || G > kMaxGroups)
        return RFPS_ERR_INVALID_ARG;
    const IndexView v = make_view(index->ws, index->n, index->n_vox, index->tile, index->shells);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // the trace buffer's first two words take the ticks and the status
    unsigned long long *out = v.trace;
    unsigned long long host[2] = {0ull, 0ull};
    const hipError_t e = launch_exchange_probe(v.board, G, words, rounds, out, reinterpret_cast<uint32_t *>(out + 1), s);
    if (e == hipErrorCooperativeLaunchTooLarge)
        return RFPS_ERR_UNSUPPORTED;
    if (e != hipSuccess || hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(host, out, sizeof host, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    if ((uint32_t)host[1] != 0)
        return (rfps_status)(uint32_t)host[1];
    *us_per_round = (double)host[0] / d->wall_hz * 1e6 / rounds;
    return RFPS_OK;
}

int32_t rfps_read_trace(const rfps_index *index, void *stream, uint64_t *out, int32_t cap, double *ticks_per_s)
{
    if (check_index(index) != RFPS_OK || !out || cap < 0)
        return -1;
    const DeviceInfo *d = device_info();
    if (!d || hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return -1;
    IndexHeader h;
    if (hipMemcpy(&h, index->ws, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    int32_t cnt = (int32_t)h.trace_n;
    cnt = std::min(std::min(cnt, cap), kTraceCap);
    const IndexLayout L = layout_index(index->n, index->n_vox, index->shells);
    if (cnt > 0 && hipMemcpy(out, static_cast<unsigned char *>(index->ws) + L.trace, 16 * (size_t)cnt,
                             hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    if (ticks_per_s)
        *ticks_per_s = d->wall_hz;
    return cnt;
}

rfps_status rfps_gather_xyz(const float *xyz, int32_t n, const int32_t *idx, int32_t m, float *out, void *stream)
{
    if (!xyz || !idx || !out || n < 1 || n > kMaxPoints || m < 1 || m > kMaxPoints)
        return RFPS_ERR_INVALID_ARG;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok)
        return RFPS_ERR_UNSUPPORTED;
    return launch_gather_xyz(xyz, n, idx, m, out, static_cast<hipStream_t>(stream)) == hipSuccess
               ? RFPS_OK
               : RFPS_ERR_DEVICE;
}

size_t rfps_fps_plain_workspace_size(int32_t n, int32_t variant)
{
    if (n < 1 || n > kMaxPoints || variant < 0 || variant > 1)
        return 0;
    return layout_plain(n).total;
}

rfps_status rfps_fps_plain(const float *xyz, int32_t n, int32_t m, int32_t start, int32_t variant, int32_t groups,
                           void *ws, size_t ws_bytes, int32_t *out_idx, float *out_d2, void *stream)
{
    if (!xyz || !out_idx || n < 1 || n > kMaxPoints || m < 1 || m > n || start < 0 || start >= n || variant < 0 ||
        variant > 1 || groups < 0 || groups > kMaxGroups)
        return RFPS_ERR_INVALID_ARG;
    const PlainLayout PL = layout_plain(n);
    if (!ws || !aligned(ws) || ws_bytes < PL.total)
        return RFPS_ERR_WORKSPACE;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok)
        return RFPS_ERR_UNSUPPORTED;
    PlainLaunch L;
    L.variant = variant;
    L.G = 1;
    L.ppt = 1;
    if (variant == 0) {
        const int max_g = std::min(d->cus, kMaxGroups);
        L.G = groups ? groups : std::max(1, std::min(max_g, (n + kBlock * 8 - 1) / (kBlock * 8)));
        if (L.G > d->cus)
            return RFPS_ERR_UNSUPPORTED;
        const long long per_thread = ((long long)n + (long long)L.G * kBlock - 1) / ((long long)L.G * kBlock);
        while (L.ppt < per_thread)
            L.ppt <<= 1;
        if (L.ppt > 32)
            return RFPS_ERR_CAPACITY;
    }
    unsigned char *b = static_cast<unsigned char *>(ws);
    hipError_t e = launch_fps_plain(xyz, n, m, start, L, reinterpret_cast<uint32_t *>(b + PL.status),
                                    reinterpret_cast<unsigned long long *>(b + PL.board),
                                    reinterpret_cast<float *>(b + PL.dist), out_idx, out_d2,
                                    static_cast<hipStream_t>(stream));
    if (e == hipErrorCooperativeLaunchTooLarge)
        return RFPS_ERR_UNSUPPORTED;
    return e == hipSuccess ? RFPS_OK : RFPS_ERR_DEVICE;
}

rfps_status rfps_read_plain_status(const void *ws, size_t ws_bytes, void *stream)
{
    if (!ws || !aligned(ws) || ws_bytes < layout_plain(1).total)
        return RFPS_ERR_WORKSPACE;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    uint32_t w = 0;
    if (hipMemcpy(&w, ws, sizeof w, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    return (rfps_status)w;
}

// ---------------------------------------------------------------------------
// Batches of clouds
// ---------------------------------------------------------------------------
size_t rfps_batched_workspace_size(int32_t n, int32_t batch, const rfps_params *params)
{
    if (n < 1 || n > kMaxPoints || batch < 1 || batch > kMaxBatch || batch > n || !params_valid(params))
        return 0;
    return layout_batch(n, batch, params ? params->n_vox : 0, use_shells(params)).total;
}

rfps_status rfps_sample_batched(const float *xyz, int32_t n, const int32_t *offsets, const int32_t *m,
                                const int32_t *starts, int32_t batch, int32_t m_total, const rfps_params *params,
                                void *ws, size_t ws_bytes, int32_t *out_idx, float *out_d2, void *stream)
{
    if (!xyz || !offsets || !m || !out_idx || n < 1 || n > kMaxPoints || batch < 1 || batch > kMaxBatch ||
        batch > n || m_total < batch || m_total > n || !params_valid(params))
        return RFPS_ERR_INVALID_ARG;
    const uint32_t flags = params ? params->flags : 0u;
    if (flags & (RFPS_F_NO_PRUNE | RFPS_F_SINGLE_PICK | RFPS_F_TRACE | RFPS_F_UNFUSED | RFPS_F_CLOCKS))
        return RFPS_ERR_UNSUPPORTED;
    const int fixed_n_vox = params ? params->n_vox : 0;
    const IndexLayout BL = layout_batch(n, batch, fixed_n_vox, use_shells(params));
    if (!ws || !aligned(ws) || ws_bytes < BL.total)
        return RFPS_ERR_WORKSPACE;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok || d->cus % kMaxXcds != 0 || d->cus > kMaxGroups)
        return RFPS_ERR_UNSUPPORTED;
    const int per_xcd = d->cus / kMaxXcds;
    const int T = (params && params->groups) ? params->groups : per_xcd;
    const long long teams = d->cus / std::max(T, 1);
    if (T < 2 || per_xcd % T != 0 || teams * (2 * T + 1) * kMaxSlotWords > kBoardWords)
        return RFPS_ERR_UNSUPPORTED;
    SampleLaunch L;
    L.G = d->cus;
    L.flags = flags;
    L.R = (params && params->lookahead) ? params->lookahead : kDefaultLookahead;
    const size_t stat = rfps_sampler_static_lds(L.R);
    if (stat == 0 || (size_t)d->max_lds <= stat + 1024)
        return RFPS_ERR_UNSUPPORTED;
    L.lds_budget = (uint32_t)((d->max_lds - stat - 256) & ~(size_t)255);

    IndexView v = make_view_l(ws, BL, n, fixed_n_vox, resolve_tile(params));
    v.bc.batch = batch;
    v.bc.team_size = T;
    v.bc.per_xcd = per_xcd;
    v.bc.fixed_n_vox = fixed_n_vox;
    v.bc.shell_inv = shell_inv_of(params);
    v.bc.m_total = m_total;
    v.bc.offsets = offsets;
    v.bc.m = m;
    v.bc.starts = starts;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_build_batch(v, xyz, s);
    if (e == hipSuccess)
        e = launch_rfps_rounds_batched(v, L, out_idx, out_d2, s);
    if (e == hipSuccess && out_d2 && (flags & RFPS_F_SQRT))
        e = launch_sqrt_out(out_d2, m_total, s);
    if (e == hipErrorCooperativeLaunchTooLarge)
        return RFPS_ERR_UNSUPPORTED;
    return e == hipSuccess ? RFPS_OK : RFPS_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// No-allocation form of the batched call: its workspace is a fixed device
// array of this file instead of a caller's buffer.  In host code `scratch`
// names a host-side stand-in, never the device memory: the device address is
// resolved once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to the kernels.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];
bool g_scratch_done[64];
hipError_t g_scratch_err[64];
}  // namespace

// Device address of this device's copy of `scratch` (nullptr on failure).
static void *noalloc_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void *ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
        g_scratch_done[dev] = true;
    }
    return g_scratch_ptr[dev];
}

size_t rfps_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

rfps_status rfps_sample_batched_noalloc(const float *xyz, int32_t n, const int32_t *offsets, const int32_t *m,
                                        const int32_t *starts, int32_t batch, int32_t m_total,
                                        const rfps_params *params, int32_t *out_idx, float *out_d2, void *stream)
{
    if (!xyz || !offsets || !m || !out_idx || n < 1 || n > kMaxPoints || batch < 1 || batch > kMaxBatch ||
        batch > n || m_total < batch || m_total > n || !params_valid(params))
        return RFPS_ERR_INVALID_ARG;
    const size_t need = layout_batch(n, batch, params ? params->n_vox : 0, use_shells(params)).total;
    if (need > kNoAllocScratchBytes)
        return RFPS_ERR_SCRATCH_LIMIT;
    void *ws = noalloc_scratch();
    if (!ws)
        return RFPS_ERR_DEVICE;
    return rfps_sample_batched(xyz, n, offsets, m, starts, batch, m_total, params, ws, need, out_idx, out_d2,
                               stream);
}

static rfps_status read_header(const void *ws, size_t ws_bytes, void *stream, IndexHeader *h)
{
    if (!ws || !aligned(ws) || ws_bytes < sizeof(IndexHeader))
        return RFPS_ERR_WORKSPACE;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return RFPS_ERR_DEVICE;
    if (hipMemcpy(h, ws, sizeof *h, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    return RFPS_OK;
}

rfps_status rfps_batched_read_status(const void *ws, size_t ws_bytes, void *stream)
{
    IndexHeader h;
    const rfps_status st = read_header(ws, ws_bytes, stream, &h);
    if (st != RFPS_OK)
        return st;
    return (rfps_status)(h.build_status ? h.build_status : h.sample_status);
}

rfps_status rfps_batched_read_telemetry(const void *ws, size_t ws_bytes, void *stream, rfps_telemetry *out)
{
    if (!out)
        return RFPS_ERR_INVALID_ARG;
    IndexHeader h;
    const rfps_status st = read_header(ws, ws_bytes, stream, &h);
    if (st != RFPS_OK)
        return st;
    memcpy(out, h.tele, sizeof *out);
    const DeviceInfo *d = device_info();
    out->tick_hz = d ? (int64_t)d->wall_hz : 0;
    return RFPS_OK;
}

rfps_status rfps_autotune_batched(const float *xyz, int32_t n, const int32_t *offsets, const int32_t *m,
                                  const int32_t *starts, int32_t batch, int32_t m_total, const rfps_params *base,
                                  int32_t reps, void *ws, size_t ws_bytes, int32_t *out_idx, float *out_d2,
                                  void *stream, rfps_params *best, float *best_ms)
{
    if (!best || reps < 1 || reps > 100 || !params_valid(base))
        return RFPS_ERR_INVALID_ARG;
    const DeviceInfo *d = device_info();
    if (!d)
        return RFPS_ERR_DEVICE;
    if (!d->ok || d->cus % kMaxXcds != 0)
        return RFPS_ERR_UNSUPPORTED;
    const int per_xcd = d->cus / kMaxXcds;
    rfps_params b0 = base ? *base : rfps_params{0, 0, 0, 0, 0u};
    std::vector<int> Ts, Rs, tiles;
    for (int t = per_xcd; t >= 4; t /= 2)
        if (per_xcd % t == 0 && (!b0.groups || b0.groups == t))
            Ts.push_back(t);
    for (int r : {2, 3, 4, 8})
        if (!b0.lookahead || b0.lookahead == r)
            Rs.push_back(r);
    for (int t : {32, 64})
        if (!b0.tile || b0.tile == t)
            tiles.push_back(t);
    if (b0.groups && Ts.empty())
        Ts.push_back(b0.groups);  // let rfps_sample_batched judge it
    if (b0.tile && tiles.empty())
        tiles.push_back(b0.tile);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev0, ev1;
    if (hipEventCreate(&ev0) != hipSuccess)
        return RFPS_ERR_DEVICE;
    if (hipEventCreate(&ev1) != hipSuccess) {
        hipEventDestroy(ev0);
        return RFPS_ERR_DEVICE;
    }
    std::vector<int32_t> ref, cur;
    bool have_ref = false;
    float best_t = INFINITY;
    rfps_params bp{};
    rfps_status result = RFPS_OK;
    for (int T : Ts) {
        for (int R : Rs) {
            for (int tile : tiles) {
                rfps_params p = b0;
                p.groups = T;
                p.lookahead = R;
                p.tile = tile;
                // one untimed run: status, and the outputs against the first candidate
                rfps_status st = rfps_sample_batched(xyz, n, offsets, m, starts, batch, m_total, &p, ws, ws_bytes,
                                                     out_idx, out_d2, stream);
                if (st == RFPS_OK)
                    st = rfps_batched_read_status(ws, ws_bytes, stream);
                if (st == RFPS_ERR_CAPACITY || st == RFPS_ERR_UNSUPPORTED)
                    continue;  // this shape does not fit the device
                if (st != RFPS_OK) {
                    result = st;
                    goto done;
                }
                cur.resize((size_t)m_total);
                if (hipMemcpy(cur.data(), out_idx, 4 * (size_t)m_total, hipMemcpyDeviceToHost) != hipSuccess) {
                    result = RFPS_ERR_DEVICE;
                    goto done;
                }
                if (!have_ref) {
                    ref = cur;
                    have_ref = true;
                } else if (cur != ref) {
                    // every partition must give the same selections
                    result = RFPS_ERR_INTERNAL;
                    goto done;
                }
                std::vector<float> times;
                for (int r = 0; r < reps; ++r) {
                    hipEventRecord(ev0, s);
                    st = rfps_sample_batched(xyz, n, offsets, m, starts, batch, m_total, &p, ws, ws_bytes, out_idx,
                                             out_d2, stream);
                    hipEventRecord(ev1, s);
                    float ms = 0.0f;
                    if (st != RFPS_OK || hipEventSynchronize(ev1) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) {
                        result = st != RFPS_OK ? st : RFPS_ERR_DEVICE;
                        goto done;
                    }
                    times.push_back(ms);
                }
                std::sort(times.begin(), times.end());
                const float med = times[times.size() / 2];
                if (med < best_t) {
                    best_t = med;
                    bp = p;
                }
            }
        }
    }
    if (!have_ref) {
        result = RFPS_ERR_CAPACITY;
        goto done;
    }
    // leave the outputs of the chosen configuration behind
    result = rfps_sample_batched(xyz, n, offsets, m, starts, batch, m_total, &bp, ws, ws_bytes, out_idx, out_d2,
                                 stream);
    if (result == RFPS_OK)
        result = rfps_batched_read_status(ws, ws_bytes, stream);
    if (result == RFPS_OK) {
        *best = bp;
        if (best_ms)
            *best_ms = best_t;
    }
done:
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    return result;
}

}  // extern "C"
