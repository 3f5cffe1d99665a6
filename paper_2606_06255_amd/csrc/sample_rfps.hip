// Persistent RadiusFPS-G sampler (Sec. 3.3, Sec. 3.4; the roles of the two
// fusion kernels of Sec. 4.2-4.3, re-designed as one persistent kernel).
//
// One launch runs every selection.  Workgroup g owns the tiles t with
// t % G == g (tiles of neighbouring voxels land on different workgroups, so
// the unpruned work near a new sample spreads over the device) and keeps
// their points (x, y, z, Dist_p, original index) and per-tile state (sphere,
// packed Dist_v key, pruning threshold) in LDS for the whole run.
//
// Per selection j:
//   1. each workgroup reduces its tile keys to its best candidate;
//   2. it publishes the candidate (key + coordinates) in its exchange slot;
//   3. every workgroup reads all slots and takes the maximum key, so all
//      agree on s_j without a separate barrier (the slots carry the epoch);
//   4. workgroup 0 writes out_idx[j], out_d2[j];
//   5. every workgroup tests its tiles against s_j (spherical bound, FP32
//      threshold form), and for each surviving tile one wavefront applies the
//      point skip and the strict update, then recomputes the tile key
//      (Dist_v resync, eq. point_skip_distv_sync) and its threshold.
#include "rfps_internal.h"

namespace rfps {

struct SampleArgs {
    IndexHeader *hdr;
    const float *xs, *ys, *zs;
    const uint32_t *orig, *inv;
    const uint32_t *tstart, *tcnt;
    const float *tcx, *tcy, *tcz, *trad;
    unsigned long long *board;
    unsigned long long *trace;
    int32_t *out_idx;
    float *out_d2;
    int32_t n, m, start, G;
    uint32_t flags;
    uint32_t lds_budget;
};

// LDS bytes a workgroup needs for `tiles` tiles holding `pts` points.
__host__ __device__ __forceinline__ uint32_t rfps_lds_need(uint32_t tiles, uint32_t pts)
{
    return tiles * 40u + pts * 20u + 64u;
}

// Capacity plan: every workgroup's share must fit the dynamic LDS budget.
__global__ __launch_bounds__(kBlock) void k_rfps_plan(IndexHeader *hdr, const uint32_t *__restrict__ tcnt, int G,
                                                      uint32_t budget)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G || hdr->build_status)
        return;
    const uint32_t NT = hdr->n_tiles;
    uint32_t tiles = 0, pts = 0;
    for (uint32_t t = g; t < NT; t += G) {
        ++tiles;
        pts += tcnt[t];
    }
    if (pts > 65535u || rfps_lds_need(tiles, pts) > budget)
        set_status(&hdr->sample_status, RFPS_ERR_CAPACITY);
}

__global__ void k_sample_reset(IndexHeader *hdr, unsigned long long *board, int G, int32_t start,
                               int32_t *out_idx, float *out_d2, int32_t m)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        hdr->sample_status = 0;
        hdr->last_m = (uint32_t)m;
        hdr->trace_n = 0;
        for (int t = 0; t < kTeleFields; ++t)
            hdr->tele[t] = 0;
        out_idx[0] = start;
        if (out_d2)
            out_d2[0] = INFINITY;
    }
    // the slots a team of G workgroups uses (both protocols fit in this span)
    const int words = 2 * G * kMaxSlotWords;
    for (int w = tid; w < words; w += gridDim.x * blockDim.x)
        board[w] = 0ull;
}

// After a sampling call: on any recorded error, every output becomes -1 / NaN.
__global__ __launch_bounds__(kBlock) void k_sample_finalize(const IndexHeader *__restrict__ hdr, int m,
                                                            int32_t *__restrict__ out_idx, float *__restrict__ out_d2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || (hdr->build_status == 0 && hdr->sample_status == 0))
        return;
    out_idx[j] = -1;
    if (out_d2)
        out_d2[j] = __uint_as_float(0x7fc00000u);
}

__global__ __launch_bounds__(kBlock) void k_rfps(SampleArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_red[kWavesPerBlock];
    __shared__ unsigned long long s_red2[kWavesPerBlock];
    __shared__ uint32_t s_scan[kWavesPerBlock];
    __shared__ uint32_t s_wgt;      // local tile holding the workgroup's best key
    __shared__ uint32_t s_list_n;   // unpruned tiles this selection
    __shared__ uint32_t s_npts;
    __shared__ uint32_t s_abort;
    __shared__ float s_s[3];
    __shared__ uint32_t s_status;

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int g = blockIdx.x, G = a.G;
    IndexHeader *hdr = a.hdr;
    if (tid == 0)
        s_status = hdr->build_status | hdr->sample_status;
    __syncthreads();
    if (s_status)
        return;  // recorded before the launch, so the whole grid leaves here
    const uint32_t NT = hdr->n_tiles;
    const int ntl = (NT > (uint32_t)g) ? (int)((NT - 1 - g) / G) + 1 : 0;
    const bool use_skip = !(a.flags & RFPS_F_NO_POINT_SKIP);
    const bool euclid = (a.flags & RFPS_F_SQRT) != 0;
    const bool no_prune = (a.flags & RFPS_F_NO_PRUNE) != 0;
    const bool tele = (a.flags & RFPS_F_TELEMETRY) != 0;
    const bool trace = (a.flags & RFPS_F_TRACE) != 0 && g == 0 && tid == 0;

    // LDS layout (the plan kernel checked that it fits).
    unsigned long long *tkey = reinterpret_cast<unsigned long long *>(smem);
    float *tcx = reinterpret_cast<float *>(tkey + ntl);
    float *tcy = tcx + ntl;
    float *tcz = tcy + ntl;
    float *trad = tcz + ntl;
    float *tthr = trad + ntl;
    uint32_t *tmeta = reinterpret_cast<uint32_t *>(tthr + ntl);  // lds start | count << 16
    uint32_t *tbest = tmeta + ntl;                                // lds index of the tile's best point
    uint32_t *tlist = tbest + ntl;                                // unpruned tiles
    float *px = reinterpret_cast<float *>(tlist + ntl);

    // ---- prologue: tile metadata and LDS offsets (block prefix sum) ----
    const int per = (ntl + kBlock - 1) / kBlock;
    const int l0 = tid * per, l1 = min(l0 + per, ntl);
    uint32_t cnt_sum = 0;
    for (int lt = l0; lt < l1; ++lt)
        cnt_sum += a.tcnt[g + (size_t)lt * G];
    uint32_t incl = cnt_sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t o = __shfl_up(incl, off, kWave);
        if (lane >= off)
            incl += o;
    }
    if (lane == kWave - 1)
        s_scan[wave] = incl;
    __syncthreads();
    uint32_t off = incl - cnt_sum, npl = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) {
        off += q < wave ? s_scan[q] : 0u;
        npl += s_scan[q];
    }
    for (int lt = l0; lt < l1; ++lt) {
        const size_t t = g + (size_t)lt * G;
        const uint32_t c = a.tcnt[t];
        tmeta[lt] = off | (c << 16);
        tcx[lt] = a.tcx[t];
        tcy[lt] = a.tcy[t];
        tcz[lt] = a.tcz[t];
        trad[lt] = a.trad[t];
        off += c;
    }
    if (tid == 0)
        s_npts = npl;
    float *py = px + npl;
    float *pz = py + npl;
    float *pd = pz + npl;
    uint32_t *po = reinterpret_cast<uint32_t *>(pd + npl);

    // Seed s_0 and the initial update (Sec. 3.3): Dist_p from the seed, then
    // Dist_v per tile.
    const uint32_t p0 = a.inv[a.start];
    float sx = a.xs[p0], sy = a.ys[p0], sz = a.zs[p0];
    __syncthreads();
    for (int lt = wave; lt < ntl; lt += kWavesPerBlock) {
        const uint32_t meta = tmeta[lt];
        const uint32_t ls = meta & 0xffffu, c = meta >> 16;
        const uint32_t gs = a.tstart[g + (size_t)lt * G];
        const bool valid = (uint32_t)lane < c;
        unsigned long long key = 0;
        if (valid) {
            const uint32_t i = gs + lane, p = ls + lane;
            const float x = a.xs[i], y = a.ys[i], z = a.zs[i];
            const uint32_t o = a.orig[i];
            const float d0 = sqdist(x, y, z, sx, sy, sz);
            const float d = euclid ? sqrt_class_top(d0) : d0;
            px[p] = x;
            py[p] = y;
            pz[p] = z;
            pd[p] = d;
            po[p] = o;
            key = pack_key(d, o);
        }
        const unsigned long long kmax = wave_max_u64(key);
        const unsigned long long hit = __ballot(valid && key == kmax);
        if (lane == 0) {
            tkey[lt] = kmax;
            tbest[lt] = ls + (uint32_t)(__ffsll((long long)hit) - 1);
            tthr[lt] = prune_threshold(trad[lt], key_d2(kmax));
        }
    }
    if (tid == 0) {
        s_abort = 0;
        s_list_n = 0;
    }
    __syncthreads();

    unsigned long long t_tests = 0, t_pruned = 0, t_visited = 0, t_skipped = 0, t_updated = 0, t_resync = 0;

    for (int j = 1; j < a.m; ++j) {
        // 1. workgroup best over its tiles
        unsigned long long loc = 0;
        for (int lt = tid; lt < ntl; lt += kBlock)
            loc = umax64(loc, tkey[lt]);
        loc = wave_max_u64(loc);
        if (lane == 0)
            s_red[wave] = loc;
        __syncthreads();
        unsigned long long wgk = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q)
            wgk = umax64(wgk, s_red[q]);
        for (int lt = tid; lt < ntl; lt += kBlock)
            if (tkey[lt] == wgk)
                s_wgt = (uint32_t)lt;
        __syncthreads();

        // 2. publish the candidate
        const uint32_t epoch = (uint32_t)j;
        unsigned long long t_pub = 0;
        if (tid == 0) {
            Candidate c;
            c.key = 0;
            c.x = c.y = c.z = 0.0f;
            if (ntl > 0) {
                const uint32_t p = tbest[s_wgt];
                c.key = wgk;
                c.x = px[p];
                c.y = py[p];
                c.z = pz[p];
            }
            if (trace)
                t_pub = wall_clock64();
            publish(slot_ptr(a.board, G, epoch, g), epoch, c);
            s_list_n = 0;
        }

        // 3. read every slot and agree on the maximum
        Candidate c;
        c.key = 0;
        c.x = c.y = c.z = 0.0f;
        bool ok = true;
        if (tid < G)
            ok = poll_slot(slot_ptr(a.board, G, epoch, tid), epoch, c);
        if (!ok)
            s_abort = 1;
        const unsigned long long wk = wave_max_u64(c.key);
        if (lane == 0)
            s_red2[wave] = wk;
        __syncthreads();
        if (s_abort) {
            if (tid == 0) {
                set_status(&hdr->sample_status, RFPS_ERR_TIMEOUT);
                publish_abort(a.board, G, g);
            }
            return;
        }
        unsigned long long win = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q)
            win = umax64(win, s_red2[q]);
        if (tid < G && c.key == win) {
            s_s[0] = c.x;
            s_s[1] = c.y;
            s_s[2] = c.z;
        }
        __syncthreads();
        sx = s_s[0];
        sy = s_s[1];
        sz = s_s[2];

        // 4. output
        if (g == 0 && tid == 0) {
            a.out_idx[j] = (int32_t)key_orig(win);
            if (a.out_d2)
                a.out_d2[j] = key_d2(win);
            if (trace && j - 1 < kTraceCap) {
                a.trace[2 * (size_t)(j - 1)] = t_pub;
                a.trace[2 * (size_t)(j - 1) + 1] = wall_clock64();
            }
        }
        if (j == a.m - 1)
            break;

        // 5a. voxel filter: conservative spherical test per tile
        for (int lt = tid; lt < ntl; lt += kBlock) {
            const float q = sqdist(tcx[lt], tcy[lt], tcz[lt], sx, sy, sz);
            const bool pruned = !no_prune && q >= tthr[lt];
            t_tests += 1;
            t_pruned += pruned;
            if (!pruned)
                tlist[atomicAdd(&s_list_n, 1u)] = (uint32_t)lt;
        }
        __syncthreads();

        // 5b. point skip + strict update + Dist_v resync, one wavefront per tile
        const uint32_t nlist = s_list_n;
        for (uint32_t e = wave; e < nlist; e += kWavesPerBlock) {
            const uint32_t lt = tlist[e];
            const uint32_t meta = tmeta[lt];
            const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
            const bool valid = (uint32_t)lane < cnt;
            const uint32_t p = ls + (valid ? lane : 0);
            float d = pd[p];
            bool upd = false, skip = false;
            if (valid) {
                const float dx = px[p] - sx;
                const float dy = py[p] - sy;
                const float dz = pz[p] - sz;
                const float xx = dx * dx;
                const float yy = dy * dy;
                const float zz = dz * dz;
                skip = use_skip && (xx >= d || yy >= d || zz >= d);
                const float s2 = xx + yy;
                float t = s2 + zz;
                if (euclid && !skip && t < d)
                    t = sqrt_class_top(t);
                upd = !skip && t < d;
                if (upd) {
                    d = t;
                    pd[p] = t;
                }
            }
            const unsigned long long um = __ballot(upd);
            if (tele && lane == 0) {
                t_visited += cnt;
                t_skipped += (unsigned long long)__popcll(__ballot(skip));
                t_updated += (unsigned long long)__popcll(um);
                t_resync += um != 0;
            }
            if (um) {
                const unsigned long long key = valid ? pack_key(d, po[p]) : 0ull;
                const unsigned long long kmax = wave_max_u64(key);
                const unsigned long long hit = __ballot(valid && key == kmax);
                if (lane == 0) {
                    tkey[lt] = kmax;
                    tbest[lt] = ls + (uint32_t)(__ffsll((long long)hit) - 1);
                    tthr[lt] = prune_threshold(trad[lt], key_d2(kmax));
                }
            }
        }
        __syncthreads();
    }

    if (tele) {
        unsigned long long v[6] = {t_tests, t_pruned, t_visited, t_skipped, t_updated, t_resync};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            unsigned long long s = v[q];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1)
                s += __shfl_xor(s, o, kWave);
            if (lane == 0 && s)
                atomicAdd(&hdr->tele[2 + q], s);
        }
        if (g == 0 && tid == 0) {
            atomicAdd(&hdr->tele[0], (unsigned long long)(a.m > 1 ? a.m - 2 : 0));
            atomicAdd(&hdr->tele[1], (unsigned long long)NT);
            atomicAdd(&hdr->tele[8], (unsigned long long)(a.m > 1 ? a.m - 1 : 0));
        }
    }
    if (g == 0 && tid == 0)
        hdr->trace_n = (uint32_t)(a.m > 1 ? a.m - 1 : 0);
}

}  // namespace rfps

namespace rfps {

size_t rfps_sampler_static_lds(int R)
{
    if (R > 0)
        return rfps_rounds_static_lds(R);
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(k_rfps)) != hipSuccess)
        return 0;
    return attr.sharedSizeBytes;
}

hipError_t launch_rfps_sample(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s)
{
    k_sample_reset<<<4, kBlock, 0, s>>>(v.hdr, v.board, L.G, start, out_idx, out_d2, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (L.flags & RFPS_F_UNFUSED) {
        e = launch_rfps_unfused(v, m, start, L.flags, out_idx, out_d2, s);
        if (e != hipSuccess)
            return e;
    } else if (L.R > 0) {
        e = launch_rfps_rounds(v, m, start, L, out_idx, out_d2, s);
        if (e != hipSuccess)
            return e;
    } else {
        k_rfps_plan<<<(L.G + kBlock - 1) / kBlock, kBlock, 0, s>>>(v.hdr, v.tcnt, L.G, L.lds_budget);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        if (m > 1) {
            SampleArgs a;
            a.hdr = v.hdr;
            a.xs = v.xs;
            a.ys = v.ys;
            a.zs = v.zs;
            a.orig = v.orig;
            a.inv = v.inv;
            a.tstart = v.tstart;
            a.tcnt = v.tcnt;
            a.tcx = v.tcx;
            a.tcy = v.tcy;
            a.tcz = v.tcz;
            a.trad = v.trad;
            a.board = v.board;
            a.trace = v.trace;
            a.out_idx = out_idx;
            a.out_d2 = out_d2;
            a.n = v.n;
            a.m = m;
            a.start = start;
            a.G = L.G;
            a.flags = L.flags;
            a.lds_budget = L.lds_budget;
            void *args[] = {&a};
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_rfps),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_budget);
            if (e != hipSuccess)
                return e;
            e = launch_persistent(reinterpret_cast<const void *>(k_rfps), L.G, args, L.lds_budget, s);
            if (e != hipSuccess)
                return e;
        }
    }
    return launch_sample_finalize(v.hdr, m, out_idx, out_d2, s);
}

hipError_t launch_sample_finalize(const IndexHeader *hdr, int m, int32_t *out_idx, float *out_d2, hipStream_t s)
{
    k_sample_finalize<<<(m + kBlock - 1) / kBlock, kBlock, 0, s>>>(hdr, m, out_idx, out_d2);
    return hipGetLastError();
}

}  // namespace rfps
