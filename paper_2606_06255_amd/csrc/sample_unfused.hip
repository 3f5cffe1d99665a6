// Unfused sampler: one stream-ordered pair of kernel launches per selection.
//
// The paper's ablation (Sec. 5.4, Tab. ablation) compares its fused persistent
// kernel with a variant that splits every iteration into separate kernels
// (selection, voxel filter, point update, voxel resync).  This is that
// variant on the same index: per selection j,
//   k_unf_select  one workgroup takes the largest tile key (largest distance,
//                 lowest original index), records s_j and writes the outputs;
//   k_unf_update  a grid-stride pass over the tiles: spherical filter
//                 (Sec. 3.4.2), point skip, strict update and the tile's key
//                 resync (Sec. 3.4.3), fused into one launch since each needs
//                 only its own tile.
// The state lives in HBM between launches: Dist_p in sorted order and the
// tile keys as two 32-bit halves.  It reuses index buffers the build no
// longer needs (the idle radix ping-pong buffer, the voxel head flags and
// their scan), so it needs no workspace of its own; a later build rewrites
// them.  The selection sequence is the plain FPS sequence, like every other
// sampler here.
#include "rfps_internal.h"

namespace rfps {

namespace {

constexpr int kSelThreads = 1024;

struct UnfusedArgs {
    IndexHeader *hdr;
    const float *xs, *ys, *zs;
    const uint32_t *orig, *inv, *tstart, *tcnt;
    const float *tcx, *tcy, *tcz, *trad;
    float *pd;                  // [n] Dist_p of every point, sorted order
    uint32_t *tb_d, *tb_o;      // [n_tiles] tile key: distance bits, ~original index
    unsigned long long *sel;    // [3] selected key, x | y << 32, z
    int32_t *out_idx;
    float *out_d2;
    int32_t start;
    uint32_t flags;
};

__device__ __forceinline__ bool fresh_less(float &t, float d, bool euclid)
{
    // strict update test of a fresh squared distance t against the state d;
    // in Euclidean mode t becomes its class top first (only when t < d)
    if (euclid && t < d)
        t = sqrt_class_top(t);
    return t < d;
}

__global__ __launch_bounds__(kBlock) void k_unf_init(UnfusedArgs a)
{
    if (a.hdr->build_status)
        return;
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
    const int nw = gridDim.x * kWavesPerBlock;
    const bool euclid = (a.flags & RFPS_F_SQRT) != 0;
    const uint32_t NT = a.hdr->n_tiles;
    const uint32_t p0 = a.inv[a.start];
    const float sx = a.xs[p0], sy = a.ys[p0], sz = a.zs[p0];
    for (uint32_t t = (uint32_t)gw; t < NT; t += (uint32_t)nw) {
        const uint32_t c = a.tcnt[t], base = a.tstart[t];
        unsigned long long key = 0;
        if ((uint32_t)lane < c) {
            const uint32_t i = base + lane;
            float d = sqdist(a.xs[i], a.ys[i], a.zs[i], sx, sy, sz);
            if (euclid)
                d = sqrt_class_top(d);
            a.pd[i] = d;
            key = pack_key(d, a.orig[i]);
        }
        const unsigned long long k = wave_max_u64(key);
        if (lane == 0) {
            a.tb_d[t] = (uint32_t)(k >> 32);
            a.tb_o[t] = (uint32_t)k;
        }
    }
}

__global__ __launch_bounds__(kSelThreads) void k_unf_select(UnfusedArgs a, int32_t j)
{
    __shared__ unsigned long long s_red[kSelThreads / kWave];
    if (a.hdr->build_status)
        return;  // the finalize pass poisons the outputs
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t NT = a.hdr->n_tiles;
    unsigned long long best = 0;
    for (uint32_t t = (uint32_t)tid; t < NT; t += kSelThreads)
        best = umax64(best, ((unsigned long long)a.tb_d[t] << 32) | a.tb_o[t]);
    best = wave_max_u64(best);
    if (lane == 0)
        s_red[wave] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kSelThreads / kWave; ++w)
            best = umax64(best, s_red[w]);
        const uint32_t o = key_orig(best);
        const uint32_t p = a.inv[o];
        a.sel[0] = best;
        a.sel[1] = (unsigned long long)__float_as_uint(a.xs[p]) | ((unsigned long long)__float_as_uint(a.ys[p]) << 32);
        a.sel[2] = (unsigned long long)__float_as_uint(a.zs[p]);
        a.out_idx[j] = (int32_t)o;
        if (a.out_d2)
            a.out_d2[j] = key_d2(best);
    }
}

__global__ __launch_bounds__(kBlock) void k_unf_update(UnfusedArgs a)
{
    if (a.hdr->build_status)
        return;
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
    const int nw = gridDim.x * kWavesPerBlock;
    const bool euclid = (a.flags & RFPS_F_SQRT) != 0;
    const bool prune = !(a.flags & RFPS_F_NO_PRUNE);
    const bool use_skip = !(a.flags & RFPS_F_NO_POINT_SKIP);
    const unsigned long long xy = a.sel[1];
    const float sx = __uint_as_float((uint32_t)xy), sy = __uint_as_float((uint32_t)(xy >> 32));
    const float sz = __uint_as_float((uint32_t)a.sel[2]);
    const uint32_t NT = a.hdr->n_tiles;
    for (uint32_t t = (uint32_t)gw; t < NT; t += (uint32_t)nw) {
        // voxel filter: the tile's distance is the largest Dist_p it holds
        if (prune) {
            const float thr = prune_threshold(a.trad[t], __uint_as_float(a.tb_d[t]));
            if (sqdist(a.tcx[t], a.tcy[t], a.tcz[t], sx, sy, sz) >= thr)
                continue;
        }
        const uint32_t c = a.tcnt[t], base = a.tstart[t];
        unsigned long long key = 0;
        bool changed = false;
        if ((uint32_t)lane < c) {
            const uint32_t i = base + lane;
            float d = a.pd[i];
            const float dx = a.xs[i] - sx, dy = a.ys[i] - sy, dz = a.zs[i] - sz;
            const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
            const bool skip = use_skip && (xx >= d || yy >= d || zz >= d);
            const float s2 = xx + yy;
            float tt = s2 + zz;
            if (!skip && fresh_less(tt, d, euclid)) {
                d = tt;
                a.pd[i] = d;
                changed = true;
            }
            key = pack_key(d, a.orig[i]);
        }
        // resync: only a tile whose points changed needs a new key
        if (__ballot(changed)) {
            const unsigned long long k = wave_max_u64(key);
            if (lane == 0) {
                a.tb_d[t] = (uint32_t)(k >> 32);
                a.tb_o[t] = (uint32_t)k;
            }
        }
    }
}

}  // namespace

hipError_t launch_rfps_unfused(const IndexView &v, int m, int start, uint32_t flags, int32_t *out_idx,
                               float *out_d2, hipStream_t s)
{
    UnfusedArgs a;
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
    // the radix buffers the sorted keys and indices do not occupy (n words each)
    a.pd = reinterpret_cast<float *>(v.skey == v.keyA ? v.keyB : v.keyA);
    a.tb_d = v.flags;  // n words each; there are at most n tiles
    a.tb_o = v.hscan;
    a.sel = v.board;
    a.out_idx = out_idx;
    a.out_d2 = out_d2;
    a.start = start;
    a.flags = flags;
    // enough waves to cover the tiles of a typical index in a few passes
    const int blocks = std::max(1, std::min(1024, (v.n + 4 * kWave - 1) / (4 * kWave)));
    k_unf_init<<<blocks, kBlock, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    for (int j = 1; j < m && e == hipSuccess; ++j) {
        k_unf_select<<<1, kSelThreads, 0, s>>>(a, j);
        k_unf_update<<<blocks, kBlock, 0, s>>>(a);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace rfps
