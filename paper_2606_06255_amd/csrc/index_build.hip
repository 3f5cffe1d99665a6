// Spherical-voxel index builder (Sec. 3.2; the GPU steps of Algorithm 2):
// bounding box, voxel size L (eq. voxel_size), clamped voxel id
// V_id = v_z n^2 + v_y n + v_x, stable LSD radix sort of (V_id, original
// index), gather to structure-of-arrays coordinates, active-voxel compaction
// (offsets per voxel), split of voxels into tiles of at most T points and an
// enclosing sphere per tile.
//
// All kernels are launched by rfps_api.hip on the caller's stream; counts
// that only the device knows (K voxels, NT tiles) stay in the index header
// and grid-stride loops read them there.
#include <algorithm>
#include <utility>

#include "rfps_internal.h"

namespace rfps {

__global__ void k_build_reset(IndexHeader *hdr)
{
    if (threadIdx.x == 0) {
        hdr->build_status = 0;
        hdr->sample_status = 0;
        hdr->n_voxels = 0;
        hdr->n_tiles = 0;
        for (int a = 0; a < 3; ++a) {
            hdr->bb[a] = 0xffffffffu;  // running minimum
            hdr->bb[3 + a] = 0u;       // running maximum
        }
        for (int t = 0; t < kTeleFields; ++t)
            hdr->tele[t] = 0;
        hdr->trace_n = 0;
    }
}

// Bounding box of the cloud; flags non-finite coordinates.
__global__ __launch_bounds__(kBlock) void k_bbox(const float *__restrict__ xyz, int n, IndexHeader *hdr)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = xyz[3 * (size_t)i + a];
            bad |= !isfinite(v);
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
    // wave, then workgroup reduction; one atomic per bound per workgroup
    __shared__ float s_mn[3][kWavesPerBlock], s_mx[3][kWavesPerBlock];
    __shared__ uint32_t s_bad;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0)
        s_bad = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min_f32(mn[a]);
        mx[a] = wave_max_f32(mx[a]);
        if (lane == 0) {
            s_mn[a][w] = mn[a];
            s_mx[a][w] = mx[a];
        }
    }
    const bool wave_bad = __any(bad);
    __syncthreads();
    if (wave_bad && lane == 0)
        s_bad = 1;
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        float lo = s_mn[a][0], hi = s_mx[a][0];
        for (int q = 1; q < kWavesPerBlock; ++q) {
            lo = fminf(lo, s_mn[a][q]);
            hi = fmaxf(hi, s_mx[a][q]);
        }
        if (lo <= hi) {
            atomicMin(&hdr->bb[a], f2ord(lo));
            atomicMax(&hdr->bb[3 + a], f2ord(hi));
        }
    }
    if (threadIdx.x == 0 && s_bad)
        set_status(&hdr->build_status, RFPS_ERR_NONFINITE);
}

// Voxel edge L = alpha * max(E) / n_vox with alpha = 1 + 1e-4 (eq. voxel_size);
// a cloud of identical points gets L = 1 (one voxel).  The range shells (if
// any) are centred on the bounding-box centre.
__global__ void k_grid(IndexHeader *hdr, int n_vox, double shell_inv, uint32_t shell_cap)
{
    if (threadIdx.x != 0)
        return;
    double E = 0.0;
    for (int a = 0; a < 3; ++a) {
        const float lo = ord2f(hdr->bb[a]), hi = ord2f(hdr->bb[3 + a]);
        hdr->pmin[a] = (double)lo;
        hdr->origin[a] = 0.5 * ((double)lo + (double)hi);
        const double e = (double)hi - (double)lo;
        E = e > E ? e : E;
    }
    const double alpha = 1.0 + 1e-4;
    // a failed build still gets a finite edge: the keys are then meaningless
    // but every index computed from them stays in range
    hdr->L = (E > 0.0 && E < INFINITY && !hdr->build_status) ? alpha * E / (double)n_vox : 1.0;
    hdr->shell_inv = shell_inv;
    hdr->shell_cap = shell_cap;
}

// Voxel key of every point and the identity payload.
__global__ __launch_bounds__(kBlock) void k_voxel_key(const float *__restrict__ xyz, int n,
                                                      const IndexHeader *__restrict__ hdr, int n_vox,
                                                      uint32_t *__restrict__ key, uint32_t *__restrict__ val)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    key[i] = voxel_key(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2], hdr->pmin, hdr->L,
                       (uint32_t)n_vox, hdr->origin, hdr->shell_inv, hdr->shell_cap);
    val[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8 bits per pass.  Tile b covers keys
// [b*kRadixTile, (b+1)*kRadixTile).  hist is digit-major: hist[d*nblk + b].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *__restrict__ keys, int n, int shift,
                                                       uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRadixTile;
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
        int i = base + r * kBlock + tid;
        if (i < n)
            atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)tid * nblk + blockIdx.x] = h[tid];
}

// Scatter with a stable rank: keys are visited in index order (round r, wave
// w, lane l); the rank among equal digits inside a wave comes from eight
// ballots, and per-digit counters carry the order across waves and rounds.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin,
                                                          uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                          int n, int shift, const uint32_t *__restrict__ hist,
                                                          int nblk)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kWavesPerBlock][256];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    base[tid] = hist[(size_t)tid * nblk + blockIdx.x];
    const int tile0 = blockIdx.x * kRadixTile;
    const unsigned long long below = lane ? (~0ull >> (kWave - lane)) : 0ull;
    for (int r = 0; r < kRadixItems; ++r) {
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q)
            wcnt[q][tid] = 0;
        __syncthreads();
        const int i = tile0 + r * kBlock + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            unsigned long long ones = __ballot(valid && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0)
            wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (int q = 0; q < w; ++q)
                off += wcnt[q][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q)
            add += wcnt[q][tid];
        base[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of uint32 (in place allowed), three kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *wsum /*[kWavesPerBlock]*/,
                                                         uint32_t &total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t o = __shfl_up(incl, off, kWave);
        if (lane >= off)
            incl += o;
    }
    if (lane == kWave - 1)
        wsum[w] = incl;
    __syncthreads();
    uint32_t woff = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < kWavesPerBlock; ++q) {
        woff += q < w ? wsum[q] : 0u;
        total += wsum[q];
    }
    __syncthreads();
    return woff + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_blocks(const uint32_t *in, uint32_t *out, int n,
                                                        uint32_t *__restrict__ partials)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        size_t i = base + q;
        v[q] = i < (size_t)n ? in[i] : 0u;
        s += v[q];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, wsum, total);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        size_t i = base + q;
        if (i < (size_t)n)
            out[i] = run;
        run += v[q];
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = total;
}

// One workgroup scans the per-block totals (nb <= kBlock * 64) and writes the
// grand total to *total_out when it is not NULL.
__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t *partials, int nb, uint32_t *total_out)
{
    __shared__ uint32_t wsum[kWavesPerBlock];
    const int per = (nb + kBlock - 1) / kBlock;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nb)
            s += partials[b0 + q];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, wsum, total);
    for (int q = 0; q < per; ++q) {
        if (b0 + q < nb) {
            uint32_t v = partials[b0 + q];
            partials[b0 + q] = run;
            run += v;
        }
    }
    if (threadIdx.x == 0 && total_out)
        *total_out = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *out, int n, const uint32_t *__restrict__ partials)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] += partials[i / kScanChunk];
}

// ---------------------------------------------------------------------------
// Gather to structure of arrays, inverse permutation, voxel compaction, tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gather(const float *__restrict__ xyz, const uint32_t *__restrict__ orig,
                                                   int n, float *__restrict__ xs, float *__restrict__ ys,
                                                   float *__restrict__ zs, uint32_t *__restrict__ inv)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    uint32_t o = orig[p];
    xs[p] = xyz[3 * (size_t)o];
    ys[p] = xyz[3 * (size_t)o + 1];
    zs[p] = xyz[3 * (size_t)o + 2];
    inv[o] = (uint32_t)p;
}

__global__ __launch_bounds__(kBlock) void k_heads(const uint32_t *__restrict__ skey, int n, uint32_t *__restrict__ flags)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n)
        flags[p] = (p == 0 || skey[p] != skey[p - 1]) ? 1u : 0u;
}

// vstart[k] = first sorted position of active voxel k; vstart[K] = n.
__global__ __launch_bounds__(kBlock) void k_voxels(const uint32_t *__restrict__ flags,
                                                   const uint32_t *__restrict__ hscan, int n,
                                                   uint32_t *__restrict__ vstart)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    if (flags[p])
        vstart[hscan[p]] = (uint32_t)p;
    if (p == n - 1)
        vstart[hscan[p] + flags[p]] = (uint32_t)n;
}

// Tiles per voxel: ceil(count / T); zero past K so the scan over n entries
// yields the tile total.
__global__ __launch_bounds__(kBlock) void k_tile_count(const uint32_t *__restrict__ vstart,
                                                       const IndexHeader *__restrict__ hdr, int n, int T,
                                                       uint32_t *__restrict__ tcount)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const uint32_t K = hdr->n_voxels;
    tcount[k] = (uint32_t)k < K ? (vstart[k + 1] - vstart[k] + (uint32_t)T - 1) / (uint32_t)T : 0u;
}

// One wavefront per tile: its points are lanes.  The sphere centre is the
// FP32-rounded centre of the tile's bounding box; the radius is the largest
// member distance to that centre, in FP64, enlarged by 2^-40 relative and
// rounded up to FP32, so it is never below the true largest distance.  Any
// sphere that encloses the members keeps the pruning test conservative.
__global__ __launch_bounds__(kBlock) void k_tiles(const uint32_t *__restrict__ vstart,
                                                  const uint32_t *__restrict__ tbase,
                                                  const IndexHeader *__restrict__ hdr, int T,
                                                  const float *__restrict__ xs, const float *__restrict__ ys,
                                                  const float *__restrict__ zs, uint32_t *__restrict__ tstart,
                                                  uint32_t *__restrict__ tcnt, float *__restrict__ tcx,
                                                  float *__restrict__ tcy, float *__restrict__ tcz,
                                                  float *__restrict__ trad)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    const uint32_t K = hdr->n_voxels, NT = hdr->n_tiles;
    for (uint32_t t = gw; t < NT; t += nw) {
        uint32_t lo = 0, hi = K - 1;  // last voxel with tbase <= t
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (tbase[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t start = vstart[lo] + (t - tbase[lo]) * (uint32_t)T;
        const uint32_t end = min(start + (uint32_t)T, vstart[lo + 1]);
        const uint32_t cnt = end - start;
        const bool valid = (uint32_t)lane < cnt;
        const uint32_t i = start + (valid ? lane : 0);
        const float x = xs[i], y = ys[i], z = zs[i];
        float c[3];
        const float p[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float lo_a = wave_min_f32(valid ? p[a] : INFINITY);
            float hi_a = wave_max_f32(valid ? p[a] : -INFINITY);
            c[a] = (float)(0.5 * ((double)lo_a + (double)hi_a));
        }
        double dx = (double)x - (double)c[0], dy = (double)y - (double)c[1], dz = (double)z - (double)c[2];
        double r2 = wave_max_f64(valid ? dx * dx + dy * dy + dz * dz : 0.0);
        double r = sqrt(r2) * (1.0 + 0x1p-40) + 0x1p-120;
        float r32 = (float)r;
        if ((double)r32 < r)
            r32 = nextafterf(r32, INFINITY);
        if (lane == 0) {
            tstart[t] = start;
            tcnt[t] = cnt;
            tcx[t] = c[0];
            tcy[t] = c[1];
            tcz[t] = c[2];
            trad[t] = r32;
        }
    }
}

// Coordinates of the picks in pick order: the input of the next stage of a
// multi-stage down-sampling.  An index outside [0, n) gives NaN coordinates,
// which the next index build reports as non-finite input.
__global__ __launch_bounds__(kBlock) void k_gather_xyz(const float *__restrict__ xyz, int n,
                                                       const int32_t *__restrict__ idx, int m,
                                                       float *__restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m)
        return;
    const int32_t i = idx[j];
    const bool ok = i >= 0 && i < n;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        out[3 * (size_t)j + a] = ok ? xyz[3 * (size_t)i + a] : NAN;
}

// Euclidean mode: the sampler keeps squared class tops; the reported
// distance is their correctly rounded root (the same root for every value of
// a class).
__global__ __launch_bounds__(kBlock) void k_sqrt_out(float *__restrict__ d, int m)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m)
        d[j] = sqrt_rn(d[j]);
}

}  // namespace rfps

namespace rfps {

static inline int blocks_for(long long n, int per_block) { return (int)((n + per_block - 1) / per_block); }

hipError_t launch_gather_xyz(const float *xyz, int n, const int32_t *idx, int m, float *out, hipStream_t s)
{
    k_gather_xyz<<<blocks_for(m, kBlock), kBlock, 0, s>>>(xyz, n, idx, m, out);
    return hipGetLastError();
}

hipError_t launch_sqrt_out(float *d, int m, hipStream_t s)
{
    k_sqrt_out<<<blocks_for(m, kBlock), kBlock, 0, s>>>(d, m);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *in, uint32_t *out, int n, uint32_t *partials, uint32_t *total,
                       hipStream_t s)
{
    const int nb = blocks_for(n, kScanChunk);
    if (nb > kBlock * 64)
        return hipErrorInvalidValue;
    k_scan_blocks<<<nb, kBlock, 0, s>>>(in, out, n, partials);
    k_scan_partials<<<1, kBlock, 0, s>>>(partials, nb, total);
    k_scan_add<<<blocks_for(n, kBlock), kBlock, 0, s>>>(out, n, partials);
    return hipGetLastError();
}

hipError_t launch_build_index(const IndexView &v, const float *xyz, hipStream_t s)
{
    const int n = v.n;
    k_build_reset<<<1, kWave, 0, s>>>(v.hdr);
    k_bbox<<<std::min(blocks_for(n, kBlock * 4), 512), kBlock, 0, s>>>(xyz, n, v.hdr);
    k_grid<<<1, kWave, 0, s>>>(v.hdr, v.n_vox, v.shell_inv, v.shell_cap);
    k_voxel_key<<<blocks_for(n, kBlock), kBlock, 0, s>>>(xyz, n, v.hdr, v.n_vox, v.keyA, v.valA);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // stable LSD radix sort of (voxel id, original index)
    const int nblk = blocks_for(n, kRadixTile);
    uint32_t *kin = v.keyA, *vin = v.valA, *kout = v.keyB, *vout = v.valB;
    for (int pass = 0; pass < v.radix_passes; ++pass) {
        const int shift = 8 * pass;
        k_radix_hist<<<nblk, kBlock, 0, s>>>(kin, n, shift, v.hist, nblk);
        e = launch_scan(v.hist, v.hist, 256 * nblk, v.partials, nullptr, s);
        if (e != hipSuccess)
            return e;
        k_radix_scatter<<<nblk, kBlock, 0, s>>>(kin, vin, kout, vout, n, shift, v.hist, nblk);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // v.skey / v.orig alias the buffers that hold the final pass
    k_gather<<<blocks_for(n, kBlock), kBlock, 0, s>>>(xyz, v.orig, n, v.xs, v.ys, v.zs, v.inv);
    k_heads<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.skey, n, v.flags);
    e = launch_scan(v.flags, v.hscan, n, v.partials, &v.hdr->n_voxels, s);
    if (e != hipSuccess)
        return e;
    k_voxels<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.flags, v.hscan, n, v.vstart);
    k_tile_count<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.vstart, v.hdr, n, v.tile, v.tcount);
    e = launch_scan(v.tcount, v.tbase, n, v.partials, &v.hdr->n_tiles, s);
    if (e != hipSuccess)
        return e;
    k_tiles<<<std::min(blocks_for(n, kWavesPerBlock), 2048), kBlock, 0, s>>>(
        v.vstart, v.tbase, v.hdr, v.tile, v.xs, v.ys, v.zs, v.tstart, v.tcnt, v.tcx, v.tcy, v.tcz, v.trad);
    return hipGetLastError();
}

}  // namespace rfps

// ---------------------------------------------------------------------------
// Batched index: the clouds of a batch share one sorted index.  A point of
// cloud c gets the key base_c + V_id (V_id on the cloud's own grid), so
// voxels and tiles never mix clouds and the tiles of every cloud are one
// contiguous range.
// ---------------------------------------------------------------------------
namespace rfps {

// Cloud of global point i: the largest c with offsets[c] <= i.
__device__ __forceinline__ int cloud_of(const int32_t *off, int B, int i)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}


// Clears the header, the per-cloud boxes, the batch state and the exchange
// board (epochs restart at 1 in every call).
__global__ __launch_bounds__(kBlock) void k_batch_reset(IndexHeader *hdr, BatchCtl bc, uint32_t *cl_bb,
                                                        BatchState *st, unsigned long long *board)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    if (tid == 0) {
        hdr->build_status = 0;
        hdr->sample_status = 0;
        hdr->n_voxels = 0;
        hdr->n_tiles = 0;
        hdr->last_m = (uint32_t)bc.m_total;
        hdr->trace_n = 0;
        for (int t = 0; t < kTeleFields; ++t)
            hdr->tele[t] = 0;
        st->joined = 0;
        st->next = 0;
        for (int x = 0; x < kMaxXcds; ++x)
            st->xcd_count[x] = 0;
    }
    for (int c = tid; c < bc.batch; c += nth) {
        for (int a = 0; a < 3; ++a) {
            cl_bb[6 * c + a] = 0xffffffffu;
            cl_bb[6 * c + 3 + a] = 0u;
        }
    }
    for (int w = tid; w < kBoardWords; w += nth)
        board[w] = 0ull;
}

// Checks the batch description (offsets from 0 to n with every cloud
// non-empty, 1 <= m_c <= N_c, start indices inside their clouds, sum of m
// equal to the output length), then computes the output offsets, the bins
// per axis and the first key of every cloud.  One workgroup; the prefix sums
// run on one thread (batch <= 4096).
__global__ void k_batch_setup(IndexHeader *hdr, BatchCtl bc, int n, uint32_t *cl_nvox, uint32_t *cl_base)
{
    __shared__ uint32_t s_bad;
    if (threadIdx.x == 0)
        s_bad = (bc.offsets[0] != 0 || bc.offsets[bc.batch] != n) ? 1u : 0u;
    __syncthreads();
    for (int c = threadIdx.x; c < bc.batch; c += blockDim.x) {
        const int nc = bc.offsets[c + 1] - bc.offsets[c];
        const int mc = bc.m[c];
        const int sc = bc.starts ? bc.starts[c] : 0;
        if (nc < 1 || mc < 1 || mc > nc || sc < 0 || sc >= nc)
            atomicOr(&s_bad, 1u);
        cl_nvox[c] = (uint32_t)(bc.fixed_n_vox ? bc.fixed_n_vox : default_n_vox_rule(nc > 0 ? nc : 1));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long base = 0, out = 0;
        for (int c = 0; c < bc.batch; ++c) {
            cl_base[c] = (uint32_t)base;
            bc.out_offsets[c] = (uint32_t)out;
            const unsigned long long nv = cl_nvox[c];
            base += nv * nv * nv * shell_cap_for(cl_nvox[c], bc.shell_inv > 0.0);
            out += (unsigned long long)(bc.m[c] > 0 ? bc.m[c] : 0);
        }
        cl_base[bc.batch] = (uint32_t)base;
        bc.out_offsets[bc.batch] = (uint32_t)out;
        if (s_bad || out != (unsigned long long)bc.m_total)
            set_status(&hdr->build_status, RFPS_ERR_INVALID_ARG);
        else if (base > 0xffffffffull)
            set_status(&hdr->build_status, RFPS_ERR_UNSUPPORTED);
    }
}

// Per-cloud bounding boxes; flags non-finite coordinates.  A wavefront whose
// points all belong to one cloud reduces before its atomics.
// Bounding box of every cloud.  A wavefront takes a run of kBboxRun
// consecutive points and keeps the running box of the cloud it is in,
// flushing it with one atomic per bound when the run moves into the next
// cloud (clouds are contiguous ranges of the input) and at its end.
constexpr int kBboxRun = 2048;

__global__ __launch_bounds__(kBlock) void k_bbox_batch(const float *__restrict__ xyz, int n, BatchCtl bc,
                                                       uint32_t *cl_bb, IndexHeader *hdr)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nw = gridDim.x * blockDim.x / kWave;
    bool bad = false;
    for (int b = gw * kBboxRun; b < n; b += nw * kBboxRun) {
        const int e = min(b + kBboxRun, n);
        // (the last cloud runs to n whatever the offsets say, so that
        // inconsistent offsets, reported by the setup kernel, stay in bounds)
        int c = cloud_of(bc.offsets, bc.batch, b);
        int cend = c + 1 < bc.batch ? bc.offsets[c + 1] : n;
        float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        auto flush = [&]() {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float lo = wave_min_f32(mn[a]);
                const float hi = wave_max_f32(mx[a]);
                if (lane == 0 && lo <= hi) {
                    atomicMin(&cl_bb[6 * c + a], f2ord(lo));
                    atomicMax(&cl_bb[6 * c + 3 + a], f2ord(hi));
                }
                mn[a] = INFINITY;
                mx[a] = -INFINITY;
            }
        };
        for (int i0 = b; i0 < e; i0 += kWave) {
            const int i = i0 + lane;
            const bool valid = i < e;
            float p[3] = {0.0f, 0.0f, 0.0f};
            if (valid) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p[a] = xyz[3 * (size_t)i + a];
                    bad |= !isfinite(p[a]);
                }
            }
            // the lanes of one step may belong to several clouds
            bool todo = valid;
            while (__any(todo)) {
                const bool mine = todo && i < cend;
                if (mine) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        mn[a] = fminf(mn[a], p[a]);
                        mx[a] = fmaxf(mx[a], p[a]);
                    }
                }
                todo = todo && !mine;
                if (__any(todo)) {
                    flush();
                    ++c;
                    cend = c + 1 < bc.batch ? bc.offsets[c + 1] : n;
                }
            }
        }
        flush();
    }
    if (__any(bad) && lane == 0)
        set_status(&hdr->build_status, RFPS_ERR_NONFINITE);
}

// Grid of every cloud: its own box and bins (eq. voxel_size).
__global__ __launch_bounds__(kBlock) void k_grid_batch(IndexHeader *hdr, BatchCtl bc, const uint32_t *cl_bb,
                                                       const uint32_t *cl_nvox, double *cl_pmin, double *cl_L)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bc.batch)
        return;
    double E = 0.0;
    for (int a = 0; a < 3; ++a) {
        const float lo = ord2f(cl_bb[6 * c + a]), hi = ord2f(cl_bb[6 * c + 3 + a]);
        cl_pmin[3 * c + a] = (double)lo;
        const double e = (double)hi - (double)lo;
        E = e > E ? e : E;
    }
    const double alpha = 1.0 + 1e-4;
    // a failed build still gets a finite edge: the keys are then meaningless
    // but every index computed from them stays in range
    cl_L[c] = (E > 0.0 && E < INFINITY && !hdr->build_status) ? alpha * E / (double)cl_nvox[c] : 1.0;
}

__global__ __launch_bounds__(kBlock) void k_voxel_key_batch(const float *__restrict__ xyz, int n, BatchCtl bc,
                                                            const uint32_t *__restrict__ cl_nvox,
                                                            const uint32_t *__restrict__ cl_base,
                                                            const double *__restrict__ cl_pmin,
                                                            const double *__restrict__ cl_L,
                                                            const uint32_t *__restrict__ cl_bb, uint32_t *key,
                                                            uint32_t *val)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int c = cloud_of(bc.offsets, bc.batch, i);
    const uint32_t nv = cl_nvox[c];
    double o[3];
    for (int a = 0; a < 3; ++a)
        o[a] = 0.5 * ((double)ord2f(cl_bb[6 * c + a]) + (double)ord2f(cl_bb[6 * c + 3 + a]));
    key[i] = cl_base[c] + voxel_key(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2],
                                    cl_pmin + 3 * c, cl_L[c], nv, o, bc.shell_inv,
                                    shell_cap_for(nv, bc.shell_inv > 0.0));
    val[i] = (uint32_t)i;
}

// First tile of every cloud.  Tiles follow the key order, so the tiles of a
// cloud are contiguous and clouds appear in index order; every cloud of a
// valid batch has at least one tile.
__global__ __launch_bounds__(kBlock) void k_tile_first(const uint32_t *__restrict__ tstart,
                                                       const uint32_t *__restrict__ orig,
                                                       const IndexHeader *__restrict__ hdr, BatchCtl bc,
                                                       uint32_t *tile_first)
{
    const uint32_t NT = hdr->n_tiles;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += gridDim.x * blockDim.x) {
        const int c = cloud_of(bc.offsets, bc.batch, (int)orig[tstart[t]]);
        const int cp = t ? cloud_of(bc.offsets, bc.batch, (int)orig[tstart[t - 1]]) : -1;
        for (int q = cp + 1; q <= c; ++q)
            tile_first[q] = t;
        if (t == NT - 1)
            tile_first[bc.batch] = NT;
    }
}

// Clouds by decreasing cost N_c * m_c, ties by index: the teams take them in
// this order, so the longest jobs start first.
__global__ void k_batch_order(BatchCtl bc, int32_t *order)
{
    for (int c = threadIdx.x; c < bc.batch; c += blockDim.x) {
        const long long cc = (long long)(bc.offsets[c + 1] - bc.offsets[c]) * (long long)bc.m[c];
        int rank = 0;
        for (int d = 0; d < bc.batch; ++d) {
            const long long cd = (long long)(bc.offsets[d + 1] - bc.offsets[d]) * (long long)bc.m[d];
            rank += (cd > cc) || (cd == cc && d < c);
        }
        order[rank] = c;
    }
}

hipError_t launch_build_batch(const IndexView &v, const float *xyz, hipStream_t s)
{
    const int n = v.n, B = v.bc.batch;
    k_batch_reset<<<32, kBlock, 0, s>>>(v.hdr, v.bc, v.cl_bb, v.bstate, v.board);
    k_batch_setup<<<1, kBlock, 0, s>>>(v.hdr, v.bc, n, v.cl_nvox, v.cl_base);
    k_bbox_batch<<<std::min(blocks_for(n, kBboxRun * kWavesPerBlock), 1024), kBlock, 0, s>>>(xyz, n, v.bc, v.cl_bb,
                                                                                          v.hdr);
    k_grid_batch<<<blocks_for(B, kBlock), kBlock, 0, s>>>(v.hdr, v.bc, v.cl_bb, v.cl_nvox, v.cl_pmin, v.cl_L);
    k_voxel_key_batch<<<blocks_for(n, kBlock), kBlock, 0, s>>>(xyz, n, v.bc, v.cl_nvox, v.cl_base, v.cl_pmin,
                                                               v.cl_L, v.cl_bb, v.keyA, v.valA);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int nblk = blocks_for(n, kRadixTile);
    uint32_t *kin = v.keyA, *vin = v.valA, *kout = v.keyB, *vout = v.valB;
    for (int pass = 0; pass < v.radix_passes; ++pass) {
        k_radix_hist<<<nblk, kBlock, 0, s>>>(kin, n, 8 * pass, v.hist, nblk);
        e = launch_scan(v.hist, v.hist, 256 * nblk, v.partials, nullptr, s);
        if (e != hipSuccess)
            return e;
        k_radix_scatter<<<nblk, kBlock, 0, s>>>(kin, vin, kout, vout, n, 8 * pass, v.hist, nblk);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    k_gather<<<blocks_for(n, kBlock), kBlock, 0, s>>>(xyz, v.orig, n, v.xs, v.ys, v.zs, v.inv);
    k_heads<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.skey, n, v.flags);
    e = launch_scan(v.flags, v.hscan, n, v.partials, &v.hdr->n_voxels, s);
    if (e != hipSuccess)
        return e;
    k_voxels<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.flags, v.hscan, n, v.vstart);
    k_tile_count<<<blocks_for(n, kBlock), kBlock, 0, s>>>(v.vstart, v.hdr, n, v.tile, v.tcount);
    e = launch_scan(v.tcount, v.tbase, n, v.partials, &v.hdr->n_tiles, s);
    if (e != hipSuccess)
        return e;
    k_tiles<<<std::min(blocks_for(n, kWavesPerBlock), 2048), kBlock, 0, s>>>(
        v.vstart, v.tbase, v.hdr, v.tile, v.xs, v.ys, v.zs, v.tstart, v.tcnt, v.tcx, v.tcy, v.tcz, v.trad);
    k_tile_first<<<std::min(blocks_for(n, kBlock), 1024), kBlock, 0, s>>>(v.tstart, v.orig, v.hdr, v.bc,
                                                                          v.tile_first);
    k_batch_order<<<1, kBlock, 0, s>>>(v.bc, v.order);
    return hipGetLastError();
}

}  // namespace rfps
