// Plain FPS comparison kernels (no index, no pruning), Algorithm 1.
//
// k_fps_regs<PPT>:  persistent; workgroup g keeps points
//   [g*kBlock*PPT, (g+1)*kBlock*PPT) and their distances in registers and
//   exchanges one candidate per selection through the same epoch-tagged
//   board as the RadiusFPS-G sampler.
// k_fps_1wg:  one workgroup of 1024 threads streams the whole cloud and the
//   distance array from device memory every selection; the conventional GPU
//   FPS kernel.
#include <algorithm>

#include "rfps_internal.h"

namespace rfps {

struct PlainArgs {
    const float *xyz;
    uint32_t *status;
    unsigned long long *board;
    float *dist;  // variant 1 only
    int32_t *out_idx;
    float *out_d2;
    int32_t n, m, start, G;
};

__global__ void k_plain_reset(PlainArgs a)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        *a.status = 0;
        a.out_idx[0] = a.start;
        if (a.out_d2)
            a.out_d2[0] = INFINITY;
    }
    if (a.board)
        for (int w = tid; w < 2 * a.G * kSlotStride; w += gridDim.x * blockDim.x)
            a.board[w] = 0ull;
}

// Non-finite coordinates are an error for the plain kernels as well.
__global__ __launch_bounds__(kBlock) void k_plain_check(PlainArgs a)
{
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * a.n; i += gridDim.x * blockDim.x)
        bad |= !isfinite(a.xyz[i]);
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0)
        set_status(a.status, RFPS_ERR_NONFINITE);
}

__global__ __launch_bounds__(kBlock) void k_plain_finalize(PlainArgs a)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.m || *a.status == 0)
        return;
    a.out_idx[j] = -1;
    if (a.out_d2)
        a.out_d2[j] = __uint_as_float(0x7fc00000u);
}

template <int PPT>
__global__ __launch_bounds__(kBlock) void k_fps_regs(PlainArgs a)
{
    __shared__ unsigned long long s_red[kWavesPerBlock];
    __shared__ unsigned long long s_red2[kWavesPerBlock];
    __shared__ float s_c[3];
    __shared__ float s_s[3];
    __shared__ uint32_t s_abort, s_status;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int g = blockIdx.x, G = a.G;
    if (tid == 0) {
        s_status = *a.status;
        s_abort = 0;
    }
    __syncthreads();
    if (s_status)
        return;
    const int base = g * kBlock * PPT + tid;
    float px[PPT], py[PPT], pz[PPT], pd[PPT];
    float sx = a.xyz[3 * (size_t)a.start], sy = a.xyz[3 * (size_t)a.start + 1],
          sz = a.xyz[3 * (size_t)a.start + 2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = base + k * kBlock;
        if (i < a.n) {
            px[k] = a.xyz[3 * (size_t)i];
            py[k] = a.xyz[3 * (size_t)i + 1];
            pz[k] = a.xyz[3 * (size_t)i + 2];
            pd[k] = INFINITY;
        } else {
            px[k] = py[k] = pz[k] = 0.0f;
            pd[k] = -1.0f;  // never a candidate
        }
    }
    for (int j = 1; j < a.m; ++j) {
        // update with the last sample (s_0 at j = 1, as in Algorithm 1) and
        // take this thread's best key
        unsigned long long loc = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const float t = sqdist(px[k], py[k], pz[k], sx, sy, sz);
            if (t < pd[k])
                pd[k] = t;
            if (pd[k] >= 0.0f)
                loc = umax64(loc, pack_key(pd[k], (uint32_t)(base + k * kBlock)));
        }
        const unsigned long long wl = wave_max_u64(loc);
        if (lane == 0)
            s_red[wave] = wl;
        __syncthreads();
        unsigned long long wgk = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q)
            wgk = umax64(wgk, s_red[q]);
        if (loc == wgk && wgk != 0) {
            const uint32_t o = key_orig(wgk);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if ((uint32_t)(base + k * kBlock) == o) {
                    s_c[0] = px[k];
                    s_c[1] = py[k];
                    s_c[2] = pz[k];
                }
            }
        }
        __syncthreads();
        const uint32_t epoch = (uint32_t)j;
        if (tid == 0) {
            Candidate c;
            c.key = wgk;
            c.x = wgk ? s_c[0] : 0.0f;
            c.y = wgk ? s_c[1] : 0.0f;
            c.z = wgk ? s_c[2] : 0.0f;
            publish(slot_ptr(a.board, G, epoch, g), epoch, c);
        }
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
                set_status(a.status, RFPS_ERR_TIMEOUT);
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
        if (g == 0 && tid == 0) {
            a.out_idx[j] = (int32_t)key_orig(win);
            if (a.out_d2)
                a.out_d2[j] = key_d2(win);
        }
    }
}

template __global__ void k_fps_regs<1>(PlainArgs);
template __global__ void k_fps_regs<2>(PlainArgs);
template __global__ void k_fps_regs<4>(PlainArgs);
template __global__ void k_fps_regs<8>(PlainArgs);
template __global__ void k_fps_regs<16>(PlainArgs);
template __global__ void k_fps_regs<32>(PlainArgs);

constexpr int k1wgThreads = 1024;

__global__ __launch_bounds__(k1wgThreads) void k_fps_1wg(PlainArgs a)
{
    __shared__ unsigned long long s_red[k1wgThreads / kWave];
    __shared__ float s_s[3];
    __shared__ uint32_t s_status;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0)
        s_status = *a.status;
    __syncthreads();
    if (s_status)
        return;
    const int n = a.n;
    for (int i = tid; i < n; i += k1wgThreads)
        a.dist[i] = INFINITY;
    float sx = a.xyz[3 * (size_t)a.start], sy = a.xyz[3 * (size_t)a.start + 1],
          sz = a.xyz[3 * (size_t)a.start + 2];
    for (int j = 1; j < a.m; ++j) {
        unsigned long long loc = 0;
        for (int i = tid; i < n; i += k1wgThreads) {
            const float t = sqdist(a.xyz[3 * (size_t)i], a.xyz[3 * (size_t)i + 1], a.xyz[3 * (size_t)i + 2], sx,
                                   sy, sz);
            float d = a.dist[i];
            if (t < d) {
                d = t;
                a.dist[i] = t;
            }
            loc = umax64(loc, pack_key(d, (uint32_t)i));
        }
        loc = wave_max_u64(loc);
        if (lane == 0)
            s_red[wave] = loc;
        __syncthreads();
        if (tid == 0) {
            unsigned long long win = 0;
            for (int q = 0; q < k1wgThreads / kWave; ++q)
                win = umax64(win, s_red[q]);
            const uint32_t o = key_orig(win);
            a.out_idx[j] = (int32_t)o;
            if (a.out_d2)
                a.out_d2[j] = key_d2(win);
            s_s[0] = a.xyz[3 * (size_t)o];
            s_s[1] = a.xyz[3 * (size_t)o + 1];
            s_s[2] = a.xyz[3 * (size_t)o + 2];
        }
        __syncthreads();
        sx = s_s[0];
        sy = s_s[1];
        sz = s_s[2];
    }
}

}  // namespace rfps

namespace rfps {

hipError_t launch_fps_plain(const float *xyz, int n, int m, int start, const PlainLaunch &L, uint32_t *status,
                            unsigned long long *board, float *dist, int32_t *out_idx, float *out_d2,
                            hipStream_t s)
{
    PlainArgs a;
    a.xyz = xyz;
    a.status = status;
    a.board = L.variant == 0 ? board : nullptr;
    a.dist = dist;
    a.out_idx = out_idx;
    a.out_d2 = out_d2;
    a.n = n;
    a.m = m;
    a.start = start;
    a.G = L.G;
    k_plain_reset<<<4, kBlock, 0, s>>>(a);
    k_plain_check<<<std::min((3 * n + kBlock - 1) / kBlock, 1024), kBlock, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (m > 1) {
        if (L.variant == 1) {
            k_fps_1wg<<<1, k1wgThreads, 0, s>>>(a);
        } else {
            const void *fn = nullptr;
            switch (L.ppt) {
            case 1: fn = reinterpret_cast<const void *>(k_fps_regs<1>); break;
            case 2: fn = reinterpret_cast<const void *>(k_fps_regs<2>); break;
            case 4: fn = reinterpret_cast<const void *>(k_fps_regs<4>); break;
            case 8: fn = reinterpret_cast<const void *>(k_fps_regs<8>); break;
            case 16: fn = reinterpret_cast<const void *>(k_fps_regs<16>); break;
            case 32: fn = reinterpret_cast<const void *>(k_fps_regs<32>); break;
            default: return hipErrorInvalidValue;
            }
            void *args[] = {&a};
            e = launch_persistent(fn, L.G, args, 0, s);
            if (e != hipSuccess)
                return e;
        }
    }
    k_plain_finalize<<<(m + kBlock - 1) / kBlock, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace rfps
