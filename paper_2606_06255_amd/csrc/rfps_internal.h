// Internal declarations shared by the host API and the kernels of librfps.
// Device helpers: the FP32 squared distance, the packed selection key, wave
// reductions, and the epoch-tagged exchange board of the persistent kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rfps.h"

// The distance must be evaluated as written: no FMA contraction anywhere.
#pragma clang fp contract(off)

namespace rfps {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per workgroup of the persistent kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxGroups = 256;      // one exchange slot per thread of a workgroup
constexpr int kSlotWords = 5;        // d2, ~orig, x, y, z, each tagged with the epoch
constexpr int kMaxNVox = 1024;
constexpr int kMaxPoints = 1 << 26;
constexpr int kRadixItems = 8;       // keys per thread per radix tile
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kScanItems = 16;       // elements per thread of the scan kernels
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kTraceCap = 1 << 17;   // iterations recorded by RFPS_F_TRACE

// Status words live in the index header.  The build status is sticky for the
// index; the sample status is cleared at the start of every sampling call.
struct IndexHeader {
    uint32_t build_status;
    uint32_t sample_status;
    uint32_t n_voxels;   // K, active voxels
    uint32_t n_tiles;    // tiles
    uint32_t bb[6];      // order-preserving encodings of min xyz, max xyz
    uint32_t last_m;     // m of the last sampling call
    uint32_t pad;
    double pmin[3];
    double L;            // voxel edge (eq. voxel_size)
    unsigned long long tele[8];  // rfps_telemetry, in its field order
};

// Device pointers into an index workspace (see layout_index in rfps_api.hip).
struct IndexView {
    IndexHeader *hdr;
    uint32_t *keyA, *keyB, *valA, *valB;  // radix ping-pong buffers
    uint32_t *skey, *orig;                // sorted voxel ids / original indices (alias A or B)
    float *xs, *ys, *zs;                  // sorted coordinates (structure of arrays)
    uint32_t *inv;                        // inv[orig] = sorted position
    uint32_t *flags, *hscan;              // voxel head flags and their exclusive scan
    uint32_t *vstart;                     // [K+1] voxel starts in sorted order
    uint32_t *tcount, *tbase;             // tiles per voxel and its exclusive scan
    uint32_t *tstart, *tcnt;              // tile start (sorted position) and size
    float *tcx, *tcy, *tcz, *trad;        // tile sphere centre and radius (rounded up)
    uint32_t *partials;                   // scan partial sums
    uint32_t *hist;                       // radix histograms [256][blocks]
    unsigned long long *board;            // exchange board [2][kMaxGroups][kSlotWords]
    unsigned long long *trace;            // [kTraceCap][2]
    int32_t n, n_vox, tile, radix_passes;
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// FP32 squared distance ((dx*dx + dy*dy) + dz*dz), dx = fl(p_x - s_x).
__device__ __forceinline__ float sqdist(float px, float py, float pz, float sx, float sy, float sz)
{
    float dx = px - sx;
    float dy = py - sy;
    float dz = pz - sz;
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

// Selection key: larger distance first, then the smaller original index.
// For non-negative floats (including +inf) the bit pattern orders like the
// value, so one unsigned 64-bit max realises the tie-break of Sec. 3.1.
__device__ __forceinline__ unsigned long long pack_key(float d2, uint32_t orig)
{
    return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned long long)(~orig);
}
__device__ __forceinline__ float key_d2(unsigned long long k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_orig(unsigned long long k) { return ~(uint32_t)k; }

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = umax64(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ float wave_min_f32(float v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = fminf(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ float wave_max_f32(float v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ double wave_max_f64(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Order-preserving map of a finite float to uint32 (for atomic min / max).
__device__ __forceinline__ uint32_t f2ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Agent-scope relaxed atomics: coherent across the XCDs of the device
// without cache write-back or invalidate fences.
__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p)
{
    return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void set_status(uint32_t *word, uint32_t code)
{
    uint32_t zero = 0;
    __hip_atomic_compare_exchange_strong(word, &zero, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Exchange board of the persistent kernels.
//
// Every workgroup owns one slot per parity; a slot is kSlotWords 64-bit words
// whose high halves carry the epoch (the selection number j) and whose low
// halves carry the candidate: d2 bits, ~orig, x, y, z.  Each word is written
// and read with single-copy-atomic 64-bit agent-scope operations, so a reader
// that sees the current epoch in all five words holds a consistent candidate.
// Two parities suffice: a workgroup can only write selection j+2 after every
// workgroup has published j+1, i.e. after everyone finished reading j.
// ---------------------------------------------------------------------------
constexpr uint32_t kAbortEpoch = 0xffffffffu;
constexpr uint32_t kSpinLimit = 1u << 22;

struct Candidate {
    unsigned long long key;
    float x, y, z;
};

__device__ __forceinline__ unsigned long long *slot_ptr(unsigned long long *board, int G, uint32_t epoch, int g)
{
    return board + ((size_t)(epoch & 1u) * G + g) * kSlotWords;
}

__device__ __forceinline__ void publish(unsigned long long *slot, uint32_t epoch, const Candidate &c)
{
    const unsigned long long e = (unsigned long long)epoch << 32;
    st_agent(slot + 0, e | (c.key >> 32));
    st_agent(slot + 1, e | (c.key & 0xffffffffull));
    st_agent(slot + 2, e | __float_as_uint(c.x));
    st_agent(slot + 3, e | __float_as_uint(c.y));
    st_agent(slot + 4, e | __float_as_uint(c.z));
}

// Polls one slot until all words carry `epoch`.  Returns false on the abort
// epoch or when the spin budget runs out.
__device__ __forceinline__ bool poll_slot(const unsigned long long *slot, uint32_t epoch, Candidate &c)
{
    for (uint32_t spin = 0; spin < kSpinLimit; ++spin) {
        unsigned long long w0 = ld_agent(slot + 0), w1 = ld_agent(slot + 1), w2 = ld_agent(slot + 2),
                           w3 = ld_agent(slot + 3), w4 = ld_agent(slot + 4);
        uint32_t e0 = (uint32_t)(w0 >> 32);
        if (e0 == kAbortEpoch || (uint32_t)(w1 >> 32) == kAbortEpoch)
            return false;
        if (e0 == epoch && (uint32_t)(w1 >> 32) == epoch && (uint32_t)(w2 >> 32) == epoch &&
            (uint32_t)(w3 >> 32) == epoch && (uint32_t)(w4 >> 32) == epoch) {
            c.key = ((w0 & 0xffffffffull) << 32) | (w1 & 0xffffffffull);
            c.x = __uint_as_float((uint32_t)w2);
            c.y = __uint_as_float((uint32_t)w3);
            c.z = __uint_as_float((uint32_t)w4);
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ void publish_abort(unsigned long long *board, int G, int g)
{
    for (int par = 0; par < 2; ++par)
        for (int w = 0; w < kSlotWords; ++w)
            st_agent(board + ((size_t)par * G + g) * kSlotWords + w, (unsigned long long)kAbortEpoch << 32);
}

// ---------------------------------------------------------------------------
// Host-side launchers (each defined next to its kernels).  All enqueue on
// `s` and return the first launch error.
// ---------------------------------------------------------------------------
hipError_t launch_build_index(const IndexView &v, const float *xyz, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, uint32_t *out, int n, uint32_t *partials, uint32_t *total,
                       hipStream_t s);

struct SampleLaunch {
    int G;
    uint32_t flags;
    uint32_t lds_budget;  // dynamic LDS bytes per workgroup
};
// Static LDS of the sampler kernel (bytes).
size_t rfps_sampler_static_lds();
hipError_t launch_rfps_sample(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s);

struct PlainLaunch {
    int variant;  // 0 persistent registers, 1 one workgroup
    int G, ppt;
};
hipError_t launch_fps_plain(const float *xyz, int n, int m, int start, const PlainLaunch &L, uint32_t *status,
                            unsigned long long *board, float *dist, int32_t *out_idx, float *out_d2,
                            hipStream_t s);

}  // namespace rfps
