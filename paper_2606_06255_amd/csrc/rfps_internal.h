// Internal declarations shared by the host API and the kernels of librfps.
// Device helpers: the FP32 squared distance, the packed selection key, wave
// reductions, and the epoch-tagged exchange board of the persistent kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rfps.h"
#include "prune_bound.h"

// The distance must be evaluated as written: no FMA contraction anywhere.
#pragma clang fp contract(off)

namespace rfps {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per workgroup of the persistent kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxGroups = 256;      // one exchange slot per thread of a workgroup
constexpr int kSlotWords = 5;        // d2, ~orig, x, y, z, each tagged with the epoch
constexpr int kMaxSlotWords = 64;    // largest slot of any exchange protocol (words)
// Exchange board: a single cloud uses 2 * G slots; a batch gives every team
// of T workgroups 2 * T slots plus a control slot, (256 / T) * (2T + 1) slots
// in all, at most 576 for T >= 4.
constexpr int kBoardWords = 640 * kMaxSlotWords;
constexpr int kMaxNVox = 1024;
constexpr int kMaxShells = 64;       // range shells of one cloud (the last one is open-ended)
constexpr int kMaxPoints = 1 << 26;
constexpr int kRadixItems = 8;       // keys per thread per radix tile
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kScanItems = 16;       // elements per thread of the scan kernels
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kTraceCap = 1 << 17;   // iterations recorded by RFPS_F_TRACE
constexpr int kTeleFields = 32;
// telemetry slots (rfps_telemetry field order)
constexpr int kTeleExchanges = 8;
constexpr int kTeleTicksLookahead = 9;
constexpr int kTeleTicksExchange = 10;
constexpr int kTeleTicksMerge = 11;
constexpr int kTeleTicksApply = 12;
constexpr int kTeleTickHz = 13;
constexpr int kTeleTicksWait = 14;
constexpr int kTeleSub = 16;        // eight finer clocks of the rounds (see rfps_telemetry)
constexpr int kTeleMergeStats = 24; // listed-above, listed, failures summed over rounds

// Status words live in the index header.  The build status is sticky for the
// index; the sample status is cleared at the start of every sampling call.
struct IndexHeader {
    uint32_t build_status;
    uint32_t sample_status;
    uint32_t n_voxels;   // K, active voxels
    uint32_t n_tiles;    // tiles
    uint32_t bb[6];      // order-preserving encodings of min xyz, max xyz
    uint32_t last_m;     // m of the last sampling call
    uint32_t trace_n;    // entries the last traced call recorded
    double pmin[3];
    double L;            // voxel edge (eq. voxel_size)
    double origin[3];    // centre of the range shells (bounding-box centre)
    double shell_inv;    // 1 / shell spacing, 0 without shells
    uint32_t shell_cap;  // shells in use (the last one is open-ended); 1 without shells
    uint32_t pad_;
    unsigned long long tele[kTeleFields];  // rfps_telemetry, in its field order
};

constexpr int kMaxXcds = 8;      // XCDs of an MI355X; batched teams never span two
constexpr int kMaxBatch = 4096;  // clouds per batched call

// Batch description, passed by value to the kernels.
struct BatchCtl {
    int32_t batch;
    int32_t team_size;       // T, workgroups sampling one cloud (divides per_xcd)
    int32_t per_xcd;         // workgroups the launch places on every XCD
    int32_t fixed_n_vox;     // 0: per-cloud default rule
    double shell_inv;        // 1 / shell spacing, 0 without shells
    int32_t m_total;         // sum of m over the batch (length of the outputs)
    const int32_t *offsets;  // [batch+1] first point of every cloud (caller's device array)
    const int32_t *m;        // [batch] selections per cloud (caller's device array)
    const int32_t *starts;   // [batch] local start indices, or nullptr (all 0)
    uint32_t *out_offsets;   // [batch+1] first output of every cloud (workspace, prefix sum of m)
};

// Per-call device state of a batch (in the workspace, cleared before every call).
struct BatchState {
    uint32_t joined, next;
    uint32_t xcd_count[kMaxXcds];
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
    unsigned long long *board;            // exchange board, kBoardWords words
    unsigned long long *trace;            // [kTraceCap][2]
    int32_t n, n_vox, tile, radix_passes;
    double shell_inv;     // 1 / shell spacing, 0 without shells
    uint32_t shell_cap;   // shells of the grid (1 without shells)
    // batched index only (batch > 0)
    int32_t batch;
    BatchCtl bc;
    double *cl_pmin, *cl_L;               // [batch][3], [batch] grid of every cloud
    uint32_t *cl_bb;                      // [batch][6] order-preserving bounding boxes
    uint32_t *cl_nvox, *cl_base;          // [batch] bins per axis, [batch+1] first key of every cloud
    uint32_t *tile_first;                 // [batch+1] first tile of every cloud
    int32_t *order;                       // [batch] clouds by decreasing cost
    BatchState *bstate;
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

// Correctly rounded FP32 square root of x in [0, +inf] (NaN passes through).
// The FP64 root rounded to FP32 is within one unit of the answer; it is then
// checked against the rounding boundaries on either side, the midpoints
// between r and its FP32 neighbours.  A midpoint has at most 25 significant
// bits, so its FP64 square is exact and never an FP32 value: the comparisons
// decide the rounding exactly and a tie cannot occur.
__device__ __forceinline__ float sqrt_rn(float x)
{
    if (!(x > 0.0f) || x == INFINITY)
        return x;
    float r = (float)sqrt((double)x);
    const double xd = (double)x;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t rb = __float_as_uint(r);
        const double up = 0.5 * ((double)r + (double)__uint_as_float(rb + 1u));
        const double dn = 0.5 * ((double)r + (double)__uint_as_float(rb - 1u));
        if (xd > up * up)
            r = __uint_as_float(rb + 1u);
        else if (xd < dn * dn)
            r = __uint_as_float(rb - 1u);
    }
    return r;
}

// Euclidean mode (RFPS_F_SQRT).  Sec. 3.4.3 (eq. point_distance_update)
// states the distance update with the Euclidean norm; its FP32 value is the rounded root of d2.  The state
// keeps squared values: every new d2 is replaced by the top of its class,
// the largest FP32 value whose rounded root equals that of d2.  This map is
// non-decreasing and idempotent, and two values share a class exactly when
// their rounded roots are equal, so min, the strict update and the arg max
// (lowest index among equals) over class tops follow FPS on rounded
// Euclidean distances step for step.  A class top is >= d2, so each pruning
// and point-skip test, which shows the fresh d2 cannot fall below the state,
// shows the same for its class top.  The reported distance is the rounded
// root of the state.
__device__ __forceinline__ float sqrt_class_top(float x)
{
    if (!(x > 0.0f) || x == INFINITY)
        return x;
    const float r = sqrt_rn(x);
    // the class is [.., b) with b = (midpoint of r and its upper neighbour)^2,
    // exact in FP64 and not an FP32 value
    const double up = 0.5 * ((double)r + (double)__uint_as_float(__float_as_uint(r) + 1u));
    const double b = up * up;
    if (b > 3.4028234663852886e38)
        return 3.4028234663852886e38f;
    float y = (float)b;
    if ((double)y > b)
        y = __uint_as_float(__float_as_uint(y) - 1u);
    return y;
}

// min(t, the state value of a fresh squared distance d2): the class top in
// Euclidean mode (only needed when d2 < t, since the top is >= d2).
__device__ __forceinline__ float min_dist(float t, float d2, bool euclid)
{
    if (euclid && d2 < t)
        d2 = sqrt_class_top(d2);
    return fminf(t, d2);
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

// Wave64 reductions on DPP lane permutes (no LDS round trip): quad swaps,
// half-row and row mirrors combine each 16-lane row, then the row_bcast15 /
// row_bcast31 broadcasts of GFX9 fold rows 0-1 into 2-3, leaving the result
// in lane 63.  They must be called with all 64 lanes active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xf, false);
}
constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

// Lane mask of the lanes where b holds.  A ballot of a single comparison
// takes the comparison's lane mask as it is, and so do masks combined with &;
// a ballot of a compound condition first turns it into a value per lane.
__device__ __forceinline__ unsigned long long ballot64(bool b) { return __builtin_amdgcn_ballot_w64(b); }

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, dpp_u32<kDppQuadSwap1>(v, v));
    v = max(v, dpp_u32<kDppQuadSwap2>(v, v));
    v = max(v, dpp_u32<kDppHalfMirror>(v, v));
    v = max(v, dpp_u32<kDppRowMirror>(v, v));
    v = max(v, dpp_u32<kDppBcast15, 0xa>(v, v));
    v = max(v, dpp_u32<kDppBcast31, 0xc>(v, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    v = min(v, dpp_u32<kDppQuadSwap1>(v, v));
    v = min(v, dpp_u32<kDppQuadSwap2>(v, v));
    v = min(v, dpp_u32<kDppHalfMirror>(v, v));
    v = min(v, dpp_u32<kDppRowMirror>(v, v));
    v = min(v, dpp_u32<kDppBcast15, 0xa>(v, v));
    v = min(v, dpp_u32<kDppBcast31, 0xc>(v, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Largest 64-bit key of the wave: the largest high half first, then the
// largest low half among the lanes that hold it.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    const uint32_t hi = (uint32_t)(v >> 32);
    const uint32_t mhi = wave_max_u32(hi);
    const unsigned long long tie = ballot64(hi == mhi);
    if (__popcll(tie) == 1)  // one lane holds the largest high half: its low half goes with it
        return ((unsigned long long)mhi << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, __ffsll((long long)tie) - 1);
    const uint32_t mlo = wave_max_u32(hi == mhi ? (uint32_t)v : 0u);
    return ((unsigned long long)mhi << 32) | mlo;
}

// Minimum of non-negative floats (distances, +inf allowed): their bit
// patterns order like the values.
__device__ __forceinline__ float wave_min_dist(float v)
{
    return __uint_as_float(wave_min_u32(__float_as_uint(v)));
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

// The pruning threshold of a tile, prune_threshold(R, dv), is defined in
// prune_bound.h, which the CPU sampler shares.

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

// Slots are padded to one 64-byte line so that workgroups polling different
// slots never contend for the same line.
constexpr int kSlotStride = 8;

__device__ __forceinline__ unsigned long long *slot_ptr(unsigned long long *board, int G, uint32_t epoch, int g)
{
    return board + ((size_t)(epoch & 1u) * G + g) * kSlotStride;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Reads the five words of a slot with three agent-scope (sc1) vector loads
// in flight at once; each aligned 64-bit word is read atomically.
__device__ __forceinline__ void load_slot_agent(const unsigned long long *p, u32x4 &a, u32x4 &b, u32x2 &c)
{
    asm volatile(
        "global_load_dwordx4 %0, %3, off sc1\n\t"
        "global_load_dwordx4 %1, %3, off offset:16 sc1\n\t"
        "global_load_dwordx2 %2, %3, off offset:32 sc1\n\t"
        "s_waitcnt vmcnt(0)"
        : "=&v"(a), "=&v"(b), "=&v"(c)
        : "v"(p)
        : "memory");
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
    // little-endian words: .x = payload (low half), .y = epoch (high half)
    for (uint32_t spin = 0; spin < kSpinLimit; ++spin) {
        u32x4 a, b;
        u32x2 e;
        load_slot_agent(slot, a, b, e);
        if (a.y == kAbortEpoch || a.w == kAbortEpoch)
            return false;
        if (a.y == epoch && a.w == epoch && b.y == epoch && b.w == epoch && e.y == epoch) {
            c.key = ((unsigned long long)a.x << 32) | a.z;
            c.x = __uint_as_float(b.x);
            c.y = __uint_as_float(b.z);
            c.z = __uint_as_float(e.x);
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ void publish_abort(unsigned long long *board, int G, int g)
{
    for (int par = 0; par < 2; ++par)
        for (int w = 0; w < kSlotWords; ++w)
            st_agent(board + ((size_t)par * G + g) * kSlotStride + w, (unsigned long long)kAbortEpoch << 32);
}

// ---------------------------------------------------------------------------
// Host-side launchers (each defined next to its kernels).  All enqueue on
// `s` and return the first launch error.
// ---------------------------------------------------------------------------
hipError_t launch_build_index(const IndexView &v, const float *xyz, hipStream_t s);
hipError_t launch_gather_xyz(const float *xyz, int n, const int32_t *idx, int m, float *out, hipStream_t s);
hipError_t launch_sqrt_out(float *d, int m, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, uint32_t *out, int n, uint32_t *partials, uint32_t *total,
                       hipStream_t s);

struct SampleLaunch {
    int G;
    int R;                // lookahead depth of the multi-pick sampler; 0 = one selection per exchange
    uint32_t flags;
    uint32_t lds_budget;  // dynamic LDS bytes per workgroup
};
// Static LDS of the sampler kernel chosen by R (bytes); 0 if R is not supported.
size_t rfps_sampler_static_lds(int R);
hipError_t launch_rfps_sample(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s);
// The unfused sampler (sample_unfused.hip): two launches per selection.
hipError_t launch_rfps_unfused(const IndexView &v, int m, int start, uint32_t flags, int32_t *out_idx,
                               float *out_d2, hipStream_t s);
// The multi-pick sampler (sample_rounds.hip); called by launch_rfps_sample.
size_t rfps_rounds_static_lds(int R);
hipError_t launch_rfps_rounds(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s);
// Exchange floor probe (sample_rounds.hip): `rounds` bare exchanges of W
// words among G workgroups; out[0] receives the ticks of workgroup 0.
hipError_t launch_exchange_probe(unsigned long long *board, int G, int W, int rounds, unsigned long long *out,
                                 uint32_t *status, hipStream_t s);
// Writes -1 / NaN to all m outputs when the header records an error (sample_rfps.hip).
hipError_t launch_sample_finalize(const IndexHeader *hdr, int m, int32_t *out_idx, float *out_d2, hipStream_t s);

// Launches a persistent kernel of G workgroups of kBlock threads.  Outside
// stream capture this is a cooperative launch, which fails unless all G
// workgroups are resident together.  Under capture (a cooperative launch
// cannot be recorded into a graph) it is an ordinary launch after the same
// residency check from the occupancy calculator; every wait in the
// persistent kernels is bounded, so even a shared device cannot hang them.
inline hipError_t launch_persistent(const void *fn, int G, void **args, size_t lds, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess)
        return e;
    if (cs == hipStreamCaptureStatusNone)
        return hipLaunchCooperativeKernel(fn, dim3(G), dim3(kBlock), args, (unsigned)lds, s);
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
        (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds)) != hipSuccess)
        return e;
    if ((long long)per_cu * cus < G)
        return hipErrorCooperativeLaunchTooLarge;
    return hipLaunchKernel(fn, dim3(G), dim3(kBlock), args, lds, s);
}

// Batched index build (index_build.hip) and batched sampling (sample_rounds.hip).
hipError_t launch_build_batch(const IndexView &v, const float *xyz, hipStream_t s);
hipError_t launch_rfps_rounds_batched(const IndexView &v, const SampleLaunch &L, int32_t *out_idx,
                                      float *out_d2, hipStream_t s);
// Shells a grid of n bins per axis may use: keys s * n^3 + V_id stay below 2^32.
__host__ __device__ inline uint32_t shell_cap_for(uint32_t n, bool shells)
{
    if (!shells)
        return 1u;
    const unsigned long long n3 = (unsigned long long)n * n * n;
    const unsigned long long cap = (1ull << 32) / n3;
    return (uint32_t)(cap < (unsigned long long)kMaxShells ? cap : (unsigned long long)kMaxShells);
}

// Voxel key of a point (Sec. 3.2): V_id = v_z n^2 + v_y n + v_x with
// v_a = clamp(floor((p_a - pmin_a) / L), 0, n - 1), the quotient in FP64.
// With range shells (shell_inv > 0), a point at distance r from `o` lies in
// shell s = min(floor(r / spacing), shell_cap - 1), which uses cubes of edge
// (s + 1) L and ceil(n / (s + 1)) bins per axis from the same corner; its key
// is s * n^3 + V_id on that coarser grid, so shells never share a voxel.
// Any partition of the points into voxels leaves the sampling result
// unchanged (the tile spheres enclose their members whatever the grid).
__device__ __forceinline__ uint32_t voxel_key(float px, float py, float pz, const double *pmin, double L,
                                              uint32_t n, const double *o, double shell_inv, uint32_t shell_cap)
{
    uint32_t s = 0;
    if (shell_inv > 0.0) {
        const double dx = (double)px - o[0], dy = (double)py - o[1], dz = (double)pz - o[2];
        const double r = floor(sqrt(dx * dx + dy * dy + dz * dz) * shell_inv);
        s = r < (double)(shell_cap - 1) ? (uint32_t)r : shell_cap - 1;
    }
    const uint32_t ns = (n + s) / (s + 1);
    const double Ls = L * (double)(s + 1);
    const double top = (double)(ns - 1);
    const float p[3] = {px, py, pz};
    uint32_t v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double q = floor(((double)p[a] - pmin[a]) / Ls);
        q = q > 0.0 ? q : 0.0;  // also maps NaN to 0
        q = q < top ? q : top;
        v[a] = (uint32_t)q;
    }
    return s * n * n * n + (v[2] * ns + v[1]) * ns + v[0];
}

// Per-cloud default voxel bins (same rule on host and device).
__host__ __device__ inline int default_n_vox_rule(int n)
{
    const int cand[11] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    const double target = sqrt((double)(n > 0 ? n : 1) / 40.0);
    int best = cand[0];
    for (int q = 0; q < 11; ++q)
        if (fabs(log((double)cand[q] / target)) < fabs(log((double)best / target)))
            best = cand[q];
    return best;
}

struct PlainLaunch {
    int variant;  // 0 persistent registers, 1 one workgroup
    int G, ppt;
};
hipError_t launch_fps_plain(const float *xyz, int n, int m, int start, const PlainLaunch &L, uint32_t *status,
                            unsigned long long *board, float *dist, int32_t *out_idx, float *out_d2,
                            hipStream_t s);

}  // namespace rfps
