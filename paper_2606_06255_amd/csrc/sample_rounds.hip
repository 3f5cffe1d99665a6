// RadiusFPS-G with certified multi-pick rounds (the default sampler), for a
// single cloud and for batches of clouds.
//
// A cloud is sampled by a team of G workgroups.  Rank r of the team owns the
// cloud's tiles t with (t - first tile) % G == r (tiles of neighbouring voxels
// land on different workgroups, so the unpruned work near a new sample
// spreads over the team) and keeps their points (x, y, z, Dist_p, a private
// lookahead copy of Dist_p, original index) and per-tile state (sphere, packed
// Dist_v key, pruning threshold) in LDS for the whole cloud.  One exchange
// settles a whole round of selections:
//
//   L  lookahead: every workgroup runs R steps of FPS on its own points only
//      (on the private copy, with the same spherical pruning), giving local
//      candidates l_1..l_R with local keys k_1 > .. > k_R, and for every step
//      h the runner-up u_h, the largest local key of the group's other points
//      when l_h was chosen.  The group's bound k_{R+1} = max(u_R, (0, l_R))
//      is at least every local key once l_R is applied too (applying it only
//      lowers the others, and its own distance becomes 0), so that last
//      update is never run;
//   X  exchange: each workgroup publishes its candidates (coordinates, local
//      distance, original index, runner-up distance) and k_{R+1};
//   M  merge: every workgroup replays the same deterministic merge.  Group g
//      keeps a head h_g (how many of its candidates were taken).  Its bound
//      B_g = k_{h_g+1} is an upper bound on the true key of every point of g
//      not taken: the true distances include every pick of the round so far,
//      among them l_1..l_{h_g}, so they are at most the local ones.  Hence the largest
//      true key anywhere is at most max_g B_g, and if the head candidate of
//      the group with the largest bound still has its true key equal to its
//      local key (no other pick of the round lowered it), that candidate is
//      exactly the next FPS selection (the Sec. 3.1 rule; keys are unique).
//      The local distance already includes the group's own earlier picks
//      (those it skipped are at least as far), so the true distance is the
//      local one lowered by the other groups' earlier picks.  When the head
//      l_h of g fails this test, its true key t is known exactly, and the
//      other points of g are bounded by u_h (their local keys at step h
//      assumed only l_1..l_{h-1}, which are picks); the later candidates of g
//      are dropped, l_h is listed again with key t, and the merge goes on
//      under the larger bound.  The merge lists the candidates above the
//      largest bound, finds with all threads of the workgroup their order and,
//      for each, the listed candidates that would lower it, and then walks the
//      order in one wavefront, re-listing at every failure;
//   A  apply: all picks of the round update the true state (spherical test
//      per tile and pick, point skip, strict update, tile-key resync).
//
// Every round certifies at least one selection (at round start the largest
// bound is attained by its own head), so the loop always terminates; the
// output equals plain FPS bit for bit.
//
// Exchange scopes: a team spread over the device exchanges through
// agent-scope atomics (coherent across XCDs); a team whose workgroups all
// sit on one XCD exchanges through that XCD's L2 (plain stores, L1
// invalidate before every poll), which halves the exchange latency.
#include <type_traits>

#include "rfps_internal.h"

namespace rfps {

struct RoundArgs {
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
    // batched mode
    BatchCtl bc;
    BatchState *bstate;
    const uint32_t *tile_first;  // [batch+1]
    const int32_t *order;        // [batch] clouds by decreasing cost
};

// Candidates one merge lists, and so the selections one round may settle
// (the merge stops there; a shorter round is always valid).
constexpr int kList = 2 * kWave;
constexpr int kMaxRoundPicks = kList;
// Words of the order of a cut list (kList + 1, rounded to whole 8-byte words).
constexpr uint32_t kOrdWords = kList + 2;

// Tiles a wavefront tests per pass of the apply phase (their sphere loads are
// in flight together; 8 measured faster than 4 or 16).
constexpr int kApplyTiles = 8;
// Listed candidates a wavefront ranks per pass of the merge's ranking loop.
constexpr int kRankPerPass = 2;


// Value of lane l of v (l uniform).
__device__ __forceinline__ float lane_f32(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
// Failed candidates a round re-lists before it ends (each failure lowers a
// listed key, so the loop ends anyway; this caps the work of one round).
constexpr uint32_t kMaxFailures = 64;

// Entries of the merge's sort buffers: the next power of two of G * R, at
// least 128 (the smallest network the merge runs).
__host__ __device__ __forceinline__ uint32_t sort_cap(uint32_t G, uint32_t R)
{
    uint32_t s = 2 * kWave;
    while (s < G * R)
        s <<= 1;
    return s;
}

// 4-byte words of the region the merge uses first for its sorted keys and
// then for the pick coordinates.
__host__ __device__ __forceinline__ uint32_t merge_words(uint32_t G, uint32_t R)
{
    const uint32_t keys = 2u * sort_cap(G, R), picks = 3u * kMaxRoundPicks;
    return keys > picks ? keys : picks;
}

// Tile spheres a workgroup keeps: its tile count rounded up to whole passes
// of the apply phase (kApplyTiles per wavefront), at least one pass; the
// padding never passes a test.
__host__ __device__ __forceinline__ uint32_t padded_tiles(uint32_t tiles)
{
    constexpr uint32_t q = (uint32_t)(kApplyTiles * kWavesPerBlock);
    return tiles ? (tiles + q - 1) / q * q : q;
}

__host__ __device__ __forceinline__ uint32_t rounds_lds_need(uint32_t tiles, uint32_t pts, uint32_t G, uint32_t R)
{
    return tiles * 40u + padded_tiles(tiles) * 16u + pts * 24u + G * (6u * R + 2u) * 4u + kOrdWords * 4u +
           sort_cap(G, R) * 4u + merge_words(G, R) * 4u + 128u;
}

// Capacity plan of one team of G workgroups over the tiles [tb, te).
__device__ __forceinline__ bool team_fits(const uint32_t *tcnt, uint32_t tb, uint32_t te, int G, int R,
                                          uint32_t budget, int rank)
{
    uint32_t tiles = 0, pts = 0;
    for (uint32_t t = tb + rank; t < te; t += G) {
        ++tiles;
        pts += tcnt[t];
    }
    return pts <= 65535u && rounds_lds_need(tiles, pts, G, R) <= budget;
}

__global__ __launch_bounds__(kBlock) void k_rounds_plan(IndexHeader *hdr, const uint32_t *__restrict__ tcnt,
                                                        int G, int R, uint32_t budget)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G || hdr->build_status)
        return;
    if (!team_fits(tcnt, 0, hdr->n_tiles, G, R, budget, g))
        set_status(&hdr->sample_status, RFPS_ERR_CAPACITY);
}

// One wavefront recomputes the key, best point and threshold of tile lt
// (points ls .. ls + cnt - 1) from each lane's distance d and original index
// o of its point, held in registers (all lanes of the wave must call it).
// The threshold goes to tthr[lt * TS].
template <int TS>
__device__ __forceinline__ void tile_rekey(int lane, uint32_t lt, uint32_t ls, uint32_t cnt, float d, uint32_t o,
                                           const float *trad, unsigned long long *tkey, uint32_t *tbest, float *tthr)
{
    const bool valid = (uint32_t)lane < cnt;
    const unsigned long long key = valid ? pack_key(d, o) : 0ull;
    const unsigned long long kmax = wave_max_u64(key);
    const unsigned long long hit = ballot64(key == kmax) & ballot64(valid);
    if (lane == 0) {
        tkey[lt] = kmax;
        tbest[lt] = ls + (uint32_t)(__ffsll((long long)hit) - 1);
        tthr[lt * TS] = prune_threshold(trad[lt], key_d2(kmax));
    }
}

// ---------------------------------------------------------------------------
// Exchange primitives for the two scopes.
// ---------------------------------------------------------------------------
enum class Scope { Agent, Xcd };

template <Scope S>
__device__ __forceinline__ void bstore(unsigned long long *p, unsigned long long v)
{
    if constexpr (S == Scope::Agent)
        st_agent(p, v);
    else
        *reinterpret_cast<volatile unsigned long long *>(p) = v;  // written through to the XCD's L2
}
template <Scope S>
__device__ __forceinline__ void binvalidate()
{
    if constexpr (S == Scope::Xcd)
        asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
}
template <Scope S>
__device__ __forceinline__ unsigned long long bload(const unsigned long long *p)
{
    if constexpr (S == Scope::Agent)
        return ld_agent(p);
    else
        return *reinterpret_cast<const volatile unsigned long long *>(p);
}

// Scalars every workgroup keeps in LDS (static shared memory of the kernels).
struct RoundShared {
    unsigned long long red[kWavesPerBlock];
    uint32_t scan[kWavesPerBlock];
    unsigned long long red2[kWavesPerBlock];
    uint32_t abort, npick, mcount, pfront, mtotal, msel;
    float4 lq[kList];                   // merge: listed candidates' coordinates and listed distance
    uint32_t lkl[kList];                // merge: low halves of their keys (~ original index)
    // merge: listed candidates with larger keys that would lower each one
    // (positions below 64, and 64 and up)
    unsigned long long lset0[kList], lset1[kList];
    uint32_t lrank[kList];              // merge: rank of each listed candidate in key order
    uint32_t repw[kWavesPerBlock];      // merge: a wavefront's groups repeat a candidate (equal keys)
    uint32_t hist[256];    // merge: candidates per key bucket
    uint32_t my[6 * 8 + 2];  // this workgroup's slot payload (R <= 8)
};

// Per-thread telemetry accumulators.
struct RoundTele {
    unsigned long long tests = 0, pruned = 0, visited = 0, skipped = 0, updated = 0, resync = 0;
    unsigned long long ph[5] = {0, 0, 0, 0, 0};  // lookahead, exchange, merge, apply, exchange wait
    // finer clocks: merge list / rank / walk / picks, lookahead copy / steps,
    // exchange poll / keys; and the merge's list lengths and failures
    unsigned long long sub[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // + apply loop, lookahead selects, apply updates
    unsigned long long apairs = 0, arekeys = 0;  // wavefront 0's apply: tile-pick pairs updated, tiles re-keyed
    unsigned long long above = 0, listed = 0, fails = 0;
    unsigned long long rounds = 0;
};

// What one team samples: tiles [tb, te) of the index, whose original indices
// start at point_base (subtracted from the output), m selections from the
// local start index, outputs at out_idx / out_d2 (already offset).
struct CloudJob {
    uint32_t tb, te, point_base;
    int32_t m, start;
    int32_t *out_idx;
    float *out_d2;
};

// Samples one cloud.  Every thread of every workgroup of the team calls it.
// `epoch` is the team's exchange counter: it only grows, so slots never need
// clearing between clouds.  Returns false when an exchange failed (abort).
template <int R, Scope S, bool E, bool T>
__device__ bool sample_cloud(const RoundArgs &a, const CloudJob &job, int rank, int G, unsigned long long *board,
                             uint32_t &epoch, unsigned char *smem, RoundShared &sh, RoundTele &tl,
                             bool record_trace, bool clocks)
{
    constexpr int W = 6 * R + 2;  // words per slot
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    // the wavefront index is uniform: as a scalar it keeps wave-strided loops
    // and their addressing off the exec mask
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const uint32_t span = job.te - job.tb;
    const int ntl = (span > (uint32_t)rank) ? (int)((span - 1 - rank) / G) + 1 : 0;
    const bool use_skip = !(a.flags & RFPS_F_NO_POINT_SKIP);
    constexpr bool euclid = E;  // Euclidean distances (RFPS_F_SQRT), a separate instantiation
    // counters, phase clocks and the exchange trace exist only in the
    // instrumented instantiation (T): the default kernels carry none of
    // their code
    const bool tele = T && (a.flags & RFPS_F_TELEMETRY) != 0;
    const bool trace = T && record_trace && tid == 0;
    clocks = T && clocks;

    // ---- LDS layout (the plan checked that it fits) ----
    unsigned long long *tkey = reinterpret_cast<unsigned long long *>(smem);
    unsigned long long *tkeyl = tkey + ntl;
    unsigned long long *obuf = tkeyl + ntl;  // order of a cut list
    // merge: the keys in sort order, then (same memory) the pick coordinates
    unsigned long long *skey = obuf + kOrdWords / 2;
    float *pkx = reinterpret_cast<float *>(skey);
    float *pky = pkx + kMaxRoundPicks;
    float *pkz = pky + kMaxRoundPicks;
    // tile spheres with their pruning thresholds: (centre, threshold), one
    // 16-byte load per tile test
    // (aligned by offset from the LDS base, so that the compiler still sees
    // an LDS pointer)
    const size_t tsph_off =
        ((size_t)(reinterpret_cast<unsigned char *>(reinterpret_cast<float *>(skey) + merge_words(G, R)) - smem) + 15) &
        ~(size_t)15;
    float4 *tsph = reinterpret_cast<float4 *>(smem + tsph_off);
    float *tthr = reinterpret_cast<float *>(tsph) + 3;  // with stride 4
    const int ntlp = (int)padded_tiles((uint32_t)ntl);
    float *trad = reinterpret_cast<float *>(tsph + ntlp);
    float *tthrl = trad + ntl;
    uint32_t *tmeta = reinterpret_cast<uint32_t *>(tthrl + ntl);
    uint32_t *tbest = tmeta + ntl;
    uint32_t *tbestl = tbest + ntl;
    uint32_t *tflag = tbestl + ntl;
    // the round's slots as published, one W-word image per group: candidate
    // s of group g is x, y, z, local d2, original index and runner-up d2 at
    // words 6 s .. 6 s + 5, the bound key's high and low halves follow
    uint32_t *simg = reinterpret_cast<uint32_t *>(tflag + ntl);
    // field f of candidate c = g * R + s
    auto cword = [&](uint32_t c, int f) -> uint32_t { return simg[(c / R) * W + 6 * (c % R) + f]; };
    uint32_t *sidx = simg + G * W;  // merge order; its first P entries are the round's picks
    float *px = reinterpret_cast<float *>(sidx + sort_cap(G, R));

    // ---- prologue: tile metadata and LDS offsets (block prefix sum) ----
    const int per = (ntl + kBlock - 1) / kBlock;
    const int l0 = tid * per, l1 = min(l0 + per, ntl);
    uint32_t cnt_sum = 0;
    for (int lt = l0; lt < l1; ++lt)
        cnt_sum += a.tcnt[job.tb + rank + (size_t)lt * G];
    uint32_t incl = cnt_sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t o = __shfl_up(incl, off, kWave);
        if (lane >= off)
            incl += o;
    }
    if (lane == kWave - 1)
        sh.scan[wave] = incl;
    __syncthreads();
    uint32_t off = incl - cnt_sum, npl = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) {
        off += q < wave ? sh.scan[q] : 0u;
        npl += sh.scan[q];
    }
    for (int lt = l0; lt < l1; ++lt) {
        const size_t t = job.tb + rank + (size_t)lt * G;
        const uint32_t c = a.tcnt[t];
        tmeta[lt] = off | (c << 16);
        tsph[lt] = make_float4(a.tcx[t], a.tcy[t], a.tcz[t], 0.0f);
        trad[lt] = a.trad[t];
        off += c;
    }
    // padding spheres: no squared distance is below a threshold of -inf
    for (int lt = ntl + tid; lt < ntlp; lt += kBlock)
        tsph[lt] = make_float4(0.0f, 0.0f, 0.0f, -INFINITY);
    float *py = px + npl;
    float *pz = py + npl;
    float *pd = pz + npl;
    float *pdl = pd + npl;
    uint32_t *po = reinterpret_cast<uint32_t *>(pdl + npl);
    // the carving must end inside the dynamic LDS the plan sized
    if (reinterpret_cast<unsigned char *>(po + npl) - smem > (ptrdiff_t)a.lds_budget) {
        if (tid == 0) {
            set_status(&a.hdr->sample_status, RFPS_ERR_INTERNAL);
            // the rest of the team must not wait for this workgroup
            for (int par = 0; par < 2; ++par)
                for (int w = 0; w < W; ++w)
                    bstore<S>(board + ((size_t)par * G + rank) * kMaxSlotWords + w,
                              (unsigned long long)kAbortEpoch << 32);
        }
        return false;
    }

    // Seed and initial update (Sec. 3.3)
    {
        const uint32_t p0 = a.inv[job.point_base + (uint32_t)job.start];
        const float sx = a.xs[p0], sy = a.ys[p0], sz = a.zs[p0];
        __syncthreads();
        for (int lt = wave; lt < ntl; lt += kWavesPerBlock) {
            const uint32_t meta = tmeta[lt];
            const uint32_t ls = meta & 0xffffu, c = meta >> 16;
            const uint32_t gs = a.tstart[job.tb + rank + (size_t)lt * G];
            float dp = 0.0f;
            uint32_t op = 0;
            if ((uint32_t)lane < c) {
                const uint32_t i = gs + lane, p = ls + lane;
                const float x = a.xs[i], y = a.ys[i], z = a.zs[i];
                px[p] = x;
                py[p] = y;
                pz[p] = z;
                const float d0 = sqdist(x, y, z, sx, sy, sz);
                dp = euclid ? sqrt_class_top(d0) : d0;
                op = a.orig[i] - job.point_base;
                pd[p] = dp;
                po[p] = op;
            }
            tile_rekey<4>(lane, lt, ls, c, dp, op, trad, tkey, tbest, tthr);
        }
        if (tid == 0)
            sh.abort = 0;
        __syncthreads();
    }

    unsigned long long t_mark = 0;
    int j = 1;
    uint32_t round = 0;
    while (j < job.m) {
        ++round;
        ++epoch;
        if (clocks)
            t_mark = wall_clock64();
        // =============== L: local lookahead on a private copy ===============
        // One wavefront runs the lookahead: the per-step reductions stay
        // inside it and its LDS operations complete in order, so the steps
        // need no workgroup barrier.  Lanes take tiles for the arg max and the
        // sphere tests; a tile that the test keeps is updated by all lanes.
        // The first step reads the true tile state, while the other
        // wavefronts copy it to the private state the later steps use.
        {
            unsigned long long lk = 0, lk2 = 0;  // the lane's two largest tile keys
            uint32_t lt_best = 0;
            float lx = 0.0f, ly = 0.0f, lz = 0.0f;  // the last candidate
            bool more = false;                     // the lookahead goes on after step 0
            // candidate s from the lane maxima (lk, lk2, lt_best): its
            // coordinates, local key, runner-up and, for the last, the bound;
            // false for a workgroup without points
            auto select = [&](int s, bool first) -> bool {
                if (clocks)
                    tl.sub[9] -= wall_clock64();
                const unsigned long long bk = wave_max_u64(lk);
                if (bk == 0) {
                    // no points: bound 0, no candidates (every point's key is
                    // above 0, so this is step 0)
                    if (lane == 0)
                        for (int w = 0; w < W; ++w)
                            sh.my[w] = 0;
                    if (clocks)
                        tl.sub[9] += wall_clock64();
                    return false;
                }
                const unsigned long long hit = ballot64(lk == bk);
                const uint32_t bt = (uint32_t)__builtin_amdgcn_readlane((int)lt_best, __ffsll((long long)hit) - 1);
                const uint32_t p = first ? tbest[bt] : tbestl[bt];
                lx = px[p];
                ly = py[p];
                lz = pz[p];
                // runner-up: the largest local key of any other point of this
                // workgroup (other tiles, and the rest of the best tile); it
                // bounds them if this candidate is not taken at its turn.  One
                // reduction takes both parts.
                unsigned long long ru;
                {
                    const uint32_t meta = tmeta[bt];
                    const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
                    const bool valid = (uint32_t)lane < cnt;
                    const uint32_t pp = ls + (valid ? lane : 0);
                    const float dpl = pdl[pp], dpt = pd[pp];
                    const float dl = (!first && tflag[bt]) ? dpl : dpt;
                    const unsigned long long k = valid ? pack_key(dl, po[pp]) : 0ull;
                    ru = wave_max_u64(umax64(lk == bk ? lk2 : lk, k == bk ? 0ull : k));
                }
                if (lane == 0) {
                    sh.my[6 * s + 0] = __float_as_uint(lx);
                    sh.my[6 * s + 1] = __float_as_uint(ly);
                    sh.my[6 * s + 2] = __float_as_uint(lz);
                    sh.my[6 * s + 3] = (uint32_t)(bk >> 32);  // local d2
                    sh.my[6 * s + 4] = po[p];
                    sh.my[6 * s + 5] = (uint32_t)(ru >> 32);  // runner-up d2
                    if (s == R - 1) {
                        // the bound: the runner-up, or l_R itself at distance
                        // 0 (l_R is never applied to the private copy)
                        const unsigned long long b = umax64(ru, pack_key(0.0f, po[p]));
                        sh.my[6 * R] = (uint32_t)(b >> 32);
                        sh.my[6 * R + 1] = (uint32_t)b;
                    }
                }
                if (clocks)
                    tl.sub[9] += wall_clock64();
                return true;
            };
            if (wave == 0) {
                // same trip count on every lane, loads clamped: no branches
                for (int lt0 = 0; lt0 < ntl; lt0 += kWave) {
                    const int lt = lt0 + lane;
                    const unsigned long long kr = tkey[lt < ntl ? lt : 0];
                    const unsigned long long k = lt < ntl ? kr : 0ull;
                    const bool top = k > lk;
                    lk2 = top ? lk : umax64(lk2, k);
                    lt_best = top ? (uint32_t)lt : lt_best;
                    lk = top ? k : lk;
                }
                more = select(0, true) && R > 1;
            } else {
                for (int lt = tid - kWave; lt < ntl; lt += kBlock - kWave) {
                    tkeyl[lt] = tkey[lt];
                    tthrl[lt] = tsph[lt].w;
                    tbestl[lt] = tbest[lt];
                    tflag[lt] = 0;
                }
            }
            __syncthreads();
            if (clocks) {
                const unsigned long long t = wall_clock64();
                tl.sub[4] += t - t_mark;
                tl.sub[5] -= t;  // the steps end at the phase mark below
            }
            if (wave == 0 && more) {
                for (int s = 1; s < R; ++s) {
                    // local update with l_{s-1} (pruned against the local thresholds)
                    for (int lt0 = 0; lt0 < ntl; lt0 += kWave) {
                        const int lt = lt0 + lane;
                        const int li = lt < ntl ? lt : 0;
                        unsigned long long m =
                            ballot64(!(sqdist(tsph[li].x, tsph[li].y, tsph[li].z, lx, ly, lz) >= tthrl[li])) &
                            ballot64(lt < ntl);
                        while (m) {
                            const int t = lt0 + (__ffsll((long long)m) - 1);
                            m &= m - 1;
                            const uint32_t meta = tmeta[t];
                            const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
                            const bool valid = (uint32_t)lane < cnt;
                            const uint32_t pp = ls + (valid ? lane : 0);
                            // the private copy starts from the true state the
                            // first time a step of this round touches the tile
                            const float dpl = pdl[pp], dpt = pd[pp];
                            float d = tflag[t] ? dpl : dpt;
                            bool upd = false;
                            if (valid) {
                                const float dx = px[pp] - lx, dy = py[pp] - ly, dz = pz[pp] - lz;
                                const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
                                const bool skip = use_skip && (xx >= d || yy >= d || zz >= d);
                                const float s2 = xx + yy;
                                float tt = s2 + zz;
                                if (euclid && !skip && tt < d)
                                    tt = sqrt_class_top(tt);
                                upd = !skip && tt < d;
                                d = upd ? tt : d;
                                pdl[pp] = d;
                            }
                            if (lane == 0)
                                tflag[t] = 1;
                            if (__ballot(upd))
                                tile_rekey<1>(lane, t, ls, cnt, d, po[pp], trad, tkeyl, tbestl, tthrl);
                        }
                    }
                    // arg max over the private tile keys (key and tile travel together)
                    lk = 0;
                    lk2 = 0;
                    lt_best = 0;
                    for (int lt0 = 0; lt0 < ntl; lt0 += kWave) {
                        const int lt = lt0 + lane;
                        const unsigned long long kr = tkeyl[lt < ntl ? lt : 0];
                        const unsigned long long k = lt < ntl ? kr : 0ull;
                        const bool top = k > lk;
                        lk2 = top ? lk : umax64(lk2, k);
                        lt_best = top ? (uint32_t)lt : lt_best;
                        lk = top ? k : lk;
                    }
                    select(s, false);
                }
            }
        }
        __syncthreads();
        if (clocks) {
            const unsigned long long t = wall_clock64();
            tl.ph[0] += t - t_mark;
            tl.sub[5] += t;
            t_mark = t;
        }

        // =============== X: publish and read every slot ===============
        // Every word carries the round's epoch.  The readers go over all words
        // of all slots word-major (neighbouring threads, neighbouring words)
        // until each word shows the epoch, keeping all of a thread's missing
        // words in flight in every pass: reading the slots that are ready
        // overlaps waiting for the rest, and words of one slot need not
        // become visible in the order they were written.
        unsigned long long t_pub = trace ? wall_clock64() : 0ull;
        if (wave == 0) {
            unsigned long long *slot = board + ((size_t)(epoch & 1u) * G + rank) * kMaxSlotWords;
            for (int w = lane; w < W; w += kWave)
                bstore<S>(slot + w, ((unsigned long long)epoch << 32) | sh.my[w]);
        }
        {
            const int total = G * W;
            const unsigned long long *sbase = board + (size_t)(epoch & 1u) * G * kMaxSlotWords;
            // Word r of this thread, e = tid + kBlock * r, is word e % W of
            // group e / W's slot; it goes to word e of the slot image, so the
            // lanes of a wavefront store to neighbouring LDS words.
            unsigned long long pend = 0;
            uint32_t off[W];
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const int e = tid + kBlock * r;
                const bool in = e < total;
                pend |= in ? (1ull << r) : 0ull;
                off[r] = in ? (uint32_t)((e / W) * kMaxSlotWords + e % W) : 0u;
            }
            bool ab = false;
            constexpr int kFast = W < 32 ? W : 32;
            unsigned long long t_first = 0;
            for (uint32_t spin = 0; pend && !ab && spin < kSpinLimit; ++spin) {
                if (clocks && spin == 1)
                    t_first = wall_clock64();  // the passes after the first are waiting
                binvalidate<S>();
#pragma unroll
                for (int r0 = 0; r0 < W; r0 += kFast) {
                    unsigned long long x[kFast];
#pragma unroll
                    for (int q = 0; q < kFast; ++q) {
                        const int r = r0 + q;
                        x[q] = (r < W && ((pend >> r) & 1ull)) ? bload<S>(sbase + off[r]) : 0ull;
                    }
                    // a word is taken once it carries the round's epoch (a
                    // word not read this pass is 0, and epochs start at 1)
#pragma unroll
                    for (int q = 0; q < kFast; ++q) {
                        const int r = r0 + q;
                        if (r >= W)
                            break;
                        const uint32_t ep = (uint32_t)(x[q] >> 32);
                        ab |= ep == kAbortEpoch;
                        const bool ok = ep == epoch;
                        if (ok)
                            simg[tid + kBlock * r] = (uint32_t)x[q];
                        pend &= ok ? ~(1ull << r) : ~0ull;
                    }
                }
            }
            if (pend)
                sh.abort = 1;
            if (clocks && t_first)
                tl.ph[4] += wall_clock64() - t_first;
            if (clocks)
                tl.sub[6] += wall_clock64() - t_mark;
        }
        __syncthreads();
        // Candidate keys, in registers: thread g (< G <= kBlock) holds group
        // g's bound and candidate keys; a workgroup without tiles publishes the
        // bound 0 and no candidates.  The merge's S* (largest bound) and
        // largest head key are reduced on the way, and repeats of one point
        // (equal keys, consecutive in a group) are flagged per wavefront.
        unsigned long long gkey[R];
        unsigned long long gbound = 0;
        if (!sh.abort) {
            const int g = tid < G ? tid : 0;
            const uint32_t *gi = simg + g * W;
            gbound = tid < G ? ((unsigned long long)gi[6 * R] << 32) | gi[6 * R + 1] : 0ull;
            const bool empty = gbound == 0ull;
            bool repeat = false;
#pragma unroll
            for (int s2 = 0; s2 < R; ++s2) {
                gkey[s2] = empty ? 0ull : ((unsigned long long)gi[6 * s2 + 3] << 32) | (~gi[6 * s2 + 4]);
                if (s2 > 0)
                    repeat = repeat || (gkey[s2] == gkey[s2 - 1] && gkey[s2] != 0ull);
            }
            const unsigned long long sk = wave_max_u64(gbound);
            const bool anyrep = ballot64(repeat) != 0ull;
            if (lane == 0) {
                sh.red[wave] = sk;
                sh.repw[wave] = anyrep ? 1u : 0u;
            }
            if (tid == 0) {
                sh.mcount = 0;
                sh.pfront = 0;
            }
        }
        __syncthreads();
        if (sh.abort) {
            if (tid == 0) {
                set_status(&a.hdr->sample_status, RFPS_ERR_TIMEOUT);
                for (int par = 0; par < 2; ++par)
                    for (int w = 0; w < W; ++w)
                        bstore<S>(board + ((size_t)par * G + rank) * kMaxSlotWords + w,
                                  (unsigned long long)kAbortEpoch << 32);
            }
            return false;
        }
        if (clocks) {
            const unsigned long long t = wall_clock64();
            tl.ph[1] += t - t_mark;
            tl.sub[7] += t - t_mark;  // the poll's share is taken off below
            t_mark = t;
        }

        // =============== M: certified merge (whole workgroup) ===============
        // Candidates are taken in descending order of local key; each one is
        // certified when its true distance (its local distance lowered by
        // every earlier pick of the round) still equals its local distance.
        // Taking the group with the largest bound B_g at every step visits
        // exactly this order until the largest published bound S* = max_g
        // k_{R+1} is reached, where it stops.  So the candidates above S* are
        // listed (at most kList: a longer list is cut at a key boundary, and
        // the bound rises to the largest key left out), and for every listed
        // candidate its rank in key order and the set of listed candidates
        // that would lower it (state value of their distance below its listed
        // distance) are computed once, by all wavefronts.  Certification is
        // then a walk over the order in one wavefront: the first candidate
        // with a member of its set at an earlier position fails.  A failed
        // candidate is re-listed (below) and the walk resumes; distances
        // between candidates do not change, so only the re-listed candidate's
        // own set is computed again, against its new key.
        {
            unsigned long long smax = 0;
#pragma unroll
            for (int q = 0; q < kWavesPerBlock; ++q)
                smax = umax64(smax, sh.red[q]);
            // Keys of different points differ, so only a group's own repeats
            // can tie: once every point of a group has local distance 0, its
            // lookahead returns its lowest index again and again, and its
            // bound equals those candidates.  A group's candidates precede its
            // own bound, so a candidate equal to S* is taken when S* is the
            // bound of its own group.  The candidates above S* are compacted
            // (in any order) from the registers, with what the ranking pass
            // reads staged for the first kList of them.
            const unsigned long long below = lane ? (~0ull >> (kWave - lane)) : 0ull;
            // what the ranking pass reads about listed candidate pos (candidate c, key k)
            auto stage = [&](uint32_t pos, uint32_t c, unsigned long long k) {
                sh.lq[pos] = make_float4(__uint_as_float(cword(c, 0)), __uint_as_float(cword(c, 1)),
                                         __uint_as_float(cword(c, 2)), __uint_as_float((uint32_t)(k >> 32)));
                sh.lkl[pos] = (uint32_t)k;
                sh.lset1[pos] = 0ull;
                sh.lrank[pos] = 0u;
            };
#pragma unroll
            for (int s2 = 0; s2 < R; ++s2) {
                const unsigned long long k = gkey[s2];
                const bool keep = tid < G && (k > smax || (k == smax && gbound == smax));
                const unsigned long long km = ballot64(keep);
                uint32_t base = 0;
                if (lane == 0 && km)
                    base = atomicAdd(&sh.mcount, (uint32_t)__popcll(km));
                base = (uint32_t)__shfl((int)base, 0, kWave);
                if (keep) {
                    const uint32_t pos = base + (uint32_t)__popcll(km & below);
                    const uint32_t c = (uint32_t)(tid * R + s2);
                    skey[pos] = k;
                    sidx[pos] = c;
                    if (pos < (uint32_t)kList)
                        stage(pos, c, k);
                }
            }
            __syncthreads();
            const uint32_t L = sh.mcount;
            const bool rep = (sh.repw[0] | sh.repw[1] | sh.repw[2] | sh.repw[3]) != 0u;
            uint32_t *ord = reinterpret_cast<uint32_t *>(obuf);
            // scur: every listed key is above it (or equals S*, see taken) and
            // every point left out of the list has its true key at most it
            unsigned long long scur = smax;
            uint32_t W = L;  // the list: skey / sidx [0, W)
            if (L > (uint32_t)kList) {
                // a histogram of the keys' high halves (distance bits, between
                // S* and the largest listed key) in 256 buckets
                unsigned long long hm = 0;
                for (uint32_t i = tid; i < L; i += kBlock)
                    hm = umax64(hm, skey[i]);
                hm = wave_max_u64(hm);
                if (lane == 0)
                    sh.red2[wave] = hm;
                sh.hist[tid] = 0;
                __syncthreads();
                unsigned long long hmax = 0;
#pragma unroll
                for (int q = 0; q < kWavesPerBlock; ++q)
                    hmax = umax64(hmax, sh.red2[q]);
                const uint32_t hlo = (uint32_t)(smax >> 32);
                const uint32_t span = (uint32_t)(hmax >> 32) - hlo;
                const int bits = span ? 32 - __clz((int)span) : 0;
                const int bshift = bits > 8 ? bits - 8 : 0;
                for (uint32_t i = tid; i < L; i += kBlock)
                    atomicAdd(&sh.hist[((uint32_t)(skey[i] >> 32) - hlo) >> bshift], 1u);
                __syncthreads();
                // msel: the highest bucket whose suffix holds kList candidates
                if (wave == 0) {
                    uint32_t c4 = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        c4 += sh.hist[4 * lane + b];
                    uint32_t suf = c4;  // candidates in the buckets of lanes >= this one
#pragma unroll
                    for (int off = 1; off < kWave; off <<= 1) {
                        const uint32_t o = (uint32_t)__shfl_down((int)suf, off, kWave);
                        suf += lane + off < kWave ? o : 0u;
                    }
                    const unsigned long long enough = __ballot(suf >= (uint32_t)kList);
                    const int lt = 63 - __clzll((long long)enough);
                    if (lane == lt) {
                        uint32_t acc = suf - c4;
                        for (int b = 3; b >= 0; --b) {
                            acc += sh.hist[4 * lane + b];
                            if (acc >= (uint32_t)kList) {
                                sh.msel = (uint32_t)(4 * lane + b);
                                sh.mtotal = acc;
                                break;
                            }
                        }
                    }
                }
                __syncthreads();
                const uint32_t bsel = sh.msel;
                const uint32_t above = sh.mtotal - sh.hist[bsel];  // fewer than kList
                // the buckets above msel are listed when they hold anything;
                // else msel alone holds kList or more (keys that agree in their
                // high bits), and its candidates are put in order below
                const uint32_t bfront = above ? bsel + 1 : bsel;
                const uint32_t nfront = above ? above : sh.mtotal;
                constexpr int kParts = (kMaxGroups * R + kBlock - 1) / kBlock;  // L <= G * R
                unsigned long long pk_[kParts];
                uint32_t pc_[kParts], pp_[kParts];
#pragma unroll
                for (int u = 0; u < kParts; ++u) {
                    const uint32_t i = tid + kBlock * u;
                    const bool in = i < L;
                    pk_[u] = in ? skey[i] : 0ull;
                    pc_[u] = in ? sidx[i] : 0u;
                    const bool front = in && (((uint32_t)(pk_[u] >> 32) - hlo) >> bshift) >= bfront;
                    const unsigned long long fm = __ballot(front);
                    uint32_t fb = 0;
                    if (lane == 0 && fm)
                        fb = atomicAdd(&sh.pfront, (uint32_t)__popcll(fm));
                    fb = (uint32_t)__shfl((int)fb, 0, kWave);
                    pp_[u] = front ? fb + (uint32_t)__popcll(fm & below) : 0xffffffffu;
                }
                __syncthreads();
#pragma unroll
                for (int u = 0; u < kParts; ++u) {
                    if (pp_[u] != 0xffffffffu) {
                        skey[pp_[u]] = pk_[u];
                        sidx[pp_[u]] = pc_[u];
                    }
                }
                __syncthreads();
                // every candidate left out lies in a bucket below bfront
                const unsigned long long edge = (unsigned long long)(hlo + (bfront << bshift)) << 32;
                if (edge)
                    scur = umax64(scur, edge - 1ull);
                W = nfront;
                if (!above && nfront > (uint32_t)kList) {
                    // order the bucket by whole keys (equal keys: list order)
                    // and keep its first kList, cut between different keys
                    for (uint32_t i = tid; i < nfront; i += kBlock) {
                        const unsigned long long ki = skey[i];
                        uint32_t r = 0;
                        for (uint32_t q = 0; q < nfront; ++q) {
                            const unsigned long long kq = skey[q];
                            r += (kq > ki || (kq == ki && q < i)) ? 1u : 0u;
                        }
                        if (r <= (uint32_t)kList)
                            ord[r] = i;
                    }
                    __syncthreads();
                    W = kList;
                    while (W > 1 && skey[ord[W - 1]] == skey[ord[W]])
                        --W;  // equal keys are repeats of one point (at most R)
                    scur = umax64(scur, skey[ord[W]]);
                    unsigned long long kk = 0;
                    uint32_t cc = 0;
                    if ((uint32_t)tid < W) {
                        kk = skey[ord[tid]];
                        cc = sidx[ord[tid]];
                    }
                    __syncthreads();
                    if ((uint32_t)tid < W) {
                        skey[tid] = kk;
                        sidx[tid] = cc;
                    }
                    __syncthreads();
                }
                // the list moved: stage it again
                if ((uint32_t)tid < W)
                    stage(tid, sidx[tid], skey[tid]);
                __syncthreads();
            }
            const uint32_t pmax = min(W, (uint32_t)(job.m - j));
            unsigned long long t_sub = 0;
            if (clocks) {
                t_sub = wall_clock64();
                tl.sub[0] += t_sub - t_mark;
                tl.above += L;
                tl.listed += W;
            }

            // Ranks and lowering sets: for every listed candidate i, the set of
            // listed candidates q with a larger key that would lower it (state
            // value of their distance below i's listed distance), as two
            // 64-bit words (q < 64, q >= 64), and its rank in key order
            // (larger keys, then equal keys listed before it: only repeats of
            // one point are equal).  For q < 64, lanes take q and the
            // wavefronts take every fourth i, kRankPerPass at a time (measured
            // faster than a contiguous quarter of the list each), and one
            // ballot gives a word; the few q >= 64 are taken the other way
            // round (lanes take i, wavefronts share the q) so that no pass
            // runs over a nearly empty chunk of lanes.  Every ballot is of a single
            // comparison, so its lane mask is used as it is.
            const bool two = W > (uint32_t)kWave;  // some candidates are q >= 64
            const unsigned long long v0 = ballot64((uint32_t)lane < W);
            const unsigned long long v1 = ballot64((uint32_t)lane + kWave < W);
            const float4 q0 = sh.lq[lane];
            const float4 q1 = sh.lq[two ? lane + kWave : lane];
            const unsigned long long k0 = ((unsigned long long)__float_as_uint(q0.w) << 32) | sh.lkl[lane];
            const unsigned long long k1 =
                ((unsigned long long)__float_as_uint(q1.w) << 32) | sh.lkl[two ? lane + kWave : lane];
            {
                uint32_t r0l = 0, r0h = 0, rrk = 0;
                int t = 0;
                constexpr int kP = kRankPerPass;
                for (uint32_t i = (uint32_t)wave; i < W; i += kP * kWavesPerBlock, t += kP) {
                    // kP independent candidates per pass (the later ones may
                    // lie past the list: their results are not kept)
                    float4 qa[kP];
                    unsigned long long ka[kP];
#pragma unroll
                    for (int u = 0; u < kP; ++u) {
                        const uint32_t iu = i + u * kWavesPerBlock < W ? i + u * kWavesPerBlock : i;
                        qa[u] = sh.lq[iu];
                        ka[u] = ((unsigned long long)__float_as_uint(qa[u].w) << 32) | sh.lkl[iu];
                    }
#pragma unroll
                    for (int u = 0; u < kP; ++u) {
                        const float da = sqdist(qa[u].x, qa[u].y, qa[u].z, q0.x, q0.y, q0.z);
                        const unsigned long long ga = ballot64(k0 > ka[u]) & v0;
                        bool ba = da < qa[u].w;
                        if (euclid)
                            ba = ba && sqrt_class_top(da) < qa[u].w;
                        const unsigned long long ma = ballot64(ba) & ga;
                        // lane t keeps the results of this wavefront's t-th candidate
                        const bool sa = lane == t + u;
                        r0l = sa ? (uint32_t)ma : r0l;
                        r0h = sa ? (uint32_t)(ma >> 32) : r0h;
                        rrk = sa ? (uint32_t)__popcll(ga) : rrk;
                    }
                }
                const uint32_t i = (uint32_t)wave + (uint32_t)kWavesPerBlock * (uint32_t)lane;
                if (i < W) {
                    sh.lset0[i] = ((unsigned long long)r0h << 32) | r0l;
                    atomicAdd(&sh.lrank[i], rrk);
                }
            }
            if (two) {
                // q >= 64: lane l takes candidates l and l + 64, wavefront w
                // the q = 64 + w, 64 + w + 4, ...
                unsigned long long s0 = 0, s1 = 0;
                uint32_t c0 = 0, c1 = 0;
                for (uint32_t q = (uint32_t)kWave + wave; q < W; q += kWavesPerBlock) {
                    const float4 qq = sh.lq[q];
                    const unsigned long long kq = ((unsigned long long)__float_as_uint(qq.w) << 32) | sh.lkl[q];
                    const unsigned long long bit = 1ull << (q - kWave);
                    const float d0 = sqdist(q0.x, q0.y, q0.z, qq.x, qq.y, qq.z);
                    const float d1 = sqdist(q1.x, q1.y, q1.z, qq.x, qq.y, qq.z);
                    bool b0 = d0 < q0.w, b1 = d1 < q1.w;
                    if (euclid) {
                        b0 = b0 && sqrt_class_top(d0) < q0.w;
                        b1 = b1 && sqrt_class_top(d1) < q1.w;
                    }
                    const bool g0 = kq > k0, g1 = kq > k1;
                    s0 |= (b0 && g0) ? bit : 0ull;
                    s1 |= (b1 && g1) ? bit : 0ull;
                    c0 += g0 ? 1u : 0u;
                    c1 += g1 ? 1u : 0u;
                }
                if ((uint32_t)lane < W) {
                    if (s0)
                        atomicOr(&sh.lset1[lane], s0);
                    atomicAdd(&sh.lrank[lane], c0);
                }
                if ((uint32_t)lane + kWave < W) {
                    if (s1)
                        atomicOr(&sh.lset1[lane + kWave], s1);
                    atomicAdd(&sh.lrank[lane + kWave], c1);
                }
            }
            if (rep) {
                // equal keys (repeats of one point): those listed before a
                // candidate also rank above it
                for (uint32_t i = (uint32_t)wave; i < W; i += kWavesPerBlock) {
                    const float4 qi = sh.lq[i];
                    const unsigned long long ki = ((unsigned long long)__float_as_uint(qi.w) << 32) | sh.lkl[i];
                    const uint32_t il = i & (kWave - 1);
                    const unsigned long long before = il ? ~0ull >> (kWave - il) : 0ull;
                    const unsigned long long e0 = ballot64(k0 == ki) & v0 & (i >= (uint32_t)kWave ? ~0ull : before);
                    const unsigned long long e1 = ballot64(k1 == ki) & v1 & (i >= (uint32_t)kWave ? before : 0ull);
                    if (lane == 0 && (e0 | e1))
                        atomicAdd(&sh.lrank[i], (uint32_t)(__popcll(e0) + __popcll(e1)));
                }
            }
            __syncthreads();
            if (clocks) {
                const unsigned long long t = wall_clock64();
                tl.sub[1] += t - t_sub;
                t_sub = t;
            }

            // Certification walk (wavefront 0), in registers: lane l holds
            // listed candidates l and l + 64 (key, set, rank, coordinates).
            // The list stays in key order, so "earlier" means "larger key":
            // a live candidate fails when a live member of its set exists
            // (every live candidate with a larger key is a pick if the walk
            // reaches it), the first failure is the failing candidate with
            // the largest key, and the picks before it are the live
            // candidates with larger keys, which stay live from then on.
            if (wave == 0) {
                unsigned long long s00 = sh.lset0[lane], s01 = sh.lset1[lane];
                unsigned long long s10 = two ? sh.lset0[lane + kWave] : 0ull;
                unsigned long long s11 = two ? sh.lset1[lane + kWave] : 0ull;
                const uint32_t rk0 = sh.lrank[lane], rk1 = two ? sh.lrank[lane + kWave] : 0u;
                const uint32_t cc0 = sidx[lane], cc1 = two ? sidx[lane + kWave] : 0u;
                unsigned long long kc0 = k0, kc1 = k1;      // current listed keys
                unsigned long long L0 = v0, L1 = v1;        // live (listed) candidates
                unsigned long long X0 = 0, X1 = 0;          // re-listed or dropped as a group's later candidate
                unsigned long long R0 = 0, R1 = 0;          // re-listed
                uint32_t nfail = 0, P;
                for (;;) {
                    const unsigned long long F0 = ballot64(((s00 & L0) | (s01 & L1)) != 0ull) & L0;
                    const unsigned long long F1 = ballot64(((s10 & L0) | (s11 & L1)) != 0ull) & L1;
                    if (!(F0 | F1)) {
                        P = min((uint32_t)(__popcll(L0) + __popcll(L1)), pmax);
                        break;
                    }
                    // the failing candidate with the largest key
                    const unsigned long long bit = 1ull << lane;
                    const unsigned long long kf = wave_max_u64(umax64((F0 & bit) ? kc0 : 0ull, (F1 & bit) ? kc1 : 0ull));
                    const unsigned long long h0 = ballot64(kc0 > kf) & L0, h1 = ballot64(kc1 > kf) & L1;
                    P = (uint32_t)(__popcll(h0) + __popcll(h1));
                    if (P >= pmax) {
                        P = pmax;
                        break;
                    }
                    if (++nfail > kMaxFailures)
                        break;
                    const unsigned long long e0 = ballot64(kc0 == kf) & F0;
                    const uint32_t fi = e0 ? (uint32_t)(__ffsll((long long)e0) - 1)
                                           : (uint32_t)kWave + (uint32_t)(__ffsll((long long)(ballot64(kc1 == kf) & F1)) - 1);
                    const bool fh = fi >= (uint32_t)kWave;
                    const int fl = (int)(fi & (kWave - 1));
                    const float xf = lane_f32(fh ? q1.x : q0.x, fl), yf = lane_f32(fh ? q1.y : q0.y, fl),
                                zf = lane_f32(fh ? q1.z : q0.z, fl);
                    const unsigned long long sfl = fh ? s10 : s00, sfh = fh ? s11 : s01;
                    const unsigned long long sf0 = ((unsigned long long)lane_u32((uint32_t)(sfl >> 32), fl) << 32) |
                                                   lane_u32((uint32_t)sfl, fl);
                    const unsigned long long sf1 = ((unsigned long long)lane_u32((uint32_t)(sfh >> 32), fl) << 32) |
                                                   lane_u32((uint32_t)sfh, fl);
                    const uint32_t cf = lane_u32(fh ? cc1 : cc0, fl);
                    // its true distance: the listed distance lowered by the
                    // live members of its set (all of them picks)
                    const float d0 = sqdist(xf, yf, zf, q0.x, q0.y, q0.z), d1 = sqdist(xf, yf, zf, q1.x, q1.y, q1.z);
                    float tv = INFINITY;
                    if ((sf0 & L0) & bit)
                        tv = min_dist(tv, d0, euclid);
                    if ((sf1 & L1) & bit)
                        tv = min_dist(tv, d1, euclid);
                    const float tf = fminf(wave_min_dist(tv), __uint_as_float((uint32_t)(kf >> 32)));
                    const unsigned long long kt = ((unsigned long long)__float_as_uint(tf) << 32) | (uint32_t)kf;
                    scur = umax64(scur, ((unsigned long long)cword(cf, 5) << 32) | 0xffffffffull);
                    const uint32_t gf = cf / R, hf = cf % R;
                    // the group's later candidates (their local keys assumed
                    // this one picked) and every key <= the bound leave; the
                    // picks so far (h0, h1: the live keys above it) stay
                    const unsigned long long g0 = ballot64(cc0 / R == gf) & ballot64(cc0 % R > hf) & L0 & ~h0;
                    const unsigned long long g1 = ballot64(cc1 / R == gf) & ballot64(cc1 % R > hf) & L1 & ~h1;
                    X0 |= g0;
                    X1 |= g1;
                    L0 &= ~((g0 | ballot64(kc0 <= scur)) & ~h0);
                    L1 &= ~((g1 | ballot64(kc1 <= scur)) & ~h1);
                    // the failed candidate goes back in with key kt if that is
                    // above the bound; its set is taken again against tf
                    const bool put = kt > scur;
                    if (fh) {
                        const unsigned long long fb = 1ull << fl;
                        L1 = put ? (L1 | fb) : (L1 & ~fb);
                        X1 |= fb;
                        R1 |= fb;
                        if (lane == fl)
                            kc1 = kt;
                    } else {
                        const unsigned long long fb = 1ull << fl;
                        L0 = put ? (L0 | fb) : (L0 & ~fb);
                        X0 |= fb;
                        R0 |= fb;
                        if (lane == fl)
                            kc0 = kt;
                    }
                    bool b0 = d0 < tf, b1 = d1 < tf;
                    if (euclid) {
                        b0 = b0 && sqrt_class_top(d0) < tf;
                        b1 = b1 && sqrt_class_top(d1) < tf;
                    }
                    const unsigned long long n0 = ballot64(b0) & ballot64(kc0 > kt) & v0;
                    const unsigned long long n1 = ballot64(b1) & ballot64(kc1 > kt) & v1;
                    // candidates now above it no longer have it earlier
                    const unsigned long long above = fh ? ~(1ull << fl) : ~0ull, abovel = fh ? ~0ull : ~(1ull << fl);
                    if (kc0 > kt) {
                        s00 &= abovel;
                        s01 &= above;
                    }
                    if (kc1 > kt) {
                        s10 &= abovel;
                        s11 &= above;
                    }
                    if (lane == fl) {
                        if (fh) {
                            s10 = n0;
                            s11 = n1;
                        } else {
                            s00 = n0;
                            s01 = n1;
                        }
                    }
                }
                // Order of the live candidates by current key.  A candidate
                // whose key never changed has its list rank less the
                // re-listed or group-dropped candidates ranked above it
                // (every other candidate that left the list lies below all
                // live ones), plus the re-listed live candidates above it; a
                // re-listed one counts the live keys above its own.
                uint32_t lr0 = rk0, lr1 = rk1;
                unsigned long long xs0 = X0, xs1 = X1;
                while (xs0 | xs1) {
                    const bool qh = xs0 == 0ull;
                    const int ql = __ffsll((long long)(qh ? xs1 : xs0)) - 1;
                    if (qh)
                        xs1 &= xs1 - 1;
                    else
                        xs0 &= xs0 - 1;
                    const uint32_t rq = lane_u32(qh ? rk1 : rk0, ql);
                    const unsigned long long kv = qh ? kc1 : kc0;
                    const unsigned long long kq =
                        ((unsigned long long)lane_u32((uint32_t)(kv >> 32), ql) << 32) | lane_u32((uint32_t)kv, ql);
                    const bool rel_live = ((qh ? R1 & L1 : R0 & L0) >> ql) & 1ull;
                    lr0 = lr0 - (rq < rk0 ? 1u : 0u) + ((rel_live && kq > kc0) ? 1u : 0u);
                    lr1 = lr1 - (rq < rk1 ? 1u : 0u) + ((rel_live && kq > kc1) ? 1u : 0u);
                }
                // a re-listed live candidate: the live keys above its own
                unsigned long long rs0 = R0 & L0, rs1 = R1 & L1;
                while (rs0 | rs1) {
                    const bool qh = rs0 == 0ull;
                    const int ql = __ffsll((long long)(qh ? rs1 : rs0)) - 1;
                    if (qh)
                        rs1 &= rs1 - 1;
                    else
                        rs0 &= rs0 - 1;
                    const unsigned long long kv = qh ? kc1 : kc0;
                    const unsigned long long kq =
                        ((unsigned long long)lane_u32((uint32_t)(kv >> 32), ql) << 32) | lane_u32((uint32_t)kv, ql);
                    const uint32_t own =
                        (uint32_t)(__popcll(ballot64(kc0 > kq) & L0) + __popcll(ballot64(kc1 > kq) & L1));
                    if (lane == ql) {
                        if (qh)
                            lr1 = own;
                        else
                            lr0 = own;
                    }
                }
                // the picks: the first P live candidates in that order.  Their
                // coordinates go to the apply phase; rank 0 writes the
                // outputs (original index and distance from the listed key)
                // straight away, long before this wavefront next waits on
                // device memory (in the next exchange)
                const bool p0 = ((L0 >> lane) & 1ull) && lr0 < P, p1 = ((L1 >> lane) & 1ull) && lr1 < P;
                if (p0) {
                    pkx[lr0] = q0.x;
                    pky[lr0] = q0.y;
                    pkz[lr0] = q0.z;
                    if (rank == 0) {
                        job.out_idx[j + (int)lr0] = (int32_t)~(uint32_t)kc0;
                        if (job.out_d2)
                            job.out_d2[j + (int)lr0] = __uint_as_float((uint32_t)(kc0 >> 32));
                    }
                }
                if (p1) {
                    pkx[lr1] = q1.x;
                    pky[lr1] = q1.y;
                    pkz[lr1] = q1.z;
                    if (rank == 0) {
                        job.out_idx[j + (int)lr1] = (int32_t)~(uint32_t)kc1;
                        if (job.out_d2)
                            job.out_d2[j + (int)lr1] = __uint_as_float((uint32_t)(kc1 >> 32));
                    }
                }
                if (lane == 0)
                    sh.npick = P;
                if (clocks) {
                    const unsigned long long t = wall_clock64();
                    tl.sub[2] += t - t_sub;
                    tl.sub[3] -= t;
                    tl.fails += nfail;
                }
            }
        }
        __syncthreads();
        const int P = (int)sh.npick;
        if (P == 0) {
            // impossible by construction (the largest bound is attained at round
            // start); kept as a guard so a violated invariant cannot spin forever
            if (tid == 0)
                set_status(&a.hdr->sample_status, RFPS_ERR_INTERNAL);
            return false;
        }
        if (trace && round - 1 < (uint32_t)kTraceCap) {
            a.trace[2 * (size_t)(round - 1)] = t_pub;
            a.trace[2 * (size_t)(round - 1) + 1] = wall_clock64() | ((unsigned long long)P << 48);
        }
        if (clocks) {
            const unsigned long long t = wall_clock64();
            tl.ph[2] += t - t_mark;
            tl.sub[3] += t;  // from the end of the walk (subtracted there)
            t_mark = t;
        }
        j += P;
        if (j >= job.m)
            break;

        // =============== A: apply the round's picks to the true state ===============
        // Lanes take picks k and k + 64 (the second set only when the round
        // has more than 64), wavefronts take tiles, kApplyTiles at a time so
        // that their sphere loads are in flight together.  A tile's test uses
        // its current threshold (only its own update can lower it); the picks
        // that survive update the tile's points (the minimum over picks does
        // not depend on their order).  The sphere array is padded to whole
        // passes with spheres that never pass, so the tests need no bounds
        // and a pass branches only when some tile of it is hit: this loop is
        // bound by the instructions one wavefront issues, not by LDS.
        {
            const int ka = lane < P ? lane : 0, kc = lane + kWave < P ? lane + kWave : 0;
            const float sax = pkx[ka], say = pky[ka], saz = pkz[ka];
            const float scx = pkx[kc], scy = pky[kc], scz = pkz[kc];
            const unsigned long long kma = P >= kWave ? ~0ull : ((1ull << P) - 1ull);
            const unsigned long long kmc =
                P >= 2 * kWave ? ~0ull : P > kWave ? ((1ull << (P - kWave)) - 1ull) : 0ull;
            constexpr int kT = kApplyTiles;
            constexpr int kStep = kT * kWavesPerBlock;
            auto pass = [&](auto two_c) {
                constexpr bool TWO = decltype(two_c)::value;
                for (int lt0 = kT * wave; lt0 < ntl; lt0 += kStep) {
                    unsigned long long ma[kT], mc[kT];
                    float4 sp[kT];
#pragma unroll
                    for (int v = 0; v < kT; ++v)
                        sp[v] = tsph[lt0 + v];  // in the padding past the tiles
                    unsigned long long any = 0;
#pragma unroll
                    for (int v = 0; v < kT; ++v) {
                        const int lt = lt0 + v;
                        ma[v] = ballot64(!(sqdist(sp[v].x, sp[v].y, sp[v].z, sax, say, saz) >= sp[v].w)) & kma;
                        mc[v] = TWO ? ballot64(!(sqdist(sp[v].x, sp[v].y, sp[v].z, scx, scy, scz) >= sp[v].w)) & kmc
                                    : 0ull;
                        any |= ma[v] | mc[v];
                        if (tele && lane == 0 && lt < ntl) {
                            const unsigned long long nh = (unsigned long long)(__popcll(ma[v]) + __popcll(mc[v]));
                            tl.tests += (unsigned long long)P;
                            tl.pruned += (unsigned long long)P - nh;
                            tl.visited += nh * (tmeta[lt] >> 16);
                        }
                    }
                    if (!any)
                        continue;
                    unsigned long long t_upd = 0;
                    if (clocks) {
                        t_upd = wall_clock64();
                        for (int v = 0; v < kT; ++v)
                            tl.apairs += (unsigned long long)(__popcll(ma[v]) + __popcll(mc[v]));
                    }
#pragma unroll
                    for (int v = 0; v < kT; ++v) {
                        if (!(ma[v] | mc[v]))
                            continue;
                        const int lt = lt0 + v;
                        const uint32_t meta = tmeta[lt];
                        const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
                        const bool valid = (uint32_t)lane < cnt;
                        const uint32_t pp = ls + (valid ? lane : 0);
                        const float x = px[pp], y = py[pp], z = pz[pp];
                        float d = pd[pp];
                        bool changed = false;
                        for (int h = 0; h < (TWO ? 2 : 1); ++h) {
                            unsigned long long mask = h ? mc[v] : ma[v];
                            while (mask) {
                                const int kk = (h ? kWave : 0) + (__ffsll((long long)mask) - 1);
                                mask &= mask - 1;
                                const float qx = pkx[kk], qy = pky[kk], qz = pkz[kk];
                                if (valid) {
                                    const float dx = x - qx, dy = y - qy, dz = z - qz;
                                    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
                                    const bool skip = use_skip && (xx >= d || yy >= d || zz >= d);
                                    const float s2 = xx + yy;
                                    float t = s2 + zz;
                                    if (euclid && !skip && t < d)
                                        t = sqrt_class_top(t);
                                    if (!skip && t < d) {
                                        d = t;
                                        changed = true;
                                    }
                                    if (tele)
                                        tl.skipped += skip;
                                }
                            }
                        }
                        if (changed)
                            pd[pp] = d;
                        const unsigned long long um = __ballot(changed);
                        if (tele && lane == 0) {
                            tl.updated += (unsigned long long)__popcll(um);
                            tl.resync += um != 0;
                        }
                        if (um)
                            tile_rekey<4>(lane, lt, ls, cnt, d, po[pp], trad, tkey, tbest, tthr);
                        if (clocks && um)
                            ++tl.arekeys;
                    }
                    if (clocks && t_upd)
                        tl.sub[10] += wall_clock64() - t_upd;
                }
            };
            if (P > kWave)
                pass(std::true_type());
            else
                pass(std::false_type());
        }
        if (clocks)
            tl.sub[8] += wall_clock64() - t_mark;
        __syncthreads();
        if (clocks)
            tl.ph[3] += wall_clock64() - t_mark;
    }
    tl.rounds += round;
    __syncthreads();  // LDS is reused by the next cloud
    return true;
}

// Adds the per-thread telemetry of a workgroup to the header counters.
__device__ void flush_telemetry(IndexHeader *hdr, const RoundTele &tl, bool clocks)
{
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long v[6] = {tl.tests, tl.pruned, tl.visited, tl.skipped, tl.updated, tl.resync};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        unsigned long long s = v[q];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1)
            s += __shfl_xor(s, o, kWave);
        if (lane == 0 && s)
            atomicAdd(&hdr->tele[2 + q], s);
    }
    if (clocks) {
        for (int q = 0; q < 4; ++q)
            atomicAdd(&hdr->tele[kTeleTicksLookahead + q], tl.ph[q]);
        atomicAdd(&hdr->tele[kTeleTicksWait], tl.ph[4]);
        // the exchange's key forming is its phase minus its polling
        const unsigned long long sub[8] = {tl.sub[0], tl.sub[1], tl.sub[2], tl.sub[3],
                                           tl.sub[4], tl.sub[5], tl.sub[6], tl.sub[7] - tl.sub[6]};
        for (int q = 0; q < 8; ++q)
            atomicAdd(&hdr->tele[kTeleSub + q], sub[q]);
        atomicAdd(&hdr->tele[kTeleMergeStats + 0], tl.above);
        atomicAdd(&hdr->tele[kTeleMergeStats + 1], tl.listed);
        atomicAdd(&hdr->tele[kTeleMergeStats + 2], tl.fails);
        atomicAdd(&hdr->tele[kTeleMergeStats + 3], tl.sub[8]);
        atomicAdd(&hdr->tele[kTeleMergeStats + 4], tl.sub[9]);
        atomicAdd(&hdr->tele[kTeleMergeStats + 5], tl.sub[10]);
        atomicAdd(&hdr->tele[kTeleMergeStats + 6], tl.apairs);
        atomicAdd(&hdr->tele[kTeleMergeStats + 7], tl.arekeys);
    }
}

// ---------------------------------------------------------------------------
// Single cloud: one team made of the whole grid, agent-scope exchange.
// ---------------------------------------------------------------------------
template <int R, bool E, bool T>
__device__ __forceinline__ void rounds_single(const RoundArgs &a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ RoundShared sh;
    __shared__ uint32_t s_status;
    const int tid = threadIdx.x;
    IndexHeader *hdr = a.hdr;
    if (tid == 0)
        s_status = hdr->build_status | hdr->sample_status;
    __syncthreads();
    if (s_status)
        return;
    const bool tele = T && (a.flags & RFPS_F_TELEMETRY) != 0;
    const bool timed = T && (a.flags & (RFPS_F_TELEMETRY | RFPS_F_CLOCKS)) != 0;
    const bool clocks = timed && blockIdx.x == 0 && tid == 0;
    CloudJob job;
    job.tb = 0;
    job.te = hdr->n_tiles;
    job.point_base = 0;
    job.m = a.m;
    job.start = a.start;
    job.out_idx = a.out_idx;
    job.out_d2 = a.out_d2;
    uint32_t epoch = 0;
    RoundTele tl;
    const bool ok = sample_cloud<R, Scope::Agent, E, T>(a, job, blockIdx.x, a.G, a.board, epoch, smem, sh, tl,
                                                  (a.flags & RFPS_F_TRACE) != 0 && blockIdx.x == 0, clocks);
    if (timed && ok) {
        flush_telemetry(hdr, tl, clocks);  // the counters stay 0 without RFPS_F_TELEMETRY
        if (blockIdx.x == 0 && tid == 0) {
            atomicAdd(&hdr->tele[0], (unsigned long long)(a.m > 1 ? a.m - 2 : 0));
            atomicAdd(&hdr->tele[1], (unsigned long long)hdr->n_tiles);
            atomicAdd(&hdr->tele[kTeleExchanges], tl.rounds);
        }
    }
    if (blockIdx.x == 0 && tid == 0)
        hdr->trace_n = (uint32_t)tl.rounds;
}

// Squared distances (the default) and Euclidean distances are separate
// kernels, and so are the instrumented ones (RFPS_F_TELEMETRY or
// RFPS_F_TRACE): the default kernel carries no code of either.  Its machine
// code is close to the instruction cache's size, and compiling the
// instrumentation out of it shortens a round measurably.
#define RFPS_ROUNDS_KERNEL(NAME, BODY, E, T)                                                                 \
    template <int R>                                                                                          \
    __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void NAME(RoundArgs a)    \
    {                                                                                                         \
        BODY<R, E, T>(a);                                                                                     \
    }                                                                                                         \
    template __global__ void NAME<2>(RoundArgs);                                                              \
    template __global__ void NAME<3>(RoundArgs);                                                              \
    template __global__ void NAME<4>(RoundArgs);                                                              \
    template __global__ void NAME<8>(RoundArgs);
RFPS_ROUNDS_KERNEL(k_rfps_rounds, rounds_single, false, false)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_euclid, rounds_single, true, false)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_tele, rounds_single, false, true)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_euclid_tele, rounds_single, true, true)


// ---------------------------------------------------------------------------
// Batches: teams of T workgroups, all on one XCD (found from the hardware
// XCC id at run time), exchange through that XCD's L2; every team takes the
// next cloud from a queue ordered by decreasing cost until it is empty.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcc_id()
{
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((16 - 1) << 11)) & 0xffu;
}

template <int R, bool E, bool I>
__device__ __forceinline__ void rounds_batched(const RoundArgs &a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ RoundShared sh;
    __shared__ uint32_t s_status, s_xcc, s_xrank, s_cloud, s_ok;
    const int tid = threadIdx.x;
    IndexHeader *hdr = a.hdr;
    const BatchCtl &bc = a.bc;
    BatchState *st = a.bstate;
    if (tid == 0) {
        s_status = hdr->build_status | hdr->sample_status;
        s_ok = 0;
        if (!s_status) {
            // join the workgroups of this XCD, then wait until all have joined
            const uint32_t x = xcc_id();
            s_xcc = x;
            s_xrank = x < kMaxXcds ? atomicAdd(&st->xcd_count[x], 1u) : 0xffffffffu;
            // release / acquire: a workgroup that sees every join also sees
            // every XCD count bumped before it
            __hip_atomic_fetch_add(&st->joined, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t spin = 0;
            while (__hip_atomic_load(&st->joined, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x &&
                   ++spin < kSpinLimit) {
            }
            if (spin >= kSpinLimit || x >= kMaxXcds) {
                set_status(&hdr->sample_status, RFPS_ERR_TIMEOUT);
            } else if (__hip_atomic_load(&st->xcd_count[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                       (uint32_t)bc.per_xcd) {
                // the teams assume per_xcd workgroups on every XCD
                set_status(&hdr->sample_status, RFPS_ERR_UNSUPPORTED);
            } else {
                s_ok = 1;
            }
        }
    }
    __syncthreads();
    if (s_status || !s_ok)
        return;
    const int T = bc.team_size;
    const int team = (int)s_xcc * (bc.per_xcd / T) + (int)s_xrank / T;
    const int rank = (int)s_xrank % T;
    unsigned long long *board = a.board + (size_t)team * (2 * T + 1) * kMaxSlotWords;
    unsigned long long *ctl = board + (size_t)2 * T * kMaxSlotWords;  // the team's control slot
    const bool tele = I && (a.flags & RFPS_F_TELEMETRY) != 0;
    RoundTele tl;
    uint32_t epoch = 0, turn = 0;
    for (;;) {
        // The team leader takes the next cloud that needs an exchange and
        // posts it.  Every posted cloud costs at least one exchange, which the
        // leader cannot finish before every member has read the post, so a
        // post is never overwritten unread.
        ++turn;
        if (tid == 0) {
            if (rank == 0) {
                uint32_t q;
                do {
                    q = atomicAdd(&st->next, 1u);
                } while (q < (uint32_t)bc.batch && bc.m[a.order[q]] < 2);
                bstore<Scope::Xcd>(ctl, ((unsigned long long)turn << 32) | q);
                s_cloud = q;
            } else {
                uint32_t spin = 0;
                unsigned long long v = 0;
                for (; spin < kSpinLimit; ++spin) {
                    binvalidate<Scope::Xcd>();
                    v = bload<Scope::Xcd>(ctl);
                    if ((uint32_t)(v >> 32) == turn)
                        break;
                }
                s_cloud = spin < kSpinLimit ? (uint32_t)v : 0xffffffffu;
                if (spin >= kSpinLimit)
                    set_status(&hdr->sample_status, RFPS_ERR_TIMEOUT);
            }
        }
        __syncthreads();
        const uint32_t q = s_cloud;
        __syncthreads();
        if (q >= (uint32_t)bc.batch)
            break;
        const int c = a.order[q];
        CloudJob job;
        job.tb = a.tile_first[c];
        job.te = a.tile_first[c + 1];
        job.point_base = (uint32_t)bc.offsets[c];
        job.m = bc.m[c];
        job.start = bc.starts ? bc.starts[c] : 0;
        job.out_idx = a.out_idx + bc.out_offsets[c];
        job.out_d2 = a.out_d2 ? a.out_d2 + bc.out_offsets[c] : nullptr;
        if (!sample_cloud<R, Scope::Xcd, E, I>(a, job, rank, T, board, epoch, smem, sh, tl, false, false))
            return;
    }
    if (tele) {
        flush_telemetry(hdr, tl, false);
        if (rank == 0 && tid == 0)
            atomicAdd(&hdr->tele[kTeleExchanges], tl.rounds);
    }
}

RFPS_ROUNDS_KERNEL(k_rfps_rounds_batched, rounds_batched, false, false)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_batched_euclid, rounds_batched, true, false)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_batched_tele, rounds_batched, false, true)
RFPS_ROUNDS_KERNEL(k_rfps_rounds_batched_euclid_tele, rounds_batched, true, true)
#undef RFPS_ROUNDS_KERNEL

// ---------------------------------------------------------------------------
// Exchange floor: G workgroups run `rounds` exchanges with nothing else in a
// round.  Each publishes W epoch-tagged words and reads every word of every
// slot until all carry the epoch, with the same agent-scope stores, loads and
// word-major polling as the sampler's exchange.  Workgroup 0 records the
// wall-clock ticks of the whole loop in out[0]; an expired wait records
// RFPS_ERR_TIMEOUT in *status and ends the workgroup.  The launcher clears
// the slots and out[0..1] first.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_exchange_clear(unsigned long long *board, int words,
                                                           unsigned long long *out)
{
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (int w = t0; w < words; w += gridDim.x * blockDim.x)
        board[w] = 0ull;
    if (t0 < 2)
        out[t0] = 0ull;
}

// NW: words per thread (G * W <= kBlock * NW), all of a thread's words in
// flight at once as in the sampler's exchange
template <int NW>
__global__ __launch_bounds__(kBlock) void k_exchange_probe(unsigned long long *board, int G, int W, int rounds,
                                                           unsigned long long *out, uint32_t *status)
{
    const int tid = threadIdx.x, rank = blockIdx.x;
    const int total = G * W;
    __shared__ uint32_t s_abort;
    if (tid == 0)
        s_abort = 0;
    __syncthreads();
    const unsigned long long t0 = wall_clock64();
    for (uint32_t epoch = 1; epoch <= (uint32_t)rounds; ++epoch) {
        unsigned long long *sbase = board + (size_t)(epoch & 1u) * G * kMaxSlotWords;
        if (tid < W)
            bstore<Scope::Agent>(sbase + (size_t)rank * kMaxSlotWords + tid,
                                 ((unsigned long long)epoch << 32) | (uint32_t)(rank * W + tid));
        unsigned long long pend = 0;
#pragma unroll
        for (int r = 0; r < NW; ++r)
            pend |= (tid + kBlock * r < total) ? (1ull << r) : 0ull;
        for (uint32_t spin = 0; pend && spin < kSpinLimit; ++spin) {
            unsigned long long x[NW];
#pragma unroll
            for (int r = 0; r < NW; ++r) {
                const int e = tid + kBlock * r;
                x[r] = ((pend >> r) & 1ull) ? bload<Scope::Agent>(sbase + (size_t)(e / W) * kMaxSlotWords + e % W)
                                            : 0ull;
            }
#pragma unroll
            for (int r = 0; r < NW; ++r)
                if (((pend >> r) & 1ull) && (uint32_t)(x[r] >> 32) == epoch)
                    pend &= ~(1ull << r);
        }
        if (pend)
            s_abort = 1;
        __syncthreads();
        if (s_abort) {
            if (tid == 0)
                set_status(status, RFPS_ERR_TIMEOUT);
            return;
        }
    }
    if (rank == 0 && tid == 0)
        out[0] = wall_clock64() - t0;
}

hipError_t launch_exchange_probe(unsigned long long *board, int G, int W, int rounds, unsigned long long *out,
                                 uint32_t *status, hipStream_t s)
{
    if (G < 1 || G > kMaxGroups || W < 1 || W > kMaxSlotWords || 2 * G * kMaxSlotWords > kBoardWords || rounds < 1)
        return hipErrorInvalidValue;
    const int per = (G * W + kBlock - 1) / kBlock;  // words per thread
    k_exchange_clear<<<64, kBlock, 0, s>>>(board, 2 * G * kMaxSlotWords, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    void *args[] = {&board, &G, &W, &rounds, &out, &status};
    // unused dynamic LDS of more than half a compute unit's keeps one
    // workgroup per compute unit, as in the sampler
    const void *fn = per <= 2    ? reinterpret_cast<const void *>(k_exchange_probe<2>)
                     : per <= 16 ? reinterpret_cast<const void *>(k_exchange_probe<16>)
                     : per <= 32 ? reinterpret_cast<const void *>(k_exchange_probe<32>)
                                 : reinterpret_cast<const void *>(k_exchange_probe<64>);
    constexpr int kOnePerCu = 96 * 1024;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kOnePerCu);
    if (e != hipSuccess)
        return e;
    return launch_persistent(fn, G, args, kOnePerCu, s);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static const void *rounds_fn(int R, bool batched, bool euclid, bool tele)
{
#define RFPS_ROUNDS_FN(K)                                                                                    \
    (R == 2 ? reinterpret_cast<const void *>(K<2>) : R == 3 ? reinterpret_cast<const void *>(K<3>)          \
     : R == 4                                            ? reinterpret_cast<const void *>(K<4>)            \
     : R == 8                                            ? reinterpret_cast<const void *>(K<8>)            \
                                                         : nullptr)
    if (batched) {
        if (tele)
            return euclid ? RFPS_ROUNDS_FN(k_rfps_rounds_batched_euclid_tele)
                          : RFPS_ROUNDS_FN(k_rfps_rounds_batched_tele);
        return euclid ? RFPS_ROUNDS_FN(k_rfps_rounds_batched_euclid) : RFPS_ROUNDS_FN(k_rfps_rounds_batched);
    }
    if (tele)
        return euclid ? RFPS_ROUNDS_FN(k_rfps_rounds_euclid_tele) : RFPS_ROUNDS_FN(k_rfps_rounds_tele);
    return euclid ? RFPS_ROUNDS_FN(k_rfps_rounds_euclid) : RFPS_ROUNDS_FN(k_rfps_rounds);
#undef RFPS_ROUNDS_FN
}

size_t rfps_rounds_static_lds(int R)
{
    size_t mx = 0;
    for (int b = 0; b < 8; ++b) {
        const void *fn = rounds_fn(R, (b & 1) != 0, (b & 2) != 0, (b & 4) != 0);
        hipFuncAttributes attr;
        if (!fn || hipFuncGetAttributes(&attr, fn) != hipSuccess)
            return 0;
        mx = attr.sharedSizeBytes > mx ? attr.sharedSizeBytes : mx;
    }
    return mx;
}

static RoundArgs round_args(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                            float *out_d2)
{
    RoundArgs a;
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
    a.bc = BatchCtl{};
    a.bstate = nullptr;
    a.tile_first = nullptr;
    a.order = nullptr;
    return a;
}

hipError_t launch_rfps_rounds(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s)
{
    k_rounds_plan<<<(L.G + kBlock - 1) / kBlock, kBlock, 0, s>>>(v.hdr, v.tcnt, L.G, L.R, L.lds_budget);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || m <= 1)
        return e;
    const void *fn = rounds_fn(L.R, false, (L.flags & RFPS_F_SQRT) != 0,
                               (L.flags & (RFPS_F_TELEMETRY | RFPS_F_TRACE | RFPS_F_CLOCKS)) != 0);
    if (!fn)
        return hipErrorInvalidValue;
    RoundArgs a = round_args(v, m, start, L, out_idx, out_d2);
    void *args[] = {&a};
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_budget);
    if (e != hipSuccess)
        return e;
    return launch_persistent(fn, L.G, args, L.lds_budget, s);
}

// Batched: per-cloud capacity check for teams of bc.team_size workgroups,
// then the first output of every cloud (its start, at distance +inf) and the
// counters the sampler does not keep.
__global__ __launch_bounds__(kBlock) void k_batch_plan(IndexHeader *hdr, const uint32_t *__restrict__ tcnt,
                                                       BatchCtl bc, const uint32_t *__restrict__ tile_first, int R,
                                                       uint32_t budget, int32_t *out_idx, float *out_d2)
{
    if (hdr->build_status)
        return;
    const int T = bc.team_size;
    const int total = bc.batch * T;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    for (int w = tid; w < total; w += nth) {
        const int c = w / T, r = w % T;
        if (!team_fits(tcnt, tile_first[c], tile_first[c + 1], T, R, budget, r))
            set_status(&hdr->sample_status, RFPS_ERR_CAPACITY);
    }
    for (int c = tid; c < bc.batch; c += nth) {
        const uint32_t o = bc.out_offsets[c];
        out_idx[o] = bc.starts ? bc.starts[c] : 0;
        if (out_d2)
            out_d2[o] = INFINITY;
    }
    if (tid == 0) {
        unsigned long long it = 0;
        for (int c = 0; c < bc.batch; ++c)
            it += bc.m[c] > 2 ? (unsigned long long)(bc.m[c] - 2) : 0ull;
        hdr->tele[0] = it;
        hdr->tele[1] = hdr->n_tiles;
    }
}

hipError_t launch_rfps_rounds_batched(const IndexView &v, const SampleLaunch &L, int32_t *out_idx,
                                      float *out_d2, hipStream_t s)
{
    const int total = v.bc.batch * v.bc.team_size;
    k_batch_plan<<<std::min((total + kBlock - 1) / kBlock, 1024), kBlock, 0, s>>>(
        v.hdr, v.tcnt, v.bc, v.tile_first, L.R, L.lds_budget, out_idx, out_d2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const void *fn = rounds_fn(L.R, true, (L.flags & RFPS_F_SQRT) != 0,
                               (L.flags & (RFPS_F_TELEMETRY | RFPS_F_TRACE | RFPS_F_CLOCKS)) != 0);
    if (!fn)
        return hipErrorInvalidValue;
    RoundArgs a = round_args(v, 0, 0, L, out_idx, out_d2);
    a.bc = v.bc;
    a.bstate = v.bstate;
    a.tile_first = v.tile_first;
    a.order = v.order;
    void *args[] = {&a};
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_budget);
    if (e != hipSuccess)
        return e;
    e = launch_persistent(fn, L.G, args, L.lds_budget, s);
    if (e != hipSuccess)
        return e;
    return launch_sample_finalize(v.hdr, v.bc.m_total, out_idx, out_d2, s);
}

}  // namespace rfps
