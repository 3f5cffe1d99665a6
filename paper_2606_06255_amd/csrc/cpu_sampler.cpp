// CPU RadiusFPS (Sec. 3): exact FPS with spherical-voxel pruning on the host
// cores, beside the GPU samplers of this library.
//
// Index (Sec. 3.2): the same grid as the GPU build (edge L = alpha * max
// extent / n_vox in FP64, alpha = 1 + 1e-4), points sorted by voxel key with
// an LSD radix sort, each voxel split into tiles of at most `tile` points,
// each tile enclosed by a sphere around the centre of its members' bounding
// box (within the voxel cube, and tighter than the cube's sphere when a
// voxel splits into several tiles) whose radius is the largest member
// distance rounded up.
// Sampling (Sec. 3.3 - 3.4): a team of threads, each owning every T-th tile
// (round-robin, so that the updates around each new sample, which are
// spatially concentrated, spread over the team).  Per selection the team
// all-reduces the largest key of each member's tiles (largest distance, then
// lowest original index), so every thread knows s_j and no barrier is
// needed besides that exchange.  Then
// each thread filters its tiles against the cached pruning thresholds and
// updates the survivors' points with the strict rule; a tile whose points
// changed gets a new key and threshold.  The point skip of Sec. 3.4.3 is not
// used: the branch-free update of a 64-point tile vectorises, and the skip
// never changes a result.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <memory>
#include <thread>
#include <vector>

#include <sched.h>

#include "../../include/rfps.h"
#include "prune_bound.h"

// The distance must be evaluated as written: no FMA contraction.
#pragma clang fp contract(off)

namespace {

constexpr int kMaxTeam = 256;

inline float sqd(float px, float py, float pz, float sx, float sy, float sz)
{
    const float dx = px - sx, dy = py - sy, dz = pz - sz;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float s = xx + yy;
    return s + zz;
}

inline uint32_t fbits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
inline float bitsf(uint32_t u)
{
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

inline uint64_t pack(float d, uint32_t orig) { return ((uint64_t)fbits(d) << 32) | (uint32_t)~orig; }

// Skip threshold of a tile with radius R and tile distance dv: the bound
// the GPU samplers use, from the one definition in prune_bound.h.
using rfps::prune_threshold;

// Euclidean mode: the largest FP32 value whose rounded root equals that of
// x (IEEE sqrtf rounds correctly); min and arg max over these class tops
// follow FPS over rounded Euclidean distances.
inline float class_top(float x)
{
    if (!(x > 0.0f) || std::isinf(x))
        return x;
    const float r = std::sqrt(x);
    const double up = 0.5 * ((double)r + (double)std::nextafter(r, INFINITY));
    const double b = up * up;  // exact; never an FP32 value
    if (b > 3.4028234663852886e38)
        return 3.4028234663852886e38f;
    float y = (float)b;
    if ((double)y > b)
        y = std::nextafter(y, 0.0f);
    return y;
}

struct Index {
    int n = 0, nt = 0;
    std::vector<float> x, y, z;        // sorted by voxel key
    std::vector<uint32_t> orig, inv;   // sorted -> original, original -> sorted
    std::vector<uint32_t> tstart, tcnt;
    std::vector<float> cx, cy, cz, rad;
};

void build_index(const float *xyz, int n, int n_vox, int tile, Index &I)
{
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = xyz[a];
    for (int i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], xyz[3 * (size_t)i + a]);
            hi[a] = std::max(hi[a], xyz[3 * (size_t)i + a]);
        }
    double E = 0.0;
    for (int a = 0; a < 3; ++a)
        E = std::max(E, (double)hi[a] - (double)lo[a]);
    const double L = E > 0.0 ? (1.0 + 1e-4) * E / (double)n_vox : 1.0;
    const double top = (double)(n_vox - 1);
    std::vector<uint64_t> kv((size_t)n), tmp((size_t)n);
    for (int i = 0; i < n; ++i) {
        uint32_t v[3];
        for (int a = 0; a < 3; ++a) {
            double q = std::floor(((double)xyz[3 * (size_t)i + a] - (double)lo[a]) / L);
            q = std::min(std::max(q, 0.0), top);
            v[a] = (uint32_t)q;
        }
        const uint64_t key = ((uint64_t)v[2] * n_vox + v[1]) * n_vox + v[0];
        kv[i] = (key << 32) | (uint32_t)i;
    }
    // LSD radix sort on the key half, 11 bits per pass (keys < 2^30)
    const uint64_t kmax = (uint64_t)n_vox * n_vox * n_vox;
    for (int shift = 32; shift < 64 && (kmax >> (shift - 32)) > 0; shift += 11) {
        std::vector<uint32_t> cnt(2049, 0);
        for (int i = 0; i < n; ++i)
            ++cnt[((kv[i] >> shift) & 2047u) + 1];
        for (int d = 0; d < 2048; ++d)
            cnt[d + 1] += cnt[d];
        for (int i = 0; i < n; ++i)
            tmp[cnt[(kv[i] >> shift) & 2047u]++] = kv[i];
        kv.swap(tmp);
    }
    I.n = n;
    I.x.resize(n);
    I.y.resize(n);
    I.z.resize(n);
    I.orig.resize(n);
    I.inv.resize(n);
    for (int p = 0; p < n; ++p) {
        const uint32_t i = (uint32_t)kv[p];
        I.x[p] = xyz[3 * (size_t)i];
        I.y[p] = xyz[3 * (size_t)i + 1];
        I.z[p] = xyz[3 * (size_t)i + 2];
        I.orig[p] = i;
        I.inv[i] = (uint32_t)p;
    }
    // tiles: runs of equal key, cut every `tile` points
    I.tstart.clear();
    I.tcnt.clear();
    for (int p = 0; p < n;) {
        const uint64_t key = kv[p] >> 32;
        int e = p;
        while (e < n && (kv[e] >> 32) == key)
            ++e;
        for (int s = p; s < e; s += tile) {
            I.tstart.push_back((uint32_t)s);
            I.tcnt.push_back((uint32_t)std::min(tile, e - s));
        }
        p = e;
    }
    I.nt = (int)I.tstart.size();
    I.cx.resize(I.nt);
    I.cy.resize(I.nt);
    I.cz.resize(I.nt);
    I.rad.resize(I.nt);
    for (int t = 0; t < I.nt; ++t) {
        const uint32_t p0 = I.tstart[t], c_n = I.tcnt[t];
        float bl[3] = {I.x[p0], I.y[p0], I.z[p0]}, bh[3] = {I.x[p0], I.y[p0], I.z[p0]};
        for (uint32_t k = 1; k < c_n; ++k) {
            const float q[3] = {I.x[p0 + k], I.y[p0 + k], I.z[p0 + k]};
            for (int a = 0; a < 3; ++a) {
                bl[a] = std::min(bl[a], q[a]);
                bh[a] = std::max(bh[a], q[a]);
            }
        }
        float c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = (float)(0.5 * ((double)bl[a] + (double)bh[a]));
        double r2 = 0.0;
        for (uint32_t k = 0; k < I.tcnt[t]; ++k) {
            const double dx = (double)I.x[p0 + k] - c[0], dy = (double)I.y[p0 + k] - c[1],
                         dz = (double)I.z[p0 + k] - c[2];
            r2 = std::max(r2, dx * dx + dy * dy + dz * dz);
        }
        const double r = std::sqrt(r2) * (1.0 + 0x1p-40) + 0x1p-120;
        float r32 = (float)r;
        if ((double)r32 < r)
            r32 = std::nextafter(r32, INFINITY);
        I.cx[t] = c[0];
        I.cy[t] = c[1];
        I.cz[t] = c[2];
        I.rad[t] = r32;
    }
}

// Team-wide maximum of one 64-bit key per member, by dissemination: in
// round k member r hands its running maximum to member (r + 2^k) mod T and
// folds in the one from (r - 2^k) mod T; after ceil(log2 T) rounds every
// member holds the maximum of all T keys (max is idempotent, so the overlap
// when T is not a power of two is harmless).  Each round is one cache line
// handed to one partner, instead of T arrivals on a shared counter followed
// by T reads.  A message is (key, epoch): the sender stores the key, then
// the epoch with release order; the receiver waits for the epoch with
// acquire order.  Messages alternate between two buffers by the parity of
// the selection: a sender reuses a buffer two selections later, and by then
// its own maximum of the selection in between depends on every member,
// including the receiver, having started that selection, so the receiver
// has read the old message.
struct alignas(64) Msg {
    std::atomic<uint64_t> key;
    std::atomic<uint64_t> epoch;
};

class MaxReduce {
public:
    explicit MaxReduce(int T) : T_(T), rounds_(0)
    {
        while ((1 << rounds_) < T)
            ++rounds_;
        const size_t n = (size_t)2 * std::max(rounds_, 1) * T;
        box_.reset(new Msg[n]);
        for (size_t i = 0; i < n; ++i) {
            box_[i].key.store(0, std::memory_order_relaxed);
            box_[i].epoch.store(0, std::memory_order_relaxed);
        }
    }
    // Returns early (with a partial maximum) once `abort` is set.
    uint64_t all(int r, uint64_t v, uint64_t epoch, const std::atomic<bool> &abort)
    {
        Msg *b = box_.get() + (size_t)(epoch & 1) * rounds_ * T_;
        for (int k = 0; k < rounds_; ++k, b += T_) {
            Msg &out = b[(r + (1 << k)) % T_];
            out.key.store(v, std::memory_order_relaxed);
            out.epoch.store(epoch, std::memory_order_release);
            Msg &in = b[r];
            int spins = 0;
            while (in.epoch.load(std::memory_order_acquire) != epoch) {
                if (abort.load(std::memory_order_relaxed))
                    return v;
                if (++spins > 4096)
                    std::this_thread::yield();
            }
            v = std::max(v, in.key.load(std::memory_order_relaxed));
        }
        return v;
    }

private:
    int T_, rounds_;
    std::unique_ptr<Msg[]> box_;
};

// One thread's tiles (every T-th tile) with their state in structure-of-arrays form.
struct Share {
    std::vector<uint32_t> tile;       // global tile ids
    std::vector<float> cx, cy, cz;    // sphere centres
    std::vector<float> rad, thr;      // radius, cached skip threshold
    std::vector<uint64_t> key;        // tile key: largest Dist_p, lowest original index
};

struct Team {
    const Index *I;
    int T, m;
    bool euclid;
    std::vector<float> pd;            // Dist_p, sorted order
    std::vector<Share> share;
    MaxReduce reduce;
    std::atomic<bool> abort{false};   // set when the team could not be started
    int32_t *out_idx;
    float *out_d2;
    explicit Team(int t) : reduce(t) {}
};

// Updates one tile for sample s; returns whether any Dist_p changed and
// refreshes the tile's key.
inline bool update_tile(const Index &I, float *pd, uint32_t t, float sx, float sy, float sz, bool euclid,
                        uint64_t &key)
{
    const uint32_t p0 = I.tstart[t], c = I.tcnt[t];
    const float *X = I.x.data() + p0, *Y = I.y.data() + p0, *Z = I.z.data() + p0;
    float *D = pd + p0;
    bool changed = false;
    float dmax = -1.0f;
    for (uint32_t k = 0; k < c; ++k) {
        float tt = sqd(X[k], Y[k], Z[k], sx, sy, sz);
        if (euclid && tt < D[k])
            tt = class_top(tt);
        const bool upd = tt < D[k];
        changed |= upd;
        D[k] = upd ? tt : D[k];
        dmax = std::max(dmax, D[k]);
    }
    if (changed) {
        uint32_t best = 0xffffffffu;  // lowest original index at the largest distance
        for (uint32_t k = 0; k < c; ++k)
            if (D[k] == dmax)
                best = std::min(best, I.orig[p0 + k]);
        key = pack(dmax, best);
    }
    return changed;
}

void run_member(Team &tm, int r)
{
    const Index &I = *tm.I;
    Share &sh = tm.share[r];
    float *pd = tm.pd.data();
    const int nl = (int)sh.tile.size();
    uint64_t local = 0;
    for (int l = 0; l < nl; ++l)
        local = std::max(local, sh.key[l]);
    for (int j = 1; j < tm.m; ++j) {
        const uint64_t best = tm.reduce.all(r, local, (uint64_t)j, tm.abort);
        if (tm.abort.load(std::memory_order_relaxed))
            return;
        const uint32_t o = ~(uint32_t)best;
        const float d = bitsf((uint32_t)(best >> 32));
        if (r == 0) {
            tm.out_idx[j] = (int32_t)o;
            if (tm.out_d2)
                tm.out_d2[j] = d;
        }
        const uint32_t ps = I.inv[o];
        const float sx = I.x[ps], sy = I.y[ps], sz = I.z[ps];
        local = 0;
        for (int l = 0; l < nl; ++l) {
            if (!(sqd(sh.cx[l], sh.cy[l], sh.cz[l], sx, sy, sz) >= sh.thr[l])) {
                uint64_t k = sh.key[l];
                if (update_tile(I, pd, sh.tile[l], sx, sy, sz, tm.euclid, k)) {
                    sh.key[l] = k;
                    sh.thr[l] = prune_threshold(sh.rad[l], bitsf((uint32_t)(k >> 32)));
                }
            }
            local = std::max(local, sh.key[l]);
        }
    }
}

bool flags_ok(uint32_t f) { return (f & ~(uint32_t)(RFPS_F_NO_POINT_SKIP | RFPS_F_SQRT)) == 0; }

// Default team: OMP_NUM_THREADS when set (the host's share of cores),
// otherwise the CPUs this process may run on.
int default_team()
{
    if (const char *e = std::getenv("OMP_NUM_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0)
            return v;
    }
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0 && CPU_COUNT(&set) > 0)
        return CPU_COUNT(&set);
    return (int)std::max(1u, std::thread::hardware_concurrency());
}

void poison(int32_t *out_idx, float *out_d2, int m)
{
    for (int j = 0; j < m; ++j) {
        out_idx[j] = -1;
        if (out_d2)
            out_d2[j] = std::nanf("");
    }
}

rfps_status cpu_sample(const float *xyz, int32_t n, int32_t m, int32_t start, const rfps_params *params,
                       int32_t threads, int32_t *out_idx, float *out_d2)
{
    if (!xyz || !out_idx || n < 1 || n > (1 << 26) || m < 1 || m > n || start < 0 || start >= n || threads < 0)
        return RFPS_ERR_INVALID_ARG;
    // default: half the GPU's bins.  Larger voxels mean fewer tiles to test
    // per selection, which costs a core more than it costs a wavefront
    // (room 80k: 24 bins 2x faster than 48; LiDAR 115k and 1M: within 15 %
    // of the best of 8..256)
    const int n_vox = (params && params->n_vox) ? params->n_vox : std::max(8, rfps_default_n_vox(n) / 2);
    const int tile = (params && params->tile) ? params->tile : 64;
    const uint32_t flags = params ? params->flags : 0u;
    if (n_vox < 1 || n_vox > 1024 || tile < 1 || tile > 64 || !flags_ok(flags))
        return RFPS_ERR_INVALID_ARG;
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(xyz[i])) {
            poison(out_idx, out_d2, m);
            return RFPS_ERR_NONFINITE;
        }
    Index I;
    build_index(xyz, n, n_vox, tile, I);
    int T = threads ? threads : default_team();
    T = std::max(1, std::min({T, kMaxTeam, I.nt}));
    Team tm(T);
    tm.I = &I;
    tm.T = T;
    tm.m = m;
    tm.euclid = (flags & RFPS_F_SQRT) != 0;
    tm.out_idx = out_idx;
    tm.out_d2 = out_d2;
    tm.pd.resize(n);
    tm.share.resize(T);
    // seed (Sec. 3.3): Dist_p of every point to the start point, tile keys
    const uint32_t ps = I.inv[start];
    const float sx = I.x[ps], sy = I.y[ps], sz = I.z[ps];
    for (int p = 0; p < n; ++p) {
        const float d = sqd(I.x[p], I.y[p], I.z[p], sx, sy, sz);
        tm.pd[p] = tm.euclid ? class_top(d) : d;
    }
    for (int t = 0; t < I.nt; ++t) {
        Share &sh = tm.share[t % T];
        const uint32_t p0 = I.tstart[t];
        float dmax = -1.0f;
        uint32_t best = 0xffffffffu;
        for (uint32_t k = 0; k < I.tcnt[t]; ++k) {
            const float d = tm.pd[p0 + k];
            if (d > dmax || (d == dmax && I.orig[p0 + k] < best)) {
                dmax = d;
                best = I.orig[p0 + k];
            }
        }
        sh.tile.push_back((uint32_t)t);
        sh.cx.push_back(I.cx[t]);
        sh.cy.push_back(I.cy[t]);
        sh.cz.push_back(I.cz[t]);
        sh.rad.push_back(I.rad[t]);
        sh.thr.push_back(prune_threshold(I.rad[t], dmax));
        sh.key.push_back(pack(dmax, best));
    }
    out_idx[0] = start;
    if (out_d2)
        out_d2[0] = INFINITY;
    std::vector<std::thread> pool;
    pool.reserve(T - 1);
    try {
        for (int r = 1; r < T; ++r)
            pool.emplace_back(run_member, std::ref(tm), r);
    } catch (...) {
        // a member could not be started: release the ones waiting for it
        tm.abort.store(true);
        for (auto &th : pool)
            th.join();
        poison(out_idx, out_d2, m);
        return RFPS_ERR_INTERNAL;
    }
    run_member(tm, 0);
    for (auto &th : pool)
        th.join();
    if (out_d2 && tm.euclid)
        for (int j = 1; j < m; ++j)
            out_d2[j] = std::sqrt(out_d2[j]);
    return RFPS_OK;
}

}  // namespace

extern "C" rfps_status rfps_cpu_sample(const float *xyz, int32_t n, int32_t m, int32_t start,
                                       const rfps_params *params, int32_t threads, int32_t *out_idx,
                                       float *out_d2)
{
    // no C++ exception may cross the C boundary: host memory that cannot be
    // obtained is reported like a team that cannot be started
    try {
        return cpu_sample(xyz, n, m, start, params, threads, out_idx, out_d2);
    } catch (...) {
        if (out_idx && m >= 1 && m <= n)
            poison(out_idx, out_d2, m);
        return RFPS_ERR_INTERNAL;
    }
}
