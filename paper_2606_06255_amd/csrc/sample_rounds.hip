// RadiusFPS-G with certified multi-pick rounds (the default sampler).
//
// Same ownership and LDS residency as k_rfps (tiles dealt round-robin to
// workgroups), but one exchange now settles many selections.  A round:
//
//   L  lookahead: every workgroup runs R steps of FPS on its own points only
//      (a private copy of Dist_p, with the same spherical pruning), giving
//      local candidates l_1..l_R with their local keys k_1 > .. > k_R and the
//      bound k_{R+1}, the largest local key left after them;
//   X  exchange: each workgroup publishes its candidates (coordinates, true
//      round-start distance, local distance) and k_{R+1};
//   M  merge: every workgroup replays the same deterministic merge.  Group g
//      keeps a head h_g (how many of its candidates were taken).  Its bound
//      B_g = k_{h_g+1} is an upper bound on the true key of every point of g:
//      the true distances contain every pick of the round so far, which
//      include l_1..l_{h_g}, so they are at most the local ones.  Hence the
//      largest true key anywhere is at most max_g B_g, and if the head
//      candidate of the group with the largest bound still has its true key
//      equal to its local key (no other pick of the round reduced it), that
//      candidate is exactly the next FPS selection (Sec. 3.1 rule, keys
//      unique).  Otherwise the round ends;
//   A  apply: all picks of the round update the true state (spherical test
//      per tile and pick, point skip, strict update, tile-key resync).
//
// Every round certifies at least one selection (the largest bound is the
// global maximum at round start, and nothing has reduced it yet), so the
// kernel always terminates; the output equals plain FPS bit for bit.
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
};

__host__ __device__ __forceinline__ uint32_t rounds_lds_need(uint32_t tiles, uint32_t pts, uint32_t G, uint32_t R)
{
    return tiles * 60u + pts * 24u + G * R * 28u + G * (R + 1u) * 8u + 128u;
}

__global__ __launch_bounds__(kBlock) void k_rounds_plan(IndexHeader *hdr, const uint32_t *__restrict__ tcnt,
                                                        int G, int R, uint32_t budget)
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
    if (pts > 65535u || rounds_lds_need(tiles, pts, G, R) > budget)
        set_status(&hdr->sample_status, RFPS_ERR_CAPACITY);
}

// One wavefront recomputes the key, best point and threshold of tile lt from
// the distances in D (all lanes of the wave must call it).
__device__ __forceinline__ void tile_rekey(int lane, uint32_t lt, uint32_t ls, uint32_t cnt, const float *D,
                                           const uint32_t *po, const float *trad, unsigned long long *tkey,
                                           uint32_t *tbest, float *tthr)
{
    const bool valid = (uint32_t)lane < cnt;
    const uint32_t p = ls + (valid ? lane : 0);
    const unsigned long long key = valid ? pack_key(D[p], po[p]) : 0ull;
    const unsigned long long kmax = wave_max_u64(key);
    const unsigned long long hit = __ballot(valid && key == kmax);
    if (lane == 0) {
        tkey[lt] = kmax;
        tbest[lt] = ls + (uint32_t)(__ffsll((long long)hit) - 1);
        tthr[lt] = prune_threshold(trad[lt], key_d2(kmax));
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_rfps_rounds(RoundArgs a)
{
    constexpr int W = 6 * R + 2;  // words per slot
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_red[kWavesPerBlock];
    __shared__ uint32_t s_redi[kWavesPerBlock];
    __shared__ uint32_t s_scan[kWavesPerBlock];
    __shared__ uint32_t s_status, s_abort, s_list_n, s_npick;
    __shared__ uint32_t s_my[W];  // this workgroup's slot payload

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int g = blockIdx.x, G = a.G;
    IndexHeader *hdr = a.hdr;
    if (tid == 0) {
        s_status = hdr->build_status | hdr->sample_status;
        s_abort = 0;
        s_list_n = 0;
    }
    __syncthreads();
    if (s_status)
        return;
    const uint32_t NT = hdr->n_tiles;
    const int ntl = (NT > (uint32_t)g) ? (int)((NT - 1 - g) / G) + 1 : 0;
    const bool use_skip = !(a.flags & RFPS_F_NO_POINT_SKIP);
    const bool tele = (a.flags & RFPS_F_TELEMETRY) != 0;
    const bool trace = (a.flags & RFPS_F_TRACE) != 0 && g == 0 && tid == 0;

    // ---- LDS layout (the plan kernel checked that it fits) ----
    unsigned long long *tkey = reinterpret_cast<unsigned long long *>(smem);
    unsigned long long *tkeyl = tkey + ntl;
    unsigned long long *bkey = tkeyl + ntl;  // [G][R+1] published local keys
    float *tcx = reinterpret_cast<float *>(bkey + (size_t)G * (R + 1));
    float *tcy = tcx + ntl;
    float *tcz = tcy + ntl;
    float *trad = tcz + ntl;
    float *tthr = trad + ntl;
    float *tthrl = tthr + ntl;
    uint32_t *tmeta = reinterpret_cast<uint32_t *>(tthrl + ntl);
    uint32_t *tbest = tmeta + ntl;
    uint32_t *tbestl = tbest + ntl;
    uint32_t *tflag = tbestl + ntl;
    uint32_t *tlist = tflag + ntl;
    float *cx = reinterpret_cast<float *>(tlist + ntl);  // [G][R] candidates
    float *cy = cx + G * R;
    float *cz = cy + G * R;
    float *ctd = cz + G * R;   // true round-start d2; becomes the selection d2 when picked
    float *cld = ctd + G * R;  // local d2
    uint32_t *corig = reinterpret_cast<uint32_t *>(cld + G * R);
    uint32_t *picks = corig + G * R;  // candidate index g*R+h of each pick of the round
    float *px = reinterpret_cast<float *>(picks + G * R);

    // ---- prologue: tile metadata, LDS offsets ----
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
    float *py = px + npl;
    float *pz = py + npl;
    float *pd = pz + npl;
    float *pdl = pd + npl;
    uint32_t *po = reinterpret_cast<uint32_t *>(pdl + npl);

    // Seed and initial update (Sec. 3.3)
    {
        const uint32_t p0 = a.inv[a.start];
        const float sx = a.xs[p0], sy = a.ys[p0], sz = a.zs[p0];
        __syncthreads();
        for (int lt = wave; lt < ntl; lt += kWavesPerBlock) {
            const uint32_t meta = tmeta[lt];
            const uint32_t ls = meta & 0xffffu, c = meta >> 16;
            const uint32_t gs = a.tstart[g + (size_t)lt * G];
            if ((uint32_t)lane < c) {
                const uint32_t i = gs + lane, p = ls + lane;
                const float x = a.xs[i], y = a.ys[i], z = a.zs[i];
                px[p] = x;
                py[p] = y;
                pz[p] = z;
                pd[p] = sqdist(x, y, z, sx, sy, sz);
                po[p] = a.orig[i];
            }
            tile_rekey(lane, lt, ls, c, pd, po, trad, tkey, tbest, tthr);
        }
        __syncthreads();
    }

    unsigned long long t_tests = 0, t_pruned = 0, t_visited = 0, t_skipped = 0, t_updated = 0, t_resync = 0;
    // phase clocks of workgroup 0 (lookahead, exchange, merge, apply)
    const bool clocks = tele && g == 0 && tid == 0;
    unsigned long long ph[4] = {0, 0, 0, 0}, t_mark = 0;
    int j = 1;
    uint32_t round = 0;
    while (j < a.m) {
        ++round;
        if (clocks)
            t_mark = wall_clock64();
        // =============== L: local lookahead on a private copy ===============
        for (int lt = tid; lt < ntl; lt += kBlock) {
            tkeyl[lt] = tkey[lt];
            tthrl[lt] = tthr[lt];
            tbestl[lt] = tbest[lt];
            tflag[lt] = 0;
        }
        __syncthreads();
        for (int s = 0; s <= R; ++s) {
            // arg max over the local tile keys (key and tile travel together)
            unsigned long long lk = 0;
            uint32_t lt_best = 0;
            for (int lt = tid; lt < ntl; lt += kBlock) {
                const unsigned long long k = tkeyl[lt];
                if (k > lk) {
                    lk = k;
                    lt_best = (uint32_t)lt;
                }
            }
            const unsigned long long wk = wave_max_u64(lk);
            const unsigned long long hit = __ballot(lk == wk && wk != 0);
            if (lane == 0) {
                s_red[wave] = wk;
                s_redi[wave] = hit ? (uint32_t)__builtin_amdgcn_readlane((int)lt_best, __ffsll((long long)hit) - 1)
                                   : 0u;
            }
            __syncthreads();
            unsigned long long bk = 0;
            uint32_t bt = 0;
#pragma unroll
            for (int q = 0; q < kWavesPerBlock; ++q) {
                if (s_red[q] > bk) {
                    bk = s_red[q];
                    bt = s_redi[q];
                }
            }
            if (s == R || bk == 0) {
                // bound (or an empty workgroup): no more local candidates
                if (tid == 0) {
                    s_my[6 * R] = (uint32_t)(bk >> 32);
                    s_my[6 * R + 1] = (uint32_t)bk;
                    for (int q = s; q < R; ++q) {
                        for (int w = 0; w < 6; ++w)
                            s_my[6 * q + w] = 0;
                    }
                }
                break;
            }
            const uint32_t p = tbestl[bt];
            const float lx = px[p], ly = py[p], lz = pz[p];
            if (tid == 0) {
                s_my[6 * s + 0] = __float_as_uint(lx);
                s_my[6 * s + 1] = __float_as_uint(ly);
                s_my[6 * s + 2] = __float_as_uint(lz);
                s_my[6 * s + 3] = __float_as_uint(pd[p]);
                s_my[6 * s + 4] = po[p];
                s_my[6 * s + 5] = (uint32_t)(bk >> 32);
            }
            // local update with l_s (pruned against the local thresholds)
            for (int lt = tid; lt < ntl; lt += kBlock) {
                const float q = sqdist(tcx[lt], tcy[lt], tcz[lt], lx, ly, lz);
                if (!(q >= tthrl[lt]))
                    tlist[atomicAdd(&s_list_n, 1u)] = (uint32_t)lt;
            }
            __syncthreads();
            const uint32_t nlist = s_list_n;
            for (uint32_t e = wave; e < nlist; e += kWavesPerBlock) {
                const uint32_t lt = tlist[e];
                const uint32_t meta = tmeta[lt];
                const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
                const bool valid = (uint32_t)lane < cnt;
                const uint32_t pp = ls + (valid ? lane : 0);
                if (!tflag[lt]) {
                    if (valid)
                        pdl[pp] = pd[pp];
                }
                float d = pdl[pp];
                bool upd = false;
                if (valid) {
                    const float dx = px[pp] - lx, dy = py[pp] - ly, dz = pz[pp] - lz;
                    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
                    const bool skip = use_skip && (xx >= d || yy >= d || zz >= d);
                    const float s2 = xx + yy;
                    const float t = s2 + zz;
                    upd = !skip && t < d;
                    if (upd) {
                        d = t;
                        pdl[pp] = t;
                    }
                }
                if (lane == 0)
                    tflag[lt] = 1;
                if (__ballot(upd))
                    tile_rekey(lane, lt, ls, cnt, pdl, po, trad, tkeyl, tbestl, tthrl);
            }
            __syncthreads();
            if (tid == 0)
                s_list_n = 0;
        }
        __syncthreads();
        if (clocks) {
            const unsigned long long t = wall_clock64();
            ph[0] += t - t_mark;
            t_mark = t;
        }

        // =============== X: publish and read every slot ===============
        const uint32_t epoch = round;
        unsigned long long t_pub = trace ? wall_clock64() : 0ull;
        if (wave == 0) {
            unsigned long long *slot = a.board + ((size_t)(epoch & 1u) * G + g) * kMaxSlotWords;
            for (int w = lane; w < W; w += kWave)
                if (w != W - 1)
                    st_agent(slot + w, ((unsigned long long)epoch << 32) | s_my[w]);
            if (lane == 0)
                st_agent(slot + W - 1, ((unsigned long long)epoch << 32) | s_my[W - 1]);
        }
        if (tid < G) {
            const unsigned long long *slot = a.board + ((size_t)(epoch & 1u) * G + tid) * kMaxSlotWords;
            bool ok = false;
            for (uint32_t spin = 0; spin < kSpinLimit && !ok; ++spin) {
                const unsigned long long r = ld_agent(slot + W - 1);
                if ((uint32_t)(r >> 32) == kAbortEpoch)
                    break;
                if ((uint32_t)(r >> 32) != epoch)
                    continue;
                uint32_t v[W];
                ok = true;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const unsigned long long x = ld_agent(slot + w);
                    ok &= (uint32_t)(x >> 32) == epoch;
                    v[w] = (uint32_t)x;
                }
                if (ok) {
                    // a workgroup without tiles publishes the bound key 0 and no candidates
                    const bool empty = v[6 * R] == 0u && v[6 * R + 1] == 0u;
#pragma unroll
                    for (int s = 0; s < R; ++s) {
                        const int c = tid * R + s;
                        cx[c] = __uint_as_float(v[6 * s + 0]);
                        cy[c] = __uint_as_float(v[6 * s + 1]);
                        cz[c] = __uint_as_float(v[6 * s + 2]);
                        ctd[c] = __uint_as_float(v[6 * s + 3]);
                        corig[c] = v[6 * s + 4];
                        cld[c] = __uint_as_float(v[6 * s + 5]);
                        bkey[tid * (R + 1) + s] =
                            empty ? 0ull : ((unsigned long long)v[6 * s + 5] << 32) | (~v[6 * s + 4]);
                    }
                    bkey[tid * (R + 1) + R] = ((unsigned long long)v[6 * R] << 32) | v[6 * R + 1];
                }
            }
            if (!ok)
                s_abort = 1;
        }
        __syncthreads();
        if (s_abort) {
            if (tid == 0) {
                set_status(&hdr->sample_status, RFPS_ERR_TIMEOUT);
                for (int par = 0; par < 2; ++par)
                    for (int w = 0; w < W; ++w)
                        st_agent(a.board + ((size_t)par * G + g) * kMaxSlotWords + w,
                                 (unsigned long long)kAbortEpoch << 32);
            }
            return;
        }
        if (clocks) {
            const unsigned long long t = wall_clock64();
            ph[1] += t - t_mark;
            t_mark = t;
        }

        // =============== M: certified merge (wavefront 0) ===============
        if (wave == 0) {
            int hq[4];
            float hx[4], hy[4], hz[4], ht[4], hl[4];
            unsigned long long hk[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gg = lane + kWave * q;
                hq[q] = R;
                hx[q] = hy[q] = hz[q] = ht[q] = hl[q] = 0.0f;
                hk[q] = 0ull;
                if (gg < G) {
                    hk[q] = bkey[gg * (R + 1)];
                    if (hk[q] != 0ull) {
                        hq[q] = 0;
                        hx[q] = cx[gg * R];
                        hy[q] = cy[gg * R];
                        hz[q] = cz[gg * R];
                        ht[q] = ctd[gg * R];
                        hl[q] = cld[gg * R];
                    }
                }
            }
            int P = 0;
            while (j + P < a.m) {
                unsigned long long lb = 0;
                int lq = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (hk[q] > lb) {
                        lb = hk[q];
                        lq = q;
                    }
                }
                const unsigned long long wb = wave_max_u64(lb);
                const unsigned long long hit = __ballot(lb == wb && wb != 0ull);
                if (!hit)
                    break;
                const int L0 = __ffsll((long long)hit) - 1;
                const int bq = __builtin_amdgcn_readlane(lq, L0);
                int mh = R;
                float mx = 0, my = 0, mz = 0, mt = 0, ml = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q == bq) {
                        mh = hq[q];
                        mx = hx[q];
                        my = hy[q];
                        mz = hz[q];
                        mt = ht[q];
                        ml = hl[q];
                    }
                }
                const int oh = __builtin_amdgcn_readlane(mh, L0);
                const float ox = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(mx), L0));
                const float oy = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(my), L0));
                const float oz = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(mz), L0));
                const float ot = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(mt), L0));
                const float ol = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(ml), L0));
                if (oh >= R || !(ot == ol))
                    break;  // bound not attained: the round ends here
                const int gs = L0 + kWave * bq;
                const int cidx = gs * R + oh;
                if (lane == 0) {
                    picks[P] = (uint32_t)cidx;
                    ctd[cidx] = ot;  // distance at selection
                }
                ++P;
                // every other head loses what this pick covers
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (hq[q] < R) {
                        const float d = sqdist(hx[q], hy[q], hz[q], ox, oy, oz);
                        ht[q] = fminf(ht[q], d);
                    }
                }
                // advance the owner's head; its true distance covers every pick so far
                const int nh = oh + 1;
                const unsigned long long nk = bkey[gs * (R + 1) + nh];
                float nx = 0, ny = 0, nz = 0, nt = 0, nl = 0;
                if (nh < R) {
                    nx = cx[gs * R + nh];
                    ny = cy[gs * R + nh];
                    nz = cz[gs * R + nh];
                    nt = ctd[gs * R + nh];
                    nl = cld[gs * R + nh];
                    for (int k = lane; k < P; k += kWave) {
                        const uint32_t pc = picks[k];
                        nt = fminf(nt, sqdist(nx, ny, nz, cx[pc], cy[pc], cz[pc]));
                    }
                    nt = wave_min_dist(nt);
                }
                if (lane == L0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (q == bq) {
                            hq[q] = nh;
                            hx[q] = nx;
                            hy[q] = ny;
                            hz[q] = nz;
                            ht[q] = nt;
                            hl[q] = nl;
                            hk[q] = nk;
                        }
                    }
                }
            }
            if (lane == 0)
                s_npick = (uint32_t)P;
            if (g == 0) {
                for (int k = lane; k < P; k += kWave) {
                    const uint32_t pc = picks[k];
                    a.out_idx[j + k] = (int32_t)corig[pc];
                    if (a.out_d2)
                        a.out_d2[j + k] = ctd[pc];
                }
            }
        }
        __syncthreads();
        const int P = (int)s_npick;
        if (P == 0) {
            // impossible by construction (the largest bound is attained at round
            // start); kept as a guard so a violated invariant cannot spin forever
            if (tid == 0)
                set_status(&hdr->sample_status, RFPS_ERR_INTERNAL);
            return;
        }
        if (trace && round - 1 < (uint32_t)kTraceCap) {
            a.trace[2 * (size_t)(round - 1)] = t_pub;
            a.trace[2 * (size_t)(round - 1) + 1] = wall_clock64() | ((unsigned long long)P << 48);
        }
        if (clocks) {
            const unsigned long long t = wall_clock64();
            ph[2] += t - t_mark;
            t_mark = t;
        }
        j += P;
        if (j >= a.m)
            break;

        // =============== A: apply the round's picks to the true state ===============
        for (int lt = tid; lt < ntl; lt += kBlock) {
            const float thr = tthr[lt];
            const float ccx = tcx[lt], ccy = tcy[lt], ccz = tcz[lt];
            int k = 0;
            for (; k < P; ++k) {
                const uint32_t pc = picks[k];
                const float q = sqdist(ccx, ccy, ccz, cx[pc], cy[pc], cz[pc]);
                if (!(q >= thr))
                    break;
            }
            t_tests += (k < P) ? (unsigned long long)(k + 1) : (unsigned long long)P;
            t_pruned += (unsigned long long)k;
            if (k < P)
                tlist[atomicAdd(&s_list_n, 1u)] = (uint32_t)lt | ((uint32_t)k << 20);
        }
        __syncthreads();
        const uint32_t nlist = s_list_n;
        for (uint32_t e = wave; e < nlist; e += kWavesPerBlock) {
            const uint32_t lt = tlist[e] & 0xfffffu;
            const int k0 = (int)(tlist[e] >> 20);
            const uint32_t meta = tmeta[lt];
            const uint32_t ls = meta & 0xffffu, cnt = meta >> 16;
            const bool valid = (uint32_t)lane < cnt;
            const uint32_t pp = ls + (valid ? lane : 0);
            const float thr = tthr[lt];
            const float ccx = tcx[lt], ccy = tcy[lt], ccz = tcz[lt];
            const float x = px[pp], y = py[pp], z = pz[pp];
            float d = pd[pp];
            bool changed = false;
            for (int k = k0; k < P; ++k) {
                const uint32_t pc = picks[k];
                const float sx = cx[pc], sy = cy[pc], sz = cz[pc];
                if (k > k0 && sqdist(ccx, ccy, ccz, sx, sy, sz) >= thr)
                    continue;  // uniform across the wave
                if (tele && lane == 0) {
                    t_visited += cnt;
                    t_tests += (k > k0);
                }
                if (valid) {
                    const float dx = x - sx, dy = y - sy, dz = z - sz;
                    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
                    const bool skip = use_skip && (xx >= d || yy >= d || zz >= d);
                    const float s2 = xx + yy;
                    const float t = s2 + zz;
                    if (!skip && t < d) {
                        d = t;
                        changed = true;
                    }
                    t_skipped += skip;
                }
            }
            if (changed)
                pd[pp] = d;
            const unsigned long long um = __ballot(changed);
            if (tele && lane == 0) {
                t_updated += (unsigned long long)__popcll(um);
                t_resync += um != 0;
            }
            if (um)
                tile_rekey(lane, lt, ls, cnt, pd, po, trad, tkey, tbest, tthr);
        }
        __syncthreads();
        if (tid == 0)
            s_list_n = 0;
        if (clocks)
            ph[3] += wall_clock64() - t_mark;
    }

    if (clocks) {
        for (int q = 0; q < 4; ++q)
            atomicAdd(&hdr->tele[kTeleTicksLookahead + q], ph[q]);
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
            atomicAdd(&hdr->tele[8], (unsigned long long)round);
        }
    }
    if (g == 0 && tid == 0)
        hdr->trace_n = round;
}

template __global__ void k_rfps_rounds<2>(RoundArgs);
template __global__ void k_rfps_rounds<4>(RoundArgs);
template __global__ void k_rfps_rounds<8>(RoundArgs);

size_t rfps_rounds_static_lds(int R)
{
    const void *fn = R == 2   ? reinterpret_cast<const void *>(k_rfps_rounds<2>)
                     : R == 4 ? reinterpret_cast<const void *>(k_rfps_rounds<4>)
                     : R == 8 ? reinterpret_cast<const void *>(k_rfps_rounds<8>)
                              : nullptr;
    hipFuncAttributes attr;
    if (!fn || hipFuncGetAttributes(&attr, fn) != hipSuccess)
        return 0;
    return attr.sharedSizeBytes;
}

hipError_t launch_rfps_rounds(const IndexView &v, int m, int start, const SampleLaunch &L, int32_t *out_idx,
                              float *out_d2, hipStream_t s)
{
    k_rounds_plan<<<(L.G + kBlock - 1) / kBlock, kBlock, 0, s>>>(v.hdr, v.tcnt, L.G, L.R, L.lds_budget);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || m <= 1)
        return e;
    const void *fn = L.R == 2   ? reinterpret_cast<const void *>(k_rfps_rounds<2>)
                     : L.R == 4 ? reinterpret_cast<const void *>(k_rfps_rounds<4>)
                     : L.R == 8 ? reinterpret_cast<const void *>(k_rfps_rounds<8>)
                                : nullptr;
    if (!fn)
        return hipErrorInvalidValue;
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
    void *args[] = {&a};
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_budget);
    if (e != hipSuccess)
        return e;
    return hipLaunchCooperativeKernel(fn, dim3(L.G), dim3(kBlock), args, L.lds_budget, s);
}

}  // namespace rfps
