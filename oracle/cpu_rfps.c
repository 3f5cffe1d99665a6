/*
 * ORACLE -- test infrastructure, not product code.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load or call anything in this directory.  It shares no source, header or
 * constant with the device path.
 *
 * CPU RadiusFPS: the paper's spherical-voxel method (Sec. 3) written as a
 * second, independent CPU implementation.  Its only job is to pin the
 * pruning logic: for every voxel resolution and every split of voxels into
 * tiles it must return exactly the index and distance sequence of the plain
 * oracle (fps_oracle.c).
 *
 * Steps, in the paper's order:
 *   Preprocessing (Sec. 3.2): bounding box, E, L = alpha * max(E) / n_vox,
 *     clamped voxel coordinates, V_id = v_z n^2 + v_y n + v_x, active voxels,
 *     voxel centre c_k and enclosing sphere radius r_k.
 *   Initial update (Sec. 3.3): Dist_p[i] = d(p_i, s_0); Dist_v[k] = max over
 *     the voxel.
 *   Iterative sampling (Sec. 3.4): two-level arg max (eq. best_voxel, then
 *     eq. best_point), spherical-voxel pruning (eq. spherical_voxel_bound,
 *     eq. radius_pruning_condition), coordinate-wise point skip
 *     (eq. point_skip_condition), exact update (eq. point_distance_update)
 *     and Dist_v resync (eq. point_skip_distv_sync).
 *
 * Readings (same as the plain oracle, plus):
 *   - Dist_p holds FP32 squared distances; the skip test compares the FP32
 *     square of one coordinate difference with Dist_p (exact: the rounded sum
 *     of non-negative squares is never below one of its terms);
 *   - the voxel level carries (Dist_v, lowest original index attaining it),
 *     which is how "the same tie-breaking at both levels" is made exact;
 *   - r_k is the largest member distance to c_k, computed in FP64 and
 *     inflated; with RFPS_CPU_PAPER_RADIUS it is sqrt(3)/2 L (eq.
 *     preprocess_voxel_radius), raised to the member radius if rounding at a
 *     cube face put a member outside;
 *   - the pruning test is evaluated in FP64 with a margin that covers the
 *     rounding of the FP32 squared distance (see prune_safe below);
 *   - alpha = 1 + 1e-4; if max(E) == 0, L = 1.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if defined(__FAST_MATH__)
#error "the oracle must not be built with fast-math"
#endif

/* option bits */
#define RFPS_CPU_NO_PRUNE 1u       /* visit every voxel */
#define RFPS_CPU_NO_SKIP 2u        /* no point skip */
#define RFPS_CPU_PAPER_RADIUS 4u   /* r_k = sqrt(3)/2 L */
/* planted mistakes, used only to show that the tests catch them */
#define RFPS_CPU_MUT_CENTROID 256u /* prune on ||s - c_k|| alone (unsafe, Sec. 3.4.2) */
#define RFPS_CPU_MUT_HALF_RADIUS 512u /* use r_k / 2 */

typedef struct {
    int64_t iters;            /* update rounds (M - 1) */
    int64_t voxels;           /* K, number of active voxels (or tiles) */
    int64_t voxel_tests;      /* sphere tests evaluated */
    int64_t voxels_pruned;    /* tests that pruned */
    int64_t points_visited;   /* points in unpruned voxels */
    int64_t points_skipped;   /* of those, removed by the point skip */
    int64_t points_updated;   /* strict decreases of Dist_p */
} rfps_cpu_telemetry;

static inline float sqdist(float px, float py, float pz, float sx, float sy, float sz)
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

/*
 * Voxel grid of Sec. 3.2.  Writes pmin (FP64 copy of the FP32 minimum) and
 * L, and the voxel id of every point.  Returns 0, or 2 on a non-finite
 * coordinate.
 */
int rfps_cpu_voxelize(const float *xyz, int64_t n, int32_t n_vox, double *pmin_L /*[4]*/,
                      uint32_t *vid)
{
    float mn[3], mx[3];
    for (int a = 0; a < 3; ++a) {
        mn[a] = xyz[a];
        mx[a] = xyz[a];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = xyz[3 * i + a];
            if (!isfinite(v))
                return 2;
            if (v < mn[a])
                mn[a] = v;
            if (v > mx[a])
                mx[a] = v;
        }
    double E = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = (double)mx[a] - (double)mn[a];
        if (e > E)
            E = e;
    }
    const double alpha = 1.0 + 1e-4;
    double L = E > 0.0 ? alpha * E / (double)n_vox : 1.0;
    for (int a = 0; a < 3; ++a)
        pmin_L[a] = (double)mn[a];
    pmin_L[3] = L;
    const uint32_t nv = (uint32_t)n_vox;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t v[3];
        for (int a = 0; a < 3; ++a) {
            double q = floor(((double)xyz[3 * i + a] - pmin_L[a]) / L);
            if (q < 0.0)
                q = 0.0;
            if (q > (double)(nv - 1))
                q = (double)(nv - 1);
            v[a] = (uint32_t)q;
        }
        vid[i] = v[2] * nv * nv + v[1] * nv + v[0];
    }
    return 0;
}

/*
 * Conservative spherical-voxel test (eq. spherical_voxel_bound and
 * eq. radius_pruning_condition), made safe under rounding.
 *
 * In real arithmetic every member p satisfies ||p - s|| >= ||s - c|| - r
 * (eq. triangle_inequality_bound).  The FP32 squared distance the update
 * computes is at least (1 - 2^-24)^5 ||p - s||^2 (five roundings of
 * non-negative quantities), so a voxel may be skipped when
 *     (||s - c|| - r)^2 * (1 - 2^-20) >= Dist_v
 * with ||s - c|| - r evaluated in FP64 and lowered by 2^-44 (||s - c|| + r)
 * to absorb the FP64 error of both terms, including cancellation.  A voxel
 * whose Dist_v is 0 is always skipped (nothing is below 0); one whose Dist_v
 * is positive but below 2^-100 is always visited, which keeps the bound away
 * from FP32 subnormals.
 */
static int prune_safe(double sx, double sy, double sz, const double *c, double r, float dv)
{
    if (dv == 0.0f)
        return 1;
    if (!(dv >= 0x1p-100f))
        return 0;
    double ex = sx - c[0], ey = sy - c[1], ez = sz - c[2];
    double delta = sqrt(ex * ex + ey * ey + ez * ez);
    double lb = (delta - r) - 0x1p-44 * (delta + r);
    if (!(lb > 0.0))
        return 0;
    return lb * lb * (1.0 - 0x1p-20) >= (double)dv;
}

typedef struct {
    int64_t begin, count;  /* range in the voxel-sorted member list */
    double c[3];           /* voxel centre */
    double r;              /* enclosing radius */
    float dv;              /* Dist_v */
    int64_t dv_idx;        /* lowest original index attaining Dist_v */
} cpu_voxel;

typedef struct { uint32_t vid; int64_t i; } vid_pair;

static int cmp_pair(const void *a, const void *b)
{
    const vid_pair *x = (const vid_pair *)a, *y = (const vid_pair *)b;
    if (x->vid != y->vid)
        return x->vid < y->vid ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/* Dist_v resync over one voxel (eq. point_skip_distv_sync). */
static void resync(cpu_voxel *v, const int64_t *member, const float *D)
{
    float best = -1.0f;
    int64_t bi = -1;
    for (int64_t q = 0; q < v->count; ++q) {
        int64_t i = member[v->begin + q];
        if (D[i] > best || (D[i] == best && i < bi)) {
            best = D[i];
            bi = i;
        }
    }
    v->dv = best;
    v->dv_idx = bi;
}

/*
 * xyz [n][3] float32.  n_vox >= 1 voxel bins per axis.  tile >= 1 splits
 * every voxel into consecutive runs of at most `tile` members (each run gets
 * its own radius about the voxel centre and its own Dist_v); tile <= 0 keeps
 * whole voxels.  opts: RFPS_CPU_* bits.  tel may be NULL.
 * Returns 0, 1 invalid arguments, 2 non-finite input, 3 out of memory.
 */
int rfps_cpu_sample(const float *xyz, int64_t n, int64_t m, int64_t start, int32_t n_vox,
                    int32_t tile, uint32_t opts, int32_t *out_idx, float *out_d2,
                    rfps_cpu_telemetry *tel)
{
    if (!xyz || !out_idx || n < 1 || m < 1 || m > n || start < 0 || start >= n || n_vox < 1 ||
        n_vox > 1625)
        return 1;
    int rc = 0;
    double g[4];
    uint32_t *vid = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    vid_pair *pr = (vid_pair *)malloc((size_t)n * sizeof(vid_pair));
    int64_t *member = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    float *D = (float *)malloc((size_t)n * sizeof(float));
    cpu_voxel *vox = (cpu_voxel *)malloc((size_t)n * sizeof(cpu_voxel));
    if (!vid || !pr || !member || !D || !vox) {
        rc = 3;
        goto done;
    }
    if (rfps_cpu_voxelize(xyz, n, n_vox, g, vid)) {
        rc = 2;
        goto done;
    }
    const double L = g[3];

    /* Active voxels: group the points by V_id. */
    for (int64_t i = 0; i < n; ++i) {
        pr[i].vid = vid[i];
        pr[i].i = i;
    }
    qsort(pr, (size_t)n, sizeof(vid_pair), cmp_pair);
    for (int64_t q = 0; q < n; ++q)
        member[q] = pr[q].i;
    int64_t K = 0;
    const uint32_t nv = (uint32_t)n_vox;
    for (int64_t q = 0; q < n;) {
        int64_t e = q;
        while (e < n && pr[e].vid == pr[q].vid)
            ++e;
        uint32_t id = pr[q].vid;
        double cc[3];
        uint32_t vv[3] = {id % nv, (id / nv) % nv, id / (nv * nv)};
        for (int a = 0; a < 3; ++a)
            cc[a] = g[a] + ((double)vv[a] + 0.5) * L;
        int64_t step = tile > 0 ? tile : (e - q);
        for (int64_t b = q; b < e; b += step) {
            cpu_voxel *v = &vox[K++];
            v->begin = b;
            v->count = (b + step <= e) ? step : (e - b);
            memcpy(v->c, cc, sizeof cc);
            double r2 = 0.0;
            for (int64_t t = 0; t < v->count; ++t) {
                const float *p = xyz + 3 * member[b + t];
                double dx = (double)p[0] - cc[0], dy = (double)p[1] - cc[1],
                       dz = (double)p[2] - cc[2];
                double d = dx * dx + dy * dy + dz * dz;
                if (d > r2)
                    r2 = d;
            }
            double r = sqrt(r2) * (1.0 + 0x1p-40) + 0x1p-100;
            if (opts & RFPS_CPU_PAPER_RADIUS) {
                double rp = 0.5 * sqrt(3.0) * L * (1.0 + 0x1p-40);
                v->r = rp > r ? rp : r;
            } else {
                v->r = r;
            }
            if (opts & RFPS_CPU_MUT_HALF_RADIUS)
                v->r *= 0.5;
        }
        q = e;
    }

    /* Initial update: Dist_p from the seed, Dist_v per voxel. */
    {
        const float *s = xyz + 3 * start;
        for (int64_t i = 0; i < n; ++i)
            D[i] = sqdist(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], s[0], s[1], s[2]);
        for (int64_t k = 0; k < K; ++k)
            resync(&vox[k], member, D);
    }
    out_idx[0] = (int32_t)start;
    if (out_d2)
        out_d2[0] = INFINITY;
    rfps_cpu_telemetry T;
    memset(&T, 0, sizeof T);
    T.voxels = K;

    for (int64_t j = 1; j < m; ++j) {
        /* eq. best_voxel: arg max over Dist_v, ties to the lowest index. */
        int64_t kb = 0;
        for (int64_t k = 1; k < K; ++k)
            if (vox[k].dv > vox[kb].dv || (vox[k].dv == vox[kb].dv && vox[k].dv_idx < vox[kb].dv_idx))
                kb = k;
        /* eq. best_point: arg max inside that voxel, same tie-break. */
        float bd = -1.0f;
        int64_t bi = -1;
        for (int64_t q = 0; q < vox[kb].count; ++q) {
            int64_t i = member[vox[kb].begin + q];
            if (D[i] > bd || (D[i] == bd && i < bi)) {
                bd = D[i];
                bi = i;
            }
        }
        out_idx[j] = (int32_t)bi;
        if (out_d2)
            out_d2[j] = bd;
        if (j == m - 1)
            break;

        const float sx = xyz[3 * bi], sy = xyz[3 * bi + 1], sz = xyz[3 * bi + 2];
        T.iters++;
        for (int64_t k = 0; k < K; ++k) {
            cpu_voxel *v = &vox[k];
            if (!(opts & RFPS_CPU_NO_PRUNE)) {
                T.voxel_tests++;
                int pruned;
                if (opts & RFPS_CPU_MUT_CENTROID) {
                    double ex = sx - v->c[0], ey = sy - v->c[1], ez = sz - v->c[2];
                    pruned = ex * ex + ey * ey + ez * ez >= (double)v->dv;
                } else {
                    pruned = prune_safe(sx, sy, sz, v->c, v->r, v->dv);
                }
                if (pruned) {
                    T.voxels_pruned++;
                    continue;
                }
            }
            int changed = 0;
            for (int64_t q = 0; q < v->count; ++q) {
                int64_t i = member[v->begin + q];
                const float *p = xyz + 3 * i;
                T.points_visited++;
                if (!(opts & RFPS_CPU_NO_SKIP)) {
                    float dx = p[0] - sx, dy = p[1] - sy, dz = p[2] - sz;
                    float xx = dx * dx, yy = dy * dy, zz = dz * dz;
                    if (xx >= D[i] || yy >= D[i] || zz >= D[i]) {
                        T.points_skipped++;
                        continue;
                    }
                }
                float t = sqdist(p[0], p[1], p[2], sx, sy, sz);
                if (t < D[i]) {
                    D[i] = t;
                    T.points_updated++;
                    changed = 1;
                }
            }
            if (changed)
                resync(v, member, D);
        }
    }
    if (tel)
        *tel = T;
done:
    free(vid);
    free(pr);
    free(member);
    free(D);
    free(vox);
    return rc;
}
