/*
 * ORACLE -- test infrastructure, not product code.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load or call anything in this directory.  It shares no source, header or
 * constant with the device path.
 *
 * Plain farthest point sampling, written as the paper's standard FPS
 * (Algorithm 1, Sec. 2.1) with the exactness contract of Sec. 3.1 (same seed,
 * same precision, arg max returns the smallest original index among equal
 * distances).
 *
 * Reading of the paper used here:
 *   - the distance state and every reported distance is the FP32 *squared*
 *     Euclidean distance, evaluated as ((dx*dx + dy*dy) + dz*dz) with
 *     dx = fl(p_x - s_x) and no fused multiply-add (build with
 *     -ffp-contract=off);
 *   - the seed is the caller's start index; the first reported distance is
 *     +inf (Algorithm 1 initialises D to +inf);
 *   - the update is strict: D[i] changes only when the new distance is
 *     smaller (Sec. 3.4.2, equality case).
 *
 * oracle_fps_euclid is the same definition with the Euclidean distance of
 * the update rule of Sec. 3.4.3 (eq. point_distance_update): d(p, s) = sqrtf
 * of the squared distance
 * above, correctly rounded as IEEE 754 requires of sqrtf.  Its state and
 * reported distances are these FP32 norms.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math [-fopenmp] -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(__FAST_MATH__)
#error "the oracle must not be built with fast-math"
#endif

/* Squared distance between p and s in FP32, fixed association. */
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

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * xyz: [n][3] float32, row-major.  Writes out_idx[m] (original indices) and,
 * if out_d2 is not NULL, out_d2[m] (the selected point's D at selection).
 * threads <= 0 uses the OpenMP default; threads == 1 is single-threaded.
 * euclid != 0 uses the Euclidean distance instead of its square.
 * Returns 0 on success, 1 on invalid arguments, 2 on a non-finite coordinate,
 * 3 when out of memory.
 */
static int fps_plain(const float *xyz, int64_t n, int64_t m, int64_t start,
                     int32_t *out_idx, float *out_d2, int threads, int euclid)
{
    if (!xyz || !out_idx || n < 1 || m < 1 || m > n || start < 0 || start >= n)
        return 1;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(xyz[i]))
            return 2;
    float *D = (float *)malloc((size_t)n * sizeof(float));
    if (!D)
        return 3;
#ifdef _OPENMP
    int nt = threads > 0 ? threads : omp_get_max_threads();
#else
    int nt = 1;
    (void)threads;
#endif

    /* Algorithm 1: D <- +inf, S <- {start}. */
    for (int64_t i = 0; i < n; ++i)
        D[i] = INFINITY;
    int64_t last = start;
    out_idx[0] = (int32_t)start;
    if (out_d2)
        out_d2[0] = INFINITY;

    for (int64_t j = 1; j < m; ++j) {
        const float sx = xyz[3 * last], sy = xyz[3 * last + 1], sz = xyz[3 * last + 2];
        /* D[i] <- min(D[i], d(p_i, s_last)), strict. */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
        for (int64_t i = 0; i < n; ++i) {
            float t = sqdist(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], sx, sy, sz);
            if (euclid)
                t = sqrtf(t);
            if (t < D[i])
                D[i] = t;
        }
        /* p_next <- arg max_i D[i], smallest index among equal maxima. */
        float best = -1.0f;
        int64_t bi = -1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
        {
            float lb = -1.0f;
            int64_t li = -1;
#ifdef _OPENMP
#pragma omp for schedule(static) nowait
#endif
            for (int64_t i = 0; i < n; ++i) {
                if (D[i] > lb) {
                    lb = D[i];
                    li = i;
                }
            }
#ifdef _OPENMP
#pragma omp critical
#endif
            {
                if (li >= 0 && (lb > best || (lb == best && li < bi))) {
                    best = lb;
                    bi = li;
                }
            }
        }
        out_idx[j] = (int32_t)bi;
        if (out_d2)
            out_d2[j] = best;
        last = bi;
    }
    free(D);
    return 0;
}

int oracle_fps(const float *xyz, int64_t n, int64_t m, int64_t start,
               int32_t *out_idx, float *out_d2, int threads)
{
    return fps_plain(xyz, n, m, start, out_idx, out_d2, threads, 0);
}

int oracle_fps_euclid(const float *xyz, int64_t n, int64_t m, int64_t start,
                      int32_t *out_idx, float *out_d2, int threads)
{
    return fps_plain(xyz, n, m, start, out_idx, out_d2, threads, 1);
}
