/*
 * Driver of the sanitizer build of the oracle (fps_oracle.c, cpu_rfps.c):
 * compiled with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py and run on the clouds that test writes.
 *
 *   oracle_san <cloud.f32> <m> <start>
 *
 * Runs plain FPS (one and two threads, both distance forms) and the CPU
 * RadiusFPS for several grids, tile splits and options, and exits non-zero
 * when any of them disagree or an argument check does not reject a bad call.
 * The sanitizers abort the process on the first error they find.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t iters, voxels, voxel_tests, voxels_pruned, points_visited, points_skipped, points_updated;
} telemetry;

int oracle_fps(const float *xyz, int64_t n, int64_t m, int64_t start, int32_t *out_idx, float *out_d2,
               int threads);
int oracle_fps_euclid(const float *xyz, int64_t n, int64_t m, int64_t start, int32_t *out_idx, float *out_d2,
                      int threads);
int rfps_cpu_sample(const float *xyz, int64_t n, int64_t m, int64_t start, int32_t n_vox, int32_t tile,
                    uint32_t opts, int32_t *out_idx, float *out_d2, telemetry *tel);

static int same(const int32_t *ia, const float *da, const int32_t *ib, const float *db, int64_t m)
{
    return memcmp(ia, ib, (size_t)m * 4) == 0 && memcmp(da, db, (size_t)m * 4) == 0;
}

int main(int argc, char **argv)
{
    if (argc < 4) {
        fprintf(stderr, "usage: %s cloud.f32 m start\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f)
        return 2;
    fseek(f, 0, SEEK_END);
    const int64_t n = ftell(f) / 12;
    fseek(f, 0, SEEK_SET);
    float *xyz = (float *)malloc((size_t)(n > 0 ? n : 1) * 12);
    if (fread(xyz, 12, (size_t)n, f) != (size_t)n)
        return 2;
    fclose(f);
    const int64_t m = atoll(argv[2]), start = atoll(argv[3]);
    int32_t *ia = (int32_t *)malloc((size_t)m * 4), *ib = (int32_t *)malloc((size_t)m * 4);
    float *da = (float *)malloc((size_t)m * 4), *db = (float *)malloc((size_t)m * 4);
    int bad = 0;

    if (oracle_fps(xyz, n, m, start, ia, da, 1) != 0)
        return 3;
    if (oracle_fps(xyz, n, m, start, ib, db, 2) != 0 || !same(ia, da, ib, db, m)) {
        fprintf(stderr, "threaded oracle differs\n");
        bad = 1;
    }
    const int32_t grids[] = {1, 3, 8, 24, 64};
    const int32_t tiles[] = {0, 1, 7, 64};
    const uint32_t opts[] = {0u, 1u, 2u, 4u};
    for (int g = 0; g < 5; ++g)
        for (int t = 0; t < 4; ++t)
            for (int o = 0; o < 4; ++o) {
                telemetry tel;
                memset(ib, 0, (size_t)m * 4);
                if (rfps_cpu_sample(xyz, n, m, start, grids[g], tiles[t], opts[o], ib, db, &tel) != 0 ||
                    !same(ia, da, ib, db, m)) {
                    fprintf(stderr, "CPU RadiusFPS differs: n_vox %d tile %d opts %u\n", grids[g], tiles[t],
                            opts[o]);
                    bad = 1;
                }
            }
    if (oracle_fps_euclid(xyz, n, m, start, ia, da, 2) != 0)
        return 3;
    if (oracle_fps_euclid(xyz, n, m, start, ib, db, 1) != 0 || !same(ia, da, ib, db, m)) {
        fprintf(stderr, "threaded Euclidean oracle differs\n");
        bad = 1;
    }
    /* argument checks: each must be refused without touching the buffers */
    if (rfps_cpu_sample(xyz, n, n + 1, 0, 8, 0, 0u, ib, db, NULL) == 0 ||
        rfps_cpu_sample(xyz, n, m, n, 8, 0, 0u, ib, db, NULL) == 0 ||
        rfps_cpu_sample(xyz, n, m, start, 0, 0, 0u, ib, db, NULL) == 0 ||
        rfps_cpu_sample(NULL, n, m, start, 8, 0, 0u, ib, db, NULL) == 0) {
        fprintf(stderr, "an invalid call was accepted\n");
        bad = 1;
    }
    free(xyz);
    free(ia);
    free(ib);
    free(da);
    free(db);
    printf("%s n=%lld m=%lld\n", bad ? "FAIL" : "ok", (long long)n, (long long)m);
    return bad;
}
