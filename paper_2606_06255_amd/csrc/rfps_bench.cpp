// rfps_bench: native driver of the C ABI (include/rfps.h).
//
//   rfps_bench <cloud.f32> <m> [steps] [n_vox] [groups] [plain_variant] [copy_mb]
//   rfps_bench --batch <clouds.f32> <offsets.i32> [steps] [groups] [lookahead]
//
// <cloud.f32> holds n*3 little-endian float32 values (x, y, z per point).
// Runs `steps` times build + sample (RadiusFPS-G), or with plain_variant 0/1
// the plain comparison kernels, and prints the mean time per cloud.  With
// --batch, <offsets.i32> holds the batch+1 int32 cloud offsets and every cloud
// is sampled to N_c / 4 points by rfps_sample_batched.  Meant for profilers
// that should see only the library's kernels.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/rfps.h"

#define CHECK_HIP(x)                                                                   \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));             \
            return 1;                                                                  \
        }                                                                              \
    } while (0)
#define CHECK_RFPS(x)                                                                  \
    do {                                                                               \
        rfps_status s_ = (x);                                                          \
        if (s_ != RFPS_OK) {                                                           \
            fprintf(stderr, "%s failed: %s\n", #x, rfps_status_str(s_));               \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

static bool read_file(const char *path, std::vector<char> &out)
{
    FILE *f = fopen(path, "rb");
    if (!f) {
        perror(path);
        return false;
    }
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    out.resize((size_t)bytes);
    const bool ok = fread(out.data(), 1, (size_t)bytes, f) == (size_t)bytes;
    fclose(f);
    return ok;
}

static int run_batch(int argc, char **argv)
{
    std::vector<char> cb, ob;
    if (argc < 4 || !read_file(argv[2], cb) || !read_file(argv[3], ob)) {
        fprintf(stderr, "usage: %s --batch clouds.f32 offsets.i32 [steps] [groups] [lookahead]\n", argv[0]);
        return 2;
    }
    const int n = (int)(cb.size() / 12);
    const int batch = (int)(ob.size() / 4) - 1;
    const int32_t *off = reinterpret_cast<const int32_t *>(ob.data());
    const int steps = argc > 4 ? atoi(argv[4]) : 3;
    rfps_params p = {0, 0, argc > 5 ? atoi(argv[5]) : 0, argc > 6 ? atoi(argv[6]) : 0, 0u, 0.0f};
    std::vector<int32_t> m(batch);
    int m_total = 0;
    for (int c = 0; c < batch; ++c) {
        m[c] = (off[c + 1] - off[c]) / 4;
        m[c] = m[c] < 1 ? 1 : m[c];
        m_total += m[c];
    }
    float *xyz, *d2;
    int32_t *idx, *doff, *dm;
    void *ws;
    const size_t ws_bytes = rfps_batched_workspace_size(n, batch, &p);
    if (ws_bytes == 0 || batch < 1) {
        fprintf(stderr, "bad size or parameters\n");
        return 2;
    }
    CHECK_HIP(hipMalloc(&xyz, cb.size()));
    CHECK_HIP(hipMalloc(&doff, ob.size()));
    CHECK_HIP(hipMalloc(&dm, 4 * (size_t)batch));
    CHECK_HIP(hipMalloc(&idx, 4 * (size_t)m_total));
    CHECK_HIP(hipMalloc(&d2, 4 * (size_t)m_total));
    CHECK_HIP(hipMalloc(&ws, ws_bytes));
    CHECK_HIP(hipMemcpy(xyz, cb.data(), cb.size(), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(doff, ob.data(), ob.size(), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dm, m.data(), 4 * (size_t)batch, hipMemcpyHostToDevice));
    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    hipEvent_t a, b;
    CHECK_HIP(hipEventCreate(&a));
    CHECK_HIP(hipEventCreate(&b));
    for (int k = 0; k <= steps; ++k) {
        if (k == 1)
            CHECK_HIP(hipEventRecord(a, s));  // step 0 is the warm-up
        CHECK_RFPS(rfps_sample_batched(xyz, n, doff, dm, nullptr, batch, m_total, &p, ws, ws_bytes, idx, d2, s));
    }
    CHECK_HIP(hipEventRecord(b, s));
    CHECK_HIP(hipEventSynchronize(b));
    float ms = 0.0f;
    CHECK_HIP(hipEventElapsedTime(&ms, a, b));
    const rfps_status st = rfps_batched_read_status(ws, ws_bytes, s);
    printf("batch=%d n=%d m_total=%d steps=%d RadiusFPS-G batched: %.3f ms per batch, status=%s\n", batch, n,
           m_total, steps, steps > 0 ? ms / steps : 0.0f, rfps_status_str(st));
    fflush(stdout);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(ws);
    hipFree(d2);
    hipFree(idx);
    hipFree(dm);
    hipFree(doff);
    hipFree(xyz);
    hipStreamDestroy(s);
    return st == RFPS_OK ? 0 : 1;
}

int main(int argc, char **argv)
{
    // every HIP object this driver creates (events, stream, buffers) is
    // released before main returns, so none is left for the runtime's
    // teardown after an attached profiler has finalised
    if (argc > 1 && strcmp(argv[1], "--batch") == 0)
        return run_batch(argc, argv);
    if (argc < 3) {
        fprintf(stderr, "usage: %s cloud.f32 m [steps] [n_vox] [groups] [plain_variant] [copy_mb] [flags]\n",
                argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) {
        perror(argv[1]);
        return 1;
    }
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    const int n = (int)(bytes / 12);
    std::vector<float> h((size_t)n * 3);
    if (fread(h.data(), 12, (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "short read\n");
        return 1;
    }
    fclose(f);
    const int m = atoi(argv[2]);
    const int steps = argc > 3 ? atoi(argv[3]) : 3;
    rfps_params p = {argc > 4 ? atoi(argv[4]) : 0, 0, argc > 5 ? atoi(argv[5]) : 0, 0, 0u, 0.0f};
    const int plain = argc > 6 ? atoi(argv[6]) : -1;
    p.flags = argc > 8 ? (uint32_t)strtoul(argv[8], nullptr, 0) : 0u;  // RFPS_F_* bits of the sampler

    float *xyz, *d2;
    int32_t *idx;
    void *ws;
    CHECK_HIP(hipMalloc(&xyz, (size_t)n * 12));
    CHECK_HIP(hipMalloc(&idx, (size_t)m * 4));
    CHECK_HIP(hipMalloc(&d2, (size_t)m * 4));
    CHECK_HIP(hipMemcpy(xyz, h.data(), (size_t)n * 12, hipMemcpyHostToDevice));
    const size_t ws_bytes =
        plain >= 0 ? rfps_fps_plain_workspace_size(n, plain) : rfps_index_workspace_size(n, &p);
    if (ws_bytes == 0) {
        fprintf(stderr, "bad size or parameters\n");
        return 2;
    }
    CHECK_HIP(hipMalloc(&ws, ws_bytes));
    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    hipEvent_t a, b;
    CHECK_HIP(hipEventCreate(&a));
    CHECK_HIP(hipEventCreate(&b));
    rfps_index index;
    for (int k = 0; k <= steps; ++k) {
        if (k == 1)
            CHECK_HIP(hipEventRecord(a, s));  // step 0 is the warm-up
        if (plain >= 0) {
            CHECK_RFPS(rfps_fps_plain(xyz, n, m, 0, plain, p.groups, ws, ws_bytes, idx, d2, s));
        } else {
            CHECK_RFPS(rfps_build_index(xyz, n, &p, ws, ws_bytes, s, &index));
            CHECK_RFPS(rfps_sample(&index, m, 0, &p, idx, d2, s));
        }
    }
    CHECK_HIP(hipEventRecord(b, s));
    CHECK_HIP(hipEventSynchronize(b));
    float ms = 0.0f;
    CHECK_HIP(hipEventElapsedTime(&ms, a, b));
    rfps_status st = plain >= 0 ? rfps_read_plain_status(ws, ws_bytes, s) : rfps_read_status(&index, s);
    std::vector<int32_t> out(m);
    CHECK_HIP(hipMemcpy(out.data(), idx, (size_t)m * 4, hipMemcpyDeviceToHost));
    // optional: one device-to-device copy of copy_mb MiB, a kernel of known
    // traffic against which hardware byte counters can be scaled
    const int copy_mb = argc > 7 ? atoi(argv[7]) : 0;
    if (copy_mb > 0) {
        void *src, *dst;
        const size_t cb = (size_t)copy_mb << 20;
        CHECK_HIP(hipMalloc(&src, cb));
        CHECK_HIP(hipMalloc(&dst, cb));
        CHECK_HIP(hipMemsetAsync(src, 1, cb, s));
        CHECK_HIP(hipMemcpyAsync(dst, src, cb, hipMemcpyDeviceToDevice, s));
        CHECK_HIP(hipStreamSynchronize(s));
        printf("copied %zu bytes device to device\n", cb);
        hipFree(src);
        hipFree(dst);
    }
    printf("n=%d m=%d steps=%d %s: %.3f ms per cloud, status=%s, idx[1..3]=%d %d %d\n", n, m, steps,
           plain >= 0 ? (plain ? "plain one-workgroup" : "plain persistent") : "RadiusFPS-G",
           steps > 0 ? ms / steps : 0.0f, rfps_status_str(st), m > 1 ? out[1] : -1, m > 2 ? out[2] : -1,
           m > 3 ? out[3] : -1);
    fflush(stdout);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(ws);
    hipFree(d2);
    hipFree(idx);
    hipFree(xyz);
    hipStreamDestroy(s);
    return st == RFPS_OK ? 0 : 1;
}
