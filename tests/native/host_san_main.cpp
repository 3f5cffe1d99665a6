// Driver of the sanitizer build of librfps's host code: every source of the
// library compiled with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host side only (the device code is built as usual and never launched),
// run by tests/test_sanitizers.py on a machine that may have no GPU.
//
//   host_san <cloud.f32> <m> <expected_idx.i32> <expected_d2.f32>
//
// 1. Calls every entry point with arguments the host must refuse and checks
//    the documented status; none of these calls reaches the device.
// 2. Runs the CPU sampler (rfps_cpu_sample) on the cloud with several team
//    sizes, grids and tiles and compares it with the expected selections,
//    which the test computes with the plain FPS oracle.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/rfps.h"

static int g_bad = 0;

#ifdef CPU_SAMPLER_ONLY
// Built with the CPU sampler's source alone (the ThreadSanitizer build): the
// library's default-grid rule lives in another source, and this driver
// always passes n_vox explicitly in that build.
extern "C" int32_t rfps_default_n_vox(int32_t) { abort(); }
extern "C" const char *rfps_status_str(rfps_status) { return "status"; }
#endif

static void expect(const char *what, int got, int want)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        g_bad = 1;
    }
}

template <typename T>
static bool read_all(const char *path, std::vector<T> &out)
{
    FILE *f = fopen(path, "rb");
    if (!f)
        return false;
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    out.resize((size_t)bytes / sizeof(T));
    const bool ok = fread(out.data(), sizeof(T), out.size(), f) == out.size();
    fclose(f);
    return ok;
}

#ifndef CPU_SAMPLER_ONLY
static void argument_checks()
{
    // a stand-in for device memory: the host refuses every call below before
    // any pointer is used
    alignas(256) static unsigned char fake[4096];
    void *ws = fake;
    float *xyz = reinterpret_cast<float *>(fake);
    int32_t *iv = reinterpret_cast<int32_t *>(fake);
    float *fv = reinterpret_cast<float *>(fake);
    rfps_params p = {0, 0, 0, 0, 0u, 0.0f};
    rfps_index ix;

    expect("workspace size n=0", rfps_index_workspace_size(0, nullptr) == 0, 1);
    expect("workspace size n=2^26+1", rfps_index_workspace_size((1 << 26) + 1, nullptr) == 0, 1);
    expect("workspace size n=1000", rfps_index_workspace_size(1000, nullptr) > 0, 1);
    rfps_params bad = p;
    bad.n_vox = 1025;
    expect("workspace size n_vox 1025", rfps_index_workspace_size(1000, &bad) == 0, 1);
    bad = p;
    bad.lookahead = 5;
    expect("workspace size lookahead 5", rfps_index_workspace_size(1000, &bad) == 0, 1);
    bad = p;
    bad.shell_spacing = -1.0f;
    expect("workspace size negative spacing", rfps_index_workspace_size(1000, &bad) == 0, 1);
    bad = p;
    bad.flags = 0x80000000u;
    expect("workspace size unknown flag", rfps_index_workspace_size(1000, &bad) == 0, 1);

    expect("build null xyz", rfps_build_index(nullptr, 10, &p, ws, sizeof fake, nullptr, &ix), RFPS_ERR_INVALID_ARG);
    expect("build n=0", rfps_build_index(xyz, 0, &p, ws, sizeof fake, nullptr, &ix), RFPS_ERR_INVALID_ARG);
    expect("build null out", rfps_build_index(xyz, 10, &p, ws, sizeof fake, nullptr, nullptr), RFPS_ERR_INVALID_ARG);
    expect("build small ws", rfps_build_index(xyz, 100000, &p, ws, sizeof fake, nullptr, &ix), RFPS_ERR_WORKSPACE);
    expect("build misaligned ws", rfps_build_index(xyz, 10, &p, fake + 8, sizeof fake - 8, nullptr, &ix),
           RFPS_ERR_WORKSPACE);

    rfps_index h = {100, 8, 64, 1, ws, sizeof fake};
    expect("sample small ws", rfps_sample(&h, 10, 0, nullptr, iv, fv, nullptr), RFPS_ERR_WORKSPACE);
    h.ws_bytes = (size_t)1 << 40;  // large enough for the layout; the host refuses before using it
    expect("sample m=0", rfps_sample(&h, 0, 0, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("sample m>n", rfps_sample(&h, 101, 0, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("sample start=n", rfps_sample(&h, 10, 100, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("sample start<0", rfps_sample(&h, 10, -1, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("sample null out", rfps_sample(&h, 10, 0, nullptr, nullptr, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("sample null index", rfps_sample(nullptr, 10, 0, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    rfps_index hb = h;
    hb.n_vox = 0;
    expect("sample bad handle", rfps_sample(&hb, 10, 0, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    hb = h;
    hb.n_vox = 1024;
    hb.shells = 64;  // n^3 * shells above 2^32
    expect("sample key overflow", rfps_sample(&hb, 10, 0, nullptr, iv, fv, nullptr), RFPS_ERR_INVALID_ARG);
    rfps_params unf = p;
    unf.flags = RFPS_F_UNFUSED | RFPS_F_TELEMETRY;
    expect("sample unfused+telemetry", rfps_sample(&h, 10, 0, &unf, iv, fv, nullptr), RFPS_ERR_UNSUPPORTED);

    expect("gather null", rfps_gather_xyz(xyz, 10, nullptr, 5, fv, nullptr), RFPS_ERR_INVALID_ARG);
    expect("gather m=0", rfps_gather_xyz(xyz, 10, iv, 0, fv, nullptr), RFPS_ERR_INVALID_ARG);

    expect("plain ws size variant 2", rfps_fps_plain_workspace_size(10, 2) == 0, 1);
    expect("plain m>n", rfps_fps_plain(xyz, 10, 11, 0, 0, 0, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_INVALID_ARG);
    expect("plain groups>256", rfps_fps_plain(xyz, 10, 5, 0, 0, 257, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_INVALID_ARG);
    expect("plain small ws", rfps_fps_plain(xyz, 100000, 5, 0, 0, 0, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_WORKSPACE);
    expect("plain status small ws", rfps_read_plain_status(ws, 8, nullptr), RFPS_ERR_WORKSPACE);

    int32_t off[3] = {0, 5, 10}, mm[2] = {2, 2};
    expect("batched ws size batch>n", rfps_batched_workspace_size(4, 5, nullptr) == 0, 1);
    expect("batched ws size batch 4097", rfps_batched_workspace_size(100000, 4097, nullptr) == 0, 1);
    expect("batched null offsets",
           rfps_sample_batched(xyz, 10, nullptr, mm, nullptr, 2, 4, nullptr, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_INVALID_ARG);
    expect("batched m_total<batch",
           rfps_sample_batched(xyz, 10, off, mm, nullptr, 2, 1, nullptr, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_INVALID_ARG);
    expect("batched m_total>n",
           rfps_sample_batched(xyz, 10, off, mm, nullptr, 2, 11, nullptr, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_INVALID_ARG);
    rfps_params np = p;
    np.flags = RFPS_F_NO_PRUNE;
    expect("batched no-prune",
           rfps_sample_batched(xyz, 10, off, mm, nullptr, 2, 4, &np, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_UNSUPPORTED);
    expect("batched small ws",
           rfps_sample_batched(xyz, 100000, off, mm, nullptr, 2, 4, nullptr, ws, sizeof fake, iv, fv, nullptr),
           RFPS_ERR_WORKSPACE);
    expect("batched telemetry null", rfps_batched_read_telemetry(ws, sizeof fake, nullptr, nullptr),
           RFPS_ERR_INVALID_ARG);
    expect("autotune reps 0",
           rfps_autotune_batched(xyz, 10, off, mm, nullptr, 2, 4, nullptr, 0, ws, sizeof fake, iv, fv, nullptr, &np,
                                 nullptr),
           RFPS_ERR_INVALID_ARG);

    for (int s = 0; s <= 9; ++s)
        if (!rfps_status_str((rfps_status)s) || !*rfps_status_str((rfps_status)s))
            g_bad = 1;
}
#endif

int main(int argc, char **argv)
{
    std::vector<float> xyz, d2ref;
    std::vector<int32_t> iref;
    if (argc < 5 || !read_all(argv[1], xyz) || !read_all(argv[3], iref) || !read_all(argv[4], d2ref)) {
        fprintf(stderr, "usage: %s cloud.f32 m expected_idx.i32 expected_d2.f32\n", argv[0]);
        return 2;
    }
    const int n = (int)(xyz.size() / 3), m = atoi(argv[2]);
    if ((int)iref.size() != m || (int)d2ref.size() != m)
        return 2;
#ifndef CPU_SAMPLER_ONLY
    argument_checks();
    const int grids[] = {0, 4, 16};
#else
    const int grids[] = {4, 16};
#endif
    std::vector<int32_t> idx(m);
    std::vector<float> d2(m);
    const int teams[] = {1, 2, 3, 4};
    const int tiles[] = {0, 5};
    for (int t : teams)
        for (int g : grids)
            for (int tl : tiles) {
                rfps_params p = {g, tl, 0, 0, 0u, 0.0f};
                const rfps_status st = rfps_cpu_sample(xyz.data(), n, m, 0, &p, t, idx.data(), d2.data());
                if (st != RFPS_OK || memcmp(idx.data(), iref.data(), 4 * (size_t)m) != 0 ||
                    memcmp(d2.data(), d2ref.data(), 4 * (size_t)m) != 0) {
                    fprintf(stderr, "rfps_cpu_sample differs: threads %d n_vox %d tile %d status %d\n", t, g, tl,
                            (int)st);
                    g_bad = 1;
                }
            }
    rfps_params p8 = {8, 0, 0, 0, 0u, 0.0f};
    expect("cpu m>n", rfps_cpu_sample(xyz.data(), n, n + 1, 0, &p8, 1, idx.data(), d2.data()),
           RFPS_ERR_INVALID_ARG);
    std::vector<float> nanc(xyz);
    nanc[3 * (n / 2) + 1] = __builtin_nanf("");
    expect("cpu non-finite", rfps_cpu_sample(nanc.data(), n, m, 0, &p8, 2, idx.data(), d2.data()),
           RFPS_ERR_NONFINITE);
    if (idx[0] != -1)
        g_bad = 1;
    printf("%s n=%d m=%d\n", g_bad ? "FAIL" : "ok", n, m);
    return g_bad;
}
