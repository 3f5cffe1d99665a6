// Voxel-parameter network: cloud features, forward pass, gradient and Adam
// training step (C ABI in include/rfps_mlp.h).
//
// The network maps 516 features of a cloud (log N, the bounding-box extents
// and the 8^3 occupancy histogram) through two hidden layers of 64 ReLU
// units to 72 outputs: a predicted relative log run time and a pruning rate
// for each of 36 candidate (n_vox, shell spacing) pairs.  Weight matrices are used in
// bfloat16 (round to nearest even of an FP32 master copy); biases,
// activations, accumulation and the optimiser state are FP32.  Whatever the
// network picks, the sampled sequence is the same (every partition is
// output-neutral); it only changes the speed.
//
// The products run on the matrix cores: v_mfma_f32_16x16x4f32, one 16 x 16
// output tile per wavefront, operands read straight from device memory (the
// matrices are at most 2048 x 516: the whole training step is a few
// microseconds of arithmetic and is bound by launch latency, not by HBM).
#include <math.h>

#include <algorithm>

#include "../../include/rfps_mlp.h"
#include "rfps_internal.h"

namespace rfps {
namespace mlp {

constexpr int kIn = RFPS_MLP_INPUTS, kH = 64, kOut = RFPS_MLP_OUTPUTS;
constexpr int kP = RFPS_MLP_PARAMS;
// packed parameter order: W1 [64][516], b1 [64], W2 [64][64], b2 [64], W3 [72][64], b3 [72]
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kOut * kH, oEnd = ob3 + kOut;
static_assert(oEnd == kP, "parameter count");

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;
constexpr int kMaxRows = 1 << 16;  // rows of one forward or training call

// Candidate table: n_vox major, shell spacing minor (0 = one shell).
constexpr int kNVox[9] = {12, 16, 24, 32, 48, 64, 96, 128, 192};
constexpr float kShell[4] = {0.0f, 5.0f, 10.0f, 20.0f};

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float load_op(const float *p) { return *p; }
__device__ __forceinline__ float load_op(const uint16_t *p) { return bf16_to_f32(*p); }

enum Epi : int {
    kPlain = 0,    // C = acc
    kBiasRelu = 1, // C = acc + bias[n]; C2 = max(C, 0)
    kBias = 2,     // C = acc + bias[n]
    kMask = 3,     // C = acc where mask[m][n] > 0, else 0
};

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m*sam + k*sak] and
// B(k, n) = B[k*sbk + n*sbn] (the strides express any transposition).
// Block = 4 wavefronts = a 32 x 32 tile of C; each wavefront accumulates a
// 16 x 16 tile over K in steps of 4.  Operand lanes: A element (i, k) in
// lane i + 16k, B element (k, j) in lane j + 16k; result element (i, j) in
// lane j + 16 (i / 4), component i % 4.
template <typename TB, int EPI>
__global__ __launch_bounds__(256) void k_mm(const float *__restrict__ A, int sam, int sak, const TB *__restrict__ B,
                                            int sbk, int sbn, float *__restrict__ C, float *__restrict__ C2,
                                            const float *__restrict__ aux, int M, int N, int K)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 32 + (wave >> 1) * 16, n0 = blockIdx.x * 32 + (wave & 1) * 16;
    const int li = lane & 15, lk = lane >> 4;
    const int am = m0 + li, bn = n0 + li;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        const float a = (am < M && k < K) ? A[(size_t)am * sam + (size_t)k * sak] : 0.0f;
        const float b = (bn < N && k < K) ? load_op(B + (size_t)k * sbk + (size_t)bn * sbn) : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    const int n = n0 + li;
    if (n >= N)
        return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = m0 + 4 * lk + r;
        if (m >= M)
            continue;
        float v = acc[r];
        const size_t o = (size_t)m * N + n;
        if constexpr (EPI == kBiasRelu) {
            v += aux[n];
            C[o] = v;
            C2[o] = v > 0.0f ? v : 0.0f;
        } else if constexpr (EPI == kBias) {
            C[o] = v + aux[n];
        } else if constexpr (EPI == kMask) {
            C[o] = aux[o] > 0.0f ? v : 0.0f;
        } else {
            C[o] = v;
        }
    }
}

template <typename TB, int EPI>
static void mm(const float *A, int sam, int sak, const TB *B, int sbk, int sbn, float *C, float *C2, const float *aux,
               int M, int N, int K, hipStream_t s)
{
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    k_mm<TB, EPI><<<grid, 256, 0, s>>>(A, sam, sak, B, sbk, sbn, C, C2, aux, M, N, K);
}

// dY = 2 w (Y - T) / B and the loss sum w (Y - T)^2 / B (one workgroup,
// fixed reduction order).
__global__ __launch_bounds__(1024) void k_loss(const float *__restrict__ Y, const float *__restrict__ T,
                                               const float *__restrict__ Wt, int total, int B,
                                               float *__restrict__ dY, float *__restrict__ loss)
{
    __shared__ double part[1024];
    double acc = 0.0;
    const float sc = 2.0f / (float)B;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const float w = Wt ? Wt[e] : 1.0f;
        const float d = Y[e] - T[e];
        dY[e] = sc * w * d;
        acc += (double)w * (double)d * (double)d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss)
        *loss = (float)(part[0] / (double)B);
}

// db[n] = sum_m dZ[m][n], one thread per column.
__global__ void k_colsum(const float *__restrict__ dZ, int M, int N, float *__restrict__ db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N)
        return;
    float s = 0.0f;
    for (int m = 0; m < M; ++m)
        s += dZ[(size_t)m * N + n];
    db[n] = s;
}

// Model state in the caller's memory (rfps_mlp_state_size bytes).
struct State {
    float *master, *m, *v;
    uint16_t *wbf;   // bf16 copy of master (packed like it; only the weight blocks are read)
    uint32_t *step;  // Adam steps taken
};

__global__ void k_step_inc(uint32_t *step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *step += 1u;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              uint16_t *__restrict__ wbf, const float *__restrict__ g,
                                              const uint32_t *__restrict__ step, float lr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kP)
        return;
    const float t = (float)*step;
    const float gi = g[i];
    const float mi = kBeta1 * m[i] + (1.0f - kBeta1) * gi;
    const float vi = kBeta2 * v[i] + (1.0f - kBeta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(kBeta1, t));
    const float vh = vi / (1.0f - powf(kBeta2, t));
    const float wi = w[i] - lr * mh / (sqrtf(vh) + kEps);
    w[i] = wi;
    wbf[i] = f32_to_bf16(wi);
}

// Load: master from the caller, moments and step cleared, bf16 copy made.
__global__ __launch_bounds__(256) void k_load(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              uint16_t *__restrict__ wbf, uint32_t *__restrict__ step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0)
        *step = 0u;
    if (i >= kP)
        return;
    m[i] = 0.0f;
    v[i] = 0.0f;
    wbf[i] = f32_to_bf16(w[i]);
}

// ---------------------------------------------------------------------------
// Features: bounding box, 8^3 occupancy histogram over a cubic grid of edge
// (1 + 1e-4) max(E) / 8 from the box minimum (FP64, clamped), then
// f0 = (ln N - 11) / 2, f1..3 = ln(1 + E_a) / 2, f(4 + cell) =
// ln(1 + 64 count / N) (the logarithm tames the dense near-sensor cells of
// a spinning scan).
// ---------------------------------------------------------------------------
struct FeatScratch {
    uint32_t status;
    uint32_t bb[6];
    uint32_t pad;
    uint32_t counts[512];
};

__global__ void k_feat_reset(FeatScratch *fs)
{
    const int t = threadIdx.x;
    if (t == 0)
        fs->status = 0;
    if (t < 3) {
        fs->bb[t] = 0xffffffffu;
        fs->bb[3 + t] = 0u;
    }
    for (int c = t; c < 512; c += blockDim.x)
        fs->counts[c] = 0;
}

__global__ __launch_bounds__(kBlock) void k_feat_bbox(const float *__restrict__ xyz, int n, FeatScratch *fs)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * (size_t)i + a];
            bad |= !isfinite(v);
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
    __shared__ float s_mn[3][kWavesPerBlock], s_mx[3][kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = wave_min_f32(mn[a]), hi = wave_max_f32(mx[a]);
        if (lane == 0) {
            s_mn[a][w] = lo;
            s_mx[a][w] = hi;
        }
    }
    if (__any(bad) && lane == 0)
        atomicOr(&fs->status, 1u);
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        float lo = s_mn[a][0], hi = s_mx[a][0];
        for (int q = 1; q < kWavesPerBlock; ++q) {
            lo = fminf(lo, s_mn[a][q]);
            hi = fmaxf(hi, s_mx[a][q]);
        }
        if (lo <= hi) {
            atomicMin(&fs->bb[a], f2ord(lo));
            atomicMax(&fs->bb[3 + a], f2ord(hi));
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_feat_hist(const float *__restrict__ xyz, int n, FeatScratch *fs)
{
    __shared__ uint32_t h[512];
    for (int c = threadIdx.x; c < 512; c += blockDim.x)
        h[c] = 0;
    double lo[3], emax = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = (double)ord2f(fs->bb[a]);
        const double e = (double)ord2f(fs->bb[3 + a]) - lo[a];
        emax = e > emax ? e : emax;
    }
    const double edge = (emax > 0.0 && emax < INFINITY) ? (1.0 + 1e-4) * emax / 8.0 : 1.0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int b[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double q = floor(((double)xyz[3 * (size_t)i + a] - lo[a]) / edge);
            q = q > 0.0 ? q : 0.0;
            q = q < 7.0 ? q : 7.0;
            b[a] = (int)q;
        }
        atomicAdd(&h[(b[2] * 8 + b[1]) * 8 + b[0]], 1u);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < 512; c += blockDim.x)
        if (h[c])
            atomicAdd(&fs->counts[c], h[c]);
}

__global__ void k_feat_final(int n, const FeatScratch *__restrict__ fs, float *__restrict__ f)
{
    for (int t = threadIdx.x; t < kIn; t += blockDim.x) {
        double v;
        if (t == 0) {
            v = (log((double)n) - 11.0) / 2.0;
        } else if (t < 4) {
            const int a = t - 1;
            v = log1p((double)ord2f(fs->bb[3 + a]) - (double)ord2f(fs->bb[a])) / 2.0;
        } else {
            v = log1p(64.0 * (double)fs->counts[t - 4] / (double)n);
        }
        f[t] = fs->status ? __uint_as_float(0x7fc00000u) : (float)v;
    }
}

// Pick: the candidate with the lowest predicted log time, unless it does
// not beat the default candidate's prediction by `margin`.
__global__ void k_choose(const float *__restrict__ y, int default_cand, float margin, int32_t *__restrict__ choice)
{
    if (threadIdx.x != 0)
        return;
    int best = default_cand;
    float bv = y[default_cand];
    for (int k = 0; k < RFPS_MLP_CANDIDATES; ++k)
        if (y[k] < bv) {
            bv = y[k];
            best = k;
        }
    const float yd = y[default_cand];
    *choice = (isfinite(bv) && bv < yd - margin) ? best : default_cand;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
inline size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct StateLayout {
    size_t master, m, v, wbf, step, total;
};
StateLayout state_layout()
{
    StateLayout L;
    L.master = 0;
    L.m = up(L.master + 4 * (size_t)kP);
    L.v = up(L.m + 4 * (size_t)kP);
    L.wbf = up(L.v + 4 * (size_t)kP);
    L.step = up(L.wbf + 2 * (size_t)kP);
    L.total = up(L.step + 4);
    return L;
}

State state_view(void *p)
{
    const StateLayout L = state_layout();
    unsigned char *b = static_cast<unsigned char *>(p);
    State s;
    s.master = reinterpret_cast<float *>(b + L.master);
    s.m = reinterpret_cast<float *>(b + L.m);
    s.v = reinterpret_cast<float *>(b + L.v);
    s.wbf = reinterpret_cast<uint16_t *>(b + L.wbf);
    s.step = reinterpret_cast<uint32_t *>(b + L.step);
    return s;
}

struct WsLayout {
    size_t feat, z1, a1, z2, a2, y, dy, dz2, dz1, grad, loss, total;
};
WsLayout ws_layout(int B)
{
    WsLayout L;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = up(cur);
        cur = o + bytes;
        return o;
    };
    const size_t b = (size_t)B;
    L.feat = take(sizeof(FeatScratch));
    L.z1 = take(4 * b * kH);
    L.a1 = take(4 * b * kH);
    L.z2 = take(4 * b * kH);
    L.a2 = take(4 * b * kH);
    L.y = take(4 * b * kOut);
    L.dy = take(4 * b * kOut);
    L.dz2 = take(4 * b * kH);
    L.dz1 = take(4 * b * kH);
    L.grad = take(4 * (size_t)kP);
    L.loss = take(4);
    L.total = up(cur);
    return L;
}

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<unsigned char *>(ws) + off);
}

// Forward pass of B rows: Z1, A1, Z2, A2 and Y in the workspace.
void forward(const State &st, const float *x, int B, void *ws, const WsLayout &L, float *y, hipStream_t s)
{
    float *z1 = at<float>(ws, L.z1), *a1 = at<float>(ws, L.a1), *z2 = at<float>(ws, L.z2),
          *a2 = at<float>(ws, L.a2);
    mm<uint16_t, kBiasRelu>(x, kIn, 1, st.wbf + oW1, 1, kIn, z1, a1, st.master + ob1, B, kH, kIn, s);
    mm<uint16_t, kBiasRelu>(a1, kH, 1, st.wbf + oW2, 1, kH, z2, a2, st.master + ob2, B, kH, kH, s);
    mm<uint16_t, kBias>(a2, kH, 1, st.wbf + oW3, 1, kH, y, nullptr, st.master + ob3, B, kOut, kH, s);
}

// Gradient of the loss with respect to the packed parameters into `grad`.
void backward(const State &st, const float *x, const float *t, const float *wt, int B, void *ws, const WsLayout &L,
              float *grad, float *loss, hipStream_t s)
{
    float *z1 = at<float>(ws, L.z1), *a1 = at<float>(ws, L.a1), *z2 = at<float>(ws, L.z2),
          *a2 = at<float>(ws, L.a2), *y = at<float>(ws, L.y), *dy = at<float>(ws, L.dy),
          *dz2 = at<float>(ws, L.dz2), *dz1 = at<float>(ws, L.dz1);
    forward(st, x, B, ws, L, y, s);
    k_loss<<<1, 1024, 0, s>>>(y, t, wt, B * kOut, B, dy, loss);
    // layer 3
    mm<float, kPlain>(dy, 1, kOut, a2, kH, 1, grad + oW3, nullptr, nullptr, kOut, kH, B, s);
    k_colsum<<<1, 128, 0, s>>>(dy, B, kOut, grad + ob3);
    mm<uint16_t, kMask>(dy, kOut, 1, st.wbf + oW3, kH, 1, dz2, nullptr, z2, B, kH, kOut, s);
    // layer 2
    mm<float, kPlain>(dz2, 1, kH, a1, kH, 1, grad + oW2, nullptr, nullptr, kH, kH, B, s);
    k_colsum<<<1, 128, 0, s>>>(dz2, B, kH, grad + ob2);
    mm<uint16_t, kMask>(dz2, kH, 1, st.wbf + oW2, kH, 1, dz1, nullptr, z1, B, kH, kH, s);
    // layer 1
    mm<float, kPlain>(dz1, 1, kH, x, kIn, 1, grad + oW1, nullptr, nullptr, kH, kIn, B, s);
    k_colsum<<<1, 128, 0, s>>>(dz1, B, kH, grad + ob1);
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

}  // namespace mlp
}  // namespace rfps

using namespace rfps::mlp;

extern "C" {

int32_t rfps_mlp_candidate(int32_t k, int32_t *n_vox, float *shell_spacing)
{
    if (k < 0 || k >= RFPS_MLP_CANDIDATES)
        return 1;
    if (n_vox)
        *n_vox = kNVox[k / 4];
    if (shell_spacing)
        *shell_spacing = kShell[k % 4];
    return 0;
}

size_t rfps_mlp_state_size(void) { return state_layout().total; }

size_t rfps_mlp_workspace_size(int32_t batch)
{
    if (batch < 1 || batch > kMaxRows)
        return 0;
    return ws_layout(batch).total;
}

static rfps_status check_state(const void *state, size_t bytes)
{
    if (!state || !aligned(state) || bytes < state_layout().total)
        return RFPS_ERR_WORKSPACE;
    return RFPS_OK;
}

static rfps_status check_ws(const void *ws, size_t bytes, int batch)
{
    if (batch < 1 || batch > kMaxRows)
        return RFPS_ERR_INVALID_ARG;
    if (!ws || !aligned(ws) || bytes < ws_layout(batch).total)
        return RFPS_ERR_WORKSPACE;
    return RFPS_OK;
}

static rfps_status launched(hipStream_t s)
{
    (void)s;
    return hipGetLastError() == hipSuccess ? RFPS_OK : RFPS_ERR_DEVICE;
}

rfps_status rfps_mlp_load(void *state, size_t state_bytes, const float *params, void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r != RFPS_OK)
        return r;
    if (!params)
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    State st = state_view(state);
    if (hipMemcpyAsync(st.master, params, 4 * (size_t)kP, hipMemcpyHostToDevice, s) != hipSuccess)
        return RFPS_ERR_DEVICE;
    k_load<<<(kP + 255) / 256, 256, 0, s>>>(st.master, st.m, st.v, st.wbf, st.step);
    if (launched(s) != RFPS_OK || hipStreamSynchronize(s) != hipSuccess)
        return RFPS_ERR_DEVICE;
    return RFPS_OK;
}

rfps_status rfps_mlp_save(const void *state, size_t state_bytes, float *params, void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r != RFPS_OK)
        return r;
    if (!params)
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess)
        return RFPS_ERR_DEVICE;
    State st = state_view(const_cast<void *>(state));
    if (hipMemcpy(params, st.master, 4 * (size_t)kP, hipMemcpyDeviceToHost) != hipSuccess)
        return RFPS_ERR_DEVICE;
    return RFPS_OK;
}

rfps_status rfps_mlp_features(const float *xyz, int32_t n, void *ws, size_t ws_bytes, float *feat, void *stream)
{
    if (!xyz || !feat || n < 1 || n > rfps::kMaxPoints)
        return RFPS_ERR_INVALID_ARG;
    rfps_status r = check_ws(ws, ws_bytes, 1);
    if (r != RFPS_OK)
        return r;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    FeatScratch *fs = at<FeatScratch>(ws, ws_layout(1).feat);
    const int blocks = std::min((n + 1023) / 1024, 512);
    k_feat_reset<<<1, 256, 0, s>>>(fs);
    k_feat_bbox<<<blocks, rfps::kBlock, 0, s>>>(xyz, n, fs);
    k_feat_hist<<<blocks, rfps::kBlock, 0, s>>>(xyz, n, fs);
    k_feat_final<<<1, 256, 0, s>>>(n, fs, feat);
    return launched(s);
}

rfps_status rfps_mlp_forward(const void *state, size_t state_bytes, const float *x, int32_t batch, void *ws,
                             size_t ws_bytes, float *y, void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r == RFPS_OK)
        r = check_ws(ws, ws_bytes, batch);
    if (r != RFPS_OK)
        return r;
    if (!x || !y)
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    forward(state_view(const_cast<void *>(state)), x, batch, ws, ws_layout(batch), y, s);
    return launched(s);
}

rfps_status rfps_mlp_gradient(const void *state, size_t state_bytes, const float *x, const float *t,
                              const float *w, int32_t batch, void *ws, size_t ws_bytes, float *grad, float *loss,
                              void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r == RFPS_OK)
        r = check_ws(ws, ws_bytes, batch);
    if (r != RFPS_OK)
        return r;
    if (!x || !t || !grad)
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout L = ws_layout(batch);
    backward(state_view(const_cast<void *>(state)), x, t, w, batch, ws, L, grad, loss ? loss : at<float>(ws, L.loss),
             s);
    return launched(s);
}

rfps_status rfps_mlp_train_step(void *state, size_t state_bytes, const float *x, const float *t, const float *w,
                                int32_t batch, float lr, void *ws, size_t ws_bytes, float *loss, void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r == RFPS_OK)
        r = check_ws(ws, ws_bytes, batch);
    if (r != RFPS_OK)
        return r;
    if (!x || !t || !(lr > 0.0f) || !isfinite(lr))
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout L = ws_layout(batch);
    const State st = state_view(state);
    float *grad = at<float>(ws, L.grad);
    backward(st, x, t, w, batch, ws, L, grad, loss ? loss : at<float>(ws, L.loss), s);
    k_step_inc<<<1, 64, 0, s>>>(st.step);
    k_adam<<<(kP + 255) / 256, 256, 0, s>>>(st.master, st.m, st.v, st.wbf, grad, st.step, lr);
    return launched(s);
}

rfps_status rfps_mlp_choose(const void *state, size_t state_bytes, const float *feat, int32_t default_cand,
                            float margin, void *ws, size_t ws_bytes, int32_t *choice, float *y, void *stream)
{
    rfps_status r = check_state(state, state_bytes);
    if (r == RFPS_OK)
        r = check_ws(ws, ws_bytes, 1);
    if (r != RFPS_OK)
        return r;
    if (!feat || !choice || default_cand < 0 || default_cand >= RFPS_MLP_CANDIDATES || !(margin >= 0.0f))
        return RFPS_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout L = ws_layout(1);
    float *out = y ? y : at<float>(ws, L.y);
    forward(state_view(const_cast<void *>(state)), feat, 1, ws, L, out, s);
    k_choose<<<1, 64, 0, s>>>(out, default_cand, margin, choice);
    return launched(s);
}

}  // extern "C"
