// The FP-safe form of the spherical pruning bound (Sec. 3.4.2, eq.
// radius_pruning_condition and eq. radius_pruning_correctness), shared by
// the GPU samplers and the CPU sampler of librfps: one definition, compiled
// for the device by hipcc and for the host by any C++ compiler.
//
// A tile with enclosing radius R (rounded up) and tile distance dv (the
// largest Dist_p of its members) is skipped for sample s when the FP32 value
// q = fl32(||s - c||^2), computed with the point-distance formula
// ((dx*dx + dy*dy) + dz*dz), satisfies q >= thr(R, dv).  Why that is safe
// (u = 2^-24, the unit roundoff of FP32):
//   - the formula rounds five times along any path (a subtraction that
//     enters squared, one product, two sums), so q lies within a factor
//     (1 +- u)^5 of the exact squared distance, barring underflow;
//   - thr >= (R + sqrt(dv / (1 - 2^-20)))^2 (1 + 2^-20) (shown below), and
//     (1 + 2^-20) >= (1 + u)^5, so q >= thr gives
//     ||s - c|| >= R + sqrt(dv / (1 - 2^-20));
//   - by the triangle inequality (eq. triangle_inequality_bound) every
//     member p then has ||p - s||^2 >= dv / (1 - 2^-20);
//   - its FP32 squared distance is at least (1 - u)^5 ||p - s||^2 >= dv,
//     since (1 - u)^5 >= 1 - 2^-20, so it is >= dv >= Dist_p[p] and the
//     strict update cannot fire.
// The threshold is evaluated in FP32, each step rounded to nearest:
//   a = fl(dv * k1), k1 = 1 + 2^-20 + 2^-22: a >= dv k1 (1 - u) >= dv / (1 - 2^-20);
//   b = sqrt(a), within one unit in the last place: b >= sqrt(a) (1 - 2u);
//   t = fl(R + b) >= (R + sqrt(a)) (1 - 2u) (1 - u);
//   thr = fl(fl(t * t) * k2) >= (R + sqrt(a))^2 (1 - 2u)^2 (1 - u)^4 k2, and
//   k2 = 1 + 2^-19 >= (1 + 2^-20) / ((1 - 2u)^2 (1 - u)^4).
// dv == 0 means no member can decrease (thr = 0 always skips); dv below
// 2^-100 or above 2^100, or a square beyond the FP32 range, gives NaN, which
// never skips and keeps the bound clear of subnormals and overflow.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#if defined(__HIP__)
#define RFPS_HOST_DEVICE __host__ __device__
#else
#define RFPS_HOST_DEVICE
#endif

namespace rfps {

// Margins of the production bound: the factor on dv before the root and the
// factor on the square (both exact in FP32).
constexpr float kPruneInner = 1.0f + 0x1p-20f + 0x1p-22f;
constexpr float kPruneOuter = 1.0f + 0x1p-19f;

RFPS_HOST_DEVICE inline float prune_nan()
{
    const uint32_t u = 0x7fc00000u;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// The bound with explicit margins (the production ones are the defaults of
// prune_threshold below); a margin of exactly 1 removes that safeguard.
RFPS_HOST_DEVICE inline float prune_threshold_with(float R, float dv, float inner, float outer)
{
    if (dv == 0.0f)
        return 0.0f;
    if (!(dv >= 0x1p-100f) || !(dv <= 0x1p100f))
        return prune_nan();
    const float a = dv * inner;
    const float t = R + sqrtf(a);
    const float t2 = t * t;
    if (!(t2 <= 3.0e38f))
        return prune_nan();
    return t2 * outer;
}

RFPS_HOST_DEVICE inline float prune_threshold(float R, float dv)
{
    return prune_threshold_with(R, dv, kPruneInner, kPruneOuter);
}

}  // namespace rfps
