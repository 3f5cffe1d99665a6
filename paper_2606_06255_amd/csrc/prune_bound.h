// The FP-safe form of the spherical pruning bound (Sec. 3.4.2, eq.
// radius_pruning_condition and eq. radius_pruning_correctness), shared by
// the GPU samplers and the CPU sampler of librfps: one definition, compiled
// for the device by hipcc and for the host by any C++ compiler.
//
// A tile with enclosing radius R (rounded up) and tile distance dv (the
// largest Dist_p of its members) is skipped for sample s when the FP32 value
// q = fl32(||s - c||^2), computed with the point-distance formula
// ((dx*dx + dy*dy) + dz*dz), satisfies q >= thr(R, dv).  Why that is safe:
//   - the formula rounds five times (three subtractions enter squared, one
//     product, two sums), so fl32(x) lies within a factor (1 +- 2^-24)^5 of
//     the exact squared distance x, barring underflow;
//   - thr >= (R + sqrt(dv / (1 - 2^-20)))^2 (1 + 2^-20) and
//     (1 + 2^-20) >= (1 + 2^-24)^5, so q >= thr gives
//     ||s - c|| >= R + sqrt(dv / (1 - 2^-20));
//   - by the triangle inequality (eq. triangle_inequality_bound) every
//     member p then has ||p - s||^2 >= dv / (1 - 2^-20);
//   - its FP32 squared distance is at least (1 - 2^-24)^5 ||p - s||^2 >= dv,
//     since (1 - 2^-24)^5 >= 1 - 2^-20, so it is >= dv >= Dist_p[p] and the
//     strict update cannot fire.
// The FP64 evaluation is rounded up: dv (1 + 2^-19) >= dv / (1 - 2^-20), and
// each remaining FP64 step (product, root, sum, square) is enlarged by a
// factor 1 + 2^-50, far above its rounding error of 2^-53.  The result is
// rounded up to FP32.  dv == 0 means no member can decrease (thr = 0 always
// skips); dv below 2^-100 or above 2^100 gives NaN, which never skips and
// keeps the bound clear of subnormals and overflow.
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

// Margins of the production bound: the factor inside the root, the factor
// applied to the squared sum, and the slack of each FP64 step.
constexpr double kPruneInner = 1.0 + 0x1p-19;
constexpr double kPruneOuter = 1.0 + 0x1p-20;
constexpr double kPruneStep = 1.0 + 0x1p-50;

RFPS_HOST_DEVICE inline float prune_nan()
{
    const uint32_t u = 0x7fc00000u;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// The bound with explicit margins (the production ones are the defaults of
// prune_threshold below); a margin of exactly 1 removes that safeguard.
RFPS_HOST_DEVICE inline float prune_threshold_with(float R, float dv, double inner, double outer, double step)
{
    if (dv == 0.0f)
        return 0.0f;
    if (!(dv >= 0x1p-100f) || !(dv <= 0x1p100f))
        return prune_nan();
    double q = (double)R + sqrt((double)dv * inner);
    q *= step;
    const double T = q * q * step;
    const double t64 = T * outer;
    if (!(t64 <= 3.0e38))
        return prune_nan();
    float thr = (float)t64;
    if ((double)thr < t64)
        thr = nextafterf(thr, INFINITY);
    return thr;
}

RFPS_HOST_DEVICE inline float prune_threshold(float R, float dv)
{
    return prune_threshold_with(R, dv, kPruneInner, kPruneOuter, kPruneStep);
}

}  // namespace rfps
