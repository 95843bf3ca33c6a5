// Screen threshold of the single-pulse search (host and device code).
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

namespace aa {

// Smallest window sum S in [0, 2^31) whose S/N, (double(S) - wmu) * r evaluated in float64
// as the search evaluates it, reaches the threshold; kNever if none does. For r >= 0 that
// S/N is non-decreasing in S (each float64 operation is monotone), so a cell's best S/N
// over the widths reaches the threshold exactly when some width's window sum reaches its
// threshold. The search starts at the real crossing point wmu + threshold / r and steps to
// the exact boundary; if it does not settle within 16 steps the result errs low (0), which
// only lets more cells through to the exact evaluation.
constexpr uint32_t kNever = 0x80000000u;   // above every window sum the screen compares
__host__ __device__ inline uint32_t min_passing_sum(double wmu, double r, double threshold) {
    auto reaches = [&](int64_t S) { return (static_cast<double>(S) - wmu) * r >= threshold; };
    if (!(r > 0.0)) return (0.0 >= threshold) ? 0u : kNever;   // r = 0: every S/N is 0
    const double x = wmu + threshold / r;
    int64_t s = x <= 0.0 ? 0 : (x >= 2147483648.0 ? static_cast<int64_t>(kNever) : static_cast<int64_t>(__builtin_ceil(x)));
    for (int i = 0; i < 16 && s > 0 && reaches(s - 1); ++i) --s;
    if (s > 0 && reaches(s - 1)) return 0u;
    for (int i = 0; i < 16 && s < static_cast<int64_t>(kNever) && !reaches(s); ++i) ++s;
    return static_cast<uint32_t>(s);
}

}  // namespace aa
