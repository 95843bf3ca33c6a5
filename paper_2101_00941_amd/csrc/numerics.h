// Exact integer-to-float64 helpers used by the statistics kernel. They are plain C++,
// so a host-only test can compile this header too.
#pragma once

#include <stdint.h>

#ifndef AA_HD
#if defined(__HIPCC__)
#define AA_HD __host__ __device__
#else
#define AA_HD
#endif
#endif

namespace aa {

// Round an unsigned 128-bit integer to the nearest double, ties to even. This is
// the rounding of IEEE 754 and of Python's float(int). It uses only integer
// operations and exact conversions of values below 2^54.
AA_HD inline double u128_to_double_rn(unsigned __int128 v) {
    if (v == 0) return 0.0;
    const uint64_t hi = static_cast<uint64_t>(v >> 64);
    const int msb = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(static_cast<uint64_t>(v));
    if (msb <= 52) return static_cast<double>(static_cast<uint64_t>(v));
    const int sh = msb - 52;
    uint64_t mant = static_cast<uint64_t>(v >> sh);                 // 53 significant bits
    const unsigned __int128 rem = v & ((static_cast<unsigned __int128>(1) << sh) - 1);
    const unsigned __int128 half = static_cast<unsigned __int128>(1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) ++mant;           // may reach 2^53: still exact
    // mant * 2^sh, sh <= 75: build the power of two exactly
    double scale = 1.0;
    int e = sh;
    while (e >= 32) { scale *= 4294967296.0; e -= 32; }
    scale *= static_cast<double>(static_cast<uint64_t>(1) << e);
    return static_cast<double>(mant) * scale;
}

}  // namespace aa
