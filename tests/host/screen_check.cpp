// Host check of the single-pulse screen threshold (min_passing_sum): over random rows and
// widths, the returned window sum reaches the threshold and the sum one below does not,
// both with the float64 S/N expression the search evaluates; when no sum below 2^31
// reaches it the result is kNever; r = 0 gives S/N 0 for every sum.
// Usage: screen_check  (prints ALL OK on success)
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_2101_00941_amd/csrc/screen.h"

using namespace aa;

static bool reaches(int64_t S, double wmu, double r, double thr) { return (static_cast<double>(S) - wmu) * r >= thr; }

int main() {
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> umu(0.0, 1.0e6), ulog(-12.0, 12.0);
    const double thrs[] = {6.0, 0.0, -1.0, 25.0, 1e-3, 3.5, 1e9};
    long bad = 0, n = 0, never = 0, zero = 0;
    for (int it = 0; it < 2000000; ++it) {
        // a row with mean mu and per-sample sigma sig, width w: wmu = w mu, r = 1 / (sig sqrt(w))
        const int w = 1 << (g() % 9);
        const double wmu = static_cast<double>(w) * umu(g);
        const double r = 1.0 / (std::exp(ulog(g)) * std::sqrt(static_cast<double>(w)));
        const double thr = thrs[g() % 7];
        const uint32_t s = min_passing_sum(wmu, r, thr);
        ++n;
        if (s == kNever) {
            ++never;
            if (reaches(static_cast<int64_t>(kNever) - 1, wmu, r, thr)) ++bad;
            continue;
        }
        if (s == 0) ++zero;
        if (!reaches(s, wmu, r, thr)) ++bad;                                // it reaches
        if (s > 0 && reaches(static_cast<int64_t>(s) - 1, wmu, r, thr)) ++bad;  // and is the smallest
        if (bad && bad < 5) printf("case wmu %.17g r %.17g thr %g -> %u\n", wmu, r, thr, s);
    }
    if (min_passing_sum(100.0, 0.0, 6.0) != kNever || min_passing_sum(100.0, 0.0, 0.0) != 0u ||
        min_passing_sum(100.0, 0.0, -1.0) != 0u)
        ++bad;
    printf("cases %ld (kNever %ld, zero %ld), bad %ld\n", n, never, zero, bad);
    printf(bad ? "FAIL\n" : "ALL OK\n");
    return bad != 0;
}
