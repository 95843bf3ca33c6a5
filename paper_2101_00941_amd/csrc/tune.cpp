// Dedispersion variant selection and the autotuner. The variants are work-group
// shapes: waves per work-group x trials per wave, so trials per DM block, and the LDS
// budget. The tuner times each variant with HIP events on the caller's stream and
// keeps the fastest. A flat JSON cache, named by AA_TUNE_CACHE, remembers the
// choice per (arch, plan shape).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "aa_internal.h"

namespace aa {
namespace {

std::mutex g_cache_mu;

std::string cache_key(const aa_plan_s* p, int64_t n_in) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    // shape class: arch, channels, trials, maximum shift and the length in 2^k buckets
    int lg = 0;
    while ((int64_t{1} << (lg + 1)) <= n_in) ++lg;
    k << arch << "|nchan=" << p->nchan << "|ndm=" << p->ndm << "|maxshift=" << p->maxshift << "|nin=2^" << lg;
    return k.str();
}

std::map<std::string, int> read_cache(const char* path) {
    std::map<std::string, int> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"');
        const size_t b = line.find('"', a + 1);
        const size_t c = line.find(':', b + 1);
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
        m[line.substr(a + 1, b - a - 1)] = std::atoi(line.c_str() + c + 1);
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace
}  // namespace aa

using namespace aa;

extern "C" int aa_variant_count(void) { return kNumDedispVariants; }

extern "C" int aa_variant_info(int32_t v, aa_variant_t* out) {
    if (!out || v < 0 || v >= kNumDedispVariants) return fail(AA_EINVAL, "aa_variant_info: bad argument");
    const DedispVariant& V = kDedispVariants[v];
    out->id = V.id;
    out->waves = V.waves;
    out->dm_per_wave = V.dpw;
    out->trials_per_block = V.waves * V.dpw;
    out->lds_bytes = V.lds_bytes;
    out->layout = V.layout;
    out->time_tile = V.tile;
    out->depth = V.depth;
    out->max_tiles = V.max_tiles;
    return AA_OK;
}

extern "C" int aa_plan_set_variant(aa_plan_t p, int32_t v) {
    if (!p || v < 0 || v >= kNumDedispVariants) return fail(AA_EINVAL, "aa_plan_set_variant: bad argument");
    const int rc = prepare_variant(p, v);
    if (rc != AA_OK) return rc;
    p->variant = v;
    return AA_OK;
}

extern "C" int aa_plan_get_variant(aa_plan_t p, int32_t* v) {
    if (!p || !v) return fail(AA_EINVAL, "aa_plan_get_variant: null argument");
    *v = p->variant;
    return AA_OK;
}

extern "C" int aa_autotune(aa_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, int32_t* d_out,
                           int64_t out_pitch, int32_t reps, void* stream_, float* ms_out) {
    if (!p || !d_in || !d_out || reps < 1) return fail(AA_EINVAL, "aa_autotune: bad argument");
    if (p->device < 0) return fail(AA_EINVAL, "aa_autotune: plan was created host-only");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const char* cache = std::getenv("AA_TUNE_CACHE");
    const std::string key = cache_key(p, n_in);
    if (cache && *cache) {
        std::lock_guard<std::mutex> g(g_cache_mu);
        const auto m = read_cache(cache);
        const auto it = m.find(key);
        if (it != m.end() && it->second >= 0 && it->second < kNumDedispVariants) {
            int rc = aa_plan_set_variant(p, it->second);
            const auto sp = m.find(key + "|split");
            if (rc == AA_OK && sp != m.end() && kDedispVariants[it->second].layout == 6 &&
                sp->second != p->tables[it->second].split)
                rc = prepare_mixed_split(p, it->second, sp->second);
            if (rc == AA_OK && ms_out)
                for (int v = 0; v < kNumDedispVariants; ++v) ms_out[v] = -1.0f;
            if (rc == AA_OK) return aa_dedisperse(p, d_in, in_pitch, n_in, d_out, out_pitch, stream_);
        }
    }
    hipEvent_t e0, e1;
    AA_HIP(hipEventCreate(&e0));
    AA_HIP(hipEventCreate(&e1));
    int best = -1;
    float best_ms = 0;
    int rc = AA_OK;
    // one warm-up and `reps` timed launches of the variant's current tables
    auto time_variant = [&](int v, float& ms) {
        int r = launch_dedisperse(p, v, d_in, in_pitch, n_in, d_out, out_pitch, stream);  // warm-up
        if (r != AA_OK) return r;
        (void)hipEventRecord(e0, stream);
        for (int i = 0; i < reps && r == AA_OK; ++i) r = launch_dedisperse(p, v, d_in, in_pitch, n_in, d_out, out_pitch, stream);
        (void)hipEventRecord(e1, stream);
        if (r != AA_OK) return r;
        const hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) return hip_fail(e, "aa_autotune: hipEventSynchronize");
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= static_cast<float>(reps);
        return AA_OK;
    };
    for (int v = 0; v < kNumDedispVariants; ++v) {
        float ms = -1.0f;
        if (variant_takes_pitch(v, in_pitch) && prepare_variant(p, v) == AA_OK) {
            rc = time_variant(v, ms);
            if (rc != AA_OK) break;
            if (kDedispVariants[v].layout == 6) {
                // mixed step shapes: also time splits around the host's estimate, in steps of
                // 128 and 256 trials, and keep the fastest
                const int s0 = p->tables[v].split;
                int best_split = s0, cand[4], nc = 0;
                for (int delta : {-256, -128, 128, 256}) {
                    const int s = std::max(0, std::min(s0 + delta, p->ndm));
                    bool seen = s == s0;
                    for (int i = 0; i < nc; ++i) seen = seen || cand[i] == s;
                    if (!seen) cand[nc++] = s;
                }
                for (int i = 0; i < nc; ++i) {
                    const int s = cand[i];
                    float m = -1.0f;
                    rc = prepare_mixed_split(p, v, s);
                    if (rc == AA_OK) rc = time_variant(v, m);
                    if (rc != AA_OK) break;
                    if (m < ms) {
                        ms = m;
                        best_split = s;
                    }
                }
                if (rc != AA_OK) break;
                if (best_split != p->tables[v].split) rc = prepare_mixed_split(p, v, best_split);
                if (rc != AA_OK) break;
            }
            if (best < 0 || ms < best_ms) {
                best = v;
                best_ms = ms;
            }
        }
        if (ms_out) ms_out[v] = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != AA_OK) return rc;
    if (best < 0) return fail(AA_EINVAL, "aa_autotune: no variant could be prepared");
    p->variant = best;
    if (cache && *cache) {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto m = read_cache(cache);
        m[key] = best;
        if (kDedispVariants[best].layout == 6) m[key + "|split"] = p->tables[best].split;
        write_cache(cache, m);
    }
    return launch_dedisperse(p, best, d_in, in_pitch, n_in, d_out, out_pitch, stream);
}
