// CPU model run of the streamed pipeline (csrc/pipeline.cpp) against the HIP stand-in
// in tests/host/hipstub. The kernels are replaced by plain host loops with the same
// interface: dedispersion is the literal sum over channels, and the "search" reports
// every (trial, start) of its range whose dedispersed value reaches an integer
// threshold. So the expected output of a whole signal is known exactly, and every
// chunk, sub-chunk, device-tail copy, stream assignment, resume and error path of the
// real scheduler code can be checked on the CPU, under ThreadSanitizer or
// AddressSanitizer, with several threads submitting, polling and adding beams at once.
#include <algorithm>
#include <atomic>
#include <climits>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "aa_internal.h"

namespace {
thread_local std::string g_err;
int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);              \
            ++fails;                                                      \
        }                                                                 \
    } while (0)
}  // namespace

extern "C" const char* aa_last_error(void) { return g_err.c_str(); }

namespace aa {
void set_error(const std::string& m) { g_err = m; }
int fail(int code, const std::string& m) {
    g_err = m;
    return code;
}
int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return AA_EHIP;
}
size_t sps_work_bytes(const aa_plan_s*, int64_t n) { return n > 0 ? 256 : 0; }
int launch_gather_rows(uint8_t* dst, int64_t dp, const uint8_t* src, int64_t sp, int64_t w, int64_t rows, hipStream_t) {
    for (int64_t r = 0; r < rows; ++r) std::memcpy(dst + r * dp, src + r * sp, static_cast<size_t>(w));
    return AA_OK;
}
int launch_dedisperse(const aa_plan_s* p, int, const uint8_t* in, int64_t ip, int64_t n_in, int32_t* out, int64_t op,
                      hipStream_t) {
    const int64_t n_out = n_in - p->maxshift;
    for (int d = 0; d < p->ndm; ++d)
        for (int64_t t = 0; t < n_out; ++t) {
            int32_t acc = 0;
            for (int c = 0; c < p->nchan; ++c) acc += in[c * ip + t + p->shifts[static_cast<size_t>(d) * p->nchan + c]];
            out[d * op + t] = acc;
        }
    return AA_OK;
}
// model search: (d, t) for t in [t_begin, t_end) with D >= threshold, in (d, t) order
int launch_single_pulse(const aa_plan_s* p, const int32_t* dd, int64_t dp, int64_t dd_t0, int64_t, int64_t t_begin,
                        int64_t t_end, int64_t, void*, aa_candidate_t* cand, int32_t cap, int32_t* count, float*, int64_t,
                        hipStream_t, int32_t beam) {
    int32_t n = 0;
    for (int d = 0; d < p->ndm; ++d)
        for (int64_t t = t_begin; t < t_end; ++t) {
            const int32_t v = dd[d * dp + (t - dd_t0)];
            if (v >= static_cast<int32_t>(p->threshold)) {
                if (n < cap) cand[n] = aa_candidate_t{d, 1, t, static_cast<float>(v), beam};
                ++n;
            }
        }
    *count = n;
    return AA_OK;
}
}  // namespace aa

namespace {

struct Sig {
    int nchan, ndm, wmax, block;
    int64_t nsamp;
    std::vector<uint8_t> x;          // [nchan][nsamp]
    std::vector<int32_t> shifts;     // [ndm][nchan]
    int64_t maxshift;
    int thr;
};

Sig make_sig(unsigned seed, int nchan, int ndm, int64_t nsamp, int block, int wmax) {
    std::mt19937 rng(seed);
    Sig s{nchan, ndm, wmax, block, nsamp, {}, {}, 0, 0};
    s.x.resize(static_cast<size_t>(nchan) * nsamp);
    for (auto& v : s.x) v = static_cast<uint8_t>(rng() % 4);
    // sparse bright samples make a few hundred threshold crossings
    for (int k = 0; k < 400; ++k) s.x[rng() % s.x.size()] = 250;
    s.shifts.resize(static_cast<size_t>(ndm) * nchan);
    for (int d = 0; d < ndm; ++d)
        for (int c = 0; c < nchan; ++c) {
            const int v = (d * c * 7) / (nchan + 3) + static_cast<int>(rng() % 2) * (c > 0);
            s.shifts[static_cast<size_t>(d) * nchan + c] = v;
            s.maxshift = std::max<int64_t>(s.maxshift, v);
        }
    for (int d = 0; d < ndm; ++d) s.shifts[static_cast<size_t>(d) * nchan] = 0;
    s.thr = 250;
    return s;
}

aa_plan_s* make_plan(const Sig& s) {
    auto* p = new aa_plan_s();
    p->nchan = s.nchan;
    p->ndm = s.ndm;
    p->nwidths = 1;
    p->wmax = s.wmax;
    p->stat_block = s.block;
    p->nsamp = s.nsamp;
    p->maxshift = s.maxshift;
    p->threshold = static_cast<float>(s.thr);
    p->shifts = s.shifts;
    p->widths = {s.wmax};
    p->device = 0;
    return p;
}

using Cand = std::tuple<int, int64_t, int>;   // (d, t, value)

std::vector<Cand> expected(const Sig& s, int64_t t_from = 0) {
    const int64_t T = s.nsamp - s.maxshift - s.wmax + 1;
    std::vector<Cand> out;
    for (int d = 0; d < s.ndm; ++d)
        for (int64_t t = t_from; t < T; ++t) {
            int32_t acc = 0;
            for (int c = 0; c < s.nchan; ++c) acc += s.x[c * s.nsamp + t + s.shifts[static_cast<size_t>(d) * s.nchan + c]];
            if (acc >= s.thr) out.emplace_back(d, t, acc);
        }
    return out;
}

aa_pipeline_t make_pipe(int nstreams, int64_t max_chunk, uint32_t flags, int64_t min_work, int beams = 1) {
    aa_pipeline_opts_t o{};
    o.nstreams = nstreams;
    o.max_beams = beams;
    o.max_chunk = max_chunk;
    o.cand_cap = 1 << 14;
    o.result_slots = 0;
    o.hbm_budget = int64_t{256} << 20;
    o.flags = flags;
    o.min_piece_work = min_work;
    aa_pipeline_t p = nullptr;
    CHECK(aa_pipeline_create(&o, &p) == AA_OK);
    return p;
}

struct Got {
    std::vector<Cand> cand;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    std::vector<int> status;
    std::vector<uint64_t> tags;
};

void poll_all(aa_pipeline_t p, size_t n, Got& g) {
    for (size_t i = 0; i < n; ++i) {
        aa_result_t r{};
        const int rc = aa_poll(p, &r, 20'000'000);
        CHECK(rc == AA_OK);
        if (rc != AA_OK) return;
        g.status.push_back(r.status);
        g.tags.push_back(r.tag);
        g.ranges.emplace_back(r.t_begin, r.t_end);
        for (int64_t k = 0; k < r.n; ++k) g.cand.emplace_back(r.cand[k].dm_idx, r.cand[k].t, static_cast<int>(r.cand[k].snr));
        CHECK(aa_release(p, r.tag) == AA_OK);
    }
}

// Submit samples [from, to) of the signal in random chunks; returns the number of submits.
size_t feed(aa_pipeline_t p, int beam, const Sig& s, int64_t from, int64_t to, int64_t max_chunk, std::mt19937& rng,
            uint64_t tag0, bool last, std::vector<uint8_t>* pageable = nullptr) {
    size_t k = 0;
    for (int64_t a = from; a < to; ++k) {
        const int64_t n = std::min<int64_t>(to - a, 1 + rng() % max_chunk);
        const uint8_t* h = s.x.data() + a;
        if (pageable) h = pageable->data() + a;
        CHECK(aa_stream_submit(p, beam, h, n, s.nsamp, tag0 + k, (last && a + n == to) ? AA_SUBMIT_LAST : 0) == AA_OK);
        a += n;
    }
    return k;
}

void sort_c(std::vector<Cand>& v) { std::sort(v.begin(), v.end()); }

void test_single_beam(unsigned seed) {
    std::mt19937 rng(seed);
    const Sig s = make_sig(seed, 12, 9, 9000 + rng() % 4000, 256, 8);
    aa_plan_s* plan = make_plan(s);
    auto want = expected(s);
    for (int cfg = 0; cfg < 8; ++cfg) {
        const int ns = 1 + cfg % 4;
        const uint32_t flags = (cfg == 3 ? AA_PIPE_SERIAL : 0u) | AA_PIPE_TIMING | (cfg == 5 ? AA_PIPE_SDMA_COPY : 0u) |
                               (cfg >= 6 ? AA_PIPE_STAGED : 0u);
        const int64_t minw = cfg % 2 ? -1 : (cfg == 4 ? int64_t{1} << 40 : 1000);
        const int64_t mc = 700 + rng() % 3000;
        aa_pipeline_t p = make_pipe(ns, mc, flags, minw);
        int32_t b = -1;
        CHECK(aa_pipeline_add_beam(p, plan, &b) == AA_OK);
        std::vector<uint8_t> pageable(s.x);
        const size_t n = feed(p, b, s, 0, s.nsamp, mc, rng, 0, true, cfg >= 6 ? &pageable : nullptr);
        Got g;
        poll_all(p, n, g);
        for (int st : g.status) CHECK(st == AA_OK);
        sort_c(g.cand);
        CHECK(g.cand == want);
        std::sort(g.ranges.begin(), g.ranges.end());
        int64_t pos = 0;
        for (auto& rg : g.ranges) {
            CHECK(rg.first == pos);
            pos = rg.second;
        }
        CHECK(pos == s.nsamp - s.maxshift - s.wmax + 1);
        aa_pipeline_stats_t st{};
        CHECK(aa_pipeline_stats(p, &st) == AA_OK);
        CHECK(st.completed == static_cast<int64_t>(n) && st.in_flight == 0 && st.queued == 0);
        CHECK(aa_pipeline_destroy(p) == AA_OK);
    }
    delete plan;
}

// Several beams, one submitting thread per beam, one poller, one thread reading stats:
// each beam's results must equal its own whole-signal result.
void test_threads(unsigned seed, bool staged) {
    const int nb = 3;
    std::vector<Sig> sigs;
    std::vector<aa_plan_s*> plans;
    for (int i = 0; i < nb; ++i) {
        sigs.push_back(make_sig(seed * 10 + i, 8 + 4 * i, 5 + i, 6000 + 1500 * i, 256, 4 << i));
        plans.push_back(make_plan(sigs.back()));
    }
    const int64_t mc = 1500;
    aa_pipeline_t p = make_pipe(3, mc, AA_PIPE_TIMING | (staged ? AA_PIPE_STAGED : 0u), 500, nb);
    std::vector<int32_t> ids(nb, -1);
    CHECK(aa_pipeline_add_beam(p, plans[0], &ids[0]) == AA_OK);
    std::vector<size_t> counts(nb, 0);
    std::vector<std::vector<uint8_t>> pageable;
    for (auto& s : sigs) pageable.push_back(s.x);
    std::atomic<int> submitted_beams{0};
    std::vector<std::thread> th;
    for (int i = 0; i < nb; ++i)
        th.emplace_back([&, i] {
            std::mt19937 rng(seed + 100 * i);
            if (i > 0) CHECK(aa_pipeline_add_beam(p, plans[i], &ids[i]) == AA_OK);   // while beam 0 streams
            counts[i] = feed(p, ids[i], sigs[i], 0, sigs[i].nsamp, mc, rng, static_cast<uint64_t>(i) << 32, true,
                             staged ? &pageable[i] : nullptr);
            ++submitted_beams;
        });
    std::atomic<bool> quit{false};
    std::thread stats([&] {
        while (!quit) {
            aa_pipeline_stats_t st{};
            CHECK(aa_pipeline_stats(p, &st) == AA_OK);
            std::this_thread::yield();
        }
    });
    std::vector<std::vector<Cand>> got(nb);
    size_t polled = 0;
    while (submitted_beams < nb || polled < counts[0] + counts[1] + counts[2]) {
        aa_result_t r{};
        const int rc = aa_poll(p, &r, 2000);
        if (rc == AA_EAGAIN) continue;
        CHECK(rc == AA_OK && r.status == AA_OK);
        const int beam = static_cast<int>(r.tag >> 32);
        CHECK(r.beam == ids[beam]);
        for (int64_t k = 0; k < r.n; ++k) {
            CHECK(r.cand[k].beam == r.beam);
            got[beam].emplace_back(r.cand[k].dm_idx, r.cand[k].t, static_cast<int>(r.cand[k].snr));
        }
        CHECK(aa_release(p, r.tag) == AA_OK);
        ++polled;
    }
    for (auto& t : th) t.join();
    quit = true;
    stats.join();
    CHECK(aa_pipeline_destroy(p) == AA_OK);
    for (int i = 0; i < nb; ++i) {
        sort_c(got[i]);
        CHECK(got[i] == expected(sigs[i]));
        delete plans[i];
    }
}

// AA_FAULT=unit:K fails exactly one chunk with AA_EHIP; every other chunk is exact.
void test_fault(unsigned seed) {
    std::mt19937 rng(seed);
    const Sig s = make_sig(seed, 10, 7, 8000, 256, 8);
    aa_plan_s* plan = make_plan(s);
    const auto want = expected(s);
    setenv("AA_FAULT", "unit:3", 1);
    aa_pipeline_t p = make_pipe(2, 1024, 0u, -1);
    unsetenv("AA_FAULT");
    int32_t b = -1;
    CHECK(aa_pipeline_add_beam(p, plan, &b) == AA_OK);
    const size_t n = feed(p, b, s, 0, s.nsamp, 1024, rng, 0, true);
    int bad = 0;
    std::vector<Cand> ok_c;
    std::vector<std::pair<int64_t, int64_t>> bad_ranges;
    for (size_t i = 0; i < n; ++i) {
        aa_result_t r{};
        CHECK(aa_poll(p, &r, 20'000'000) == AA_OK);
        if (r.status != AA_OK) {
            ++bad;
            CHECK(r.status == AA_EHIP);
            CHECK(std::string(aa_last_error()).find("AA_FAULT") != std::string::npos);
            bad_ranges.emplace_back(r.t_begin, r.t_end);
        } else {
            for (int64_t k = 0; k < r.n; ++k) ok_c.emplace_back(r.cand[k].dm_idx, r.cand[k].t, static_cast<int>(r.cand[k].snr));
        }
        CHECK(aa_release(p, r.tag) == AA_OK);
    }
    CHECK(bad == 1);
    std::vector<Cand> w2;
    for (auto& c : want) {
        bool in_bad = false;
        for (auto& rg : bad_ranges) in_bad |= std::get<1>(c) >= rg.first && std::get<1>(c) < rg.second;
        if (!in_bad) w2.push_back(c);
    }
    sort_c(ok_c);
    // the faulted chunk's other sub-chunks may still report theirs; the rest must be exact
    std::vector<Cand> ok_out;
    for (auto& c : ok_c) {
        bool in_bad = false;
        for (auto& rg : bad_ranges) in_bad |= std::get<1>(c) >= rg.first && std::get<1>(c) < rg.second;
        if (!in_bad) ok_out.push_back(c);
    }
    CHECK(ok_out == w2);
    CHECK(aa_pipeline_destroy(p) == AA_OK);
    delete plan;
}

// Checkpoint after some chunks, tear the pipeline down, resume in a new one at the last
// t_end with the samples from the resume column on: the union equals an uninterrupted run.
void test_resume(unsigned seed) {
    std::mt19937 rng(seed);
    const Sig s = make_sig(seed, 10, 6, 12000, 512, 16);
    aa_plan_s* plan = make_plan(s);
    const auto want = expected(s);
    aa_pipeline_t p = make_pipe(2, 2000, 0u, 0);
    int32_t b = -1;
    CHECK(aa_pipeline_add_beam(p, plan, &b) == AA_OK);
    const int64_t cut = 4000 + rng() % 3000;
    const size_t n1 = feed(p, b, s, 0, cut, 2000, rng, 0, false);
    Got g1;
    poll_all(p, n1, g1);
    CHECK(aa_pipeline_destroy(p) == AA_OK);
    int64_t ckpt = 0;
    for (auto& rg : g1.ranges) ckpt = std::max(ckpt, rg.second);
    CHECK(ckpt % s.block == 0 && ckpt > 0);
    aa_pipeline_t q = make_pipe(3, 2000, 0u, -1);
    CHECK(aa_pipeline_add_beam_at(q, plan, ckpt + 1, &b) == AA_EINVAL);   // not block-aligned
    CHECK(aa_pipeline_add_beam_at(q, plan, ckpt, &b) == AA_OK);
    const int64_t h = (ckpt - 1) & ~int64_t{15};
    const size_t n2 = feed(q, b, s, h, s.nsamp, 2000, rng, 1000, true);
    Got g2;
    poll_all(q, n2, g2);
    for (int st : g2.status) CHECK(st == AA_OK);
    int64_t lo = INT64_MAX;
    for (auto& rg : g2.ranges) lo = std::min(lo, rg.first);
    CHECK(lo == ckpt);
    CHECK(aa_pipeline_destroy(q) == AA_OK);
    std::vector<Cand> all = g1.cand;
    all.insert(all.end(), g2.cand.begin(), g2.cand.end());
    sort_c(all);
    CHECK(all == want);
    delete plan;
}

// AA_LOG: one JSON line per finished chunk.
void test_log(const char* path) {
    std::mt19937 rng(5);
    const Sig s = make_sig(5, 8, 4, 5000, 256, 4);
    aa_plan_s* plan = make_plan(s);
    std::remove(path);
    setenv("AA_LOG", path, 1);
    aa_pipeline_t p = make_pipe(2, 900, 0u, 0);
    unsetenv("AA_LOG");
    int32_t b = -1;
    CHECK(aa_pipeline_add_beam(p, plan, &b) == AA_OK);
    const size_t n = feed(p, b, s, 0, s.nsamp, 900, rng, 0, true);
    Got g;
    poll_all(p, n, g);
    CHECK(aa_pipeline_destroy(p) == AA_OK);
    FILE* f = std::fopen(path, "r");
    CHECK(f != nullptr);
    size_t lines = 0;
    if (f) {
        char buf[512];
        while (std::fgets(buf, sizeof buf, f)) {
            ++lines;
            CHECK(std::string(buf).find("\"tag\": ") != std::string::npos);
        }
        std::fclose(f);
    }
    CHECK(lines == n);
    delete plan;
}

}  // namespace

int main(int argc, char** argv) {
    const char* logpath = argc > 1 ? argv[1] : "/tmp/aa_pipeline_model.jsonl";
    for (unsigned seed = 1; seed <= 3; ++seed) test_single_beam(seed);
    test_threads(7, false);
    test_threads(8, true);
    test_fault(9);
    test_resume(10);
    test_resume(11);
    test_log(logpath);
    std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
