// Streamed pipeline and serving loop: time chunks split over HIP streams (section 1,
// Fig. 2 of the paper), pinned asynchronous copies tagged with a stream, and no
// blocking synchronisation on the hot path (section 2). Allocations are hoisted into
// a device arena sized at create time, as section 2.2 does for the search.
//
// Runtime pieces:
//  * Arena: one hipMalloc of the HBM budget. A host-side first-fit allocator
//    (256-byte granules) serves beam histories and per-sub-chunk planes. Admission
//    waits for arena space: that is the HBM-budget admission of the serving loop.
//  * Beam state: two device history buffers used in turn. A chunk's buffer gets
//    the beam's overlap tail by D2D copy, then the new samples by H2D copy, split in
//    pieces with one event per piece. Only new samples cross PCIe.
//  * Scheduler thread: admits queued requests (arrival order, in order per beam),
//    issues copies and kernels, polls events (hipEventQuery, never blocking), and
//    completes results. The atomics in the search kernels are stream-private
//    counters, so no wait here depends on another stream's atomics.
//  * Staged pageable input (AA_PIPE_STAGED, the paper's section 2 remedy for pageable
//    buffers): a ring of small pinned bounce buffers, allocated when a beam is added,
//    is filled by host-to-host copies split over one host thread per compute stream,
//    and each filled buffer is copied to the device like pinned input. A bounce
//    buffer is refilled only after the event of its previous device copy.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <new>

#include "aa_internal.h"
#include "aa_sched.h"

namespace aa {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = kArenaAlign;
size_t up(size_t x) { return arena_round(x); }

struct Unit {                       // one sub-chunk on one compute stream
    int stream = 0;
    int64_t a = 0, b = 0;
    size_t off = 0, len = 0;        // arena block
    int slot = -1;                  // pinned result slot
    hipEvent_t done = nullptr, k0 = nullptr, k1 = nullptr;
    bool complete = false;
};

struct Request {
    uint64_t tag = 0;
    int beam = 0;
    const uint8_t* h = nullptr;
    int64_t n = 0, pitch = 0;
    uint32_t flags = 0;
    uint64_t seq = 0;               // per-beam submission order
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t t_begin = 0, t_end = 0;
    int status = AA_OK;
    std::string err;                // message of the first failure, handed to the aa_poll caller
    int64_t n_true = 0;
    std::vector<aa_candidate_t> cand;
    std::vector<Unit> units;
    hipEvent_t c0 = nullptr, c1 = nullptr;
    size_t pending = 0;
};

// Fork-join pool of host threads for the staging copies: run(n, fn) calls fn(i) for
// i < n, spread over the pool and the calling thread, and returns when all are done.
class StagePool {
  public:
    void start(int nthreads) {
        for (int i = 0; i < nthreads; ++i) th_.emplace_back([this] { loop(); });
    }
    ~StagePool() {
        {
            std::lock_guard<std::mutex> g(m_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    template <class F>
    void run(int n, F fn) {
        if (th_.empty() || n <= 1) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        std::unique_lock<std::mutex> lk(m_);
        job_ = fn;
        next_ = 0;
        total_ = n;
        left_ = n;
        ++gen_;
        cv_.notify_all();
        while (next_ < total_) {          // the caller works too
            const int i = next_++;
            lk.unlock();
            fn(i);
            lk.lock();
            --left_;
        }
        done_cv_.wait(lk, [&] { return left_ == 0; });
        job_ = nullptr;
    }

  private:
    void loop() {
        std::unique_lock<std::mutex> lk(m_);
        uint64_t seen = 0;
        for (;;) {
            cv_.wait(lk, [&] { return quit_ || (gen_ != seen && next_ < total_); });
            if (quit_) return;
            while (next_ < total_) {
                const int i = next_++;
                auto fn = job_;
                lk.unlock();
                fn(i);
                lk.lock();
                if (--left_ == 0) done_cv_.notify_all();
            }
            seen = gen_;
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    std::function<void(int)> job_;
    int next_ = 0, total_ = 0, left_ = 0;
    uint64_t gen_ = 0;
    bool quit_ = false;
};

struct Beam {
    aa_plan_t plan = nullptr;
    int64_t pitch = 0, cols = 0;
    size_t off[2] = {0, 0};
    uint8_t* buf[2] = {nullptr, nullptr};
    int cur = -1;
    int64_t h0 = 0, R = 0, e = 0;
    bool finished = false;
    Request* last_user[2] = {nullptr, nullptr};   // request whose units read buf[k] last
    uint64_t next_seq = 0, issued_seq = 0;
};

}  // namespace
}  // namespace aa

using namespace aa;

struct aa_pipeline_s {
    aa_pipeline_opts_t opt{};
    int device = 0;
    int cap = 0;
    hipStream_t copy = nullptr;
    std::vector<hipStream_t> comp;
    Arena arena;
    uint8_t* d_arena = nullptr;
    uint8_t* h_slots = nullptr;
    size_t slot_bytes = 0;
    std::vector<int> free_slots;
    std::vector<hipEvent_t> ev_pool, tev_pool;
    hipEvent_t ref = nullptr;
    std::vector<Beam> beams;
    std::deque<Request*> queue;
    std::vector<Request*> inflight;
    std::deque<Request*> done;
    std::unordered_map<uint64_t, Request*> returned;
    std::unordered_map<uint64_t, int> live_tags;
    std::vector<std::pair<double, double>> copy_iv, kern_iv;
    int64_t submitted = 0, completed = 0;
    unsigned rr = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool started = false;
    std::thread thr;
    std::string thread_error;
    // staged pageable input
    std::vector<uint8_t*> bounce;
    std::vector<hipEvent_t> bounce_ev;
    size_t bounce_bytes = 0;
    unsigned bounce_next = 0;
    StagePool stagers;
    bool staging_active = false;         // the scheduler is filling a bounce buffer, lock released
    std::condition_variable cv_stage;
    // sub-chunk split, fault hook (AA_FAULT) and per-chunk log (AA_LOG)
    int64_t min_piece_work = int64_t{1} << 33;
    int64_t fault_unit = -1, units_issued = 0;
    FILE* log = nullptr;
    void log_result(const Request* r);
    bool staged() const { return opt.flags & AA_PIPE_STAGED; }
    int grow_bounce(size_t bytes);

    hipEvent_t get_event(bool timing) {
        auto& pool = timing ? tev_pool : ev_pool;
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e, bool timing) {
        if (e) (timing ? tev_pool : ev_pool).push_back(e);
    }
    bool timing() const { return opt.flags & AA_PIPE_TIMING; }
    bool serial() const { return opt.flags & AA_PIPE_SERIAL; }

    // ---- issue one request (lock held); returns false if resources are short ----
    bool try_issue(Request* r, std::unique_lock<std::mutex>& lk);
    void complete_units();
    void run();
};

bool aa_pipeline_s::try_issue(Request* r, std::unique_lock<std::mutex>& lk) {
    Beam& bm = beams[r->beam];
    const aa_plan_s* p = bm.plan;
    const int64_t M = p->maxshift, W = p->wmax, B = p->stat_block;
    const bool last = r->flags & AA_SUBMIT_LAST;
    const int64_t R2 = bm.R + r->n;
    const ChunkRange cr = chunk_range(bm.e, R2, M, W, B, last);
    const int64_t e2 = cr.e2, t_total = cr.t_total;
    const int64_t work = static_cast<int64_t>(p->ndm) * p->nchan * (e2 - bm.e);
    const std::vector<Piece> pieces = split_blocks(bm.e, e2, B, sub_chunks(work, min_piece_work, opt.nstreams));
    // keep the history from the left-halo column of the next start, rounded down to 16 bytes
    const int64_t h0n = bm.e > 0 ? ((bm.e - 1) & ~int64_t{15}) : 0;
    if (R2 - h0n > bm.cols) {
        r->status = fail(AA_EINVAL, "aa_stream_submit: chunk does not fit the beam history");
        r->err = aa_last_error();
        return true;  // completes with an error below
    }
    // resources: one arena block and one pinned slot per piece
    if (static_cast<int>(free_slots.size()) < static_cast<int>(pieces.size())) return false;
    std::vector<size_t> need(pieces.size());
    std::vector<size_t> offs(pieces.size());
    for (size_t j = 0; j < pieces.size(); ++j) {
        int64_t w0, w1;
        piece_window(pieces[j], h0n, R2, M, W, &w0, &w1);
        const int64_t n_out = w1 - w0 - M;
        const int64_t opitch = (n_out + 63) / 64 * 64;
        need[j] = up(static_cast<size_t>(p->ndm) * opitch * 4) + up(sps_work_bytes(p, pieces[j].b - pieces[j].a)) +
                  up(static_cast<size_t>(cap) * sizeof(aa_candidate_t)) + kAlign;
    }
    size_t got = 0;
    for (; got < pieces.size(); ++got)
        if (!arena.alloc(need[got], &offs[got])) break;
    if (got < pieces.size()) {
        for (size_t j = 0; j < got; ++j) arena.release(offs[j], need[j]);
        return false;
    }
    const int64_t nchan = p->nchan;
    // copy pieces (each with an event, so that a sub-chunk waits only for its window); the
    // staged path keeps nstreams pieces, the size its bounce buffers were made for
    const int npc = std::max<int>(1, std::min<int>(staged() ? opt.nstreams : static_cast<int>(std::max<size_t>(pieces.size(), 1)),
                                                   static_cast<int>((r->n + 4095) / 4096)));
    if (staged() && r->n > 0) {
        // the widest piece the loop below can cut, against the bounce size set at add_beam
        const int64_t widest = (r->n + npc - 1) / npc + 15 * (npc - 1);
        if (static_cast<size_t>((widest + 15) & ~int64_t{15}) * static_cast<size_t>(nchan) > bounce_bytes) {
            r->status = fail(AA_EINVAL, "aa_stream_submit: staged piece exceeds the bounce buffers");
            r->err = aa_last_error();
            for (size_t j = 0; j < pieces.size(); ++j) arena.release(offs[j], need[j]);
            return true;
        }
    }
    // Every enqueue below is checked. The first failure becomes the chunk's status; the
    // remaining steps are still enqueued where they are safe, so that every sub-chunk ends
    // with a recorded completion event (or a synchronised stream) before its memory is reused.
    auto ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        (void)hipGetLastError();
        if (r->status == AA_OK || r->status == AA_EOVERFLOW) {
            r->status = hip_fail(e, what);
            r->err = aa_last_error();
        }
        return false;
    };

    // ---- copies (copy stream) ----
    const int nb = bm.cur < 0 ? 0 : (bm.cur + 1) % 2;
    hipStream_t cs = copy;
    bool copies_ok = true;
    if (Request* prev = bm.last_user[nb]) {
        for (Unit& u : prev->units)
            if (!u.complete && u.done && !serial())
                copies_ok &= ok(hipStreamWaitEvent(cs, u.done, 0), "pipeline: copy stream wait");
    }
    if (timing()) {
        r->c0 = get_event(true);
        if (!r->c0 || !ok(hipEventRecord(r->c0, cs), "pipeline: event record")) {
            put_event(r->c0, true);
            r->c0 = nullptr;
        }
    }
    if (!copies_ok) {
        // the history buffer may still be read by the previous chunk: writing it now would race
        (void)hipStreamSynchronize(cs);
        for (Unit& u : bm.last_user[nb]->units)
            if (!u.complete) (void)hipStreamSynchronize(u.stream < 0 ? cs : comp[u.stream]);
    }
    if (bm.cur >= 0 && bm.R > h0n) {
        ok(hipMemcpy2DAsync(bm.buf[nb], bm.pitch, bm.buf[bm.cur] + (h0n - bm.h0), bm.pitch, bm.R - h0n, nchan,
                            hipMemcpyDeviceToDevice, cs),
           "pipeline: device tail copy");
    }
    // H2D of the new samples in pieces, with an event after each. Mapped pinned rows are
    // gathered by a kernel when every row start is 16-byte aligned; otherwise the
    // runtime's 2-D copy is used.
    const uint8_t* hdev = nullptr;
    int64_t col = bm.R - h0n, src = 0;
    if (!(opt.flags & AA_PIPE_SDMA_COPY) && !staged() && r->n > 0 && (reinterpret_cast<uintptr_t>(r->h) & 15) == 0 &&
        (r->pitch & 15) == 0 && (col & 15) == 0 && (bm.pitch & 15) == 0) {
        void* dp = nullptr;
        if (hipHostGetDevicePointer(&dp, const_cast<uint8_t*>(r->h), 0) == hipSuccess && dp)
            hdev = static_cast<const uint8_t*>(dp);
        else
            (void)hipGetLastError();
    }
    std::vector<hipEvent_t> pev;
    std::vector<int64_t> pend;   // end column (exclusive) covered after piece i
    for (int i = 0; i < npc; ++i) {
        int64_t w = (r->n - src) / (npc - i);
        if (i + 1 < npc) w &= ~int64_t{15};
        else w = r->n - src;
        if (w > 0 && staged()) {
            // host-to-host into a pinned bounce buffer (rows split over the stage threads),
            // then the device copy from it. The wait for the buffer's previous device copy
            // and the host copies run with the pipeline lock released, so submit, poll and
            // release callers are not blocked; add_beam waits for staging_active to clear
            // before it may replace the bounce buffers.
            const unsigned j = bounce_next++ % static_cast<unsigned>(bounce.size());
            const int64_t bp = (w + 15) & ~int64_t{15};   // bp * nchan <= bounce_bytes, checked above
            uint8_t* hb = bounce[j];
            const hipEvent_t prev_copy = bounce_ev[j];
            const uint8_t* hs = r->h + src;
            const int64_t sp = r->pitch;
            const int parts = std::min<int>(opt.nstreams, static_cast<int>(nchan));
            staging_active = true;
            lk.unlock();
            const hipError_t se = prev_copy ? hipEventSynchronize(prev_copy) : hipSuccess;
            if (se == hipSuccess)
                stagers.run(parts, [&](int q) {
                    const int64_t c0 = nchan * q / parts, c1 = nchan * (q + 1) / parts;
                    for (int64_t c = c0; c < c1; ++c) std::memcpy(hb + c * bp, hs + c * sp, static_cast<size_t>(w));
                });
            lk.lock();
            staging_active = false;
            cv_stage.notify_all();
            if (ok(se, "pipeline: bounce buffer wait")) {
                void* dp = nullptr;
                const bool mapped = hipHostGetDevicePointer(&dp, hb, 0) == hipSuccess && dp;
                if (!mapped) (void)hipGetLastError();
                const int64_t body = (mapped && (col & 15) == 0 && (bm.pitch & 15) == 0) ? (w & ~int64_t{15}) : 0;
                if (body)
                    ok(launch_gather_rows(bm.buf[nb] + col, bm.pitch, static_cast<const uint8_t*>(dp), bp, body, nchan, cs) ==
                               AA_OK ? hipSuccess : hipErrorLaunchFailure,
                       "pipeline: staged row gather");
                if (w > body)
                    ok(hipMemcpy2DAsync(bm.buf[nb] + col + body, bm.pitch, hb + body, bp, w - body, nchan,
                                        hipMemcpyHostToDevice, cs),
                       "pipeline: staged copy");
            }
            if (!bounce_ev[j]) bounce_ev[j] = get_event(false);
            if (!bounce_ev[j] || !ok(hipEventRecord(bounce_ev[j], cs), "pipeline: event record")) {
                (void)hipStreamSynchronize(cs);   // the buffer's copy must be over before its next fill
                put_event(bounce_ev[j], false);
                bounce_ev[j] = nullptr;
            }
        } else if (w > 0) {
            if (hdev && (w & 15) == 0)
                ok(launch_gather_rows(bm.buf[nb] + col, bm.pitch, hdev + src, r->pitch, w, nchan, cs) == AA_OK
                       ? hipSuccess : hipErrorLaunchFailure,
                   "pipeline: row gather");
            else if (hdev) {   // 16-byte body by the kernel, ragged tail by the runtime copy
                const int64_t body = w & ~int64_t{15};
                if (body)
                    ok(launch_gather_rows(bm.buf[nb] + col, bm.pitch, hdev + src, r->pitch, body, nchan, cs) == AA_OK
                           ? hipSuccess : hipErrorLaunchFailure,
                       "pipeline: row gather");
                ok(hipMemcpy2DAsync(bm.buf[nb] + col + body, bm.pitch, r->h + src + body, r->pitch, w - body, nchan,
                                    hipMemcpyHostToDevice, cs),
                   "pipeline: H2D copy");
            } else
                ok(hipMemcpy2DAsync(bm.buf[nb] + col, bm.pitch, r->h + src, r->pitch, w, nchan, hipMemcpyHostToDevice, cs),
                   "pipeline: H2D copy");
        }
        col += w;
        src += w;
        hipEvent_t ev = get_event(false);
        if (!ev || !ok(hipEventRecord(ev, cs), "pipeline: event record")) {
            put_event(ev, false);
            ev = nullptr;   // sub-chunks that need this piece wait by synchronising the copy stream
        }
        pev.push_back(ev);
        pend.push_back(col);
    }
    if (timing()) {
        r->c1 = get_event(true);
        if (!r->c1 || !ok(hipEventRecord(r->c1, cs), "pipeline: event record")) {
            put_event(r->c1, true);
            r->c1 = nullptr;
        }
    }
    bm.cur = nb;
    bm.h0 = h0n;
    bm.R = R2;
    bm.last_user[nb] = r;

    // ---- sub-chunks (compute streams) ----
    r->t_begin = bm.e;
    r->t_end = e2;
    r->units.resize(pieces.size());
    for (size_t j = 0; j < pieces.size(); ++j) {
        Unit& u = r->units[j];
        u.a = pieces[j].a;
        u.b = pieces[j].b;
        u.off = offs[j];
        u.len = need[j];
        u.slot = free_slots.back();
        free_slots.pop_back();
        u.stream = serial() ? -1 : static_cast<int>(rr++ % opt.nstreams);
        hipStream_t s = u.stream < 0 ? cs : comp[u.stream];
        int64_t w0, w1;
        piece_window(pieces[j], h0n, R2, M, W, &w0, &w1);
        const int64_t n_in = w1 - w0, n_out = n_in - M;
        const int64_t opitch = (n_out + 63) / 64 * 64;
        uint8_t* blk = arena.base + u.off;
        int32_t* dplane = reinterpret_cast<int32_t*>(blk);
        blk += up(static_cast<size_t>(p->ndm) * opitch * 4);
        void* work_buf = blk;
        blk += up(sps_work_bytes(p, u.b - u.a));
        aa_candidate_t* dcand = reinterpret_cast<aa_candidate_t*>(blk);
        blk += up(static_cast<size_t>(cap) * sizeof(aa_candidate_t));
        int32_t* dcount = reinterpret_cast<int32_t*>(blk);
        uint8_t* hs = h_slots + static_cast<size_t>(u.slot) * slot_bytes;
        std::memset(hs, 0, sizeof(int32_t));   // a chunk whose count copy fails reads 0, not a stale count
        bool launch = true;
        if (u.stream >= 0) {
            size_t k = 0;
            while (k + 1 < pend.size() && pend[k] < w1 - h0n) ++k;
            if (!pev[k] || !ok(hipStreamWaitEvent(s, pev[k], 0), "pipeline: compute stream wait")) {
                // without the wait the kernels could read the history before its copy lands
                if (!ok(hipStreamSynchronize(cs), "pipeline: copy stream synchronise")) launch = false;
            }
        }
        if (fault_unit >= 0 && units_issued == fault_unit) {
            launch = false;
            if (r->status == AA_OK || r->status == AA_EOVERFLOW) {
                r->status = fail(AA_EHIP, "pipeline: injected fault (AA_FAULT) at sub-chunk " + std::to_string(units_issued));
                r->err = aa_last_error();
            }
        }
        ++units_issued;
        if (timing()) {
            u.k0 = get_event(true);
            if (u.k0 && !ok(hipEventRecord(u.k0, s), "pipeline: event record")) {
                put_event(u.k0, true);
                u.k0 = nullptr;
            }
        }
        if (launch) {
            int rc = launch_dedisperse(p, p->variant, bm.buf[nb] + (w0 - h0n), bm.pitch, n_in, dplane, opitch, s);
            if (rc == AA_OK)
                rc = launch_single_pulse(p, dplane, opitch, w0, n_out, u.a, u.b, t_total, work_buf, dcand, cap, dcount,
                                         nullptr, 0, s);
            if (rc != AA_OK && (r->status == AA_OK || r->status == AA_EOVERFLOW)) {
                r->status = rc;
                r->err = aa_last_error();
            }
            if (rc == AA_OK) {
                ok(hipMemcpyAsync(hs, dcount, sizeof(int32_t), hipMemcpyDeviceToHost, s), "pipeline: D2H count");
                ok(hipMemcpyAsync(hs + kAlign, dcand, static_cast<size_t>(cap) * sizeof(aa_candidate_t),
                                  hipMemcpyDeviceToHost, s),
                   "pipeline: D2H candidates");
            }
        }
        if (timing()) {
            u.k1 = get_event(true);
            if (u.k1 && !ok(hipEventRecord(u.k1, s), "pipeline: event record")) {
                put_event(u.k1, true);
                u.k1 = nullptr;
            }
        }
        u.done = get_event(false);
        if (!u.done || !ok(hipEventRecord(u.done, s), "pipeline: event record")) {
            // no completion event: wait here (error path only) so the arena block and the
            // result slot are not reused while the stream may still write them
            (void)hipStreamSynchronize(s);
            put_event(u.done, false);
            u.done = nullptr;
        }
    }
    // piece events are only waited on above, so they can be recycled now: a later record
    // on the same event does not change a wait already enqueued
    for (hipEvent_t ev : pev) put_event(ev, false);
    bm.e = e2;
    if (last) bm.finished = true;
    r->pending = r->units.size();
    r->t_admit = now_s();
    return true;
}

void aa_pipeline_s::log_result(const Request* r) {
    if (!log) return;
    std::fprintf(log,
                 "{\"tag\": %llu, \"beam\": %d, \"t_begin\": %lld, \"t_end\": %lld, \"samples\": %lld, "
                 "\"sub_chunks\": %zu, \"candidates\": %lld, \"status\": %d, \"queue_s\": %.6f, \"latency_s\": %.6f}\n",
                 static_cast<unsigned long long>(r->tag), r->beam, static_cast<long long>(r->t_begin),
                 static_cast<long long>(r->t_end), static_cast<long long>(r->n), r->units.size(),
                 static_cast<long long>(r->n_true), r->status, r->t_admit - r->t_submit, r->t_done - r->t_submit);
    std::fflush(log);
}

void aa_pipeline_s::complete_units() {
    for (size_t i = 0; i < inflight.size();) {
        Request* r = inflight[i];
        for (Unit& u : r->units) {
            if (u.complete) continue;
            // a unit without a completion event had its stream synchronised when it was issued
            const hipError_t q = u.done ? hipEventQuery(u.done) : hipSuccess;
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                r->status = hip_fail(q, "pipeline: asynchronous failure");
                r->err = aa_last_error();
            }
            const uint8_t* hs = h_slots + static_cast<size_t>(u.slot) * slot_bytes;
            int32_t cnt = 0;
            std::memcpy(&cnt, hs, sizeof(cnt));
            const int32_t nget = std::min(cnt, cap);
            const aa_candidate_t* c = reinterpret_cast<const aa_candidate_t*>(hs + kAlign);
            for (int32_t k = 0; k < nget; ++k) {
                aa_candidate_t x = c[k];
                x.beam = r->beam;
                r->cand.push_back(x);
            }
            r->n_true += cnt;
            if (cnt > cap && r->status == AA_OK) r->status = AA_EOVERFLOW;
            if (timing() && u.k0 && u.k1) {
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, ref, u.k0) == hipSuccess && hipEventElapsedTime(&b, ref, u.k1) == hipSuccess)
                    kern_iv.emplace_back(a, b);
            }
            put_event(u.k0, true);
            put_event(u.k1, true);
            put_event(u.done, false);
            u.k0 = u.k1 = u.done = nullptr;
            arena.release(u.off, u.len);
            free_slots.push_back(u.slot);
            u.complete = true;
            --r->pending;
        }
        if (r->pending == 0) {
            if (timing() && r->c0 && r->c1) {
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, ref, r->c0) == hipSuccess && hipEventElapsedTime(&b, ref, r->c1) == hipSuccess)
                    copy_iv.emplace_back(a, b);
            }
            put_event(r->c0, true);
            put_event(r->c1, true);
            r->c0 = r->c1 = nullptr;
            std::sort(r->cand.begin(), r->cand.end(), [](const aa_candidate_t& x, const aa_candidate_t& y) {
                return x.dm_idx != y.dm_idx ? x.dm_idx < y.dm_idx : x.t < y.t;
            });
            r->t_done = now_s();
            log_result(r);
            for (Beam& bm : beams)
                for (auto& lu : bm.last_user)
                    if (lu == r) lu = nullptr;
            done.push_back(r);
            ++completed;
            inflight.erase(inflight.begin() + i);
            cv_done.notify_all();
        } else {
            ++i;
        }
    }
}

void aa_pipeline_s::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        const size_t before = inflight.size() + queue.size();
        complete_units();
        // admission: arrival order, in order per beam, head-of-line for resources. Requests
        // are addressed by index: try_issue may release the lock (staged input), and a
        // submit in that window appends to the queue, which invalidates deque iterators
        // but not the positions of the requests already queued (only this thread erases).
        for (size_t i = 0; i < queue.size();) {
            Request* r = queue[i];
            Beam& bm = beams[r->beam];
            if (r->seq != bm.issued_seq) {   // an earlier chunk of this beam is still queued
                ++i;
                continue;
            }
            if (!try_issue(r, lk)) {
                if (inflight.empty()) {
                    // nothing in flight can release memory or slots: this request never fits
                    r->status = fail(AA_ENOMEM, "pipeline: chunk needs more arena memory or result slots than exist");
                    r->err = aa_last_error();
                    ++bm.issued_seq;
                    queue.erase(queue.begin() + static_cast<std::ptrdiff_t>(i));
                    r->t_admit = r->t_done = now_s();
                    log_result(r);
                    done.push_back(r);
                    ++completed;
                    cv_done.notify_all();
                    progress = true;
                    continue;
                }
                break;
            }
            ++bm.issued_seq;
            queue.erase(queue.begin() + static_cast<std::ptrdiff_t>(i));
            inflight.push_back(r);
            progress = true;
        }
        if (inflight.size() + queue.size() != before) progress = true;
        if (stop && queue.empty() && inflight.empty()) break;
        if (!progress) cv_work.wait_for(lk, std::chrono::microseconds(inflight.empty() ? 2000 : 50));
    }
}

// ---------------------------------------------------------------------------------

extern "C" int aa_pipeline_create(const aa_pipeline_opts_t* opts, aa_pipeline_t* out) {
    if (!opts || !out) return fail(AA_EINVAL, "aa_pipeline_create: null argument");
    *out = nullptr;
    aa_pipeline_opts_t o = *opts;
    if (o.nstreams < 1 || o.nstreams > 16) return fail(AA_EINVAL, "aa_pipeline_create: nstreams must be 1..16");
    if (o.max_beams < 1 || o.max_chunk < 1) return fail(AA_EINVAL, "aa_pipeline_create: need max_beams, max_chunk >= 1");
    if (o.cand_cap <= 0) o.cand_cap = 65536;
    if (o.result_slots <= 0) o.result_slots = 4 * o.nstreams;
    if (o.hbm_budget <= 0) return fail(AA_EINVAL, "aa_pipeline_create: hbm_budget must be > 0");
    auto* p = new (std::nothrow) aa_pipeline_s();
    if (!p) return fail(AA_ENOMEM, "aa_pipeline_create: out of host memory");
    p->opt = o;
    p->cap = o.cand_cap;
    if (o.min_piece_work != 0) p->min_piece_work = o.min_piece_work;
    p->beams.reserve(static_cast<size_t>(o.max_beams));   // Beam references stay valid while the lock is released
    if (const char* f = std::getenv("AA_FAULT")) {
        if (std::strncmp(f, "unit:", 5) == 0) p->fault_unit = std::strtoll(f + 5, nullptr, 10);
    }
    auto cleanup = [&](int rc) {
        if (p->d_arena) (void)hipFree(p->d_arena);
        if (p->h_slots) (void)hipHostFree(p->h_slots);
        if (p->copy) (void)hipStreamDestroy(p->copy);
        for (hipStream_t s : p->comp) (void)hipStreamDestroy(s);
        if (p->ref) (void)hipEventDestroy(p->ref);
        if (p->log) std::fclose(p->log);
        delete p;
        return rc;
    };
    if (const char* lp = std::getenv("AA_LOG")) {
        if (*lp && !(p->log = std::fopen(lp, "a"))) return cleanup(fail(AA_EINVAL, "aa_pipeline_create: cannot open AA_LOG"));
    }
    if (hipGetDevice(&p->device) != hipSuccess) return cleanup(fail(AA_EHIP, "aa_pipeline_create: no device"));
    // streams at the default priority (section 2, step 1)
    if (hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(AA_EHIP, "aa_pipeline_create: stream"));
    for (int i = 0; i < o.nstreams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(AA_EHIP, "aa_pipeline_create: stream"));
        p->comp.push_back(s);
    }
    // the arena and the pinned result slots (section 2, step 2) are allocated once, here
    if (hipMalloc(reinterpret_cast<void**>(&p->d_arena), static_cast<size_t>(o.hbm_budget)) != hipSuccess)
        return cleanup(fail(AA_ENOMEM, "aa_pipeline_create: cannot allocate the HBM budget"));
    p->arena.init(p->d_arena, static_cast<size_t>(o.hbm_budget));
    p->slot_bytes = up(kAlign + static_cast<size_t>(p->cap) * sizeof(aa_candidate_t));
    if (hipHostMalloc(reinterpret_cast<void**>(&p->h_slots), p->slot_bytes * o.result_slots, hipHostMallocDefault) !=
        hipSuccess)
        return cleanup(fail(AA_ENOMEM, "aa_pipeline_create: cannot pin result slots"));
    for (int i = o.result_slots - 1; i >= 0; --i) p->free_slots.push_back(i);
    if (hipEventCreate(&p->ref) != hipSuccess) return cleanup(fail(AA_EHIP, "aa_pipeline_create: event"));
    (void)hipEventRecord(p->ref, p->copy);
    (void)hipEventSynchronize(p->ref);
    if (o.flags & AA_PIPE_STAGED) p->stagers.start(o.nstreams - 1);
    p->thr = std::thread([p] { p->run(); });
    *out = p;
    return AA_OK;
}

// Bounce buffers for staged pageable input: 2 * nstreams pinned buffers of `bytes`
// (one piece of a chunk each). Plan-time work: waits for copies still using the old
// buffers before it replaces them.
int aa_pipeline_s::grow_bounce(size_t bytes) {
    if (bytes <= bounce_bytes) return AA_OK;
    for (hipEvent_t e : bounce_ev)
        if (e) (void)hipEventSynchronize(e);
    for (uint8_t* b : bounce) (void)hipHostFree(b);
    bounce.clear();
    const int n = 2 * opt.nstreams;
    for (int i = 0; i < n; ++i) {
        uint8_t* b = nullptr;
        if (hipHostMalloc(reinterpret_cast<void**>(&b), bytes, hipHostMallocDefault) != hipSuccess) {
            for (uint8_t* q : bounce) (void)hipHostFree(q);
            bounce.clear();
            bounce_bytes = 0;
            return fail(AA_ENOMEM, "aa_pipeline_add_beam: cannot pin staging buffers");
        }
        bounce.push_back(b);
    }
    bounce_ev.resize(n, nullptr);
    bounce_bytes = bytes;
    return AA_OK;
}

namespace {
int add_beam(aa_pipeline_t p, aa_plan_t plan, int64_t t_resume, int32_t* beam) {
    if (!p || !plan || !beam) return fail(AA_EINVAL, "aa_pipeline_add_beam: null argument");
    if (plan->device != p->device) return fail(AA_EINVAL, "aa_pipeline_add_beam: plan is not on the pipeline's device");
    if (plan->nwidths > 32) return fail(AA_EINVAL, "aa_pipeline_add_beam: more than 32 widths");
    if (t_resume < 0 || t_resume % plan->stat_block)
        return fail(AA_EINVAL, "aa_pipeline_add_beam_at: t_resume must be a non-negative multiple of the stat block");
    std::unique_lock<std::mutex> lk(p->mu);
    if (static_cast<int>(p->beams.size()) >= p->opt.max_beams) return fail(AA_EBUSY, "aa_pipeline_add_beam: max_beams reached");
    Beam b;
    b.plan = plan;
    b.cols = p->opt.max_chunk + plan->maxshift + plan->wmax + plan->stat_block + 32;
    b.pitch = static_cast<int64_t>(up(static_cast<size_t>(b.cols)));
    // a resumed beam starts with an empty history whose column 0 is the left-halo column
    // of its first start, rounded down to 16 samples: the first submit begins there
    b.e = t_resume;
    b.h0 = b.R = t_resume > 0 ? ((t_resume - 1) & ~int64_t{15}) : 0;
    const size_t bytes = static_cast<size_t>(b.pitch) * plan->nchan;
    if (!p->arena.alloc(bytes, &b.off[0])) return fail(AA_ENOMEM, "aa_pipeline_add_beam: HBM budget exhausted");
    if (!p->arena.alloc(bytes, &b.off[1])) {
        p->arena.release(b.off[0], bytes);
        return fail(AA_ENOMEM, "aa_pipeline_add_beam: HBM budget exhausted");
    }
    b.buf[0] = p->arena.base + b.off[0];
    b.buf[1] = p->arena.base + b.off[1];
    if (p->staged()) {
        // try_issue cuts a chunk of n samples into npc <= nstreams pieces, each but the
        // last rounded down to 16 columns, so a piece spans at most n / npc + 15 (npc - 1)
        // columns, with n / npc <= max(ceil(max_chunk / nstreams), 4096); it is packed
        // with a 16-byte pitch
        const int64_t piece = std::max<int64_t>((p->opt.max_chunk + p->opt.nstreams - 1) / p->opt.nstreams, 4096) +
                              16 * static_cast<int64_t>(p->opt.nstreams);
        // the scheduler may be filling a bounce buffer with the lock released
        p->cv_stage.wait(lk, [&] { return !p->staging_active; });
        const int rc = p->grow_bounce(static_cast<size_t>((piece + 15) & ~int64_t{15}) * plan->nchan);
        if (rc != AA_OK) {
            p->arena.release(b.off[0], bytes);
            p->arena.release(b.off[1], bytes);
            return rc;
        }
    }
    p->beams.push_back(b);
    *beam = static_cast<int32_t>(p->beams.size() - 1);
    return AA_OK;
}
}  // namespace

extern "C" int aa_pipeline_add_beam(aa_pipeline_t p, aa_plan_t plan, int32_t* beam) {
    return add_beam(p, plan, 0, beam);
}

extern "C" int aa_pipeline_add_beam_at(aa_pipeline_t p, aa_plan_t plan, int64_t t_resume, int32_t* beam) {
    if (!plan) return fail(AA_EINVAL, "aa_pipeline_add_beam_at: null argument");
    return add_beam(p, plan, t_resume, beam);
}

extern "C" int aa_stream_submit(aa_pipeline_t p, int32_t beam, const uint8_t* h_chunk, int64_t nsamp, int64_t pitch,
                                uint64_t tag, uint32_t flags) {
    if (!p || (!h_chunk && nsamp > 0)) return fail(AA_EINVAL, "aa_stream_submit: null argument");
    std::lock_guard<std::mutex> g(p->mu);
    if (p->stop) return fail(AA_EINVAL, "aa_stream_submit: pipeline is shutting down");
    if (beam < 0 || beam >= static_cast<int32_t>(p->beams.size())) return fail(AA_EINVAL, "aa_stream_submit: unknown beam");
    Beam& bm = p->beams[beam];
    if (bm.finished) return fail(AA_EINVAL, "aa_stream_submit: beam already received its last chunk");
    if (nsamp < 0 || nsamp > p->opt.max_chunk || (nsamp > 0 && pitch < nsamp))
        return fail(AA_EINVAL, "aa_stream_submit: need 0 <= nsamp <= max_chunk and pitch >= nsamp");
    if (p->live_tags.count(tag)) return fail(AA_EINVAL, "aa_stream_submit: tag already in use");
    auto* r = new (std::nothrow) Request();
    if (!r) return fail(AA_ENOMEM, "aa_stream_submit: out of host memory");
    r->tag = tag;
    r->beam = beam;
    r->h = h_chunk;
    r->n = nsamp;
    r->pitch = pitch;
    r->flags = flags;
    r->seq = bm.next_seq++;
    if (flags & AA_SUBMIT_LAST) bm.finished = true;
    r->t_submit = now_s();
    p->live_tags[tag] = 1;
    p->queue.push_back(r);
    ++p->submitted;
    p->cv_work.notify_all();
    return AA_OK;
}

extern "C" int aa_poll(aa_pipeline_t p, aa_result_t* out, int32_t timeout_us) {
    if (!p || !out) return fail(AA_EINVAL, "aa_poll: null argument");
    std::unique_lock<std::mutex> lk(p->mu);
    auto ready = [&] { return !p->done.empty(); };
    if (!ready()) {
        if (timeout_us < 0)
            p->cv_done.wait(lk, ready);
        else if (timeout_us > 0)
            p->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    }
    if (!ready()) return AA_EAGAIN;
    Request* r = p->done.front();
    p->done.pop_front();
    p->returned[r->tag] = r;
    std::memset(out, 0, sizeof(*out));
    out->tag = r->tag;
    out->beam = r->beam;
    out->status = r->status;
    out->t_begin = r->t_begin;
    out->t_end = r->t_end;
    out->n_true = r->n_true;
    out->n = static_cast<int64_t>(r->cand.size());
    out->cand = r->cand.data();
    out->latency_s = r->t_done - r->t_submit;
    out->queue_s = r->t_admit - r->t_submit;
    if (r->status < 0) set_error(r->err);   // the chunk's failure, readable by the caller
    return AA_OK;
}

extern "C" int aa_release(aa_pipeline_t p, uint64_t tag) {
    if (!p) return fail(AA_EINVAL, "aa_release: null argument");
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->returned.find(tag);
    if (it == p->returned.end()) return fail(AA_EINVAL, "aa_release: tag not returned by aa_poll");
    delete it->second;
    p->returned.erase(it);
    p->live_tags.erase(tag);
    return AA_OK;
}

namespace {
double union_len(std::vector<std::pair<double, double>> v) {
    std::sort(v.begin(), v.end());
    double tot = 0, s = 0, e = -1e300;
    for (auto& iv : v) {
        if (iv.first > e) {
            if (e > s) tot += e - s;
            s = iv.first;
            e = iv.second;
        } else {
            e = std::max(e, iv.second);
        }
    }
    if (e > s) tot += e - s;
    return tot;
}
std::vector<std::pair<double, double>> merged(std::vector<std::pair<double, double>> v) {
    std::sort(v.begin(), v.end());
    std::vector<std::pair<double, double>> m;
    for (auto& iv : v) {
        if (m.empty() || iv.first > m.back().second)
            m.push_back(iv);
        else
            m.back().second = std::max(m.back().second, iv.second);
    }
    return m;
}
}  // namespace

extern "C" int aa_pipeline_stats(aa_pipeline_t p, aa_pipeline_stats_t* out) {
    if (!p || !out) return fail(AA_EINVAL, "aa_pipeline_stats: null argument");
    std::lock_guard<std::mutex> g(p->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = p->submitted;
    out->completed = p->completed;
    out->in_flight = static_cast<int64_t>(p->inflight.size());
    out->queued = static_cast<int64_t>(p->queue.size());
    out->arena_bytes = static_cast<int64_t>(p->arena.size);
    out->arena_used = static_cast<int64_t>(p->arena.used);
    out->arena_peak = static_cast<int64_t>(p->arena.peak);
    if (!p->copy_iv.empty() || !p->kern_iv.empty()) {
        const auto c = merged(p->copy_iv), k = merged(p->kern_iv);
        out->copy_ms = union_len(p->copy_iv);
        out->kernel_ms = union_len(p->kern_iv);
        double ov = 0;
        size_t i = 0, j = 0;
        while (i < c.size() && j < k.size()) {
            const double lo = std::max(c[i].first, k[j].first), hi = std::min(c[i].second, k[j].second);
            if (hi > lo) ov += hi - lo;
            if (c[i].second < k[j].second) ++i; else ++j;
        }
        out->overlap_ms = ov;
        double lo = 1e300, hi = -1e300;
        for (auto& iv : p->copy_iv) { lo = std::min(lo, iv.first); hi = std::max(hi, iv.second); out->copy_sum_ms += iv.second - iv.first; }
        for (auto& iv : p->kern_iv) { lo = std::min(lo, iv.first); hi = std::max(hi, iv.second); out->kernel_sum_ms += iv.second - iv.first; }
        out->span_ms = hi > lo ? hi - lo : 0;
    }
    return AA_OK;
}

extern "C" int aa_pipeline_destroy(aa_pipeline_t p) {
    if (!p) return fail(AA_EINVAL, "aa_pipeline_destroy: null argument");
    {
        std::lock_guard<std::mutex> g(p->mu);
        p->stop = true;
        p->cv_work.notify_all();
    }
    if (p->thr.joinable()) p->thr.join();   // drains queued and in-flight work
    (void)hipStreamSynchronize(p->copy);
    for (hipStream_t s : p->comp) (void)hipStreamSynchronize(s);
    for (Request* r : p->done) delete r;
    for (auto& kv : p->returned) delete kv.second;
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->tev_pool) (void)hipEventDestroy(e);
    (void)hipEventDestroy(p->ref);
    (void)hipStreamDestroy(p->copy);
    for (hipStream_t s : p->comp) (void)hipStreamDestroy(s);
    (void)hipFree(p->d_arena);
    (void)hipHostFree(p->h_slots);
    for (hipEvent_t e : p->bounce_ev)
        if (e) (void)hipEventDestroy(e);
    for (uint8_t* b : p->bounce) (void)hipHostFree(b);
    if (p->log) std::fclose(p->log);
    delete p;
    return AA_OK;
}
