"""Host-logic tests of the streamed pipeline's scheduler pieces (CPU only): the device
arena allocator, the computable start range per chunk, and the block-aligned split.
csrc/aa_sched.h is plain C++, so a small harness is compiled here with g++."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2101_00941_amd", "csrc")

HARNESS = r'''
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include "aa_sched.h"
using namespace aa;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static void test_arena(unsigned seed) {
    std::mt19937_64 rng(seed);
    Arena a; a.init(nullptr, 1 << 24);
    struct Blk { size_t off, n; };
    std::vector<Blk> live;
    size_t used = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            size_t n = 1 + rng() % 100000, off;
            if (a.alloc(n, &off)) {
                CHECK(off % kArenaAlign == 0 && off + arena_round(n) <= a.size);
                for (auto& b : live) CHECK(off + arena_round(n) <= b.off || b.off + arena_round(b.n) <= off);
                live.push_back({off, n});
                used += arena_round(n);
            } else {
                CHECK(a.largest_free() < arena_round(n));
            }
        } else {
            size_t k = rng() % live.size();
            a.release(live[k].off, live[k].n);
            used -= arena_round(live[k].n);
            live.erase(live.begin() + k);
        }
        CHECK(a.used == used);
    }
    for (auto& b : live) a.release(b.off, b.n);
    CHECK(a.used == 0 && a.free_blocks() == 1 && a.largest_free() == a.size);
}

static void test_ranges(unsigned seed) {
    std::mt19937_64 rng(seed);
    for (int trial = 0; trial < 300; ++trial) {
        const int64_t M = rng() % 80000, W = 1 + rng() % 256, B = 256 * (1 + rng() % 128);
        const int64_t max_chunk = 1 + rng() % 300000;
        const int parts = 1 + rng() % 8;
        const int64_t total = M + W + 1 + rng() % 2000000;
        const int64_t T = total - M - W + 1;
        int64_t R = 0, e = 0;
        while (R < total) {
            const int64_t n = std::min<int64_t>(total - R, 1 + rng() % max_chunk);
            const int64_t R2 = R + n;
            const bool last = R2 == total;
            const int64_t h0n = e > 0 ? ((e - 1) & ~int64_t{15}) : 0;
            CHECK(R2 - h0n <= max_chunk + M + W + B + 32);           // history capacity
            ChunkRange c = chunk_range(e, R2, M, W, B, last);
            CHECK(c.e2 >= e);
            if (!last) {
                CHECK(c.e2 % B == 0);
                CHECK(c.e2 == e || c.e2 + W - 1 + M <= R2 - 1);        // right neighbour present
                CHECK(c.t_total == -1);
            } else {
                CHECK(c.e2 == T && c.t_total == T);
            }
            auto ps = split_blocks(e, c.e2, B, parts);
            int64_t a = e;
            for (auto& p : ps) {
                CHECK(p.a == a && p.b > p.a && p.a % B == 0);
                CHECK(p.b == c.e2 || p.b % B == 0);
                int64_t w0, w1;
                piece_window(p, h0n, R2, M, W, &w0, &w1);
                CHECK(w0 >= h0n && (w0 - h0n) % 16 == 0 && w0 <= std::max<int64_t>(p.a - 1, 0));
                CHECK(w1 <= R2 && w1 - w0 - M >= 1);
                a = p.b;
            }
            CHECK(a == c.e2 || ps.empty());
            CHECK((int)ps.size() <= parts);
            e = c.e2;
            R = R2;
        }
        CHECK(e == T);                                                  // every start covered once
    }
}

int main() {
    for (unsigned s = 1; s <= 3; ++s) { test_arena(s); test_ranges(s); }
    std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
'''


def test_scheduler_host_logic(tmp_path):
    src = tmp_path / "h.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "h"
    # host code only: built with g++, with the sanitizers on
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-I", INC, str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


MODEL = os.path.join(ROOT, "tests", "host", "pipeline_model_check.cpp")
STUB = os.path.join(ROOT, "tests", "host", "hipstub")
PIPELINE = os.path.join(INC, "pipeline.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _model_build(tmp_path, compiler, sanitize):
    exe = tmp_path / f"model_{sanitize.replace(',', '_')}"
    # host code only (the HIP calls resolve to the host stand-in in tests/host/hipstub)
    subprocess.run([compiler, "-O1", "-g", "-std=c++17", f"-fsanitize={sanitize}", "-I", STUB, "-I", INC,
                    "-I", os.path.join(ROOT, "include"), PIPELINE, MODEL, "-o", str(exe), "-lpthread"], check=True)
    return exe


def _model_run(exe, tmp_path):
    r = subprocess.run([str(exe), str(tmp_path / "chunks.jsonl")], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-4000:] + r.stderr[-4000:]
    assert "WARNING" not in r.stderr, r.stderr[-4000:]


def test_pipeline_model_address_sanitizer(tmp_path):
    """The real scheduler code (pipeline.cpp) over a host model of the device: chunks,
    sub-chunks, device tails, multi-beam threads, staged input, fault hook, resume, log."""
    _model_run(_model_build(tmp_path, "g++", "address,undefined"), tmp_path)


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ with ThreadSanitizer not installed")
def test_pipeline_model_thread_sanitizer(tmp_path):
    """Same model under ThreadSanitizer: submitting, polling, stats and add_beam threads
    against the scheduler and its stage threads. Built with clang: the ThreadSanitizer
    runtime of g++ 11 does not intercept the clock-based condition-variable wait that
    libstdc++ uses for wait_for, and then reports false races and runs for minutes."""
    _model_run(_model_build(tmp_path, CLANG, "thread"), tmp_path)
