// Dedispersion tiling tables. Built on the host and uploaded once, at plan time or
// when the tuner prepares a variant. Nothing here runs in the hot loop.
#include <algorithm>
#include <climits>
#include <cstring>

#include "aa_internal.h"

namespace aa {

// LDS budgets are sized so that 3 (52 KB) or 2 (80 KB) work-groups fit in one CU's
// 160 KB of LDS.
const DedispVariant kDedispVariants[kNumDedispVariants] = {
    {0, 4, 4, 53248, 1, kTimeTile, 2, 0},    // 256 threads, 16 trials per block, interleaved lanes
    {1, 8, 2, 53248, 1, kTimeTile, 2, 0},    // 512 threads, 16 trials per block, interleaved lanes
    {2, 8, 4, 81920, 1, kTimeTile, 2, 0},    // 512 threads, 32 trials per block, interleaved lanes
    {3, 16, 2, 81920, 1, kTimeTile, 2, 0},   // 1024 threads, 32 trials per block, interleaved lanes
    {4, 8, 2, 53248, 0, kTimeTile, 2, 0},    // 512 threads, 16 trials per block, contiguous lanes
    {5, 4, 4, 53248, 0, kTimeTile, 2, 0},    // 256 threads, 16 trials per block, contiguous lanes
    {6, 8, 2, 53248, 3, kTimeTile, 2, 0},    // 512 threads, 16 trials per block, contiguous lanes, 16-way switch
    {7, 4, 4, 53248, 3, kTimeTile, 2, 0},    // 256 threads, 16 trials per block, contiguous lanes, 16-way switch
    {8, 8, 2, 53248, 2, kTimeTile, 2, 0},    // 512 threads, 16 trials per block, interleaved, equal-offset reuse
    {9, 8, 4, 81920, 2, kTimeTile, 2, 0},    // 512 threads, 32 trials per block, interleaved, equal-offset reuse
    {10, 4, 4, 53248, 2, kTimeTile, 2, 0},   // 256 threads, 16 trials per block, interleaved, equal-offset reuse
    // 32 trials per block, i8 matrix cores; waves, time tile, staging depth and the
    // channel-block span vary. The kernel table in dedisp.hip repeats these parameters.
    {11, 8, 4, mfma_lds_bytes(1024, 3, 63), 4, 1024, 3, 63},   // 512 threads, 8 tiles per wave
    {12, 16, 2, mfma_lds_bytes(1024, 3, 63), 4, 1024, 3, 63},  // 1024 threads, 4 tiles per wave
    {13, 16, 2, mfma_lds_bytes(768, 7, 63), 4, 768, 7, 63},    // 1024 threads, 4 tiles per wave
    // two work-groups per CU (LDS <= 80 KB, registers for 4 or 8 waves per SIMD)
    {14, 8, 4, mfma_lds_bytes(512, 3, 31), 4, 512, 3, 31},     // 512 threads, 4 tiles per wave
    {15, 16, 2, mfma_lds_bytes(512, 3, 31), 4, 512, 3, 31},    // 1024 threads, 2 tiles per wave
    {16, 8, 4, mfma_lds_bytes(480, 4, 31), 4, 480, 4, 31},     // 512 threads, 4 tiles per wave
    // 8 channels x 4 residuals per step
    {17, 16, 2, mfma_lds_bytes(864, 3, 63, 8), 5, 864, 3, 63},  // 1024 threads, 4 tiles per wave
    // deeper staging rings (loads 3 or 4 steps ahead) for slightly smaller tiles
    {18, 16, 2, mfma_lds_bytes(960, 4, 63), 4, 960, 4, 63},     // 1024 threads, 4 tiles per wave
    {19, 16, 2, mfma_lds_bytes(896, 5, 63), 4, 896, 5, 63},     // 1024 threads, 4 tiles per wave
    // step shape per DM block: 8 x 4 below a split trial, 4 x 8 above it
    {20, 16, 2, mfma_lds_bytes(864, 3, 63, 8), 6, 864, 3, 63},  // 1024 threads, 4 tiles per wave
    // shift-and-add with v_sad_u8 on channel quads staged per residual pattern, 32 trials
    // per block; tile = 64 * waves * samples per lane, depth = staging chunks per step
    {21, 4, 8, quad_lds_bytes(16), 7, 512, 16, 0},    // 256 threads, 2 samples per lane
    {22, 8, 4, quad_lds_bytes(32), 7, 1024, 32, 0},   // 512 threads, 2 samples per lane
    {23, 16, 2, quad_lds_bytes(32), 7, 1024, 32, 0},  // 1024 threads, 1 sample per lane
    {24, 8, 4, quad_lds_bytes(16), 7, 512, 16, 0},    // 512 threads, 1 sample per lane
};

void free_tables(DedispTables& t) {
    if (t.d_blocks) (void)hipFree(t.d_blocks);
    if (t.d_base) (void)hipFree(t.d_base);
    if (t.d_offs) (void)hipFree(t.d_offs);
    if (t.d_pad) (void)hipFree(t.d_pad);
    t = DedispTables();
}

namespace {
template <class T>
int upload(T** dst, const std::vector<T>& src) {
    AA_HIP(hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(src.size(), 1) * sizeof(T)));
    AA_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return AA_OK;
}
}  // namespace

// Tables of the matrix-core variants (layouts 4, 5 and 6). f(d, c) = s[d][c] - s[d0][c];
// a step is `cps` consecutive channels and R = 32 / cps is the residual range.
//  * DM blocks: up to 32 consecutive trials such that every step on its own has a
//    residual range below R (so a channel block always holds at least one step) and,
//    for every channel, the spread of f over the block's trials is at most
//    (max_tiles * 32 - tile). The spread of E over a channel block is bounded
//    by that, so a channel block never needs more than max_tiles tiles of t'.
//    A single trial always qualifies (f = 0).
//  * Channel blocks: greedy runs of steps whose residual range stays below R.
//    E[d] = min over the run of f(d, c), r = f - E, e = E - min E, and the staged row
//    of channel c starts at s[d0][c] + min E (16-aligned start + phase).
//  * Padded channels (c >= nchan) are staged from a row of 0x80 bytes, which the kernel
//    maps to 0, so their residuals are 0. Absent trials of a short block have r = 0,
//    e = 0 and are not written out.
//  * Layout 6 mixes the two step shapes by trial range: blocks below a split trial use
//    8 channels x 4 residuals, the others 4 x 8. Each block records its shape and where
//    its records start.
namespace {

struct MfmaGeom {
    int tile, depth, max_tiles, spread_max, row;
};

// Trials of the block that starts at d0 under the cps rules.
int grow_block(const aa_plan_s* p, int d0, int cps, const MfmaGeom& g, std::vector<int32_t>& fmin,
               std::vector<int32_t>& fmax) {
    const int nchan = p->nchan, R = 32 / cps;
    auto S = [&](int d, int c) { return p->shifts[static_cast<size_t>(d) * nchan + c]; };
    std::fill(fmin.begin(), fmin.end(), 0);
    std::fill(fmax.begin(), fmax.end(), 0);
    int count = 1;
    while (count < 32 && d0 + count < p->ndm) {
        const int d = d0 + count;
        bool ok = true;
        for (int c0 = 0; c0 < nchan && ok; c0 += cps) {
            int lo = INT32_MAX, hi = INT32_MIN;
            for (int c = c0; c < std::min(c0 + cps, nchan); ++c) {
                const int32_t f = S(d, c) - S(d0, c);
                lo = std::min(lo, f);
                hi = std::max(hi, f);
                if (std::max(fmax[c], f) - std::min(fmin[c], f) > g.spread_max) ok = false;
            }
            if (hi - lo > R - 1) ok = false;
        }
        if (!ok) break;
        for (int c = 0; c < nchan; ++c) {
            const int32_t f = S(d, c) - S(d0, c);
            fmin[c] = std::min(fmin[c], f);
            fmax[c] = std::max(fmax[c], f);
        }
        ++count;
    }
    return count;
}

// Row starts (npad entries) and records (npad / cps of them) of one block. When not null,
// mfma_tiles and flush_tiles receive the block's tile-steps (one matrix op per 32-row tile
// and step) and flushed tiles, per time tile.
int block_tables(const aa_plan_s* p, DmBlock& blk, int cps, const MfmaGeom& g, int npad, int32_t* rsv, uint8_t* Rb,
                 int64_t* mfma_tiles, int64_t* flush_tiles) {
    const int nchan = p->nchan, R = 32 / cps, K = npad / cps;
    const MfmaRec RL = mfma_rec(cps);
    auto S = [&](int d, int c) { return p->shifts[static_cast<size_t>(d) * nchan + c]; };
    const int d0 = blk.first, count = blk.count;
    std::vector<int32_t> lo(32), hi(32);
    int64_t mt = 0, ft = 0;
    for (int k0 = 0; k0 < K;) {
        // grow the channel block [k0, k1) step by step
        std::fill(lo.begin(), lo.end(), INT32_MAX);
        std::fill(hi.begin(), hi.end(), INT32_MIN);
        int k1 = k0;
        while (k1 < K) {
            bool ok = true;
            for (int i = 0; i < count && ok; ++i) {
                int l = lo[i], h = hi[i];
                for (int c = cps * k1; c < std::min(cps * k1 + cps, nchan); ++c) {
                    const int32_t f = S(d0 + i, c) - S(d0, c);
                    l = std::min(l, f);
                    h = std::max(h, f);
                }
                if (h - l > R - 1) ok = false;
            }
            if (!ok) break;
            for (int i = 0; i < count; ++i)
                for (int c = cps * k1; c < std::min(cps * k1 + cps, nchan); ++c) {
                    const int32_t f = S(d0 + i, c) - S(d0, c);
                    lo[i] = std::min(lo[i], f);
                    hi[i] = std::max(hi[i], f);
                }
            ++k1;
        }
        if (k1 == k0) return fail(AA_EINVAL, "matrix-core tiling: a step exceeds the residual range");
        int32_t emin = INT32_MAX, emax = INT32_MIN;
        for (int i = 0; i < count; ++i) {
            emin = std::min(emin, lo[i]);
            emax = std::max(emax, lo[i]);
        }
        const int tiles = (emax - emin + g.tile + 31) / 32;
        if (tiles > g.max_tiles) return fail(AA_EINVAL, "matrix-core tiling: channel block spread too large");
        mt += static_cast<int64_t>(tiles) * (k1 - k0);
        ft += tiles;
        for (int k = k0; k < k1; ++k) {
            uint8_t* rk = Rb + static_cast<size_t>(k) * RL.size;
            for (int j = 0; j < cps; ++j) {
                const int c = cps * k + j;
                const int32_t v = c < nchan ? S(d0, c) + emin : 0;
                rsv[c] = v & ~15;
                rk[RL.phase + j] = static_cast<uint8_t>(v & 15);
                for (int i = 0; i < count && c < nchan; ++i) {
                    const int32_t r = S(d0 + i, c) - S(d0, c) - lo[i];
                    rk[cps * i + j] = static_cast<uint8_t>(8 * r);
                }
            }
            for (int i = 0; i < count; ++i) {
                const int16_t e = static_cast<int16_t>(lo[i] - emin);
                std::memcpy(rk + RL.e + 2 * i, &e, 2);
            }
            const int32_t left = k1 - k, emax_rel = emax - emin;
            std::memcpy(rk + RL.tiles, &tiles, 4);
            std::memcpy(rk + RL.left, &left, 4);
            std::memcpy(rk + RL.max_e, &emax_rel, 4);
        }
        k0 = k1;
    }
    blk.rs_lo = *std::min_element(rsv, rsv + npad);
    blk.rs_hi = *std::max_element(rsv, rsv + npad);
    // row starts and lengths of step k + depth - 1, read by the kernel when it issues
    // that step's loads. A row needs the bytes [0, 32 tiles + phase + 11).
    for (int k = 0; k + g.depth - 1 < K; ++k) {
        uint8_t* rk = Rb + static_cast<size_t>(k) * RL.size;
        const uint8_t* rn = Rb + static_cast<size_t>(k + g.depth - 1) * RL.size;
        std::memcpy(rk + RL.next_rs, &rsv[cps * (k + g.depth - 1)], 4 * cps);
        int32_t tiles;
        std::memcpy(&tiles, rn + RL.tiles, 4);
        const int32_t need = std::min(g.row / 16, (32 * tiles + 15 + 11 + 15) / 16);
        std::memcpy(rk + RL.next_need, &need, 4);
    }
    if (mfma_tiles) *mfma_tiles = mt;
    if (flush_tiles) *flush_tiles = ft;
    return AA_OK;
}

// Estimated launch time (ns) of a block's work on MI355X, fitted to timings of the two
// step shapes over trial ranges of the survey plan: a work-group step (its staging, wait
// and barrier) costs 1.63 ns of launch time with 4 channels and 2.17 ns with 8, a
// tile-step 0.018 ns and a flushed tile 0.16 ns.
double block_cost_ns(int cps, int64_t ntile, int K, int64_t tile_steps, int64_t flush_tiles) {
    const double step = cps == 8 ? 2.17 : 1.63;
    return static_cast<double>(ntile) * (step * K + 0.018 * static_cast<double>(tile_steps) +
                                         0.16 * static_cast<double>(flush_tiles));
}

}  // namespace

int build_mfma_tables(const aa_plan_s* p, int tile, int depth, int max_tiles, int cps, std::vector<DmBlock>& blocks,
                      std::vector<int32_t>& rsv, std::vector<uint8_t>& rec, int split_at, int* split_out) {
    if (cps != 4 && cps != 8 && cps != 0) return fail(AA_EINVAL, "matrix-core tiling: 4, 8 or mixed channels per step");
    const MfmaGeom g{tile, depth, max_tiles, max_tiles * 32 - tile, mfma_row_bytes(max_tiles)};
    if (tile % 32 || tile < 256 || g.spread_max < 0 || depth < 3 || (max_tiles != 31 && max_tiles != 63))
        return fail(AA_EINVAL, "matrix-core tiling: bad tile, depth or channel-block span");
    const int nchan = p->nchan;
    const int npad = cps == 4 ? (nchan + 3) / 4 * 4 : (nchan + 7) / 8 * 8;
    std::vector<int32_t> fmin(nchan), fmax(nchan);
    // block shapes: the split trial below which blocks use 8 channels per step
    int split = cps == 8 ? p->ndm : 0;
    if (cps == 0 && split_at >= 0) {
        split = std::min(split_at, p->ndm);
    } else if (cps == 0) {
        // price each shape's own partition, then take the split (at an 8-channel block
        // boundary) with the lowest estimated launch time
        const int64_t n_out = std::max<int64_t>(p->nsamp - p->maxshift, 1);
        std::vector<int32_t> rsv_tmp(npad);
        std::vector<std::pair<int, double>> c8, c4;   // (first trial, cost)
        for (int shape : {8, 4}) {
            const int64_t ntile = (n_out + g.tile - 1) / g.tile;
            std::vector<uint8_t> rec_tmp(static_cast<size_t>(npad / shape) * mfma_rec(shape).size);
            for (int d0 = 0; d0 < p->ndm;) {
                DmBlock b{d0, grow_block(p, d0, shape, g, fmin, fmax), 0, 0, 0, shape, 0};
                int64_t mt = 0, ft = 0;
                const int rc = block_tables(p, b, shape, g, npad, rsv_tmp.data(), rec_tmp.data(), &mt, &ft);
                if (rc != AA_OK) return rc;
                (shape == 8 ? c8 : c4).push_back({d0, block_cost_ns(shape, ntile, npad / shape, mt, ft)});
                d0 += b.count;
            }
        }
        double best = -1.0;
        for (size_t i = 0; i <= c8.size(); ++i) {
            const int d = i < c8.size() ? c8[i].first : p->ndm;
            double cost = 0.0;
            for (size_t k = 0; k < i; ++k) cost += c8[k].second;
            for (const auto& b : c4)
                if (b.first >= d) cost += b.second;
            if (best < 0.0 || cost < best) {
                best = cost;
                split = d;
            }
        }
    }
    if (split_out) *split_out = split;
    blocks.clear();
    for (int d0 = 0; d0 < p->ndm;) {
        const int shape = d0 < split ? 8 : 4;
        int count = grow_block(p, d0, shape, g, fmin, fmax);
        if (shape == 8 && d0 + count > split) count = split - d0;   // the 4-channel part starts at the split
        blocks.push_back(DmBlock{d0, count, 0, 0, 0, shape, 0});
        d0 += count;
    }
    const size_t nblk = blocks.size();
    size_t rec_bytes = 0;
    for (auto& b : blocks) {
        b.rec256 = static_cast<int32_t>(rec_bytes / 256);
        rec_bytes += static_cast<size_t>(npad / b.cps) * mfma_rec(b.cps).size;
    }
    rsv.assign(nblk * npad, 0);
    rec.assign(rec_bytes, 0);
    for (size_t bi = 0; bi < nblk; ++bi) {
        DmBlock& b = blocks[bi];
        const int rc = block_tables(p, b, b.cps, g, npad, &rsv[bi * npad],
                                    &rec[static_cast<size_t>(b.rec256) * 256], nullptr, nullptr);
        if (rc != AA_OK) return rc;
    }
    return AA_OK;
}

// Tables of the quad variants (layout 7). A DM block grows trial by trial while, in
// every step (quad of channels), the block's trials form at most kQuadMaxPat residual
// patterns whose staged dwords fill at most `chunks` 64-unit chunks. One trial always
// fits: its step has one pattern of tile / 4 units.
namespace {

struct QuadPat {
    int32_t r1, r2, r3, lo, hi;
};

int64_t quad_units(int tile, int32_t lo, int32_t hi) { return (static_cast<int64_t>(tile) + hi - lo + 3) / 4; }

}  // namespace

int build_quad_tables(const aa_plan_s* p, int tile, int chunks, std::vector<DmBlock>& blocks,
                      std::vector<int32_t>& rec) {
    const int nchan = p->nchan, nq = (nchan + 3) / 4;
    if (tile % 256 != 0 || static_cast<int64_t>(tile) / 256 > chunks || chunks > kQuadMaxChunks)
        return fail(AA_EINVAL, "quad tiling: a one-trial step does not fit the chunks");
    auto S = [&](int d, int c) { return p->shifts[static_cast<size_t>(d) * nchan + c]; };
    auto key = [&](int d, int q, int32_t (&r)[3]) {
        const int32_t s0 = S(d, 4 * q);
        for (int i = 1; i < 4; ++i) r[i - 1] = 4 * q + i < nchan ? S(d, 4 * q + i) - s0 : 0;
        return s0;
    };
    for (int d = 0; d < p->ndm; ++d)
        for (int q = 0; q < nq; ++q) {
            int32_t r[3];
            key(d, q, r);
            for (int32_t v : r)
                if (v < 0 || v > kQuadMaxResidual)
                    return fail(AA_EINVAL, "quad tiling: a residual within a channel quad exceeds 1023 samples");
        }
    blocks.clear();
    std::vector<std::vector<QuadPat>> st(nq);
    for (int d0 = 0; d0 < p->ndm;) {
        for (auto& v : st) v.clear();
        int count = 0;
        while (count < kQuadTrials && d0 + count < p->ndm) {
            const int d = d0 + count;
            bool ok = true;
            for (int q = 0; q < nq && ok; ++q) {
                int32_t r[3];
                const int32_t s0 = key(d, q, r);
                int64_t used = 0;
                bool found = false;
                for (const QuadPat& P : st[q]) {
                    int32_t lo = P.lo, hi = P.hi;
                    if (P.r1 == r[0] && P.r2 == r[1] && P.r3 == r[2]) {
                        lo = std::min(lo, s0);
                        hi = std::max(hi, s0);
                        found = true;
                    }
                    used += (quad_units(tile, lo, hi) + 63) / 64;
                }
                if (!found) {
                    if (static_cast<int>(st[q].size()) >= kQuadMaxPat) ok = false;
                    used += (quad_units(tile, s0, s0) + 63) / 64;
                }
                if (used > chunks) ok = false;
            }
            if (!ok) break;
            for (int q = 0; q < nq; ++q) {
                int32_t r[3];
                const int32_t s0 = key(d, q, r);
                bool found = false;
                for (QuadPat& P : st[q])
                    if (P.r1 == r[0] && P.r2 == r[1] && P.r3 == r[2]) {
                        P.lo = std::min(P.lo, s0);
                        P.hi = std::max(P.hi, s0);
                        found = true;
                    }
                if (!found) st[q].push_back(QuadPat{r[0], r[1], r[2], s0, s0});
            }
            ++count;
        }
        if (count < 1) return fail(AA_EINVAL, "quad tiling: a single trial does not fit");
        blocks.push_back(DmBlock{d0, count, 0, 0, 0, 4, 0});
        d0 += count;
    }
    // records: entry e of a block holds the trial offsets of step e - 1 and the chunks
    // of step e (entries 0 .. nq)
    const size_t nblk = blocks.size(), nrec = static_cast<size_t>(nq) + 1;
    const size_t rd = static_cast<size_t>(quad_rec_dwords(chunks));
    rec.assign(nblk * nrec * rd, 0);
    for (size_t bi = 0; bi < nblk; ++bi) {
        DmBlock& b = blocks[bi];
        b.rec256 = static_cast<int32_t>(bi * nrec * rd / 64);
        for (int q = 0; q < nq; ++q) {
            std::vector<QuadPat> pats;
            std::vector<int> which(b.count);
            for (int i = 0; i < b.count; ++i) {
                int32_t r[3];
                const int32_t s0 = key(b.first + i, q, r);
                int k = 0;
                while (k < static_cast<int>(pats.size()) &&
                       !(pats[k].r1 == r[0] && pats[k].r2 == r[1] && pats[k].r3 == r[2]))
                    ++k;
                if (k == static_cast<int>(pats.size())) pats.push_back(QuadPat{r[0], r[1], r[2], s0, s0});
                pats[k].lo = std::min(pats[k].lo, s0);
                pats[k].hi = std::max(pats[k].hi, s0);
                which[i] = k;
            }
            int32_t* P = &rec[(bi * nrec + q) * rd];        // chunks of step q
            int32_t* O = &rec[(bi * nrec + q + 1) * rd];    // trial offsets of step q
            int64_t nch = 0;
            std::vector<int64_t> first_chunk(pats.size());
            for (size_t k = 0; k < pats.size(); ++k) {
                const QuadPat& Q = pats[k];
                const int64_t units = quad_units(tile, Q.lo, Q.hi), n = (units + 63) / 64;
                first_chunk[k] = nch;
                if (pats.size() > static_cast<size_t>(kQuadMaxPat) || nch + n > chunks)
                    return fail(AA_EINVAL, "quad tiling: step tables exceed the chunk budget");
                for (int64_t c = 0; c < n; ++c) {
                    int32_t* C = P + 64 + 4 * (nch + c);
                    C[0] = static_cast<int32_t>(Q.lo + 256 * c);
                    C[1] = static_cast<int32_t>(Q.lo + Q.r1 + 256 * c);
                    C[2] = static_cast<int32_t>(Q.lo + Q.r2 + 256 * c);
                    C[3] = static_cast<int32_t>(Q.lo + Q.r3 + 256 * c);
                    for (int i = 1; i < 4; ++i)
                        if (4 * q + i >= nchan) C[i] = kQuadNoRow;
                }
                nch += n;
            }
            P[32] = static_cast<int32_t>(nch);
            for (int i = 0; i < b.count; ++i) {
                const QuadPat& Q = pats[which[i]];
                const uint32_t off = static_cast<uint32_t>(4 * (256 * first_chunk[which[i]] + S(b.first + i, 4 * q) - Q.lo));
                O[i / 2] = static_cast<int32_t>(static_cast<uint32_t>(O[i / 2]) | (off << (16 * (i & 1))));
            }
        }
    }
    return AA_OK;
}

namespace {
int prepare_quad(const aa_plan_s* p, const DedispVariant& V, DedispTables& t) {
    std::vector<DmBlock> blocks;
    std::vector<int32_t> rec;
    const int rc0 = build_quad_tables(p, V.tile, V.depth, blocks, rec);
    if (rc0 != AA_OK) return rc0;
    t.bd = kQuadTrials;
    t.nchan_pad = (p->nchan + 3) / 4 * 4;
    t.max_row = 0;
    t.blocks = blocks;
    if (p->device >= 0) {
        int rc = upload(&t.d_blocks, blocks);
        if (rc == AA_OK) rc = upload(&t.d_offs, rec);
        if (rc != AA_OK) return rc;
    }
    return AA_OK;
}

int prepare_mfma(const aa_plan_s* p, const DedispVariant& V, DedispTables& t, int split_at = -1) {
    std::vector<DmBlock> blocks;
    std::vector<int32_t> rsv;
    std::vector<uint8_t> rec;
    const int cps = mfma_cps(V.layout);   // 0: mixed by trial range
    const int rc0 = build_mfma_tables(p, V.tile, V.depth, V.max_tiles, cps, blocks, rsv, rec, split_at, &t.split);
    if (rc0 != AA_OK) return rc0;
    t.bd = 32;
    t.nchan_pad = cps == 4 ? (p->nchan + 3) / 4 * 4 : (p->nchan + 7) / 8 * 8;
    t.max_row = mfma_row_bytes(V.max_tiles);
    t.blocks = blocks;
    if (p->device >= 0) {
        std::vector<uint8_t> pad(t.max_row, 0x80);
        int rc = upload(&t.d_blocks, blocks);
        if (rc == AA_OK) rc = upload(&t.d_base, rsv);
        if (rc == AA_OK) rc = upload(reinterpret_cast<uint8_t**>(&t.d_offs), rec);
        if (rc == AA_OK) rc = upload(&t.d_pad, pad);
        if (rc != AA_OK) return rc;
    }
    return AA_OK;
}
}  // namespace

int prepare_mixed_split(aa_plan_s* p, int v, int split) {
    if (v < 0 || v >= kNumDedispVariants || kDedispVariants[v].layout != 6)
        return fail(AA_EINVAL, "prepare_mixed_split: not a mixed-shape variant");
    DedispTables t;
    t.variant = v;
    const int rc = prepare_mfma(p, kDedispVariants[v], t, std::max(0, std::min(split, p->ndm)));
    if (rc != AA_OK) {
        free_tables(t);
        return rc;
    }
    free_tables(p->tables[v]);
    p->tables[v] = t;
    return AA_OK;
}

int prepare_variant(aa_plan_s* p, int v) {
    if (v < 0 || v >= kNumDedispVariants) return fail(AA_EINVAL, "unknown dedispersion variant");
    DedispTables& T = p->tables[v];
    if (T.variant == v) return AA_OK;
    const DedispVariant& V = kDedispVariants[v];
    if (V.layout >= 4) {
        DedispTables t;
        t.variant = v;
        const int rc = V.layout == 7 ? prepare_quad(p, V, t) : prepare_mfma(p, V, t);
        if (rc != AA_OK) {
            free_tables(t);
            return rc;
        }
        T = t;
        return AA_OK;
    }
    const int bd = V.waves * V.dpw;
    const int row_max = (V.lds_bytes / (2 * kChanPerPass)) & ~15;
    const int nchan = p->nchan;
    const int nchan_pad = (nchan + kChanPerPass - 1) / kChanPerPass * kChanPerPass;

    // Greedy blocks: up to bd consecutive trials whose windows fit one staged row.
    std::vector<DmBlock> blocks;
    int32_t max_row = 0;
    for (int d = 0; d < p->ndm;) {
        const int32_t* s0 = &p->shifts[static_cast<size_t>(d) * nchan];
        int32_t omax = 0;
        int count = 0;
        while (count < bd && d + count < p->ndm) {
            const int32_t* sd = &p->shifts[static_cast<size_t>(d + count) * nchan];
            int32_t m = 0;
            for (int c = 0; c < nchan; ++c) m = std::max(m, sd[c] - (s0[c] & ~15));
            const int32_t row = kTimeTile + 16 + (std::max(omax, m) & ~15);
            if (count > 0 && row > row_max) break;
            omax = std::max(omax, m);
            ++count;
        }
        DmBlock b{d, count, kTimeTile + 16 + (omax & ~15), 0, 0, 0, 0};
        if (b.row > row_max) return fail(AA_EINVAL, "dedispersion tiling: a single trial does not fit the LDS row");
        max_row = std::max(max_row, b.row);
        blocks.push_back(b);
        d += count;
    }
    const size_t nblk = blocks.size();
    std::vector<int32_t> base(nblk * nchan_pad, 0);
    std::vector<int32_t> offs(nblk * nchan_pad * bd, 0);
    for (size_t k = 0; k < nblk; ++k) {
        const DmBlock& b = blocks[k];
        const int32_t* s0 = &p->shifts[static_cast<size_t>(b.first) * nchan];
        for (int c = 0; c < nchan; ++c) {
            const int32_t bc = s0[c] & ~15;
            base[k * nchan_pad + c] = bc;
            for (int i = 0; i < b.count; ++i)
                offs[(k * nchan_pad + c) * bd + i] = p->shifts[static_cast<size_t>(b.first + i) * nchan + c] - bc;
        }
    }
    DedispTables t;
    t.variant = v;
    t.bd = bd;
    t.nchan_pad = nchan_pad;
    t.max_row = max_row;
    t.blocks = blocks;
    if (p->device >= 0) {
        int rc = upload(&t.d_blocks, blocks);
        if (rc == AA_OK) rc = upload(&t.d_base, base);
        if (rc == AA_OK) rc = upload(&t.d_offs, offs);
        if (rc != AA_OK) {
            free_tables(t);
            return rc;
        }
    }
    T = t;
    return AA_OK;
}

}  // namespace aa
