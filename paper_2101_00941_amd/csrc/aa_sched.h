// Host-side scheduling logic of the streamed pipeline, kept free of HIP so that CPU
// tests can compile it on its own: the device-arena allocator, the computable start
// range of a chunk, and the block-aligned split of a range into sub-chunks.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>
#include <vector>

namespace aa {

constexpr size_t kArenaAlign = 256;
inline size_t arena_round(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size) in 256-byte granules, with coalescing on free.
class Arena {
public:
    uint8_t* base = nullptr;
    size_t size = 0, used = 0, peak = 0;
    void init(uint8_t* b, size_t n) {
        base = b;
        size = n / kArenaAlign * kArenaAlign;
        used = peak = 0;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t* off) {
        n = arena_round(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = arena_round(n ? n : 1);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;
};

// Starts that become computable once R2 samples have been received: [e, e2).
// Without `last`, the right neighbour column (boxcars included) must be present
// (e2 + wmax - 1 + maxshift <= R2 - 1), and e2 is a multiple of the stat block. With
// `last`, e2 is the total number of starts T = R2 - maxshift - wmax + 1.
struct ChunkRange {
    int64_t e2;
    int64_t t_total;   // T with `last`, else -1
};

inline ChunkRange chunk_range(int64_t e, int64_t R2, int64_t maxshift, int64_t wmax, int64_t block, bool last) {
    ChunkRange c{e, -1};
    if (last) {
        c.t_total = std::max<int64_t>(R2 - maxshift - wmax + 1, 0);
        c.e2 = c.t_total;
    } else {
        const int64_t lim = R2 - wmax - maxshift;
        c.e2 = lim >= 0 ? lim / block * block : 0;
    }
    if (c.e2 < e) c.e2 = e;
    return c;
}

struct Piece {
    int64_t a, b;
};

// Split [e, e2) into at most `parts` pieces of whole stat blocks (the last may be partial).
inline std::vector<Piece> split_blocks(int64_t e, int64_t e2, int64_t block, int parts) {
    std::vector<Piece> out;
    if (e2 <= e || parts < 1) return out;
    const int64_t nb = (e2 - e + block - 1) / block;
    const int64_t n = std::min<int64_t>(parts, nb);
    int64_t a = e;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t blocks = nb / n + (j < nb % n ? 1 : 0);
        const int64_t b = std::min(e2, a + blocks * block);
        out.push_back({a, b});
        a = b;
    }
    return out;
}

// Number of sub-chunks for a range of `work` DM-trial x channel x start units. The
// range is split over at most `nstreams` compute streams, but no piece gets less than
// `min_work` units: splitting a small chunk only adds launches, events and copies per
// piece, and the streams still overlap consecutive chunks. min_work <= 0 always splits
// into nstreams pieces.
inline int sub_chunks(int64_t work, int64_t min_work, int nstreams) {
    if (nstreams < 1) return 1;
    if (min_work <= 0) return nstreams;
    const int64_t k = work / min_work;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nstreams, k)));
}

// Input window [w0, w1) of a piece, with w0 rounded down to a 16-byte column of the
// beam history (whose column 0 holds absolute sample h0).
inline void piece_window(const Piece& pc, int64_t h0, int64_t R2, int64_t maxshift, int64_t wmax, int64_t* w0,
                         int64_t* w1) {
    *w0 = h0 + ((std::max<int64_t>(pc.a - 1, 0) - h0) & ~int64_t{15});
    *w1 = std::min(pc.b + wmax + maxshift, R2);
}

}  // namespace aa
