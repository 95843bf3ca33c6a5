// Dedispersion tiling tables. Built on the host and uploaded once, at plan time or
// when the tuner prepares a variant. Nothing here runs in the hot loop.
#include <algorithm>

#include "aa_internal.h"

namespace aa {

// LDS budgets are sized so that 3 (52 KB) or 2 (80 KB) work-groups fit in one CU's
// 160 KB of LDS.
const DedispVariant kDedispVariants[kNumDedispVariants] = {
    {0, 4, 4, 53248, 1},    // 256 threads, 16 trials per block, interleaved lanes
    {1, 8, 2, 53248, 1},    // 512 threads, 16 trials per block, interleaved lanes
    {2, 8, 4, 81920, 1},    // 512 threads, 32 trials per block, interleaved lanes
    {3, 16, 2, 81920, 1},   // 1024 threads, 32 trials per block, interleaved lanes
    {4, 8, 2, 53248, 0},    // 512 threads, 16 trials per block, contiguous lanes
    {5, 4, 4, 53248, 0},    // 256 threads, 16 trials per block, contiguous lanes
    {6, 8, 2, 53248, 3},    // 512 threads, 16 trials per block, contiguous lanes, 16-way switch
    {7, 4, 4, 53248, 3},    // 256 threads, 16 trials per block, contiguous lanes, 16-way switch
    {8, 8, 2, 53248, 2},    // 512 threads, 16 trials per block, interleaved, equal-offset reuse
    {9, 8, 4, 81920, 2},    // 512 threads, 32 trials per block, interleaved, equal-offset reuse
    {10, 4, 4, 53248, 2},   // 256 threads, 16 trials per block, interleaved, equal-offset reuse
};

void free_tables(DedispTables& t) {
    if (t.d_blocks) (void)hipFree(t.d_blocks);
    if (t.d_base) (void)hipFree(t.d_base);
    if (t.d_offs) (void)hipFree(t.d_offs);
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

int prepare_variant(aa_plan_s* p, int v) {
    if (v < 0 || v >= kNumDedispVariants) return fail(AA_EINVAL, "unknown dedispersion variant");
    DedispTables& T = p->tables[v];
    if (T.variant == v) return AA_OK;
    const DedispVariant& V = kDedispVariants[v];
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
        DmBlock b{d, count, kTimeTile + 16 + (omax & ~15), 0};
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
