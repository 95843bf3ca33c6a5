// Host check of the quad dedispersion tables (layout 7): a scalar model of the kernel's
// steps over the tables that build_quad_tables produces, compared with
// D[d][t] = sum_c X[c][t + s[d][c]] computed directly. The model stages each step the
// way the kernel does (64-unit chunks at recorded row offsets, two aligned dwords per
// channel and unit, byte alignment, 4x4 transpose, whole chunks written), then sums every
// trial's dwords at its recorded offset. Loads follow the kernel's per-quad buffer range
// (a row's loads past its n_in16 read the next row's bytes, and the pitch padding, which
// only samples past n_out see; rows past nchan read zero and are never touched); the
// model also checks that every LDS access stays inside the step buffer.
// Host-only plan: no GPU needed. Usage: quad_tables_check TILE CHUNKS
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include "../../paper_2101_00941_amd/csrc/aa_internal.h"

using namespace aa;

static int TILE = 1024, CHUNKS = 24;

static int run_case(int nchan, int nsamp, double ftop, double foff, double tsamp, std::vector<double> dms, unsigned seed,
                    int max_tiles_check = 1 << 30) {
    aa_plan_desc_t d{};
    d.nchan = nchan; d.nsamp = nsamp; d.f_top_mhz = ftop; d.foff_mhz = foff; d.tsamp_s = tsamp;
    d.dm = dms.data(); d.ndm = (int)dms.size();
    int32_t widths[2] = {1, 2};
    d.widths = widths; d.nwidths = 2; d.snr_threshold = 1e9f; d.stat_block = 0; d.flags = AA_PLAN_HOST_ONLY;
    aa_plan_t p = nullptr;
    if (aa_plan(&d, &p) != AA_OK) { printf("plan failed: %s\n", aa_last_error()); return 1; }
    std::vector<DmBlock> blocks;
    std::vector<int32_t> rec;
    if (build_quad_tables(p, TILE, CHUNKS, blocks, rec) != AA_OK) { printf("tables failed: %s\n", aa_last_error()); return 1; }
    const int nq = (nchan + 3) / 4;
    {
        int next = 0;
        for (size_t bi = 0; bi < blocks.size(); ++bi) {
            const DmBlock& b = blocks[bi];
            if (b.first != next || b.count < 1 || b.count > kQuadTrials) {
                printf("blocks do not tile the trials\n");
                return 1;
            }
            next += b.count;
        }
        const size_t rd = quad_rec_dwords(CHUNKS);
        if (next != (int)dms.size() || rec.size() != blocks.size() * (nq + 1) * rd) { printf("table sizes\n"); return 1; }
        for (size_t bi = 0; bi < blocks.size(); ++bi)
            if ((size_t)blocks[bi].rec256 * 64 != bi * (nq + 1) * rd) { printf("record offsets\n"); return 1; }
    }
    const int64_t M = p->maxshift, n_out = nsamp - M;
    const int64_t pitch = (nsamp + 255) / 256 * 256;
    const int64_t n_in16 = (nsamp + 15) & ~15;
    std::vector<uint8_t> x(nchan * pitch, 0xEE);
    std::mt19937 g(seed);
    for (int c = 0; c < nchan; ++c) for (int t = 0; t < nsamp; ++t) x[c * pitch + t] = g() & 255;
    auto S = [&](int dd, int c) { return p->shifts[(size_t)dd * nchan + c]; };
    const int64_t ntile = (n_out + TILE - 1) / TILE;
    const int BUFD = CHUNKS * 256;   // dwords per step buffer
    long bad = 0, checked = 0, oob = 0;
    int full = 0;
    double chunks_used = 0, steps = 0;
    int tiles_done = 0;
    std::vector<uint32_t> buf(BUFD);
    for (size_t bi = 0; bi < blocks.size(); ++bi) {
        const DmBlock& b = blocks[bi];
        full += b.count == kQuadTrials;
        for (int64_t ti = 0; ti < ntile && tiles_done < max_tiles_check; ++ti, ++tiles_done) {
            // take the first tiles, the last two and every 7th in between
            if (ti > 2 && ti + 2 < ntile && ti % 7 != 0) continue;
            const int64_t t0 = ti * TILE;
            std::vector<uint64_t> acc((size_t)kQuadTrials * TILE, 0);
            const size_t rd = quad_rec_dwords(CHUNKS);
            for (int q = 0; q < nq; ++q) {
                const int32_t* P = &rec[(size_t)b.rec256 * 64 + (size_t)q * rd];        // chunks of step q
                const int32_t* R = &rec[(size_t)b.rec256 * 64 + (size_t)(q + 1) * rd];  // trial offsets of step q
                const int nch = P[32];
                if (nch < 1 || nch > CHUNKS) { printf("bad chunk count\n"); return 1; }
                chunks_used += nch;
                steps += 1;
                std::fill(buf.begin(), buf.end(), 0xDEADBEEFu);
                for (int j = 0; j < nch; ++j) {
                    for (int lane = 0; lane < 64; ++lane) {
                        uint32_t v[4];
                        for (int i = 0; i < 4; ++i) {
                            const int c = 4 * q + i;
                            const int32_t o = P[64 + 4 * j + i];
                            if (c >= nchan && o != kQuadNoRow) { printf("a row past nchan without the no-row offset\n"); return 1; }
                            // one range per quad from its first row to n_in16 past the start of
                            // its last existing row; row i at i * pitch within it; dword loads
                            const int64_t a = t0 + (o & ~3) + 4 * lane;
                            const int64_t last = std::min(3, nchan - 1 - 4 * q);
                            const int64_t range = last * pitch + n_in16;
                            uint32_t w[2] = {0, 0};
                            for (int h = 0; h < 2; ++h) {
                                const int64_t ah = a + 4 * h;
                                if (ah < 0) { ++oob; continue; }
                                const int64_t at = i * pitch + ah;   // offset from the quad's first row
                                if (at + 4 <= range) {
                                    if (c >= nchan) { printf("a load of a row past nchan\n"); return 1; }
                                    if ((size_t)(4 * q) * pitch + at + 4 > x.size()) { printf("a load past the input\n"); return 1; }
                                    memcpy(&w[h], &x[(size_t)(4 * q) * pitch + at], 4);
                                }
                            }
                            v[i] = (uint32_t)((((uint64_t)w[1] << 32) | w[0]) >> (8 * (o & 3)));
                        }
                        const int64_t k = 256 * (int64_t)j + 4 * lane;
                        if (k < 0 || k + 4 > BUFD) { printf("staging write past the buffer\n"); return 1; }
                        for (int m = 0; m < 4; ++m)
                            buf[k + m] = ((v[0] >> (8 * m)) & 255u) | (((v[1] >> (8 * m)) & 255u) << 8) |
                                         (((v[2] >> (8 * m)) & 255u) << 16) | (((v[3] >> (8 * m)) & 255u) << 24);
                    }
                }
                for (int dd = 0; dd < kQuadTrials; ++dd) {
                    const int32_t off = (int32_t)(((uint32_t)R[dd / 2] >> (16 * (dd & 1))) & 0xFFFFu);
                    if (off & 3) { printf("unaligned trial offset\n"); return 1; }
                    if (dd >= b.count && off != 0) { printf("absent trial with an offset\n"); return 1; }
                    for (int t = 0; t < TILE; ++t) {
                        const int64_t k = off / 4 + t;
                        if (k < 0 || k >= BUFD) { printf("trial read past the buffer\n"); return 1; }
                        if (dd >= b.count) continue;
                        const uint32_t y = buf[k];
                        acc[(size_t)dd * TILE + t] += (y & 255u) + ((y >> 8) & 255u) + ((y >> 16) & 255u) + (y >> 24);
                    }
                }
            }
            for (int dd = 0; dd < b.count; ++dd)
                for (int t = 0; t < TILE && t0 + t < n_out; ++t) {
                    int64_t want = 0;
                    const int dm = b.first + dd;
                    for (int c = 0; c < nchan; ++c) want += x[c * pitch + t0 + t + S(dm, c)];
                    ++checked;
                    const int64_t got = (int64_t)acc[(size_t)dd * TILE + t];
                    if (got != want && bad++ < 5)
                        printf("mismatch blk %zu d %d t %lld got %lld want %lld\n", bi, dm, (long long)(t0 + t), (long long)got,
                               (long long)want);
                }
        }
    }
    printf("nchan %d nsamp %d ndm %zu: blocks %zu (%d full), mean chunks per step %.2f, checked %ld, bad %ld, "
           "negative offsets %ld\n",
           nchan, nsamp, dms.size(), blocks.size(), full, chunks_used / (steps > 0 ? steps : 1), checked, bad, oob);
    aa_plan_destroy(p);
    return bad != 0 || oob != 0;
}

int main(int argc, char** argv) {
    if (argc > 2) { TILE = atoi(argv[1]); CHUNKS = atoi(argv[2]); }
    printf("tile %d chunks %d\n", TILE, CHUNKS);
    int rc = 0;
    rc |= run_case(1, 3000, 1400.0, 1.0, 64e-6, {0.0, 10.0, 100.0}, 1);
    rc |= run_case(7, 5003, 1500.0, 3.0, 64e-6, {0, 12.5, 25, 37.5, 50}, 2);
    std::vector<double> d17; for (int i = 0; i < 17; ++i) d17.push_back(3.0 * i);
    rc |= run_case(33, 4099, 1500.0, 1.0, 64e-6, d17, 3);
    std::vector<double> d40; for (int i = 0; i < 40; ++i) d40.push_back(2.0 * i);
    rc |= run_case(300, 10000, 1450.0, 1.0, 64e-6, d40, 4);
    std::vector<double> d9; for (int i = 0; i < 9; ++i) d9.push_back(60.0 * i);
    rc |= run_case(48, 60000, 1200.0, 4.0, 64e-6, d9, 5, 6);
    std::vector<double> d21; for (int i = 0; i < 21; ++i) d21.push_back(1.0 * i);
    rc |= run_case(257, 8000, 1500.0, 0.5, 64e-6, d21, 6);
    // survey-like: 4096 channels, steep DMs (many patterns per quad), a few time tiles only
    std::vector<double> ds; for (int i = 0; i < 64; ++i) ds.push_back(1500.0 + 2.0 * i);
    rc |= run_case(4096, 40000, 1450.0, 300.0 / 4096, 64e-6, ds, 7, 3);
    // low DMs on the survey band: long runs of one pattern
    std::vector<double> dl; for (int i = 0; i < 40; ++i) dl.push_back(i / 16.0);
    rc |= run_case(4096, 12000, 1450.0, 300.0 / 4096, 64e-6, dl, 8, 3);
    printf(rc ? "FAIL\n" : "ALL OK\n");
    return rc;
}
namespace aa {
size_t sps_work_bytes(const aa_plan_s*, int64_t) { return 0; }
int launch_dedisperse(const aa_plan_s*, int, const uint8_t*, int64_t, int64_t, int32_t*, int64_t, hipStream_t) { return -1; }
}
extern "C" int aa_dedisperse(aa_plan_t, const uint8_t*, int64_t, int64_t, int32_t*, int64_t, void*) { return -1; }
