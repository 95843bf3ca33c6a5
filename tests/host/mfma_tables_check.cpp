// Host check of the matrix-core dedispersion tables (layouts 4-6): a scalar model of the
// kernel's steps (staging with the same row starts, lengths and clamps, one-hot
// residual selection, per-block flush at t' - e) over the tables that build_mfma_tables
// produces, compared with D[d][t] = sum_c X[c][t + s[d][c]] computed directly.
// Host-only plan: no GPU needed. Usage: mfma_tables_check TILE DEPTH [MAX_TILES [CPS [SPLIT]]]
// CPS 0 mixes the step shapes by trial range; SPLIT (a fraction of the trials, or -1 for
// the cost estimate's choice) places the change of shape.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include "../../paper_2101_00941_amd/csrc/aa_internal.h"

using namespace aa;

static int TILE = 1024, DEPTH = 3, MAXT = 63, CPS_ARG = 4;
static double SPLIT = -1.0;
static int run_case(int nchan, int nsamp, double ftop, double foff, double tsamp, std::vector<double> dms, unsigned seed,
                    int max_tiles_check = 1 << 30) {
    aa_plan_desc_t d{};
    d.nchan = nchan; d.nsamp = nsamp; d.f_top_mhz = ftop; d.foff_mhz = foff; d.tsamp_s = tsamp;
    d.dm = dms.data(); d.ndm = (int)dms.size();
    int32_t widths[2] = {1, 2};
    d.widths = widths; d.nwidths = 2; d.snr_threshold = 1e9f; d.stat_block = 0; d.flags = AA_PLAN_HOST_ONLY;
    aa_plan_t p = nullptr;
    if (aa_plan(&d, &p) != AA_OK) { printf("plan failed: %s\n", aa_last_error()); return 1; }
    std::vector<DmBlock> blocks; std::vector<int32_t> rsv; std::vector<uint8_t> rec;
    const int ROW = mfma_row_bytes(MAXT);
    const int split = SPLIT < 0 ? -1 : (int)(SPLIT * dms.size());
    if (build_mfma_tables(p, TILE, DEPTH, MAXT, CPS_ARG, blocks, rsv, rec, split) != AA_OK) { printf("tables failed: %s\n", aa_last_error()); return 1; }
    const int npad = CPS_ARG == 4 ? (nchan + 3) / 4 * 4 : (nchan + 7) / 8 * 8;
    // blocks cover the trials in order; a mixed table has its 8-channel blocks first
    {
        int next = 0, prev_cps = 8;
        size_t rec_at = 0;
        for (const DmBlock& b : blocks) {
            if (b.first != next || b.count < 1 || b.count > 32) { printf("blocks do not tile the trials\n"); return 1; }
            if (b.cps != 4 && b.cps != 8) { printf("bad block shape %d\n", b.cps); return 1; }
            if (CPS_ARG != 0 && b.cps != CPS_ARG) { printf("block shape differs from the variant's\n"); return 1; }
            if (CPS_ARG == 0 && b.cps > prev_cps) { printf("8-channel block after a 4-channel block\n"); return 1; }
            if ((size_t)b.rec256 * 256 != rec_at) { printf("record offsets not packed\n"); return 1; }
            rec_at += (size_t)(npad / b.cps) * mfma_rec(b.cps).size;
            next += b.count;
            prev_cps = b.cps;
        }
        if (next != (int)dms.size() || rec_at != rec.size() || rsv.size() != blocks.size() * npad) {
            printf("table sizes\n");
            return 1;
        }
        if (CPS_ARG == 0 && split >= 0)
            for (const DmBlock& b : blocks)
                if ((b.cps == 8) != (b.first < split) || (b.cps == 8 && b.first + b.count > split)) {
                    printf("block shape does not follow the split\n");
                    return 1;
                }
    }
    int n8 = 0;
    for (const DmBlock& b : blocks) n8 += b.cps == 8;
    const int64_t M = p->maxshift, n_out = nsamp - M;
    const int64_t pitch = (nsamp + 255) / 256 * 256;
    const int64_t n_in16 = (nsamp + 15) & ~15;
    std::vector<uint8_t> x(nchan * pitch, 0xEE);
    std::mt19937 g(seed);
    for (int c = 0; c < nchan; ++c) for (int t = 0; t < nsamp; ++t) x[c * pitch + t] = g() & 255;
    auto S = [&](int dd, int c) { return p->shifts[(size_t)dd * nchan + c]; };
    const int64_t ntile = (n_out + TILE - 1) / TILE;
    long bad = 0, checked = 0;
    int maxnr = 0; double sumcb = 0; int ncb = 0;
    int tiles_done = 0;
    for (size_t bi = 0; bi < blocks.size(); ++bi) {
        const int CPS = blocks[bi].cps;
        const MfmaRec RL = mfma_rec(CPS);
        const int RES = 32 / CPS;                      // residual range
        const int nchan4 = npad, K4 = nchan4 / CPS;
        const uint8_t* R = &rec[(size_t)blocks[bi].rec256 * 256];
        for (int k = 0; k < K4; ++k) if (*(int32_t*)(R + k * RL.size + RL.left) == 1) ncb++;
        for (int64_t ti = 0; ti < ntile && tiles_done < max_tiles_check; ++ti, ++tiles_done) {
            const int64_t t0 = ti * TILE;
            std::vector<int64_t> acc(TILE * 32, 0);
            std::vector<int64_t> C(64 * 32 * 32, 0);
            std::vector<int32_t> rs_hist(K4 * 4);
            for (int k = 0; k < K4; ++k) {
                const uint8_t* rk = R + (size_t)k * RL.size;
                // row starts as the kernel obtains them
                int rs[8];
                int need = ROW / 16;
                for (int i = 0; i < CPS; ++i)
                    rs[i] = k < DEPTH - 1 ? rsv[bi * nchan4 + CPS * k + i] : *(const int32_t*)(R + (size_t)(k - DEPTH + 1) * RL.size + RL.next_rs + 4 * i);
                if (k >= DEPTH - 1) need = *(const int32_t*)(R + (size_t)(k - DEPTH + 1) * RL.size + RL.next_need);
                static uint8_t row[8][2048];
                for (int i = 0; i < CPS; ++i) {
                    const int c = CPS * k + i;
                    for (int v0 = 0; v0 < ROW / 16; ++v0) {
                        const int v = v0 < need ? v0 : 0;
                        int64_t pos = t0 + rs[i] + 16 * v;
                        pos = pos < 0 ? 0 : (pos > n_in16 - 16 ? n_in16 - 16 : pos);
                        for (int b = 0; b < 16; ++b) row[i][16 * v0 + b] = c < nchan ? x[c * pitch + pos + b] : 0x80;
                    }
                }
                const int nr = *(const int32_t*)(rk + RL.tiles);
                const int left = *(const int32_t*)(rk + RL.left);
                const int endf = left == 1;
                // a channel block is a run of steps with one tile count and a step count
                // that counts down to 1
                if (k > 0) {
                    const uint8_t* rp = rk - RL.size;
                    const int pleft = *(const int32_t*)(rp + RL.left);
                    if (pleft > 1 && (pleft != left + 1 || *(const int32_t*)(rp + RL.tiles) != *(const int32_t*)(rk + RL.tiles))) {
                        printf("inconsistent block record at step %d\n", k);
                        return 1;
                    }
                }
                if (left < 1 || k + left > K4) { printf("bad step count %d at step %d\n", left, k); return 1; }
                {
                    int emax = 0;
                    for (int dd = 0; dd < blocks[bi].count; ++dd) {
                        const int e = *(const int16_t*)(rk + RL.e + 2 * dd);
                        if (e < 0) { printf("negative e\n"); return 1; }
                        emax = e > emax ? e : emax;
                    }
                    if (emax != *(const int32_t*)(rk + RL.max_e)) { printf("max e mismatch at step %d\n", k); return 1; }
                }
                if (nr > maxnr) maxnr = nr;
                if (nr > MAXT || nr < TILE / 32) { printf("bad nr %d\n", nr); return 1; }
                for (int q = 0; q < nr; ++q)
                    for (int mrow = 0; mrow < 32; ++mrow)
                        for (int dd = 0; dd < 32; ++dd) {
                            int64_t s = 0;
                            for (int ch = 0; ch < CPS; ++ch) {
                                const int r = rk[CPS * dd + ch] / 8;
                                if (r >= RES) { printf("residual out of range\n"); return 1; }
                                const int ph = rk[RL.phase + ch];
                                // the kernel reads the aligned dwords covering the R-byte window
                                const int a = 32 * q + mrow + ph;
                                if ((a & ~3) + (RES == 8 ? 12 : 8) > ROW) { printf("window past row\n"); return 1; }
                                const int P = a + r;
                                s += (int)(int8_t)(row[ch][P] ^ 0x80);   // (x ^ 0x80) as int8 = x - 128
                            }
                            C[(q * 32 + mrow) * 32 + dd] += s;
                        }
                if (endf) {
                    for (int q = 0; q < nr; ++q)
                        for (int mrow = 0; mrow < 32; ++mrow)
                            for (int dd = 0; dd < 32; ++dd) {
                                const int e = *(const int16_t*)(rk + RL.e + 2 * dd);
                                const int t = 32 * q + mrow - e;
                                if (t >= 0 && t < TILE) acc[t * 32 + dd] += C[(q * 32 + mrow) * 32 + dd];
                            }
                    std::fill(C.begin(), C.end(), 0);
                }
            }
            for (int dd = 0; dd < blocks[bi].count; ++dd)
                for (int t = 0; t < TILE && t0 + t < n_out; ++t) {
                    const int64_t got = acc[t * 32 + dd] + 128 * nchan;
                    int64_t want = 0;
                    const int dm = blocks[bi].first + dd;
                    for (int c = 0; c < nchan; ++c) want += x[c * pitch + t0 + t + S(dm, c)];
                    ++checked;
                    if (got != want && bad++ < 5) printf("mismatch blk %zu d %d t %lld got %lld want %lld\n", bi, dm, (long long)(t0 + t), (long long)got, (long long)want);
                }
        }
    }
    printf("nchan %d nsamp %d ndm %zu: blocks %zu (%d of 8 channels per step), channel blocks %d, max nr %d, checked %ld, bad %ld\n",
           nchan, nsamp, dms.size(), blocks.size(), n8, ncb, maxnr, checked, bad);
    aa_plan_destroy(p);
    return bad != 0;
}
int main(int argc, char** argv) {
    if (argc > 2) { TILE = atoi(argv[1]); DEPTH = atoi(argv[2]); }
    if (argc > 3) MAXT = atoi(argv[3]);
    if (argc > 4) CPS_ARG = atoi(argv[4]);
    if (argc > 5) SPLIT = atof(argv[5]);
    printf("tile %d depth %d max tiles %d channels per step %d split %g\n", TILE, DEPTH, MAXT, CPS_ARG, SPLIT);
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
    // survey-like: 4096 channels, steep DMs, a few time tiles only
    std::vector<double> ds; for (int i = 0; i < 64; ++i) ds.push_back(1500.0 + 2.0 * i);
    rc |= run_case(4096, 40000, 1450.0, 300.0 / 4096, 64e-6, ds, 7, 2);
    printf(rc ? "FAIL\n" : "ALL OK\n");
    return rc;
}
namespace aa {
size_t sps_work_bytes(const aa_plan_s*, int64_t) { return 0; }
int launch_dedisperse(const aa_plan_s*, int, const uint8_t*, int64_t, int64_t, int32_t*, int64_t, hipStream_t) { return -1; }
}
extern "C" int aa_dedisperse(aa_plan_t, const uint8_t*, int64_t, int64_t, int32_t*, int64_t, void*) { return -1; }
