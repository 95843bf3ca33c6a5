// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/aa.h"

namespace aa {

// Thread-local error message behind aa_last_error().
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define AA_HIP(call)                                         \
    do {                                                     \
        hipError_t aa_e_ = (call);                           \
        if (aa_e_ != hipSuccess) return ::aa::hip_fail(aa_e_, #call); \
    } while (0)

// Dedispersion tiling. A work-group of `waves` waves owns one DM block of up to
// waves * dpw consecutive trials and one time tile of 1024 samples (16 per lane).
// Each wave owns dpw trials. A channel pass stages `cp` input rows of `row` bytes
// in LDS, double-buffered.
constexpr int kSampPerLane = 16;
constexpr int kTimeTile = 64 * kSampPerLane;
constexpr int kChanPerPass = 16;

struct DedispVariant {
    int id;          // index into the kernel table (dedisp.hip)
    int waves;       // waves per work-group
    int dpw;         // DM trials per wave
    int lds_bytes;   // LDS budget per work-group (both buffers)
    int layout;      // 0/3: lane owns 16 contiguous samples (ds_read_b128; 4-way or 16-way switch)
                     // 1/2: four 4-sample groups (ds_read2_b32; 2 reuses equal-offset windows)
                     // 4: matrix-core contraction (v_mfma_i32_32x32x32_i8), 4 channels x 8
                     //    residuals per step, see below
                     // 5: the same contraction with 8 channels x 4 residuals per step
                     // 6: layouts 5 and 4 mixed by trial range (per DM block)
                     // 7: quads of channels staged per residual pattern, v_sad_u8 sums
    int tile;        // output samples per work-group (time tile)
    int depth;       // staging buffers in the LDS ring (loads run depth - 1 steps ahead);
                     // layout 7: staging chunks per step (64 units of 16 bytes each)
    int max_tiles;   // layouts 4-6: a channel block spans at most 32 * max_tiles rows of t' (31 or 63)
};
constexpr int kNumDedispVariants = 25;
static_assert(kNumDedispVariants <= AA_MAX_VARIANTS, "aa_batch_info_t::tune_ms holds every variant");

// Matrix-core variants (layouts 4-6). Within a block of up to 32 trials (first trial d0)
// and a run of channels, the shift splits exactly as
//   s[d][c] = base[c] + E[d] + r[d][c],  base[c] = s[d0][c],  0 <= r < 8.
// For rows t' of a shifted time axis, the partial sum over the run,
//   P[t'][d] = sum_c X[c][t' + base[c] + r[d][c]],
// is a product of the matrix A[t'][(c, r)] = X[c][t' + base[c] + r] with the one-hot
// matrix B[(c, r)][d] = (r == r[d][c]). D[d][t] receives P[t + E[d]][d]. One MFMA step
// contracts CPS channels x 32/CPS residuals: 4 x 8 (layout 4) or 8 x 4 (layout 5). A
// channel block ends where the residual range of the next CPS channels would reach
// 32/CPS.
// A channel block spans at most 32 * max_tiles rows of t', with max_tiles 63 or 31. A
// staged row then needs at most 32 * max_tiles + 26 bytes: 2048 or 1024 bytes of LDS.
// Layout 6 takes the step shape per DM block (DmBlock::cps); mfma_cps is 0 for it.
constexpr int mfma_cps(int layout) { return layout == 5 ? 8 : layout == 6 ? 0 : 4; }
constexpr int mfma_row_bytes(int max_tiles) { return max_tiles <= 31 ? 1024 : 2048; }
// Record of one DM block and step k (D = the variant's depth), CPS channels per step:
//   [0, 32 CPS)   u8  8*r[d][CPS k + i] at CPS d + i (d < 32, i < CPS)
//   e             i16 e[d] = E[d] - min E of the channel block holding step k (32 of them)
//   phase         u8  phase of the CPS staged rows (their start mod 16)
//   tiles         i32 rows of t' in 32-row tiles for that channel block
//   left          i32 steps of the channel block from step k on (k included)
//   next_need     i32 16-byte chunks each row of step k + D - 1 needs
//   max_e         i32 max e over the channel block's trials
//   next_rs       i32 16-aligned row starts (relative to the time tile) of step k + D - 1
struct MfmaRec {
    int size, e, phase, tiles, left, next_need, max_e, next_rs;
};
constexpr MfmaRec mfma_rec(int cps) {
    return cps == 8 ? MfmaRec{512, 256, 320, 328, 332, 336, 340, 352} : MfmaRec{256, 128, 192, 200, 204, 208, 212, 224};
}
// LDS of a work-group: int32 accumulator tile [tile + 2][32] (rows -1 and tile take the
// adds that fall outside the tile and are never read), then `depth` staging buffers of
// CPS rows, then `depth` records.
constexpr int mfma_lds_bytes(int tile, int depth, int max_tiles, int cps = 4) {
    return (tile + 2) * 32 * 4 + depth * (cps * mfma_row_bytes(max_tiles) + mfma_rec(cps).size);
}
// Quad variants (layout 7): shift-and-add on the vector ALUs, no matrix cores. A step
// is one quad of channels c_i = 4q + i. Within a DM block, trials whose residuals
// r_i = s[d][c_i] - s[d][c_0] (i = 1..3) agree share a pattern. Per step, each pattern
// is staged once as dwords holding one sample of the four channels,
//   Y[k] = (X[c0][t0 + lo + k], X[c1][t0 + lo + r1 + k], X[c2][.. + r2 ..], X[c3][.. + r3 ..]),
// with lo the smallest s[d][c0] over the pattern's trials, and trial d adds the dword
// Y[s[d][c0] - lo + t] into output sample t with one v_sad_u8 (four byte-adds).
// A work-group stages a step in 64-unit chunks (a unit is 4 dwords); chunk j belongs
// to wave j % waves and fills dwords [256 j, 256 j + 256) of the step buffer. Pattern p
// takes ceil(units_p / 64) consecutive chunks from chunk cb_p (the earlier patterns'
// chunks), units_p = ceil((tile + hi - lo) / 4).
// Records, nq + 1 per DM block, quad_rec_dwords(chunks) int32 each (a multiple of 64):
// record e holds
//   [0, 16)           byte offsets in the step buffer of the trials' windows at step e - 1,
//                     4 (256 cb_p + s[d][c0] - lo_p), two u16 per dword (trial 2i in the
//                     low half of dword i; 0 for absent trials and for e = 0)
//   32                chunks of step e (0 for e = nq)
//   64 + 4 j + i      row offset of channel i for chunk j of step e: lo_p + r_i + 256 c,
//                     c = j - cb_p (relative to the time tile; its low 2 bits are the
//                     byte phase of the row within a dword); kQuadNoRow for channels
//                     past nchan
// so that one record serves the sums of step e - 1 and the staging of step e.
// Channels past nchan have r = 0 and stage zero bytes: their loads start at or beyond
// 2^30, outside the quad's load range (at most four row pitches of at most 2^28 bytes).
constexpr int kQuadTrials = 32;
constexpr int kQuadMaxPat = 8;
constexpr int quad_rec_dwords(int chunks) { return (64 + 4 * chunks + 63) / 64 * 64; }
constexpr int kQuadMaxResidual = 1023;
constexpr int kQuadMaxChunks = 64;   // trial offsets stay below 64 KB
constexpr int32_t kQuadNoRow = int32_t{1} << 30;
constexpr int64_t kQuadMaxPitch = int64_t{1} << 28;   // four row pitches stay below kQuadNoRow
constexpr int quad_lds_bytes(int chunks) { return 2 * chunks * 1024; }

extern const DedispVariant kDedispVariants[kNumDedispVariants];
// Input row pitches a variant can take (the quad variants address four rows from one
// 32-bit range).
inline bool variant_takes_pitch(int variant, int64_t in_pitch) {
    return kDedispVariants[variant].layout != 7 || in_pitch <= kQuadMaxPitch;
}
constexpr int kDefaultDedispVariant = 12;   // i8 matrix cores, 16 waves

// Single-pulse-search tiling: a work-group covers kSpsRows DM rows and kSpsTile starts.
constexpr int kSpsTile = 256;
constexpr int kSpsRows = 8;

struct DmBlock {
    int32_t first;   // first DM trial of the block
    int32_t count;   // trials in the block (<= waves * dpw)
    int32_t row;     // LDS row length (bytes) the block needs, multiple of 16 (layouts 0-3)
    int32_t rs_lo;   // layouts 4-6: smallest and largest staged-row start over the block's
    int32_t rs_hi;   // channels, relative to the time tile (0 for the other layouts)
    int32_t cps;     // layouts 4-6: channels per matrix step of this block (4 or 8)
    int32_t rec256;  // layouts 4-7: offset of the block's records in 256-byte units
};

// Per-variant tables. For block b and channel c:
//   base[b][c]       = s[first][c] & ~15   (16-byte-aligned start of the staged row)
//   offs[b][c][i]    = s[first+i][c] - base[b][c], for i < waves*dpw (0 for absent trials)
// Channels are padded to a multiple of kChanPerPass. Padded rows are zero.
struct DedispTables {
    int variant = -1;
    int bd = 0;                      // trials per block
    int nchan_pad = 0;
    int32_t max_row = 0;
    std::vector<DmBlock> blocks;
    DmBlock* d_blocks = nullptr;
    int32_t* d_base = nullptr;
    int32_t* d_offs = nullptr;
    uint8_t* d_pad = nullptr;        // layouts 4-6: one staged row of 0x80 bytes (padded channels)
    int split = -1;                  // layout 6: first trial of the 4-channel blocks
};

// Arguments of one dedispersion launch (one beam), passed by value or from a device table.
struct DedispArgs {
    const uint8_t* in;
    int64_t in_pitch, n_in16;
    const int32_t* base;
    const int32_t* offs;
    const DmBlock* blocks;
    int32_t nblk, nchan, nchan_pad, row;
    int32_t* out;
    int64_t out_pitch, n_out, ntile;
    const uint8_t* pad;
    int64_t tile;    // output samples per work-group
};

}  // namespace aa

struct aa_plan_s {
    int32_t nchan = 0, ndm = 0, nwidths = 0, wmax = 0, stat_block = 0;
    int64_t nsamp = 0, maxshift = 0, n_dd = 0, n_start = 0, nblocks = 0;
    double f_top = 0, foff = 0, tsamp = 0;
    float threshold = 0;
    float clip_sigma = 0;                 // outlier clipping of the block statistics (0: off)
    int32_t clip_iters = 0;
    int32_t boxcar_full_width = 0;        // decimated boxcar hierarchy (0: every width at every start)
    uint32_t flags = 0;
    std::vector<double> dm;
    std::vector<int32_t> widths;
    std::vector<double> sqrtw;            // sqrt(double(w)), rounded once on the host
    std::vector<int32_t> shifts;          // [ndm][nchan]
    // dedispersion tiling tables, one set per kernel variant that has been prepared
    aa::DedispTables tables[aa::kNumDedispVariants];
    int variant = aa::kDefaultDedispVariant;   // variant used by aa_dedisperse
    // device copies (uploaded once at plan time)
    int device = -1;
    int32_t* d_shifts = nullptr;
    int32_t* d_widths = nullptr;
};

namespace aa {
// Builds (host) and uploads (device, unless the plan is host-only) the tables of a variant.
int prepare_variant(aa_plan_s* p, int variant);
// Host tables of the matrix-core variants: DM blocks, 16-aligned staged-row starts
// [nblk][nchan_pad] and the per-step records [nblk][nchan_pad / cps][record size], with
// nchan_pad = nchan rounded up to cps channels.
// cps 4 or 8: one step shape; cps 0: 8 channels per step below a split trial and 4 from
// it on, the split taken from a cost estimate, or split_at when that is >= 0.
int build_mfma_tables(const aa_plan_s* p, int tile, int depth, int max_tiles, int cps, std::vector<DmBlock>& blocks,
                      std::vector<int32_t>& rsv, std::vector<uint8_t>& rec, int split_at = -1, int* split_out = nullptr);
// Rebuild the tables of a mixed-shape variant (layout 6) with its 4-channel blocks starting
// at trial `split` (the autotuner's search around the host estimate).
int prepare_mixed_split(aa_plan_s* p, int variant, int split);
// Host tables of the quad variants: DM blocks (rec256 = first record, in 256-byte
// units) and the records [block][nq + 1][quad_rec_dwords(chunks)].
int build_quad_tables(const aa_plan_s* p, int tile, int chunks, std::vector<DmBlock>& blocks,
                      std::vector<int32_t>& rec);
void free_tables(DedispTables& t);
// Launchers (dedisp.hip, sps.hip). Arguments are validated by the callers.
int launch_dedisperse(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                      int32_t* d_out, int64_t out_pitch, hipStream_t stream);
DedispArgs dedisp_args(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                       int32_t* d_out, int64_t out_pitch);
int launch_dedisperse_batch(int variant, const DedispArgs* d_args, const int64_t* d_item_begin, int nbeams,
                            int64_t total, unsigned long long* d_counter, int max_row, hipStream_t stream);
size_t sps_work_bytes(const aa_plan_s* p, int64_t n_starts);
// One halving of each row: out[c][j] = (in[c][2j] + in[c][2j+1] + 1) >> 1, j < n_in / 2.
int launch_halve(const uint8_t* in, int64_t in_pitch, int64_t n_in, int32_t nchan, uint8_t* out, int64_t out_pitch,
                 hipStream_t stream);
int launch_gather_rows(uint8_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch, int64_t width,
                       int64_t nrows, hipStream_t stream);
int launch_single_pulse(const aa_plan_s* p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0,
                        int64_t dd_n, int64_t t_begin, int64_t t_end, int64_t t_total, void* d_work,
                        aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, float* d_best,
                        int64_t best_pitch, hipStream_t stream, int32_t beam_id = 0);
}  // namespace aa
