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
};
constexpr int kNumDedispVariants = 11;
extern const DedispVariant kDedispVariants[kNumDedispVariants];
constexpr int kDefaultDedispVariant = 0;

// Single-pulse-search tiling: a work-group covers kSpsRows DM rows and kSpsTile starts.
constexpr int kSpsTile = 256;
constexpr int kSpsRows = 8;

struct DmBlock {
    int32_t first;   // first DM trial of the block
    int32_t count;   // trials in the block (<= waves * dpw)
    int32_t row;     // LDS row length (bytes) the block needs, multiple of 16
    int32_t pad;
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
};

}  // namespace aa

struct aa_plan_s {
    int32_t nchan = 0, ndm = 0, nwidths = 0, wmax = 0, stat_block = 0;
    int64_t nsamp = 0, maxshift = 0, n_dd = 0, n_start = 0, nblocks = 0;
    double f_top = 0, foff = 0, tsamp = 0;
    float threshold = 0;
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
void free_tables(DedispTables& t);
// Launchers (dedisp.hip, sps.hip). Arguments are validated by the callers.
int launch_dedisperse(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                      int32_t* d_out, int64_t out_pitch, hipStream_t stream);
DedispArgs dedisp_args(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                       int32_t* d_out, int64_t out_pitch);
int launch_dedisperse_batch(int variant, const DedispArgs* d_args, const int64_t* d_item_begin, int nbeams,
                            int64_t total, unsigned long long* d_counter, int max_row, hipStream_t stream);
size_t sps_work_bytes(const aa_plan_s* p, int64_t n_starts);
int launch_gather_rows(uint8_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch, int64_t width,
                       int64_t nrows, hipStream_t stream);
int launch_single_pulse(const aa_plan_s* p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0,
                        int64_t dd_n, int64_t t_begin, int64_t t_end, int64_t t_total, void* d_work,
                        aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, float* d_best,
                        int64_t best_pitch, hipStream_t stream, int32_t beam_id = 0);
}  // namespace aa
