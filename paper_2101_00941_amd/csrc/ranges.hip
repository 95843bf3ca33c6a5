// Per-range time decimation for gfx950. Beyond the paper's brute-force dedispersion
// (section 2.1): the trials are split into consecutive ranges, and range r is
// dedispersed and searched on the input decimated by f_r = 2^k (k halvings, each the
// rounding average of adjacent samples), at sampling time f_r * t_samp. With f_r
// doubling where the survey plan's DM step doubles, the bottom channel's shift step
// stays near one sample per trial while the adds fall by the factor.
//
// Kernels:
//   halve_kernel    y[c][j] = (x[c][2j] + x[c][2j+1] + 1) >> 1. HBM-bound: 2 bytes read
//                   and 1 written per output. A thread takes 16 outputs from two 16-byte
//                   loads; the even and odd bytes of each dword are split into 16-bit
//                   lanes, added with the rounding one and shifted, in packed integer
//                   adds that cannot carry across lanes (at most 255 + 255 + 1).
//   gather_kernel   concatenates the ranges' candidate lists in range (so trial) order,
//                   scaling start and width by f_r and offsetting the trial index.
// Host: aa_range_plan builds one ordinary plan per range (aa_plan with f_r * t_samp,
// the range's trials, nsamp >> k and stat block / f_r). aa_range_run decimates level by
// level into the work buffer, then runs aa_dedisperse and the search of each range on
// one stream, reusing one plane and one search scratch for every range.
#include <algorithm>
#include <cstring>
#include <vector>

#include "aa_internal.h"

namespace aa {
namespace {

constexpr int kMaxRanges = 16;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 8 input bytes (two dwords) -> 4 rounded pair averages in one dword
__device__ __forceinline__ uint32_t halve8(uint32_t lo, uint32_t hi) {
    const uint32_t m = 0x00FF00FFu;
    const uint32_t a = ((lo & m) + ((lo >> 8) & m) + 0x00010001u) >> 1;   // bytes 0,1 | 2,3 of lo
    const uint32_t b = ((hi & m) + ((hi >> 8) & m) + 0x00010001u) >> 1;
    // a holds averages in bits 0-7 and 16-23 (bit 8 and 24 are 0 after the shift of a
    // sum <= 511): pack them as bytes 0,1 from a and 2,3 from b
    return __builtin_amdgcn_perm(b, a, 0x06040200u);
}

__global__ __launch_bounds__(256) void halve_kernel(const uint8_t* __restrict__ in, int64_t in_pitch,
                                                    uint8_t* __restrict__ out, int64_t out_pitch, int64_t n_out,
                                                    int64_t groups_per_row) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;   // 16-output group in the row
    const int64_t c = blockIdx.y;
    if (g >= groups_per_row) return;
    const uint8_t* src = in + c * in_pitch;
    uint8_t* dst = out + c * out_pitch;
    const int64_t j0 = 16 * g;
    if (j0 + 16 <= n_out) {
        // 32 valid input bytes at 2 j0 (16-byte aligned: pitches and bases are)
        const u32x4 x0 = *reinterpret_cast<const u32x4*>(src + 2 * j0);
        const u32x4 x1 = *reinterpret_cast<const u32x4*>(src + 2 * j0 + 16);
        u32x4 y;
        y.x = halve8(x0.x, x0.y);
        y.y = halve8(x0.z, x0.w);
        y.z = halve8(x1.x, x1.y);
        y.w = halve8(x1.z, x1.w);
        *reinterpret_cast<u32x4*>(dst + j0) = y;
    } else {
        for (int64_t j = j0; j < n_out; ++j)
            dst[j] = static_cast<uint8_t>((static_cast<uint32_t>(src[2 * j]) + src[2 * j + 1] + 1u) >> 1);
    }
}

struct GatherArgs {
    int32_t nranges;
    int32_t cap;          // output capacity
    int32_t stage_cap;    // capacity of each range's staged list
    int32_t lo[kMaxRanges];
    int32_t f[kMaxRanges];
};

__global__ __launch_bounds__(256) void gather_kernel(const aa_candidate_t* __restrict__ stage,
                                                     const int32_t* __restrict__ counts, GatherArgs g,
                                                     aa_candidate_t* __restrict__ out, int32_t* __restrict__ count) {
    const int r = blockIdx.x;
    int64_t off = 0;
    for (int q = 0; q < r; ++q) off += counts[q];
    if (r == g.nranges - 1 && threadIdx.x == 0) *count = static_cast<int32_t>(min<int64_t>(off + counts[r], 0x7fffffff));
    const int n = min(counts[r], g.stage_cap);
    const aa_candidate_t* src = stage + static_cast<int64_t>(r) * g.stage_cap;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (off + i >= g.cap) break;
        aa_candidate_t c = src[i];
        c.dm_idx += g.lo[r];
        c.t *= g.f[r];
        c.width *= g.f[r];
        out[off + i] = c;
    }
}

size_t up256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }
int log2i(int f) {
    int k = 0;
    while ((1 << k) < f) ++k;
    return k;
}

}  // namespace

int launch_halve(const uint8_t* in, int64_t in_pitch, int64_t n_in, int32_t nchan, uint8_t* out, int64_t out_pitch,
                 hipStream_t stream) {
    const int64_t n_out = n_in / 2;
    if (n_out < 1) return AA_OK;
    const int64_t groups = (n_out + 15) / 16;
    const int64_t gx = (groups + 255) / 256;
    if (gx > 0x7fffffff || nchan > 65535) return fail(AA_EINVAL, "decimation: grid too large");
    hipLaunchKernelGGL(halve_kernel, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(nchan)), dim3(256), 0, stream,
                       in, in_pitch, out, out_pitch, n_out, groups);
    AA_HIP(hipGetLastError());
    return AA_OK;
}

}  // namespace aa

using namespace aa;

struct aa_range_plan_s {
    int32_t nranges = 0, nchan = 0, ndm = 0;
    int64_t nsamp = 0;
    std::vector<int32_t> first, factor;
    std::vector<aa_plan_t> plans;
};

extern "C" int aa_decimate2(const uint8_t* d_in, int64_t in_pitch, int64_t n_in, int32_t nchan, uint8_t* d_out,
                            int64_t out_pitch, void* stream) {
    if (!d_in || !d_out || nchan < 1 || n_in < 2 || in_pitch < n_in || out_pitch < n_in / 2)
        return fail(AA_EINVAL, "aa_decimate2: bad argument");
    if ((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_out)) & 15 || (in_pitch | out_pitch) & 15)
        return fail(AA_EINVAL, "aa_decimate2: buffers and pitches must be multiples of 16 bytes");
    return launch_halve(d_in, in_pitch, n_in, nchan, d_out, out_pitch, static_cast<hipStream_t>(stream));
}

extern "C" void aa_range_plan_destroy(aa_range_plan_t rp) {
    if (!rp) return;
    for (aa_plan_t p : rp->plans) aa_plan_destroy(p);
    delete rp;
}

extern "C" int aa_range_plan(const aa_plan_desc_t* desc, const int32_t* first, const int32_t* factor, int32_t nranges,
                             aa_range_plan_t* out) {
    if (!desc || !first || !factor || !out) return fail(AA_EINVAL, "aa_range_plan: null argument");
    *out = nullptr;
    if (nranges < 1 || nranges > kMaxRanges) return fail(AA_EINVAL, "aa_range_plan: 1..16 ranges");
    if (desc->ndm < 1 || !desc->dm) return fail(AA_EINVAL, "aa_range_plan: need DM trials");
    const int32_t B = desc->stat_block == 0 ? 32768 : desc->stat_block;
    if (first[0] != 0) return fail(AA_EINVAL, "aa_range_plan: the first range starts at trial 0");
    for (int r = 0; r < nranges; ++r) {
        const int32_t hi = r + 1 < nranges ? first[r + 1] : desc->ndm;
        if (hi <= first[r]) return fail(AA_EINVAL, "aa_range_plan: range first trials must ascend below ndm");
        const int32_t f = factor[r];
        if (f < 1 || (f & (f - 1)) || f > (1 << 20)) return fail(AA_EINVAL, "aa_range_plan: factors must be powers of two");
        if (r > 0 && f < factor[r - 1]) return fail(AA_EINVAL, "aa_range_plan: factors must not decrease");
        if (B % f) return fail(AA_EINVAL, "aa_range_plan: every factor must divide the stat block");
    }
    auto* rp = new (std::nothrow) aa_range_plan_s();
    if (!rp) return fail(AA_ENOMEM, "aa_range_plan: out of host memory");
    rp->nranges = nranges;
    rp->nchan = desc->nchan;
    rp->ndm = desc->ndm;
    rp->nsamp = desc->nsamp;
    rp->first.assign(first, first + nranges);
    rp->factor.assign(factor, factor + nranges);
    for (int r = 0; r < nranges; ++r) {
        const int32_t hi = r + 1 < nranges ? first[r + 1] : desc->ndm;
        aa_plan_desc_t d = *desc;
        d.dm = desc->dm + first[r];
        d.ndm = hi - first[r];
        d.tsamp_s = static_cast<double>(factor[r]) * desc->tsamp_s;   // exact: a power of two
        d.nsamp = desc->nsamp >> log2i(factor[r]);
        d.stat_block = B / factor[r];
        aa_plan_t p = nullptr;
        const int rc = aa_plan(&d, &p);
        if (rc != AA_OK) {
            aa_range_plan_destroy(rp);
            return rc;
        }
        rp->plans.push_back(p);
    }
    *out = rp;
    return AA_OK;
}

extern "C" int aa_range_plan_get(aa_range_plan_t rp, int32_t r, aa_plan_t* plan, int32_t* first, int32_t* factor) {
    if (!rp || r < 0 || r >= rp->nranges) return fail(AA_EINVAL, "aa_range_plan_get: bad argument");
    if (plan) *plan = rp->plans[r];
    if (first) *first = rp->first[r];
    if (factor) *factor = rp->factor[r];
    return AA_OK;
}

namespace {
struct RangeLayout {
    std::vector<size_t> level_off;      // decimated input of level k (k >= 1), in the work buffer
    std::vector<int64_t> level_pitch, level_n;
    size_t plane = 0, scratch = 0, stage = 0, counts = 0, total = 0;
    int64_t plane_pitch_max = 0;
};

int range_layout(const aa_range_plan_s* rp, int64_t n_in, int32_t cap, RangeLayout* L) {
    const int kmax = log2i(rp->factor.back());
    size_t off = 0;
    L->level_off.assign(kmax + 1, 0);
    L->level_pitch.assign(kmax + 1, 0);
    L->level_n.assign(kmax + 1, n_in);
    for (int k = 1; k <= kmax; ++k) {
        L->level_n[k] = L->level_n[k - 1] / 2;
        L->level_pitch[k] = (L->level_n[k] + 255) / 256 * 256;
        L->level_off[k] = off;
        off += up256(static_cast<size_t>(rp->nchan) * static_cast<size_t>(L->level_pitch[k]));
    }
    size_t plane = 0, scratch = 0;
    for (int r = 0; r < rp->nranges; ++r) {
        const aa_plan_s* p = rp->plans[r];
        const int64_t n = L->level_n[log2i(rp->factor[r])];
        const int64_t n_out = n - p->maxshift, T = n_out - p->wmax + 1;
        if (T < 1) return fail(AA_ESHORT, "aa_range_run: a range is shorter than its maxshift + widest boxcar");
        const int64_t op = (n_out + 63) / 64 * 64;
        plane = std::max(plane, up256(static_cast<size_t>(p->ndm) * op * 4));
        scratch = std::max(scratch, up256(sps_work_bytes(p, T)));
    }
    L->plane = off;
    off += plane;
    L->scratch = off;
    off += scratch;
    L->stage = off;
    off += up256(static_cast<size_t>(rp->nranges) * static_cast<size_t>(std::max(cap, 1)) * sizeof(aa_candidate_t));
    L->counts = off;
    off += 256;
    L->total = off;
    return AA_OK;
}
}  // namespace

extern "C" int aa_range_work_bytes(aa_range_plan_t rp, int64_t n_in, int32_t cap, size_t* out) {
    if (!rp || !out || n_in < 1 || cap < 0) return fail(AA_EINVAL, "aa_range_work_bytes: bad argument");
    RangeLayout L;
    const int rc = range_layout(rp, n_in, cap, &L);
    if (rc != AA_OK) return rc;
    *out = L.total;
    return AA_OK;
}

namespace {
// Decimation levels 1 .. kmax into the work buffer, each from the one before.
int decimate_levels(const aa_range_plan_s* rp, const RangeLayout& L, const uint8_t* d_in, int64_t in_pitch, uint8_t* W,
                    hipStream_t stream) {
    const int kmax = static_cast<int>(L.level_off.size()) - 1;
    for (int k = 1; k <= kmax; ++k) {
        const uint8_t* src = k == 1 ? d_in : W + L.level_off[k - 1];
        const int64_t sp = k == 1 ? in_pitch : L.level_pitch[k - 1];
        const int rc = launch_halve(src, sp, L.level_n[k - 1], rp->nchan, W + L.level_off[k], L.level_pitch[k], stream);
        if (rc != AA_OK) return rc;
    }
    return AA_OK;
}

int check_run_args(const aa_range_plan_s* rp, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, const void* d_work) {
    if (!rp || !d_in || !d_work) return fail(AA_EINVAL, "aa_range: null argument");
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15) || n_in > in_pitch || n_in < 2)
        return fail(AA_EINVAL, "aa_range: d_in and in_pitch must be multiples of 16 with 2 <= n_in <= in_pitch");
    if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(AA_EINVAL, "aa_range: d_work must be 256-byte aligned");
    for (aa_plan_t p : rp->plans)
        if (p->device < 0) return fail(AA_EINVAL, "aa_range: plan was created host-only");
    return AA_OK;
}
}  // namespace

extern "C" int aa_range_autotune(aa_range_plan_t rp, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, void* d_work,
                                 size_t work_bytes, int32_t reps, void* stream_, float* ms_out) {
    int rc = check_run_args(rp, d_in, in_pitch, n_in, d_work);
    if (rc != AA_OK) return rc;
    RangeLayout L;
    rc = range_layout(rp, n_in, 0, &L);
    if (rc != AA_OK) return rc;
    if (work_bytes < L.total) return fail(AA_EINVAL, "aa_range_autotune: work buffer too small (aa_range_work_bytes)");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    uint8_t* W = static_cast<uint8_t*>(d_work);
    rc = decimate_levels(rp, L, d_in, in_pitch, W, stream);
    if (rc != AA_OK) return rc;
    for (int r = 0; r < rp->nranges; ++r) {
        aa_plan_s* p = rp->plans[r];
        const int k = log2i(rp->factor[r]);
        const int64_t n = L.level_n[k];
        const int64_t op = (n - p->maxshift + 63) / 64 * 64;
        rc = aa_autotune(p, k == 0 ? d_in : W + L.level_off[k], k == 0 ? in_pitch : L.level_pitch[k], n,
                         reinterpret_cast<int32_t*>(W + L.plane), op, reps, stream_,
                         ms_out ? ms_out + static_cast<int64_t>(r) * kNumDedispVariants : nullptr);
        if (rc != AA_OK) return rc;
    }
    return AA_OK;
}

extern "C" int aa_range_run(aa_range_plan_t rp, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, void* d_work,
                            size_t work_bytes, aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, void* stream_) {
    if (!d_count || cap < 0 || (cap > 0 && !d_cand)) return fail(AA_EINVAL, "aa_range_run: null argument");
    int rc = check_run_args(rp, d_in, in_pitch, n_in, d_work);
    if (rc != AA_OK) return rc;
    RangeLayout L;
    rc = range_layout(rp, n_in, cap, &L);
    if (rc != AA_OK) return rc;
    if (work_bytes < L.total) return fail(AA_EINVAL, "aa_range_run: work buffer too small (aa_range_work_bytes)");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    uint8_t* W = static_cast<uint8_t*>(d_work);
    rc = decimate_levels(rp, L, d_in, in_pitch, W, stream);
    if (rc != AA_OK) return rc;
    const int32_t stage_cap = std::max(cap, 1);
    aa_candidate_t* stage = reinterpret_cast<aa_candidate_t*>(W + L.stage);
    int32_t* counts = reinterpret_cast<int32_t*>(W + L.counts);
    int32_t* plane = reinterpret_cast<int32_t*>(W + L.plane);
    GatherArgs g{};
    g.nranges = rp->nranges;
    g.cap = cap;
    g.stage_cap = stage_cap;
    for (int r = 0; r < rp->nranges; ++r) {
        aa_plan_s* p = rp->plans[r];
        const int k = log2i(rp->factor[r]);
        const uint8_t* x = k == 0 ? d_in : W + L.level_off[k];
        const int64_t xp = k == 0 ? in_pitch : L.level_pitch[k];
        const int64_t n = L.level_n[k];
        const int64_t n_out = n - p->maxshift, T = n_out - p->wmax + 1;
        const int64_t op = (n_out + 63) / 64 * 64;
        rc = launch_dedisperse(p, p->variant, x, xp, n, plane, op, stream);
        if (rc != AA_OK) return rc;
        rc = launch_single_pulse(p, plane, op, 0, n_out, 0, T, T, W + L.scratch, stage + static_cast<int64_t>(r) * stage_cap,
                                 stage_cap, counts + r, nullptr, 0, stream);
        if (rc != AA_OK) return rc;
        g.lo[r] = rp->first[r];
        g.f[r] = rp->factor[r];
    }
    hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(rp->nranges)), dim3(256), 0, stream, stage, counts, g,
                       d_cand, d_count);
    AA_HIP(hipGetLastError());
    return AA_OK;
}
