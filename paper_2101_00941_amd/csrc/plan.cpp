// Plan: validation, the float64 shift table, sizes, dedispersion tiling tables and
// the one-time device upload. Section 1 of the paper fixes every size and
// allocation in its "mapping tasks to resources and allocation" part, before
// the search runs. Section 2.2 moves the search's dynamic allocations there too.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

#include "aa_internal.h"

namespace aa {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return AA_EHIP;
}

namespace {

constexpr double kDispersion = 4.148808e3;  // MHz^2 s per (pc cm^-3)

// floor(((K*dm) * inv) / tsamp + 0.5), one IEEE double operation per step.
int64_t shift_of(double dm, double inv, double tsamp) {
    volatile double kdm = kDispersion * dm;
    volatile double prod = kdm * inv;
    volatile double q = prod / tsamp;
    volatile double x = q + 0.5;
    return static_cast<int64_t>(std::floor(x));
}

void free_device(aa_plan_s* p) {
    int cur = 0;
    const bool on_dev = p->device >= 0;
    if (on_dev) {
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
    }
    for (auto& t : p->tables) free_tables(t);
    if (on_dev) {
        if (p->d_shifts) (void)hipFree(p->d_shifts);
        if (p->d_widths) (void)hipFree(p->d_widths);
        (void)hipSetDevice(cur);
    }
    p->d_shifts = p->d_widths = nullptr;
}

template <class T>
int upload(T** dst, const T* src, size_t n) {
    AA_HIP(hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T)));
    AA_HIP(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return AA_OK;
}

}  // namespace
}  // namespace aa

using namespace aa;

extern "C" const char* aa_last_error(void) { return aa::g_err.c_str(); }

extern "C" const char* aa_version(void) { return "aa-mi355x 0.1 gfx950"; }

extern "C" int aa_plan(const aa_plan_desc_t* desc, aa_plan_t* out) {
    if (!desc || !out) return fail(AA_EINVAL, "aa_plan: null argument");
    *out = nullptr;
    const aa_plan_desc_t& q = *desc;
    if (q.nchan < 1 || q.nchan > AA_MAX_NCHAN) return fail(AA_EINVAL, "aa_plan: nchan out of range");
    if (q.ndm < 1 || !q.dm) return fail(AA_EINVAL, "aa_plan: need at least one DM trial");
    if (q.nwidths < 1 || !q.widths) return fail(AA_EINVAL, "aa_plan: need at least one boxcar width");
    if (!(q.foff_mhz > 0) || !(q.tsamp_s > 0) || !(q.f_top_mhz > 0) || !std::isfinite(q.f_top_mhz) ||
        !std::isfinite(q.foff_mhz) || !std::isfinite(q.tsamp_s))
        return fail(AA_EINVAL, "aa_plan: f_top, foff and tsamp must be positive and finite");
    if (!(q.f_top_mhz - (q.nchan - 1) * q.foff_mhz > 0))
        return fail(AA_EINVAL, "aa_plan: the bottom channel frequency must be positive");
    for (int i = 0; i < q.ndm; ++i) {
        if (!std::isfinite(q.dm[i]) || q.dm[i] < 0) return fail(AA_EINVAL, "aa_plan: DMs must be finite and >= 0");
        if (i > 0 && q.dm[i] < q.dm[i - 1]) return fail(AA_EINVAL, "aa_plan: DMs must be ascending");
    }
    for (int i = 0; i < q.nwidths; ++i) {
        if (q.widths[i] < 1) return fail(AA_EINVAL, "aa_plan: widths must be >= 1");
        if (i > 0 && q.widths[i] <= q.widths[i - 1]) return fail(AA_EINVAL, "aa_plan: widths must be ascending and unique");
    }
    const int32_t wmax = q.widths[q.nwidths - 1];
    if (wmax > AA_MAX_WIDTH) return fail(AA_EINVAL, "aa_plan: widest boxcar exceeds AA_MAX_WIDTH");
    if (static_cast<uint64_t>(q.nchan) * 255u * static_cast<uint64_t>(wmax) >= (1ull << 32))
        return fail(AA_EINVAL, "aa_plan: nchan*255*wmax must stay below 2^32");
    if (!std::isfinite(q.snr_threshold)) return fail(AA_EINVAL, "aa_plan: threshold must be finite");
    if (!std::isfinite(q.clip_sigma) || q.clip_sigma < 0 || q.clip_iters < 0 || q.clip_iters > 16)
        return fail(AA_EINVAL, "aa_plan: clip_sigma must be finite and >= 0, clip_iters 0..16");
    if (q.boxcar_full_width < 0 || (q.boxcar_full_width > 0 && q.boxcar_full_width < q.widths[0]))
        return fail(AA_EINVAL, "aa_plan: boxcar_full_width must be 0 or at least the first width");
    const int32_t B = q.stat_block == 0 ? 32768 : q.stat_block;
    if (B < kSpsTile || B % kSpsTile) return fail(AA_EINVAL, "aa_plan: stat_block must be a positive multiple of 256");
    {
        const unsigned __int128 dmax = static_cast<unsigned __int128>(q.nchan) * 255u;
        if (dmax * dmax * static_cast<unsigned>(B) >= (static_cast<unsigned __int128>(1) << 63))
            return fail(AA_EINVAL, "aa_plan: stat_block too large for exact int64 moments");
    }

    aa_plan_s* p = new (std::nothrow) aa_plan_s();
    if (!p) return fail(AA_ENOMEM, "aa_plan: out of host memory");
    p->nchan = q.nchan;
    p->ndm = q.ndm;
    p->nwidths = q.nwidths;
    p->wmax = wmax;
    p->stat_block = B;
    p->nsamp = q.nsamp;
    p->f_top = q.f_top_mhz;
    p->foff = q.foff_mhz;
    p->tsamp = q.tsamp_s;
    p->threshold = q.snr_threshold;
    p->clip_sigma = q.clip_sigma;
    p->clip_iters = q.clip_sigma > 0 ? q.clip_iters : 0;
    p->boxcar_full_width = q.boxcar_full_width;
    p->flags = q.flags;
    p->dm.assign(q.dm, q.dm + q.ndm);
    p->widths.assign(q.widths, q.widths + q.nwidths);
    for (int32_t w : p->widths) p->sqrtw.push_back(std::sqrt(static_cast<double>(w)));

    // float64 shift table, one rounding per operation
    std::vector<double> inv(q.nchan);
    {
        volatile double ft2 = q.f_top_mhz * q.f_top_mhz;
        volatile double itop = 1.0 / ft2;
        for (int c = 0; c < q.nchan; ++c) {
            volatile double cf = static_cast<double>(c) * q.foff_mhz;
            volatile double fc = q.f_top_mhz - cf;
            volatile double fc2 = fc * fc;
            volatile double ic = 1.0 / fc2;
            inv[c] = ic - itop;
        }
    }
    p->shifts.resize(static_cast<size_t>(q.ndm) * q.nchan);
    int64_t m = 0;
    for (int d = 0; d < q.ndm; ++d) {
        for (int c = 0; c < q.nchan; ++c) {
            const int64_t s = shift_of(q.dm[d], inv[c], q.tsamp_s);
            if (s < 0 || s > std::numeric_limits<int32_t>::max() / 2) {
                delete p;
                return fail(AA_EINVAL, "aa_plan: shift out of range");
            }
            p->shifts[static_cast<size_t>(d) * q.nchan + c] = static_cast<int32_t>(s);
            m = std::max(m, s);
        }
    }
    p->maxshift = m;
    p->n_dd = q.nsamp - m;
    p->n_start = p->n_dd - wmax + 1;
    if (p->n_start < 1) {
        delete p;
        return fail(AA_ESHORT, "aa_plan: nsamp < maxshift + widest boxcar");
    }
    p->nblocks = (p->n_start + B - 1) / B;

    if (!(q.flags & AA_PLAN_HOST_ONLY)) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "aa_plan: hipGetDevice");
        }
        p->device = dev;
        int rc = upload(&p->d_shifts, p->shifts.data(), p->shifts.size());
        if (rc == AA_OK) rc = upload(&p->d_widths, p->widths.data(), p->widths.size());
        if (rc != AA_OK) {
            free_device(p);
            delete p;
            return rc;
        }
    }
    {
        const int rc = prepare_variant(p, p->variant);
        if (rc != AA_OK) {
            free_device(p);
            delete p;
            return rc;
        }
    }
    *out = p;
    return AA_OK;
}

extern "C" int aa_plan_info(aa_plan_t p, aa_plan_info_t* out) {
    if (!p || !out) return fail(AA_EINVAL, "aa_plan_info: null argument");
    std::memset(out, 0, sizeof(*out));
    out->nchan = p->nchan;
    out->ndm = p->ndm;
    out->nwidths = p->nwidths;
    out->wmax = p->wmax;
    out->nsamp = p->nsamp;
    out->maxshift = p->maxshift;
    out->n_dd = p->n_dd;
    out->n_start = p->n_start;
    out->stat_block = p->stat_block;
    out->nblocks = p->nblocks;
    out->in_pitch = (p->nsamp + 255) / 256 * 256;
    out->out_pitch = (p->n_dd + 63) / 64 * 64;
    out->work_bytes = sps_work_bytes(p, p->n_start);
    out->device = p->device;
    return AA_OK;
}

extern "C" int aa_plan_shifts(aa_plan_t p, int32_t* h_out) {
    if (!p || !h_out) return fail(AA_EINVAL, "aa_plan_shifts: null argument");
    std::memcpy(h_out, p->shifts.data(), p->shifts.size() * sizeof(int32_t));
    return AA_OK;
}

extern "C" void aa_plan_destroy(aa_plan_t p) {
    if (!p) return;
    free_device(p);
    delete p;
}
