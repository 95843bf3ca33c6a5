// Batched beams: groups of beams of any shape go through one persistent dedispersion
// launch each (items pulled from a device counter), then each beam's single-pulse
// search. Host side: validation, grouping by the work budget, tables, events.
#include <algorithm>
#include <vector>

#include "aa_internal.h"

using namespace aa;

namespace {

size_t up256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct BeamPlan {
    int index;
    int64_t n_out, T, opitch;
    size_t plane, work;
};

}  // namespace

extern "C" int aa_batch_run(const aa_batch_beam_t* beams, int32_t nbeams, int32_t variant, void* d_work,
                            size_t work_bytes, aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, uint32_t flags,
                            aa_batch_info_t* info, void* stream_) {
    if (!beams || nbeams < 1 || !d_work || !d_count || cap < 0 || (cap > 0 && !d_cand))
        return fail(AA_EINVAL, "aa_batch_run: bad argument");
    if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(AA_EINVAL, "aa_batch_run: d_work must be 256-byte aligned");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    int dev = 0;
    AA_HIP(hipGetDevice(&dev));
    std::vector<BeamPlan> bp(nbeams);
    int64_t best_adds = -1;
    int biggest = 0;
    for (int i = 0; i < nbeams; ++i) {
        const aa_batch_beam_t& b = beams[i];
        const aa_plan_s* p = b.plan;
        if (!p || !b.d_in) return fail(AA_EINVAL, "aa_batch_run: beam without plan or input");
        if (p->device != dev) return fail(AA_EINVAL, "aa_batch_run: a plan is not on the current device");
        if (p->nwidths > 32) return fail(AA_EINVAL, "aa_batch_run: more than 32 widths");
        if ((reinterpret_cast<uintptr_t>(b.d_in) & 15) || (b.in_pitch & 15) || b.n_in > b.in_pitch)
            return fail(AA_EINVAL, "aa_batch_run: inputs must be 16-byte aligned with n_in <= in_pitch");
        BeamPlan& q = bp[i];
        q.index = i;
        q.n_out = b.n_in - p->maxshift;
        q.T = q.n_out - p->wmax + 1;
        if (q.T < 1) return fail(AA_ESHORT, "aa_batch_run: a beam is shorter than maxshift + widest boxcar");
        q.opitch = (q.n_out + 63) / 64 * 64;
        q.plane = up256(static_cast<size_t>(p->ndm) * q.opitch * 4);
        q.work = up256(sps_work_bytes(p, q.T));
        const int64_t adds = static_cast<int64_t>(p->ndm) * q.n_out * p->nchan;
        if (adds > best_adds) {
            best_adds = adds;
            biggest = i;
        }
    }
    const size_t header = up256(static_cast<size_t>(nbeams) * sizeof(DedispArgs)) +
                          up256(static_cast<size_t>(nbeams + 1) * sizeof(int64_t)) + 256;
    for (const BeamPlan& q : bp)
        if (header + q.plane + q.work > work_bytes)
            return fail(AA_ENOMEM, "aa_batch_run: one beam's plane does not fit the work buffer");

    // variant: given, or tuned on the beam with the most work
    float tune_ms[AA_MAX_VARIANTS];
    for (float& m : tune_ms) m = -1.0f;
    int tuned_beam = -1;
    if (variant < 0) {
        const aa_batch_beam_t& b = beams[biggest];
        int32_t* plane = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(d_work) + header);
        const int rc = aa_autotune(b.plan, b.d_in, b.in_pitch, b.n_in, plane, bp[biggest].opitch, 1, stream_, tune_ms);
        if (rc != AA_OK) return rc;
        variant = b.plan->variant;
        tuned_beam = biggest;
    }
    if (variant >= kNumDedispVariants) return fail(AA_EINVAL, "aa_batch_run: unknown variant");
    for (int i = 0; i < nbeams; ++i)
        if (!variant_takes_pitch(variant, beams[i].in_pitch))
            return fail(AA_EINVAL, "aa_batch_run: the quad variants take row pitches of at most 2^28 bytes");
    for (int i = 0; i < nbeams; ++i) {
        const int rc = prepare_variant(beams[i].plan, variant);
        if (rc != AA_OK) return rc;
    }

    hipEvent_t e[3];
    for (auto& ev : e) AA_HIP(hipEventCreate(&ev));
    float ms_d = 0, ms_s = 0;
    int groups = 0;
    int64_t items_all = 0;
    int rc = AA_OK;
    uint8_t* W = static_cast<uint8_t*>(d_work);
    for (int g0 = 0; g0 < nbeams && rc == AA_OK;) {
        // pack beams g0 .. g1-1 into the work buffer
        size_t used = header;
        int g1 = g0;
        while (g1 < nbeams && used + bp[g1].plane + bp[g1].work <= work_bytes) {
            used += bp[g1].plane + bp[g1].work;
            ++g1;
        }
        const int nb = g1 - g0;
        DedispArgs* d_args = reinterpret_cast<DedispArgs*>(W);
        int64_t* d_begin = reinterpret_cast<int64_t*>(W + up256(nbeams * sizeof(DedispArgs)));
        unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(
            W + up256(nbeams * sizeof(DedispArgs)) + up256((nbeams + 1) * sizeof(int64_t)));
        std::vector<DedispArgs> args(nb);
        std::vector<int64_t> begin(nb + 1, 0);
        std::vector<int32_t*> planes(nb);
        std::vector<void*> works(nb);
        size_t off = header;
        int max_row = 0;
        for (int k = 0; k < nb; ++k) {
            const BeamPlan& q = bp[g0 + k];
            const aa_batch_beam_t& b = beams[g0 + k];
            planes[k] = reinterpret_cast<int32_t*>(W + off);
            off += q.plane;
            works[k] = W + off;
            off += q.work;
            args[k] = dedisp_args(b.plan, variant, b.d_in, b.in_pitch, b.n_in, planes[k], q.opitch);
            begin[k + 1] = begin[k] + static_cast<int64_t>(args[k].nblk) * args[k].ntile;
            max_row = std::max(max_row, args[k].row);
        }
        const int64_t total = begin[nb];
        items_all += total;
        hipError_t ue = hipMemcpyAsync(d_args, args.data(), nb * sizeof(DedispArgs), hipMemcpyHostToDevice, stream);
        if (ue == hipSuccess)
            ue = hipMemcpyAsync(d_begin, begin.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream);
        if (ue != hipSuccess) {
            rc = hip_fail(ue, "aa_batch_run: table upload");
            break;
        }
        (void)hipEventRecord(e[0], stream);
        if (flags & AA_BATCH_STATIC) {
            for (int k = 0; k < nb && rc == AA_OK; ++k) {
                const aa_batch_beam_t& b = beams[g0 + k];
                rc = launch_dedisperse(b.plan, variant, b.d_in, b.in_pitch, b.n_in, planes[k], bp[g0 + k].opitch,
                                       stream);
            }
        } else {
            rc = launch_dedisperse_batch(variant, d_args, d_begin, nb, total, d_counter, max_row, stream);
        }
        (void)hipEventRecord(e[1], stream);
        for (int k = 0; k < nb && rc == AA_OK; ++k) {
            const BeamPlan& q = bp[g0 + k];
            rc = launch_single_pulse(beams[g0 + k].plan, planes[k], q.opitch, 0, q.n_out, 0, q.T, q.T, works[k],
                                     d_cand + static_cast<int64_t>(q.index) * cap, cap, d_count + q.index, nullptr, 0,
                                     stream, q.index);
        }
        (void)hipEventRecord(e[2], stream);
        const hipError_t se = hipEventSynchronize(e[2]);   // args/begin host vectors live until here
        if (se != hipSuccess && rc == AA_OK) rc = hip_fail(se, "aa_batch_run: synchronize");
        float a = 0, b2 = 0;
        (void)hipEventElapsedTime(&a, e[0], e[1]);
        (void)hipEventElapsedTime(&b2, e[1], e[2]);
        ms_d += a;
        ms_s += b2;
        ++groups;
        g0 = g1;
    }
    for (auto& ev : e) (void)hipEventDestroy(ev);
    if (info) {
        info->groups = groups;
        info->variant = variant;
        info->items = items_all;
        info->ms_dedisp = ms_d;
        info->ms_search = ms_s;
        info->tuned_beam = tuned_beam;
        for (int v = 0; v < AA_MAX_VARIANTS; ++v) info->tune_ms[v] = tune_ms[v];
    }
    return rc;
}
