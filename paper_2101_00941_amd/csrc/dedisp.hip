// Brute-force incoherent dedispersion for gfx950 (the paper's dedispersion phase,
// section 2.1):  D[d][t] = sum_c X[c][t + s[d][c]], exact in integers.
//
// Shape of the kernel:
//  * A work-group of 4 waves owns one DM block (up to 16 consecutive trials) and one
//    time tile of 1024 samples. Each wave owns 4 trials. Each lane owns 16
//    consecutive samples of each of its trials.
//  * The input is consumed in channel passes. A pass stages 16 channel rows in LDS
//    with coalesced 16-byte global loads. A row holds the bytes
//    [t0 + (s[first][c] & ~15), + row), which covers every trial of the block. Each
//    staged byte is then reused by all trials of the block.
//  * The inner step for one (channel, trial): two aligned ds_read_b128 give the 32
//    bytes around the lane's 16-sample window. Eight v_perm_b32 extract the window
//    as zero-extended 16-bit pairs. The byte offset (o & 3) picks the selector, and
//    (o >> 2) & 3 picks the registers through a uniform branch. The pairs are then
//    added into packed u16x2 accumulators. A u16 half holds up to 257 * 255, so the
//    pairs are widened into int32 accumulators every 256 channels.
//  * MFMA is not used: this is shift-and-add, not a dense contraction.
#include "aa_internal.h"

namespace aa {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Work-group i runs on XCD i % 8. Give each XCD a contiguous run of logical tiles
// (adjacent DM blocks of the same time tile), so that their overlapping input rows
// are shared in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + min(x, r) + k;
}

template <int Q>
__device__ __forceinline__ void extract16(const uint32_t (&w)[8], uint32_t sel0, uint32_t sel1,
                                          uint32_t (&p)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = Q + (j >> 1);
        p[j] = __builtin_amdgcn_perm(w[i + 1], w[i], (j & 1) ? sel1 : sel0);
    }
}

template <int KS, int DPW, int WAVES, int CP>
__global__ __launch_bounds__(64 * WAVES) void dedisp_kernel(
    const uint8_t* __restrict__ in, int64_t in_pitch, const int32_t* __restrict__ shifts,
    const int32_t* __restrict__ offs, const DmBlock* __restrict__ blocks, int nblk, int nchan,
    int32_t* __restrict__ out, int64_t out_pitch, int64_t n_out, int row) {
    static_assert(KS == 16, "the extraction below is written for 16 samples per lane");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    constexpr int NT = 64 * WAVES;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = bid % nblk;
    const int64_t t0 = static_cast<int64_t>(bid / nblk) * (64 * KS);
    const DmBlock b = blocks[blk];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int ndw = min(max(b.count - wave * DPW, 0), DPW);
    const int dfirst = b.first + wave * DPW;

    uint32_t a16[DPW][KS / 2];
    uint32_t a32[DPW][KS];
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) a16[i][j] = 0;
#pragma unroll
        for (int k = 0; k < KS; ++k) a32[i][k] = 0;
    }

    const int vec_per_row = row >> 4;
    const int32_t* s_first = shifts + static_cast<int64_t>(b.first) * nchan;
    int since_flush = 0;
    for (int c0 = 0; c0 < nchan; c0 += CP) {
        const int ncp = min(CP, nchan - c0);
        __syncthreads();
        for (int v = threadIdx.x; v < ncp * vec_per_row; v += NT) {
            const int cr = v / vec_per_row;
            const int k = v - cr * vec_per_row;
            const int c = c0 + cr;
            const int64_t g = t0 + (s_first[c] & ~15) + 16 * k;
            u32x4 val = {0u, 0u, 0u, 0u};
            if (g + 16 <= in_pitch) val = *reinterpret_cast<const u32x4*>(in + c * in_pitch + g);
            *reinterpret_cast<u32x4*>(lds + cr * row + 16 * k) = val;
        }
        __syncthreads();
        if (since_flush + ncp > 256) {
#pragma unroll
            for (int i = 0; i < DPW; ++i) {
#pragma unroll
                for (int j = 0; j < KS / 2; ++j) {
                    a32[i][2 * j] += a16[i][j] & 0xFFFFu;
                    a32[i][2 * j + 1] += a16[i][j] >> 16;
                    a16[i][j] = 0;
                }
            }
            since_flush = 0;
        }
        since_flush += ncp;
        for (int cr = 0; cr < ncp; ++cr) {
            const uint8_t* rowp = lds + cr * row + 16 * lane;
#pragma unroll
            for (int i = 0; i < DPW; ++i) {
                if (i < ndw) {
                    const int o = offs[static_cast<int64_t>(dfirst + i) * nchan + c0 + cr];
                    const u32x4* p = reinterpret_cast<const u32x4*>(rowp + (o & ~15));
                    const u32x4 x0 = p[0], x1 = p[1];
                    const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                    const uint32_t r = static_cast<uint32_t>(o & 3);
                    const uint32_t sel0 = 0x0C000C00u | ((r + 1u) << 16) | r;
                    const uint32_t sel1 = sel0 + 0x00020002u;
                    uint32_t pr[8];
                    switch ((o >> 2) & 3) {
                        case 0: extract16<0>(w, sel0, sel1, pr); break;
                        case 1: extract16<1>(w, sel0, sel1, pr); break;
                        case 2: extract16<2>(w, sel0, sel1, pr); break;
                        default: extract16<3>(w, sel0, sel1, pr); break;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) a16[i][j] += pr[j];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            a32[i][2 * j] += a16[i][j] & 0xFFFFu;
            a32[i][2 * j + 1] += a16[i][j] >> 16;
        }
    }

    const int64_t t = t0 + KS * lane;
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
        if (i >= ndw) continue;
        int32_t* o = out + static_cast<int64_t>(dfirst + i) * out_pitch + t;
        if (t + KS <= n_out) {
#pragma unroll
            for (int k = 0; k < KS; k += 4) {
                u32x4 v = {a32[i][k], a32[i][k + 1], a32[i][k + 2], a32[i][k + 3]};
                *reinterpret_cast<u32x4*>(o + k) = v;
            }
        } else {
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (t + k < n_out) o[k] = static_cast<int32_t>(a32[i][k]);
        }
    }
}

}  // namespace

int launch_dedisperse(const aa_plan_s* p, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                      int32_t* d_out, int64_t out_pitch, hipStream_t stream) {
    const int64_t n_out = n_in - p->maxshift;
    const int64_t ntile = (n_out + kTimeTile - 1) / kTimeTile;
    const int64_t nblk = static_cast<int64_t>(p->blocks.size());
    const int64_t grid = ntile * nblk;
    if (grid > 0x7fffffff) return fail(AA_EINVAL, "aa_dedisperse: too many tiles for one launch");
    const size_t lds = static_cast<size_t>(kChanPerPass) * p->max_row;
    hipLaunchKernelGGL((dedisp_kernel<kSampPerLane, kDmPerWave, kDedispWaves, kChanPerPass>),
                       dim3(static_cast<unsigned>(grid)), dim3(64 * kDedispWaves), lds, stream, d_in,
                       in_pitch, p->d_shifts, p->d_offs, p->d_blocks, static_cast<int>(nblk), p->nchan,
                       d_out, out_pitch, n_out, p->max_row);
    AA_HIP(hipGetLastError());
    return AA_OK;
}

}  // namespace aa

extern "C" int aa_dedisperse(aa_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                             int32_t* d_out, int64_t out_pitch, void* stream) {
    using namespace aa;
    if (!p || !d_in || !d_out) return fail(AA_EINVAL, "aa_dedisperse: null argument");
    if (p->device < 0) return fail(AA_EINVAL, "aa_dedisperse: plan was created host-only");
    if (n_in < p->maxshift + 1 || n_in > in_pitch)
        return fail(AA_EINVAL, "aa_dedisperse: need maxshift + 1 <= n_in <= in_pitch");
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15))
        return fail(AA_EINVAL, "aa_dedisperse: d_in and in_pitch must be multiples of 16 bytes");
    if ((reinterpret_cast<uintptr_t>(d_out) & 15) || (out_pitch & 3) || out_pitch < n_in - p->maxshift)
        return fail(AA_EINVAL, "aa_dedisperse: d_out must be 16-byte aligned, out_pitch a multiple of 4 and >= n_out");
    return launch_dedisperse(p, d_in, in_pitch, n_in, d_out, out_pitch, static_cast<hipStream_t>(stream));
}
