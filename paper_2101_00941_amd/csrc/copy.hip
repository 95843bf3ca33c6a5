// Host->device row gather for the streamed pipeline (the H2D step of section 2's
// recipe). A chunk of a [nchan][pitch] pinned host filterbank is a strided 2-D region.
// The runtime's 2-D copy moves it at a fraction of the PCIe rate: about 12 GB/s,
// against 56 GB/s for 1-D copies, measured on this chip. This kernel reads the mapped
// pinned rows directly over PCIe with 16-byte loads, several in flight per lane, and
// writes them into the beam's history buffer.
#include "aa_internal.h"

namespace aa {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gather_rows_kernel(uint8_t* __restrict__ dst, int64_t dpitch,
                                                          const uint8_t* __restrict__ src, int64_t spitch,
                                                          int64_t vec_per_row, int64_t total_vec) {
    constexpr int U = 4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i0 < total_vec; i0 += stride * U) {
        u32x4 v[U];
        int64_t idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            idx[u] = i0 + u * stride;
            if (idx[u] < total_vec) {
                const int64_t r = idx[u] / vec_per_row, c = idx[u] - r * vec_per_row;
                v[u] = *reinterpret_cast<const u32x4*>(src + r * spitch + 16 * c);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (idx[u] < total_vec) {
                const int64_t r = idx[u] / vec_per_row, c = idx[u] - r * vec_per_row;
                *reinterpret_cast<u32x4*>(dst + r * dpitch + 16 * c) = v[u];
            }
        }
    }
}

}  // namespace

// dst/src row starts, both pitches and width must be multiples of 16 bytes. src is a
// device-visible pointer to pinned host memory.
int launch_gather_rows(uint8_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch, int64_t width,
                       int64_t nrows, hipStream_t stream) {
    const int64_t vpr = width / 16;
    const int64_t total = vpr * nrows;
    if (total == 0) return AA_OK;
    const int64_t want = (total + 256 * 4 - 1) / (256 * 4);
    // The copy is bound by PCIe reads of mapped host memory, not by the CUs: 32 work-groups
    // of 4 waves, each lane with 4 x 16 bytes in flight, keep 512 KB of reads outstanding,
    // which holds the full host-link rate (measured: 56 GB/s from 24 to 160 work-groups,
    // slower at 16), and leave the other CUs to the kernels it overlaps. At 160 work-groups
    // the overlapped dedispersion launches ran 3.5-5x longer than alone.
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(want, 32));
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid), dim3(256), 0, stream, dst, dpitch, src, spitch, vpr, total);
    AA_HIP(hipGetLastError());
    return AA_OK;
}

}  // namespace aa
