// Single-pulse search on a dedispersed plane, for gfx950 (the paper's SPDT phase,
// section 2.2). Three kernels run in order on the caller's stream:
//   sps_stats   exact int64 moments per (DM row, stat block), then mu and sigma in
//               float64, then the per-width normalisation wmu_w = w*mu and
//               r_w = 1/(sigma*sqrt(w)), and each width's smallest window sum whose
//               S/N reaches the threshold.
//   sps_detect  per (8 DM rows, 256 starts) tile: LDS prefix sums give the boxcars,
//               an integer screen against those sums drops the cells whose best S/N
//               is below the threshold, and the rest get the float64 best S/N and a
//               3x3 peak test on a one-sample, one-row halo. The result is a bit mask
//               of candidates per row, plus integer per-row counts.
//   sps_emit    one work-group per DM row. The row's output offset is the sum of
//               the counts of the rows before it. A block scan of the mask ranks each
//               candidate, and the candidate is written in (dm, t) order. Its S/N and
//               width are recomputed with the same float64 operations.
// No float atomics and no cross-stream waits are involved. The only atomics are
// integer counter adds, and their sum does not depend on order. Output order comes
// from the scan, not from the atomics. The paper's section 2.2 notes that its
// streamed search stalled on atomics combined with event waits.
#pragma clang fp contract(off)

#include <mutex>
#include <string>

#include "aa_internal.h"
#include "numerics.h"
#include "screen.h"
#include "xcd.h"

namespace aa {
namespace {

constexpr int kMaxWidths = 32;

struct SpsConst {
    int32_t nw;
    int32_t wmax;
    int32_t widths[kMaxWidths];
    double sqrtw[kMaxWidths];
    // decimated boxcar hierarchy: widths kfull .. nw-1 are tried only at starts t with
    // (t & smask[k]) == 0 (stride - 1); kfull = nw when the hierarchy is off
    int32_t kfull;
    int32_t smask[kMaxWidths];
};

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Inclusive prefix sum over the 64 lanes of a wave (modulo 2^32): shifts by 1, 2, 4 and
// 8 lanes inside each row of 16, then the last lane of row 0 (and of row 2) is added to
// row 1 (and 3), and the last lane of row 1 to rows 2 and 3. Lanes whose source falls
// outside the row, or rows masked off, add 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---- statistics -------------------------------------------------------------
// Exact count, sum and sum of squares over the block's values that pass keep(v),
// reduced over the work-group; the totals are returned to every thread.
template <class Keep>
__device__ __forceinline__ void block_moments(const int32_t* row, int64_t lo, int64_t hi, Keep keep, uint64_t* n_out,
                                              uint64_t* s1_out, uint64_t* s2_out) {
    uint64_t s1 = 0, s2 = 0, cnt = 0;
    // elements up to the first 16-byte boundary, then 4 per lane, then the tail
    const uint32_t* p = reinterpret_cast<const uint32_t*>(row + lo);
    const int64_t n = hi - lo;
    const int64_t head = min<int64_t>(static_cast<int64_t>(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) >> 2), n);
    const int64_t n4 = (n - head) >> 2;
    auto add = [&](uint32_t v) {
        if (keep(v)) {
            s1 += v;
            s2 += static_cast<uint64_t>(v) * v;
            ++cnt;
        }
    };
    if (threadIdx.x < head) add(p[threadIdx.x]);
    const u32x4_t* q = reinterpret_cast<const u32x4_t*>(p + head);
    for (int64_t i = threadIdx.x; i < n4; i += 256) {
        const u32x4_t v = q[i];
        add(v[0]);
        add(v[1]);
        add(v[2]);
        add(v[3]);
    }
    for (int64_t t = head + 4 * n4 + threadIdx.x; t < n; t += 256) add(p[t]);
    s1 = wave_sum_u64(s1);
    s2 = wave_sum_u64(s2);
    cnt = wave_sum_u64(cnt);
    __shared__ uint64_t part[3][4];
    const int wave = threadIdx.x >> 6;
    __syncthreads();   // part[] may still be read from a previous call
    if ((threadIdx.x & 63) == 0) {
        part[0][wave] = s1;
        part[1][wave] = s2;
        part[2][wave] = cnt;
    }
    __syncthreads();
    *s1_out = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    *s2_out = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    *n_out = part[2][0] + part[2][1] + part[2][2] + part[2][3];
}

// mu and sigma from exact moments, with the rounding points of the definition
__device__ __forceinline__ void mu_sigma(uint64_t n, uint64_t s1, uint64_t s2, double* mu, double* sigma) {
    *mu = static_cast<double>(s1) / static_cast<double>(n);
    const unsigned __int128 num = static_cast<unsigned __int128>(n) * s2 - static_cast<unsigned __int128>(s1) * s1;
    *sigma = __builtin_sqrt(u128_to_double_rn(num) / static_cast<double>(n * n));
}

// Per (stat block j, DM row d): exact moments, optionally clipped (clip_iters rounds of
// keeping the values within clip_c * sigma of mu, recomputing exact moments over the
// kept values; a round that would keep nothing ends the clipping), then the per-width
// normalisation and each width's smallest passing window sum.
__global__ __launch_bounds__(256) void sps_stats_kernel(const int32_t* __restrict__ dd, int64_t dd_pitch,
                                                        int64_t dd_t0, int64_t t_begin, int64_t t_end,
                                                        int32_t B, int32_t ndm, SpsConst sc,
                                                        double threshold, double clip_c, int32_t clip_iters,
                                                        double* __restrict__ norms, uint32_t* __restrict__ smin,
                                                        int32_t* __restrict__ rowcount) {
    const int j = blockIdx.x;
    const int d = blockIdx.y;
    const int64_t lo = t_begin + static_cast<int64_t>(j) * B;
    const int64_t hi = min(lo + B, t_end);
    const int32_t* row = dd + static_cast<int64_t>(d) * dd_pitch - dd_t0;
    uint64_t n, s1, s2;
    block_moments(row, lo, hi, [](uint32_t) { return true; }, &n, &s1, &s2);
    double mu, sigma;
    mu_sigma(n, s1, s2, &mu, &sigma);
    for (int it = 0; it < clip_iters; ++it) {
        const double lim = clip_c * sigma;
        uint64_t m, a, b;
        block_moments(row, lo, hi, [=](uint32_t v) { return __builtin_fabs(static_cast<double>(v) - mu) <= lim; }, &m,
                      &a, &b);
        if (m == 0) break;   // uniform: every thread holds the same totals
        n = m;
        s1 = a;
        s2 = b;
        mu_sigma(n, s1, s2, &mu, &sigma);
    }
    if (threadIdx.x == 0) {
        double* out = norms + (static_cast<int64_t>(j) * ndm + d) * (2 * sc.nw);
        uint32_t* so = smin + (static_cast<int64_t>(j) * ndm + d) * sc.nw;
        for (int k = 0; k < sc.nw; ++k) {
            out[k] = static_cast<double>(sc.widths[k]) * mu;
            out[sc.nw + k] = sigma == 0.0 ? 0.0 : 1.0 / (sigma * sc.sqrtw[k]);
            so[k] = min_passing_sum(out[k], out[sc.nw + k], threshold);
        }
        if (j == 0) rowcount[d] = 0;
    }
}

// ---- detection ----------------------------------------------------------------
constexpr int kHaloRows = kSpsRows + 2;
constexpr int kHaloCols = kSpsTile + 2;

// LDS of a detection work-group, in this order: 8 bytes, prefix sums [kHaloRows][ps]
// (u32, row stride ps >= kSpsTile + 2 + wmax, a multiple of 4, so that entry 2 of every
// row is 16-byte aligned), then (EXACT only) the float64 best S/N of every halo cell
// [kHaloRows][kHaloCols]. The float64 normalisation is read from global memory (cached)
// by the exact evaluations, which only cells passing the screen need.
struct DetectLds {
    int tail, total;   // byte offsets
};
__host__ __device__ inline int detect_row_stride(int wmax) { return 4 * ((kSpsTile + wmax + 3) / 4 + 1); }
__host__ __device__ inline DetectLds detect_lds(int wmax, int nw, bool exact) {
    DetectLds L;
    (void)nw;
    L.tail = (8 + kHaloRows * detect_row_stride(wmax) * 4 + 15) / 16 * 16;
    L.total = L.tail + (exact ? kHaloRows * kHaloCols * 8 : 0);
    return L;
}

// Exact value of one halo cell: best S/N over the widths, float64, same operation order
// as the oracle. -inf outside the range of rows and starts.
__device__ __forceinline__ double exact_best(const uint32_t* pre, int stride, const double* nj, int d0,
                                             const SpsConst& sc, int r, int c, bool valid, uint32_t t) {
    if (!valid) return -__builtin_huge_val();
    const uint32_t* pr = pre + r * stride + c;
    const double* nr = nj + static_cast<int64_t>(d0 - 1 + r) * (2 * sc.nw);   // halo row r is trial d0 - 1 + r
    double v = 0.0;
    for (int k = 0; k < sc.nw; ++k) {
        if (k >= sc.kfull && (t & static_cast<uint32_t>(sc.smask[k]))) continue;   // not on this width's grid
        const uint32_t s = pr[sc.widths[k]] - pr[0];
        const double snr = (static_cast<double>(s) - nr[k]) * nr[sc.nw + k];
        if (k == 0 || snr > v) v = snr;
    }
    return v;
}

// EXACT: every halo cell in float64 (needed when the best plane is an output).
// Otherwise an integer screen runs first (min_passing_sum): cells whose best S/N cannot
// reach the threshold are dropped, and only the others, with their 8 neighbours, are
// evaluated in float64 for the 3x3 peak decision. The launcher takes this path only when
// every window sum is below 2^31.
template <bool EXACT>
__global__ __launch_bounds__(256) void sps_detect_kernel(
    const int32_t* __restrict__ dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n, int64_t t_begin,
    int64_t t_end, int64_t t_total, int32_t B, int32_t ndm, double threshold, SpsConst sc,
    const double* __restrict__ norms, const uint32_t* __restrict__ smin_g, int32_t* __restrict__ rowcount,
    uint32_t* __restrict__ mask, int64_t nwords, float* __restrict__ best_out, int64_t best_pitch) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int nw = sc.nw;
    const int tw = kSpsTile + 1 + sc.wmax;            // D columns t_tile0-1 .. t_tile0+255+wmax
    const int pw = tw + 1;                            // prefix entries per row
    const int ps = detect_row_stride(sc.wmax);        // row stride of the prefix sums
    const DetectLds L = detect_lds(sc.wmax, nw, EXACT);
    uint32_t* pre = reinterpret_cast<uint32_t*>(smem + 8);               // [kHaloRows][ps]

    // XCD-aware order: each XCD walks consecutive time tiles of a row block, which share
    // their halo columns in its L2
    const int item = xcd_remap(static_cast<int>(blockIdx.x + blockIdx.y * gridDim.x),
                               static_cast<int>(gridDim.x * gridDim.y));
    const int bx = item % static_cast<int>(gridDim.x), by = item / static_cast<int>(gridDim.x);
    const int64_t tt0 = t_begin + static_cast<int64_t>(bx) * kSpsTile;
    const int64_t tile_end = min(tt0 + kSpsTile, t_end);
    const int d0 = by * kSpsRows;
    const int j = static_cast<int>((static_cast<uint64_t>(bx) * kSpsTile) / static_cast<uint32_t>(B));
    const int64_t lo = max(tt0 - 1, static_cast<int64_t>(0));
    const int64_t hi = (t_total < 0 || tile_end < t_total) ? tile_end + 1 : tile_end;  // best valid in [lo, hi)
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const double* nj = norms + static_cast<int64_t>(j) * ndm * (2 * nw);

    // halo row r (trial d0 - 1 + r) belongs to wave r % 4: the prefix sums of its D
    // columns, pre[r][j] = sum of D[t_tile0 - 1 + i] for i < j
    // (modulo 2^32: every window sum is exact below 2^32), for j < pw
    {
        const int64_t col0 = tt0 - 1 - dd_t0;          // plane column of i = 0
        const int nq = (kSpsTile + sc.wmax + 3) / 4;   // 4-column groups from t_tile0 on
        // a tile inside an aligned plane loads 16 bytes per lane and scans in registers
        const bool fast = col0 >= 0 && col0 + 1 + 4 * nq <= dd_n && ((col0 + 1) & 3) == 0 && (dd_pitch & 3) == 0 &&
                          (reinterpret_cast<uintptr_t>(dd) & 15) == 0;
        const int ilo = col0 < 0 ? static_cast<int>(-col0) : 0;
        const int ihi = static_cast<int>(min<int64_t>(tw, dd_n - col0));
        // up to 128 groups (wmax <= 256): all of the wave's loads are issued before any
        // scan, so their latencies overlap
        const bool fast2 = fast && nq <= 128;
        u32x4_t xs[3][2];
        uint32_t firsts[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            firsts[i] = 0u;
            xs[i][0] = xs[i][1] = u32x4_t{0u, 0u, 0u, 0u};
            const int r = wave + 4 * i, d = d0 - 1 + r;
            if (fast2 && r < kHaloRows && d >= 0 && d < ndm) {
                const int32_t* src = dd + static_cast<int64_t>(d) * dd_pitch + col0;
                firsts[i] = static_cast<uint32_t>(src[0]);
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (64 * c + lane < nq) xs[i][c] = *reinterpret_cast<const u32x4_t*>(src + 1 + 4 * (64 * c + lane));
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int r = wave + 4 * i;
            if (r >= kHaloRows) break;
            const int d = d0 - 1 + r;
            const bool in = d >= 0 && d < ndm;
            uint32_t* prow = pre + r * ps;
            if (!in) {
                for (int k = lane; k < ps; k += 64) prow[k] = 0u;
                continue;
            }
            const int32_t* src = dd + static_cast<int64_t>(d) * dd_pitch + col0;
            if (fast2) {
                uint32_t carry = firsts[i];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int u = 64 * c + lane;
                    const u32x4_t x = xs[i][c];
                    const uint32_t a = x[0], b = a + x[1], cc = b + x[2], e = cc + x[3];
                    const uint32_t incl = wave_incl_scan(e);
                    const uint32_t base = carry + (incl - e);
                    if (u < nq) *reinterpret_cast<u32x4_t*>(prow + 2 + 4 * u) = u32x4_t{base + a, base + b, base + cc, base + e};
                    carry += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
                }
                if (lane == 0) {
                    prow[0] = 0u;
                    prow[1] = firsts[i];
                }
            } else if (fast) {
                // lane holds columns t_tile0 + 4u .. + 3, u = lane, lane + 64, ...
                const uint32_t first = static_cast<uint32_t>(src[0]);
                uint32_t carry = first;
                for (int u0 = 0; u0 < nq; u0 += 64) {
                    const int u = u0 + lane;
                    u32x4_t x = {0u, 0u, 0u, 0u};
                    if (u < nq) x = *reinterpret_cast<const u32x4_t*>(src + 1 + 4 * u);
                    const uint32_t a = x[0], b = a + x[1], c = b + x[2], e = c + x[3];
                    const uint32_t incl = wave_incl_scan(e);
                    const uint32_t base = carry + (incl - e);
                    if (u < nq) *reinterpret_cast<u32x4_t*>(prow + 2 + 4 * u) = u32x4_t{base + a, base + b, base + c, base + e};
                    carry += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
                }
                if (lane == 0) {
                    prow[0] = 0u;
                    prow[1] = first;
                }
            } else {
                // columns outside the plane count as 0; then the prefix in place, by the
                // same wave (LDS operations of one wave complete in order)
                if (lane == 0) prow[0] = 0u;
                for (int i = lane; i < tw; i += 64) prow[1 + i] = (i >= ilo && i < ihi) ? static_cast<uint32_t>(src[i]) : 0u;
                const int per = (pw + 63) / 64;
                const int a = lane * per, b = min(a + per, pw);
                uint32_t s = 0;
                for (int i = a; i < b; ++i) s += prow[i];
                uint32_t run = wave_incl_scan(s) - s;
                for (int i = a; i < b; ++i) {
                    run += prow[i];
                    prow[i] = run;
                }
            }
        }
    }
    // screen thresholds of the inner rows wave + 1 and wave + 5 (from the statistics
    // kernel): lane k holds width k's smallest passing window sum (kNever if none)
    uint32_t smin[2] = {kNever, kNever};
    const int wlane = lane < nw ? sc.widths[lane < kMaxWidths ? lane : 0] : 0;   // width of lane k
    if constexpr (!EXACT) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int d = d0 + wave + 4 * h;
            if (lane < nw && d < ndm) smin[h] = smin_g[(static_cast<int64_t>(j) * ndm + d) * nw + lane];
        }
    }
    __syncthreads();
    if constexpr (EXACT) {
        double* best = reinterpret_cast<double*>(smem + L.tail);         // [kHaloRows][kHaloCols]
        __shared__ int32_t cnt[kSpsRows];
        if (tid < kSpsRows) cnt[tid] = 0;
        for (int i = tid; i < kHaloRows * kHaloCols; i += 256) {
            const int r = i / kHaloCols, c = i - r * kHaloCols;
            const int d = d0 - 1 + r;
            const int64_t t = tt0 - 1 + c;
            best[i] = exact_best(pre, ps, nj, d0, sc, r, c, d >= 0 && d < ndm && t >= lo && t < hi,
                                 static_cast<uint32_t>(t));
        }
        __syncthreads();
        // 3x3 peak test for the inner rows, 64 consecutive starts per wave step
        for (int item = tid; item < kSpsRows * kSpsTile; item += 256) {
            const int ri = item / kSpsTile, tc = item - ri * kSpsTile;
            const int d = d0 + ri;
            const int64_t t = tt0 + tc;
            bool ok = false;
            if (d < ndm && t < tile_end) {
                const double* m = best + (ri + 1) * kHaloCols + (tc + 1);
                const double v = m[0];
                ok = v >= threshold && v > m[-kHaloCols - 1] && v > m[-kHaloCols] && v > m[-kHaloCols + 1] &&
                     v > m[-1] && v >= m[1] && v >= m[kHaloCols - 1] && v >= m[kHaloCols] && v >= m[kHaloCols + 1];
                if (best_out) best_out[static_cast<int64_t>(d) * best_pitch + (t - t_begin)] = static_cast<float>(v);
            }
            const uint64_t bal = __ballot(ok);
            if (lane == 0 && d < ndm) {
                const int64_t w = (tt0 - t_begin) / 32 + tc / 32;
                *reinterpret_cast<uint64_t*>(mask + static_cast<int64_t>(d) * nwords + w) = bal;
                if (bal) atomicAdd(&cnt[ri], __popcll(bal));
            }
        }
        __syncthreads();
        if (tid < kSpsRows && d0 + tid < ndm && cnt[tid] > 0) atomicAdd(&rowcount[d0 + tid], cnt[tid]);
    } else {
        // wave w screens inner rows w and w + 4; lane l holds starts 64 q + l, q < 4. A cell
        // passes if some width's window sum reaches that width's smallest passing sum,
        // which is exactly the float64 rule best >= threshold. The same lanes take the exact
        // peak test of the cells that pass, so each row's mask words and count come from
        // one wave.
        // both rows in one width loop (row wave + 5 reads the prefix of row wave + 1 if it
        // is past the last trial; its result is not used)
        int32_t margin[2][4];   // max over widths of (window sum - smallest passing sum)
        {
            const uint32_t* pr0 = pre + (wave + 1) * ps + 1 + lane;   // prefix at start tt0 + 64 q + lane
            const uint32_t* pr1 = d0 + wave + 4 < ndm ? pre + (wave + 5) * ps + 1 + lane : pr0;
            uint32_t neg0[2][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                neg0[0][q] = 0u - pr0[64 * q];
                neg0[1][q] = 0u - pr1[64 * q];
                asm volatile("" : "+v"(neg0[0][q]), "+v"(neg0[1][q]));   // keep each sum one three-way add
                margin[0][q] = margin[1][q] = INT32_MIN;
            }
            const int nsm0 = static_cast<int>(0u - smin[0]);   // lane k: minus width k's threshold
            const int nsm1 = static_cast<int>(0u - smin[1]);
#pragma unroll 3
            for (int k = 0; k < sc.kfull; ++k) {
                const int w = __builtin_amdgcn_readlane(wlane, k);
                const uint32_t nsk0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(nsm0, k));
                const uint32_t nsk1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(nsm1, k));
                // sum - smin lies in (-2^31, 2^31): sums are below 2^31 and smin <= 2^31
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    margin[0][q] = max(margin[0][q], static_cast<int32_t>(pr0[64 * q + w] + neg0[0][q] + nsk0));
                    margin[1][q] = max(margin[1][q], static_cast<int32_t>(pr1[64 * q + w] + neg0[1][q] + nsk1));
                }
            }
            // widths of the decimated hierarchy: only starts on the width's grid count
#pragma unroll 1
            for (int k = sc.kfull; k < nw; ++k) {
                const int w = __builtin_amdgcn_readlane(wlane, k);
                const uint32_t nsk0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(nsm0, k));
                const uint32_t nsk1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(nsm1, k));
                const uint32_t sm = static_cast<uint32_t>(sc.smask[k]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if ((static_cast<uint32_t>(tt0 + 64 * q + lane) & sm) == 0) {
                        margin[0][q] = max(margin[0][q], static_cast<int32_t>(pr0[64 * q + w] + neg0[0][q] + nsk0));
                        margin[1][q] = max(margin[1][q], static_cast<int32_t>(pr1[64 * q + w] + neg0[1][q] + nsk1));
                    }
                }
            }
        }
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int ri = wave + 4 * h, r = ri + 1;
            const int d = d0 + ri;
            if (d >= ndm) break;
            uint32_t pass = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if ((h ? margin[1][q] : margin[0][q]) >= 0 && tt0 + 64 * q + lane < tile_end) pass |= 1u << q;
            int pop = 0;
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                bool ok = false;
                if ((pass >> q) & 1u) {
                    auto val = [&](int rr_, int cc) {
                        const int dr = d0 - 1 + rr_;
                        const int64_t tr = tt0 - 1 + cc;
                        return exact_best(pre, ps, nj, d0, sc, rr_, cc, dr >= 0 && dr < ndm && tr >= lo && tr < hi,
                                          static_cast<uint32_t>(tr));
                    };
                    const int c0 = 64 * q + lane + 1;
                    const double x = val(r, c0);
                    ok = x >= threshold && x > val(r - 1, c0 - 1) && x > val(r - 1, c0) && x > val(r - 1, c0 + 1) &&
                         x > val(r, c0 - 1) && x >= val(r, c0 + 1) && x >= val(r + 1, c0 - 1) &&
                         x >= val(r + 1, c0) && x >= val(r + 1, c0 + 1);
                }
                const uint64_t bal = __ballot(ok);
                if (lane == 0)
                    *reinterpret_cast<uint64_t*>(mask + static_cast<int64_t>(d) * nwords + (tt0 - t_begin) / 32 + 2 * q) = bal;
                pop += __popcll(bal);
            }
            if (lane == 0 && pop > 0) atomicAdd(&rowcount[d], pop);
        }
    }
}

// ---- emission -------------------------------------------------------------------
constexpr int kEmitList = 1024;   // candidates listed per batch in LDS
__device__ int block_excl_scan(int v, int* total, int* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wave) base += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ __launch_bounds__(256) void sps_emit_kernel(
    const int32_t* __restrict__ dd, int64_t dd_pitch, int64_t dd_t0, int64_t t_begin, int32_t B,
    int32_t ndm, SpsConst sc, const double* __restrict__ norms, const int32_t* __restrict__ rowcount,
    const uint32_t* __restrict__ mask, int64_t nwords, aa_candidate_t* __restrict__ cand, int32_t cap,
    int32_t* __restrict__ count, int32_t beam_id) {
    __shared__ int sh[4];
    __shared__ int64_t red[4];
    const int d = blockIdx.x;
    int64_t off = 0;
    for (int i = threadIdx.x; i < d; i += 256) off += rowcount[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = off;
    __syncthreads();
    off = red[0] + red[1] + red[2] + red[3];
    const int mine = rowcount[d];
    if (d == ndm - 1 && threadIdx.x == 0) *count = static_cast<int32_t>(min<int64_t>(off + mine, 0x7fffffff));
    if (mine == 0 || off >= cap) return;
    const int32_t* row = dd + static_cast<int64_t>(d) * dd_pitch - dd_t0;
    int64_t running = off;
    __shared__ int64_t tl[kEmitList];   // starts of one batch of the row's candidates, in order
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t k0 = 0; k0 < nwords; k0 += 256) {
        const int64_t k = k0 + threadIdx.x;
        const uint32_t word = k < nwords ? mask[static_cast<int64_t>(d) * nwords + k] : 0u;
        int total;
        const int excl = block_excl_scan(__popc(word), &total, sh);
        for (int b0 = 0; b0 < total; b0 += kEmitList) {
            // list the batch's starts, then one wave per candidate
            uint32_t wv = word;
            for (int idx = excl; wv; ++idx) {
                const int b = __ffs(wv) - 1;
                wv &= wv - 1;
                if (idx >= b0 && idx < b0 + kEmitList) tl[idx - b0] = t_begin + 32 * k + b;
            }
            __syncthreads();
            const int nb = min(kEmitList, total - b0);
            for (int i = wave; i < nb && running + b0 + i < cap; i += 4) {
                const int64_t t = tl[i];
                const int jb = static_cast<int>((t - t_begin) / B);
                const double* nr = norms + (static_cast<int64_t>(jb) * ndm + d) * (2 * sc.nw);
                // window sums from a wave scan: lane l holds samples c0 + 4 l .. c0 + 4 l + 3
                // of each 256-sample chunk; S/N and the smallest best width in the order
                // of the detection's exact evaluation
                double v = 0.0;
                int wbest = sc.widths[0];
                uint32_t carry = 0;
                int q = 0;
                for (int c0 = 0; c0 < sc.wmax; c0 += 256) {
                    uint32_t x[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ix = c0 + 4 * lane + e;
                        x[e] = ix < sc.wmax ? static_cast<uint32_t>(row[t + ix]) : 0u;
                    }
                    const uint32_t p1 = x[0] + x[1], p2 = p1 + x[2], p3 = p2 + x[3];
                    const uint32_t incl = wave_incl_scan(p3);
                    const uint32_t base = carry + (incl - p3);
                    const uint32_t pre4[4] = {base + x[0], base + p1, base + p2, base + p3};
                    for (; q < sc.nw && sc.widths[q] <= c0 + 256; ++q) {
                        if (q >= sc.kfull && (static_cast<uint32_t>(t) & static_cast<uint32_t>(sc.smask[q]))) continue;
                        const int ix = sc.widths[q] - 1 - c0;    // sum of the first widths[q] samples
                        const uint32_t sel = pre4[ix & 3];
                        const uint32_t S = static_cast<uint32_t>(__shfl(static_cast<int>(sel), ix >> 2, 64));
                        const double snr = (static_cast<double>(S) - nr[q]) * nr[sc.nw + q];
                        if (q == 0 || snr > v) {
                            v = snr;
                            wbest = sc.widths[q];
                        }
                    }
                    carry += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
                }
                if (lane == 0) {
                    aa_candidate_t c;
                    c.dm_idx = d;
                    c.width = wbest;
                    c.t = t;
                    c.snr = static_cast<float>(v);
                    c.beam = beam_id;
                    cand[running + b0 + i] = c;
                }
            }
            __syncthreads();
        }
        running += total;
        if (running >= cap) break;
    }
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct WorkLayout {
    size_t norms, smin, rowcount, mask, total;
    int64_t nblk, ntiles, nwords;
};

WorkLayout layout(const aa_plan_s* p, int64_t n_starts) {
    WorkLayout L{};
    L.nblk = (n_starts + p->stat_block - 1) / p->stat_block;
    L.ntiles = (n_starts + kSpsTile - 1) / kSpsTile;
    L.nwords = L.ntiles * (kSpsTile / 32);
    L.norms = 0;
    L.smin = align256(static_cast<size_t>(L.nblk) * p->ndm * 2 * p->nwidths * sizeof(double));
    L.rowcount = L.smin + align256(static_cast<size_t>(L.nblk) * p->ndm * p->nwidths * sizeof(uint32_t));
    L.mask = L.rowcount + align256(static_cast<size_t>(p->ndm) * sizeof(int32_t));
    L.total = L.mask + align256(static_cast<size_t>(p->ndm) * L.nwords * sizeof(uint32_t));
    return L;
}

}  // namespace

size_t sps_work_bytes(const aa_plan_s* p, int64_t n_starts) { return n_starts > 0 ? layout(p, n_starts).total : 0; }

int launch_single_pulse(const aa_plan_s* p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n,
                        int64_t t_begin, int64_t t_end, int64_t t_total, void* d_work, aa_candidate_t* d_cand,
                        int32_t cap, int32_t* d_count, float* d_best, int64_t best_pitch, hipStream_t stream,
                        int32_t beam_id) {
    const int64_t n = t_end - t_begin;
    const WorkLayout L = layout(p, n);
    uint8_t* w = static_cast<uint8_t*>(d_work);
    double* norms = reinterpret_cast<double*>(w + L.norms);
    uint32_t* smin = reinterpret_cast<uint32_t*>(w + L.smin);
    int32_t* rowcount = reinterpret_cast<int32_t*>(w + L.rowcount);
    uint32_t* mask = reinterpret_cast<uint32_t*>(w + L.mask);
    SpsConst sc{};
    sc.nw = p->nwidths;
    sc.wmax = p->wmax;
    sc.kfull = p->nwidths;
    for (int k = 0; k < p->nwidths; ++k) {
        sc.widths[k] = p->widths[k];
        sc.sqrtw[k] = p->sqrtw[k];
        int64_t stride = 1;   // smallest power of two with full_width * stride >= width
        if (p->boxcar_full_width > 0)
            while (static_cast<int64_t>(p->boxcar_full_width) * stride < p->widths[k]) stride *= 2;
        sc.smask[k] = static_cast<int32_t>(stride - 1);
        if (stride > 1 && sc.kfull == p->nwidths) sc.kfull = k;   // widths ascend: the rest are strided too
    }
    hipLaunchKernelGGL(sps_stats_kernel, dim3(static_cast<unsigned>(L.nblk), static_cast<unsigned>(p->ndm)), dim3(256),
                       0, stream, d_dd, dd_pitch, dd_t0, t_begin, t_end, p->stat_block, p->ndm, sc,
                       static_cast<double>(p->threshold), static_cast<double>(p->clip_sigma),
                       p->clip_sigma > 0.0f ? p->clip_iters : 0, norms, smin, rowcount);
    AA_HIP(hipGetLastError());
    const unsigned rowblocks = static_cast<unsigned>((p->ndm + kSpsRows - 1) / kSpsRows);
    if (L.ntiles * static_cast<int64_t>(rowblocks) > 0x7fffffff)
        return fail(AA_EINVAL, "aa_single_pulse: too many detection tiles for one launch");
    // the integer screen compares window sums below 2^31
    const bool screen = !d_best && static_cast<uint64_t>(p->nchan) * 255u * static_cast<uint64_t>(p->wmax) < (1ull << 31);
    const size_t lds = static_cast<size_t>(detect_lds(p->wmax, p->nwidths, !screen).total);
    hipLaunchKernelGGL(screen ? sps_detect_kernel<false> : sps_detect_kernel<true>,
                       dim3(static_cast<unsigned>(L.ntiles), rowblocks), dim3(256), lds, stream,
                       d_dd, dd_pitch, dd_t0, dd_n, t_begin, t_end, t_total, p->stat_block, p->ndm,
                       static_cast<double>(p->threshold), sc, norms, smin, rowcount, mask, L.nwords, d_best, best_pitch);
    AA_HIP(hipGetLastError());
    hipLaunchKernelGGL(sps_emit_kernel, dim3(static_cast<unsigned>(p->ndm)), dim3(256), 0, stream, d_dd, dd_pitch,
                       dd_t0, t_begin, p->stat_block, p->ndm, sc, norms, rowcount, mask, L.nwords, d_cand, cap,
                       d_count, beam_id);
    AA_HIP(hipGetLastError());
    return AA_OK;
}

}  // namespace aa

extern "C" int aa_single_pulse_work_bytes(aa_plan_t p, int64_t n_starts, size_t* out) {
    using namespace aa;
    if (!p || !out || n_starts < 1) return fail(AA_EINVAL, "aa_single_pulse_work_bytes: bad argument");
    *out = sps_work_bytes(p, n_starts);
    return AA_OK;
}

namespace aa {
namespace {
// Argument checks shared by aa_single_pulse and aa_single_pulse_noalloc.
int check_single_pulse(const char* fn, aa_plan_t p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n,
                       int64_t t_begin, int64_t t_end, int64_t t_total, aa_candidate_t* d_cand, int32_t cap,
                       int32_t* d_count, float* d_best, int64_t best_pitch) {
    const std::string f(fn);
    if (!p || !d_dd || !d_count || (cap > 0 && !d_cand)) return fail(AA_EINVAL, f + ": null argument");
    if (p->device < 0) return fail(AA_EINVAL, f + ": plan was created host-only");
    if (p->nwidths > kMaxWidths) return fail(AA_EINVAL, f + ": more than 32 widths");
    if (cap < 0) return fail(AA_EINVAL, f + ": cap < 0");
    if (t_begin < 0 || t_end <= t_begin || t_begin % p->stat_block)
        return fail(AA_EINVAL, f + ": need 0 <= t_begin < t_end and t_begin a multiple of stat_block");
    if (t_total >= 0 && t_end > t_total) return fail(AA_EINVAL, f + ": t_end > t_total");
    if (dd_n < 1 || dd_n > dd_pitch) return fail(AA_EINVAL, f + ": need 1 <= dd_n <= dd_pitch");
    if (dd_t0 > (t_begin > 0 ? t_begin - 1 : t_begin)) return fail(AA_EINVAL, f + ": plane misses the left halo column");
    const int64_t right = (t_total >= 0 && t_end >= t_total) ? t_end : t_end + 1;
    if (dd_t0 + dd_n < right + p->wmax - 1) return fail(AA_EINVAL, f + ": plane too short for the right edge");
    if (d_best && best_pitch < t_end - t_begin) return fail(AA_EINVAL, f + ": best_pitch too small");
    return AA_OK;
}

// Scratch of aa_single_pulse_noalloc: one copy per GPU, alive until the process ends.
// Host code never passes `scratch` itself to a kernel (in host code the name is only a
// stand-in for the symbol): it passes the device address that hipGetSymbolAddress
// returned for the current device.
__device__ __align__(256) uint8_t scratch[AA_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[256] = {};

// The device address of `scratch` on the current device, looked up once per device.
int scratch_ptr(void** out) {
    int dev = 0;
    AA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) return fail(AA_EINVAL, "aa_single_pulse_noalloc: device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "aa_single_pulse_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return AA_OK;
}
}  // namespace
}  // namespace aa

extern "C" int aa_single_pulse(aa_plan_t p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n,
                               int64_t t_begin, int64_t t_end, int64_t t_total, void* d_work, size_t work_bytes,
                               aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, float* d_best,
                               int64_t best_pitch, void* stream) {
    using namespace aa;
    if (!d_work) return fail(AA_EINVAL, "aa_single_pulse: null argument");
    const int rc = check_single_pulse("aa_single_pulse", p, d_dd, dd_pitch, dd_t0, dd_n, t_begin, t_end, t_total, d_cand,
                                      cap, d_count, d_best, best_pitch);
    if (rc != AA_OK) return rc;
    if (work_bytes < sps_work_bytes(p, t_end - t_begin)) return fail(AA_EINVAL, "aa_single_pulse: work buffer too small");
    if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(AA_EINVAL, "aa_single_pulse: d_work must be 256-byte aligned");
    return launch_single_pulse(p, d_dd, dd_pitch, dd_t0, dd_n, t_begin, t_end, t_total, d_work, d_cand, cap, d_count,
                               d_best, best_pitch, static_cast<hipStream_t>(stream));
}

extern "C" int aa_single_pulse_noalloc(aa_plan_t p, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n,
                                       int64_t t_begin, int64_t t_end, int64_t t_total, aa_candidate_t* d_cand,
                                       int32_t cap, int32_t* d_count, float* d_best, int64_t best_pitch, void* stream) {
    using namespace aa;
    int rc = check_single_pulse("aa_single_pulse_noalloc", p, d_dd, dd_pitch, dd_t0, dd_n, t_begin, t_end, t_total,
                                d_cand, cap, d_count, d_best, best_pitch);
    if (rc != AA_OK) return rc;
    const size_t need = sps_work_bytes(p, t_end - t_begin);
    if (need > static_cast<size_t>(AA_NOALLOC_SCRATCH_BYTES))
        return fail(AA_EINVAL, "aa_single_pulse_noalloc: the search needs " + std::to_string(need) +
                                   " bytes of scratch, more than the fixed " +
                                   std::to_string(static_cast<size_t>(AA_NOALLOC_SCRATCH_BYTES)) +
                                   "; use aa_single_pulse with a work buffer or search fewer starts per call");
    void* ptr = nullptr;
    rc = scratch_ptr(&ptr);
    if (rc != AA_OK) return rc;
    // every scratch word the kernels read is written first in the same call (moments,
    // norms, row counts cleared by the statistics kernel, every mask word by detection)
    return launch_single_pulse(p, d_dd, dd_pitch, dd_t0, dd_n, t_begin, t_end, t_total, ptr, d_cand, cap, d_count,
                               d_best, best_pitch, static_cast<hipStream_t>(stream));
}
