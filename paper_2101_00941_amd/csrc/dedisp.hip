// Brute-force incoherent dedispersion for gfx950 (the paper's dedispersion phase,
// section 2.1):  D[d][t] = sum_c X[c][t + s[d][c]], exact in integers.
//
// Shape of the kernel:
//  * A work-group of W waves owns one DM block of up to W * DPW consecutive trials
//    and one time tile of 1024 samples. Each wave owns DPW trials. Each lane owns
//    16 consecutive samples of each of its trials.
//  * The input is consumed in passes of 16 channel rows. A pass is staged in LDS
//    with direct global->LDS 16-byte loads (global_load_lds_dwordx4), with no
//    register round trip, into one of two buffers. The next pass streams in while
//    the current one is summed. A staged row holds the bytes
//    [t0 + (s[first][c] & ~15), + row), which cover every trial of the block. So
//    each staged byte is reused by all trials of the block.
//  * The inner step for one (channel, trial): two aligned ds_read_b128 bring in
//    the 32 bytes around the lane's 16-sample window. Eight v_perm_b32 extract the
//    window as zero-extended 16-bit pairs. The byte phase (o & 3) picks the
//    selector, and (o >> 2) & 3 picks the registers through a uniform branch. Two
//    channels are folded per v_add3_u32 into packed u16x2 accumulators. A 16-bit
//    half holds up to 257 * 255, so the pairs are widened into int32 accumulators
//    every 256 channels.
//  * The shift-and-add variants (layouts 0-3) use no matrix cores. The layouts 4-6
//    variants below recast each block of 32 trials as an exact one-hot int8 contraction
//    on the matrix cores (v_mfma_i32_32x32x32_i8), which is faster on this chip although
//    most of its multiply-accumulates are by zero; see dedisp_mfma_tile.
#include "aa_internal.h"
#include "xcd.h"

namespace aa {
namespace {

// A DM block's table entry, read through the constant address space: it is the same in
// every lane and read-only for the launch, so its loads are scalar even where the table
// pointer comes from memory (the persistent batch kernel reads it from the beam's
// argument block).
__device__ __forceinline__ DmBlock load_block(const DmBlock* blocks, int blk) {
    static_assert(sizeof(DmBlock) % 4 == 0, "a DM block entry is whole dwords");
    typedef const __attribute__((address_space(4))) int32_t* word_ptr;
    const word_ptr p = (word_ptr)(const void*)(blocks + blk);
    int32_t w[sizeof(DmBlock) / 4];
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(DmBlock) / 4); ++i) w[i] = p[i];
    DmBlock b;
    __builtin_memcpy(&b, w, sizeof(b));
    return b;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

// Work-group i runs on XCD i % 8. Give each XCD a contiguous run of logical tiles
// (adjacent DM blocks of the same time tile), so that their overlapping input rows
// are shared in that XCD's L2.

template <int Q>
__device__ __forceinline__ void extract16(const u32x4& x0, const u32x4& x1, uint32_t sel0, uint32_t sel1,
                                          uint32_t (&p)[8]) {
    const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = Q + (j >> 1);
        p[j] = __builtin_amdgcn_perm(w[i + 1], w[i], (j & 1) ? sel1 : sel0);
    }
}

// The 16 samples of a lane's window, as 8 zero-extended u16 pairs (sample 2j in the
// low half, 2j+1 in the high half). x0 and x1 are the two aligned 16-byte reads at
// the lane's slot + (o & ~15), where o is the trial's byte offset within the row.
__device__ __forceinline__ void window16(const u32x4& x0, const u32x4& x1, int o, uint32_t (&p)[8]) {
    const uint32_t r = static_cast<uint32_t>(o & 3);
    const uint32_t sel0 = 0x0C000C00u | ((r + 1u) << 16) | r;
    const uint32_t sel1 = sel0 + 0x00020002u;
    switch ((o >> 2) & 3) {
        case 0: extract16<0>(x0, x1, sel0, sel1, p); break;
        case 1: extract16<1>(x0, x1, sel0, sel1, p); break;
        case 2: extract16<2>(x0, x1, sel0, sel1, p); break;
        default: extract16<3>(x0, x1, sel0, sel1, p); break;
    }
}

// Interleaved layout: lane l owns the four 4-sample groups t0 + 256 m + 4 l + [0, 4),
// m = 0..3. A group's window starts at byte o + 256 m + 4 l of the row. Two dwords at
// the 4-byte-aligned address below it (one ds_read2_b32) hold all 4 bytes, for any
// phase r = o & 3. So the perm selector depends only on r, and there is no
// register selection: this path is branch-free. Consecutive lanes read consecutive
// dwords, so there are no bank conflicts.
__device__ __forceinline__ void window4x4(const uint8_t* lanep, int o, uint32_t (&p)[8]) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(lanep + (o & ~3));
    const uint32_t r = static_cast<uint32_t>(o & 3);
    const uint32_t sel0 = 0x0C010C00u + r * 0x00010001u;
    const uint32_t sel1 = sel0 + 0x00020002u;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t lo = w[64 * m], hi = w[64 * m + 1];
        p[2 * m] = __builtin_amdgcn_perm(hi, lo, sel0);
        p[2 * m + 1] = __builtin_amdgcn_perm(hi, lo, sel1);
    }
}

// Contiguous layout, two channels at once: the register offsets QA, QB of the two
// windows are template constants. So each case of the 16-way uniform switch below
// perms straight from the loaded dwords into the accumulators, with no register copies.
template <int QA, int QB>
__device__ __forceinline__ void acc_pair16(uint32_t (&acc)[8], const u32x4& a0, const u32x4& a1, const u32x4& b0,
                                           const u32x4& b1, uint32_t sa0, uint32_t sa1, uint32_t sb0,
                                           uint32_t sb1) {
    const uint32_t wa[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
    const uint32_t wb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int ia = QA + (j >> 1), ib = QB + (j >> 1);
        acc[j] = acc[j] + __builtin_amdgcn_perm(wa[ia + 1], wa[ia], (j & 1) ? sa1 : sa0) +
                 __builtin_amdgcn_perm(wb[ib + 1], wb[ib], (j & 1) ? sb1 : sb0);
    }
    // keep the adds inside this case: without the barrier the compiler sinks the common
    // adds below the switch and merges the perm results through register copies
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                 "+v"(acc[6]), "+v"(acc[7]));
}

#define AA_PAIR_CASE(QA, QB) \
    case QA * 4 + QB: acc_pair16<QA, QB>(acc, a0, a1, b0, b1, sa0, sa1, sb0, sb1); break;

__device__ __forceinline__ void acc_pair16_dispatch(uint32_t (&acc)[8], const u32x4& a0, const u32x4& a1,
                                                    const u32x4& b0, const u32x4& b1, int oa, int ob) {
    const uint32_t sa0 = 0x0C010C00u + static_cast<uint32_t>(oa & 3) * 0x00010001u, sa1 = sa0 + 0x00020002u;
    const uint32_t sb0 = 0x0C010C00u + static_cast<uint32_t>(ob & 3) * 0x00010001u, sb1 = sb0 + 0x00020002u;
    switch (((oa >> 2) & 3) * 4 + ((ob >> 2) & 3)) {
        AA_PAIR_CASE(0, 0) AA_PAIR_CASE(0, 1) AA_PAIR_CASE(0, 2) AA_PAIR_CASE(0, 3)
        AA_PAIR_CASE(1, 0) AA_PAIR_CASE(1, 1) AA_PAIR_CASE(1, 2) AA_PAIR_CASE(1, 3)
        AA_PAIR_CASE(2, 0) AA_PAIR_CASE(2, 1) AA_PAIR_CASE(2, 2) AA_PAIR_CASE(2, 3)
        AA_PAIR_CASE(3, 0) AA_PAIR_CASE(3, 1) AA_PAIR_CASE(3, 2) default: AA_PAIR_CASE(3, 3)
    }
}
#undef AA_PAIR_CASE

// One (DM block, time tile) of one beam. Used by the per-plan launch and by the
// batched persistent launch.
template <int DPW, int W, int LAYOUT>
__device__ __forceinline__ void dedisp_tile(const DedispArgs& A, int blk, int64_t t0) {
    constexpr int BD = DPW * W;
    constexpr int CP = kChanPerPass;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const uint8_t* __restrict__ in = A.in;
    const int64_t in_pitch = A.in_pitch, n_in16 = A.n_in16, out_pitch = A.out_pitch, n_out = A.n_out;
    const int32_t* __restrict__ base = A.base;
    const int32_t* __restrict__ offs = A.offs;
    const int nchan = A.nchan, nchan_pad = A.nchan_pad, row = A.row;
    int32_t* __restrict__ out = A.out;
    const DmBlock b = load_block(A.blocks, blk);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t* bbase = base + static_cast<int64_t>(blk) * nchan_pad;
    const int32_t* woffs = offs + static_cast<int64_t>(blk) * nchan_pad * BD + wave * DPW;
    const int nvec = row >> 4;

    // Stage channel rows c0 .. c0+CP-1 into buffer `buf`. Wave w loads rows w, w+W, ...
    auto stage = [&](int c0, int buf) {
        uint8_t* dst = lds + buf * CP * row;
        for (int cr = wave; cr < CP; cr += W) {
            const int c = c0 + cr;
            uint8_t* drow = dst + cr * row;
            if (c < nchan) {
                const int64_t rs = t0 + bbase[c];               // first staged sample, 16-aligned
                const uint8_t* g = in + static_cast<int64_t>(c) * in_pitch + rs;
                for (int v0 = 0; v0 < nvec; v0 += 64) {
                    const int v = v0 + lane;
                    if (v < nvec && rs + 16 * (v + 1) <= n_in16)
                        __builtin_amdgcn_global_load_lds(g + 16 * v, (lds_void*)(drow + 16 * v0),
                                                         16, 0, 0);
                }
            } else {
                for (int v = lane; v < nvec; v += 64) *reinterpret_cast<u32x4*>(drow + 16 * v) = u32x4{0u, 0u, 0u, 0u};
            }
        }
    };

    uint32_t a16[DPW][8];
    uint32_t a32[DPW][16];
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a16[i][j] = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) a32[i][k] = 0;
    }

    const int npass = nchan_pad / CP;
    stage(0, 0);
    int since_flush = 0;
    for (int p = 0; p < npass; ++p) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (p + 1 < npass) stage((p + 1) * CP, (p + 1) & 1);
        if (since_flush + CP > 256) {
#pragma unroll
            for (int i = 0; i < DPW; ++i) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    a32[i][2 * j] += a16[i][j] & 0xFFFFu;
                    a32[i][2 * j + 1] += a16[i][j] >> 16;
                    a16[i][j] = 0;
                }
            }
            since_flush = 0;
        }
        since_flush += CP;
        const uint8_t* bufp = lds + (p & 1) * CP * row + ((LAYOUT == 0 || LAYOUT == 3) ? 16 : 4) * lane;
        const int32_t* po = woffs + static_cast<int64_t>(p) * CP * BD;
        // offsets of the first channel pair; the next pair's are fetched one step ahead
        int oa[DPW], ob[DPW];
#pragma unroll
        for (int i = 0; i < DPW; ++i) {
            oa[i] = po[i];
            ob[i] = po[BD + i];
        }
#pragma unroll 1
        for (int cr = 0; cr < CP; cr += 2) {
            const uint8_t* ra = bufp + cr * row;
            const uint8_t* rb = ra + row;
            int na[DPW], nb[DPW];
            const int cn = cr + 2 < CP ? cr + 2 : cr;
            if constexpr (LAYOUT == 0) {
                u32x4 xa[DPW][2], xb[DPW][2];
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    const u32x4* va = reinterpret_cast<const u32x4*>(ra + (oa[i] & ~15));
                    const u32x4* vb = reinterpret_cast<const u32x4*>(rb + (ob[i] & ~15));
                    xa[i][0] = va[0];
                    xa[i][1] = va[1];
                    xb[i][0] = vb[0];
                    xb[i][1] = vb[1];
                }
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    na[i] = po[cn * BD + i];
                    nb[i] = po[(cn + 1) * BD + i];
                }
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    uint32_t pa[8], pb[8];
                    window16(xa[i][0], xa[i][1], oa[i], pa);
                    window16(xb[i][0], xb[i][1], ob[i], pb);
#pragma unroll
                    for (int j = 0; j < 8; ++j) a16[i][j] = a16[i][j] + pa[j] + pb[j];
                }
            } else if constexpr (LAYOUT == 3) {
                u32x4 xa[DPW][2], xb[DPW][2];
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    const u32x4* va = reinterpret_cast<const u32x4*>(ra + (oa[i] & ~15));
                    const u32x4* vb = reinterpret_cast<const u32x4*>(rb + (ob[i] & ~15));
                    xa[i][0] = va[0];
                    xa[i][1] = va[1];
                    xb[i][0] = vb[0];
                    xb[i][1] = vb[1];
                }
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    na[i] = po[cn * BD + i];
                    nb[i] = po[(cn + 1) * BD + i];
                }
#pragma unroll
                for (int i = 0; i < DPW; ++i)
                    acc_pair16_dispatch(a16[i], xa[i][0], xa[i][1], xb[i][0], xb[i][1], oa[i], ob[i]);
            } else if constexpr (LAYOUT == 2) {
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    na[i] = po[cn * BD + i];
                    nb[i] = po[(cn + 1) * BD + i];
                }
                // a trial whose window offset equals the previous trial's reuses its pairs
                uint32_t pa[8], pb[8];
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    if (i == 0 || oa[i] != oa[i - 1]) window4x4(ra, oa[i], pa);
                    if (i == 0 || ob[i] != ob[i - 1]) window4x4(rb, ob[i], pb);
#pragma unroll
                    for (int j = 0; j < 8; ++j) a16[i][j] = a16[i][j] + pa[j] + pb[j];
                }
            } else {
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    na[i] = po[cn * BD + i];
                    nb[i] = po[(cn + 1) * BD + i];
                }
#pragma unroll
                for (int i = 0; i < DPW; ++i) {
                    uint32_t pa[8], pb[8];
                    window4x4(ra, oa[i], pa);
                    window4x4(rb, ob[i], pb);
#pragma unroll
                    for (int j = 0; j < 8; ++j) a16[i][j] = a16[i][j] + pa[j] + pb[j];
                }
            }
#pragma unroll
            for (int i = 0; i < DPW; ++i) {
                oa[i] = na[i];
                ob[i] = nb[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < DPW; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a32[i][2 * j] += a16[i][j] & 0xFFFFu;
            a32[i][2 * j + 1] += a16[i][j] >> 16;
        }
    }

#pragma unroll
    for (int i = 0; i < DPW; ++i) {
        if (wave * DPW + i >= b.count) continue;
        int32_t* orow = out + static_cast<int64_t>(b.first + wave * DPW + i) * out_pitch;
        // a32[i][k] holds sample t0 + 16 lane + k (contiguous layout) or
        // t0 + 256 (k >> 2) + 4 lane + (k & 3) (interleaved layout)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int64_t t = (LAYOUT == 0 || LAYOUT == 3) ? t0 + 16 * lane + 4 * g : t0 + 256 * g + 4 * lane;
            if (t + 4 <= n_out) {
                const u32x4 v = {a32[i][4 * g], a32[i][4 * g + 1], a32[i][4 * g + 2], a32[i][4 * g + 3]};
                *reinterpret_cast<u32x4*>(orow + t) = v;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (t + k < n_out) orow[t + k] = static_cast<int32_t>(a32[i][4 * g + k]);
            }
        }
    }
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

// s_waitcnt vmcnt(n) for a wave-uniform n in [0, 24].
template <int N>
__device__ __forceinline__ void vmcnt_le() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void wait_vmcnt(int n) {
    switch (n) {
#define AA_VM(N) \
    case N: vmcnt_le<N>(); break;
        AA_VM(0) AA_VM(1) AA_VM(2) AA_VM(3) AA_VM(4) AA_VM(5) AA_VM(6) AA_VM(7) AA_VM(8) AA_VM(9) AA_VM(10) AA_VM(11)
        AA_VM(12) AA_VM(13) AA_VM(14) AA_VM(15) AA_VM(16) AA_VM(17) AA_VM(18) AA_VM(19) AA_VM(20) AA_VM(21) AA_VM(22)
        AA_VM(23)
#undef AA_VM
        default: vmcnt_le<24>(); break;
    }
}

// Matrix-core dedispersion of one (DM block, time tile), layouts 4-6. The shift
// of a trial d of the block at channel c is s = base[c] + E[d] + r[d][c], with
// 0 <= r < R inside a channel block (the tables are built on the host, tiling.cpp). So
//   D[d][t] = sum over channel blocks of P[t + e[d]][d],
//   P[t'][d] = sum_{c in block} X[c][t' + base[c] + min E + r[d][c]],
// where t' runs over a shifted time axis and e[d] = E[d] - min E. P is a product of
// the data matrix A[t'][(c, r)] (a sliding R-byte window per channel) and the one-hot
// matrix B[(c, r)][d], computed exactly by v_mfma_i32_32x32x32_i8: rows are 32 values
// of t', columns the 32 trials, and one step contracts CPS channels x R residuals,
// CPS x R = 32 (4 x 8 for layout 4, 8 x 4 for layout 5, the block's own shape for 6).
// Input bytes enter as x - 128 (signed 8-bit), and 128 * nchan is added back at the end.
//  * W = 8 or 16 waves. Wave w owns the tiles w + W j of 32 rows of t' (a channel block
//    needs TILE / 32 to MAXT tiles, MAXT = 63 or 31, so a wave owns NT = TILE / (32 W)
//    .. ceil(MAXT / W) of them) and holds their 32 x 32 int32 accumulators in
//    registers. Each channel block runs a loop specialised for the wave's NT, so the hot
//    loop has no per-tile branches.
//  * At the end of a channel block, each accumulator row t' of trial d is added into
//    the work-group's [TILE][32] int32 tile in LDS at t = t' - e[d] (ds_add_u32). Lanes
//    hold 32 distinct trials of one row, so these adds are conflict-free.
//  * Input rows are staged CPS channels per step, up to ROW = 2048 (MAXT 63) or 1024
//    (MAXT 31) bytes each, by direct global->LDS loads into a ring of DEPTH buffers,
//    issued DEPTH - 1 steps ahead. Each staging wave loads 1024 bytes of one row.
//    Each step's table record (residuals, e, phases, tile and step counts, and the row
//    starts and lengths of the step DEPTH - 1 ahead) rides along in the same ring.
//    Every staging wave issues exactly one data load per step, and wave 0 also the
//    record, so waiting until only the newer steps' loads are in flight makes a step's
//    data complete. Lanes past a row's needed length load a duplicate of its first chunk.
//  * A lane (row m, half h) holds channels CPS/2 h .. CPS/2 h + CPS/2 - 1 of the step.
//    It reads each channel's R-byte window as aligned dwords (3 for R = 8, 2 for R = 4)
//    and aligns them with v_alignbyte_b32. Every staged chunk that a needed byte lives
//    in is in range; chunks wholly outside [0, n_in16) are clamped to a valid address,
//    and their bytes only reach rows that are never written out.
struct MfmaCtx {
    const DedispArgs* A;
    const uint8_t* recg;   // this DM block's records
    int64_t t0, last16;
    int K, wave, lane, m, h, row, part0, ps;
    bool interior;         // every staged row of the tile lies inside [0, n_in16)
};

template <int TILE, int DEPTH, int MAXT, int CPS>
struct MfmaLayout {
    static constexpr int ROW = mfma_row_bytes(MAXT);  // staged bytes per channel row
    static constexpr int PARTS = ROW / 1024;          // 1024-byte loads per staged row
    // staging waves per row: two for 4-channel steps with 2048-byte rows (waves 0-7, one
    // load each), else one (waves 0-7 stage the 8-channel steps' rows, two loads each)
    static constexpr int SPLIT = (CPS == 4 && PARTS == 2) ? 2 : 1;
    static constexpr int LPW = PARTS / SPLIT;                        // loads per staging wave
    static constexpr int SW = CPS * SPLIT;            // staging waves
    static constexpr int STAGE = CPS * ROW;
    static constexpr MfmaRec RL = mfma_rec(CPS);      // record layout
    static constexpr int ACC = (TILE + 2) * 32 * 4;   // accumulator rows -1 .. TILE
    static constexpr int ACC0 = 32 * 4;               // byte offset of row 0
    static constexpr int RING = ACC;                  // byte offsets into LDS
    static constexpr int RECS = ACC + DEPTH * STAGE;
};

// Where the next step's loads go: `c` is the wave's channel, `rowp` its input row
// at the time tile (A.in + c * in_pitch + t0) and `recp` the step's record.
template <int CPS>
struct MfmaNext {
    int c;
    const uint8_t* rowp;
    const uint8_t* recp;
    __device__ __forceinline__ void advance(int64_t step_bytes) {
        c += CPS;
        rowp += step_bytes;
        recp += mfma_rec(CPS).size;
    }
};

// Loads of step k into ring slot `slot`: the staging waves (L::SW of them, L::SPLIT per
// row) each load L::LPW 1024-byte parts of their row (16 bytes per lane, `need` chunks of
// the row), then wave 0 the step's record. The staging waves are the oldest of the
// work-group (waves w, w + 4, w + 8, w + 12 share a SIMD, and older waves win issue),
// which wait longest at the step's barrier; the youngest waves, whose chain sets the
// step's length, issue no loads and do not queue behind the work-group's loads in the
// address unit.
template <int TILE, int DEPTH, int MAXT, int CPS>
__device__ __forceinline__ void mfma_issue(const MfmaCtx& cx, uint8_t* lds, const MfmaNext<CPS>& nx, int slot, int rs,
                                           int need) {
    using L = MfmaLayout<TILE, DEPTH, MAXT, CPS>;
    const DedispArgs& A = *cx.A;
    if (cx.wave >= L::SW) return;                      // waves 0 .. SW - 1 stage the rows
    // plain pointer types keep the load builtins' arguments out of template dependence
    const uint8_t* rowp = nx.rowp;
    const uint8_t* recp = nx.recp;
#pragma unroll
    for (int pi = 0; pi < L::LPW; ++pi) {
        const int part = cx.part0 + pi;
        const int vlane = 64 * part + cx.lane;
        const int v = vlane < need ? vlane : 0;
        uint8_t* dst = lds + L::RING + slot * L::STAGE + cx.row * L::ROW + part * 1024;
        if (nx.c < A.nchan) {
            if (cx.interior) {
                __builtin_amdgcn_global_load_lds(rowp + rs + 16 * v, (lds_void*)dst, 16, 0, 0);
            } else {
                const int64_t first = cx.t0 + rs;           // wave-uniform
                const int top = need < 64 * part + 64 ? need : 64 * part + 64;
                const uint8_t* row0 = rowp - cx.t0;         // the row at sample 0
                if (first >= 0 && first + 16 * top <= A.n_in16) {
                    __builtin_amdgcn_global_load_lds(row0 + first + 16 * v, (lds_void*)dst, 16, 0, 0);
                } else {
                    int64_t pos = first + 16 * v;
                    pos = pos < 0 ? 0 : (pos > cx.last16 ? cx.last16 : pos);
                    __builtin_amdgcn_global_load_lds(row0 + pos, (lds_void*)dst, 16, 0, 0);
                }
            }
        } else {
            __builtin_amdgcn_global_load_lds(A.pad + 16 * v, (lds_void*)dst, 16, 0, 0);
        }
    }
    if (cx.wave == 0) {
        uint8_t* rdst = lds + L::RECS + slot * L::RL.size;
        if constexpr (L::RL.size == 256) {
            __builtin_amdgcn_global_load_lds(recp + 4 * cx.lane, (lds_void*)rdst, 4, 0, 0);
        } else {
            static_assert(L::RL.size == 512, "record size");
            if (cx.lane < 32) __builtin_amdgcn_global_load_lds(recp + 16 * cx.lane, (lds_void*)rdst, 16, 0, 0);
        }
    }
}

// Wait until step k's loads are complete: the steps k + 1 .. k + DEPTH - 2 may still
// be in flight (constant count in the steady state), then barrier.
template <int DEPTH>
__device__ __forceinline__ void mfma_wait(const MfmaCtx& cx, int k) {
    if (k + DEPTH - 2 < cx.K) {
        if (cx.ps == 3)
            vmcnt_le<3 * (DEPTH - 2)>();
        else if (cx.ps == 2)
            vmcnt_le<2 * (DEPTH - 2)>();
        else if (cx.ps == 1)
            vmcnt_le<DEPTH - 2>();
    } else {
        wait_vmcnt((cx.K - 1 - k) * cx.ps);
    }
    __builtin_amdgcn_s_barrier();
}

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

// The steps [k0, k1) of one channel block, with NT tiles for this wave (tiles
// wave + W j). `slot` is the ring slot of step k0 on entry and of step k1 on exit.
template <int NT, int W, int TILE, int DEPTH, int MAXT, int CPS>
__device__ __forceinline__ void mfma_block(const MfmaCtx& cx, uint8_t* lds, int k0, int k1, int& slot,
                                           MfmaNext<CPS>& nx, int64_t step_bytes, uint32_t acc_base, int e,
                                           int emax) {
    using L = MfmaLayout<TILE, DEPTH, MAXT, CPS>;
    i32x16 acc[NT];
    constexpr int HC = CPS / 2;                        // channels per lane
    const int lane_base = L::RING + HC * cx.h * L::ROW + 32 * cx.wave + cx.m;
    // one step; the first step of a channel block starts its accumulators from zero
    // (the matrix op's zero operand), so a flush needs no register clears
    auto step = [&](int k, auto first) {
        constexpr bool FIRST = decltype(first)::value;
        const int rec = L::RECS + slot * L::RL.size;
        // every wave is done with the buffer of step k - 1: refill it with step k + DEPTH - 1
        // (the staging waves only: the others skip the refill's record reads as well)
        if (k + DEPTH - 1 < cx.K && cx.wave < L::SW) {
            const int need = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int32_t*>(lds + rec + L::RL.next_need));
            const int rs = __builtin_amdgcn_readfirstlane(
                *reinterpret_cast<const int32_t*>(lds + rec + L::RL.next_rs + 4 * cx.row));
            mfma_issue<TILE, DEPTH, MAXT, CPS>(cx, lds, nx, slot == 0 ? DEPTH - 1 : slot - 1, rs, need);
            nx.advance(step_bytes);
        }
        const int base = lane_base + slot * L::STAGE;
        if constexpr (CPS == 4) {
            // one-hot B: lane (trial m, half h) holds channels 2h, 2h+1 of the step
            const uint32_t r32 = *reinterpret_cast<const uint32_t*>(lds + rec + 4 * cx.m);
            const uint32_t ph = *reinterpret_cast<const uint16_t*>(lds + rec + L::RL.phase + 2 * cx.h);
            const uint32_t sh0 = (r32 >> (16 * cx.h)) & 0xFFu, sh1 = (r32 >> (16 * cx.h + 8)) & 0xFFu;
            const uint64_t o0 = 1ull << sh0, o1 = 1ull << sh1;
            const i32x4 B = {static_cast<int32_t>(o0), static_cast<int32_t>(o0 >> 32), static_cast<int32_t>(o1),
                             static_cast<int32_t>(o1 >> 32)};
            // data A: lane (row m, half h) reads 8-byte windows of channels 2h, 2h+1
            const int a0 = base + static_cast<int>(ph & 0xFFu), a1 = base + L::ROW + static_cast<int>(ph >> 8);
            const int w0 = a0 & ~3, w1 = a1 & ~3;
            const uint32_t u0 = static_cast<uint32_t>(a0 & 3), u1 = static_cast<uint32_t>(a1 & 3);
            uint32_t x[NT][3], y[NT][3];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const uint32_t* p0 = reinterpret_cast<const uint32_t*>(lds + w0 + 32 * W * j);
                const uint32_t* p1 = reinterpret_cast<const uint32_t*>(lds + w1 + 32 * W * j);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    x[j][i] = p0[i];
                    y[j][i] = p1[i];
                }
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const i32x4 Av = {static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][1], x[j][0], u0) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][2], x[j][1], u0) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(y[j][1], y[j][0], u1) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(y[j][2], y[j][1], u1) ^ 0x80808080u)};
                acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Av, B, FIRST ? i32x16{} : acc[j], 0, 0, 0);
            }
        } else {
            // one-hot B: lane (trial m, half h) holds channels 4h .. 4h+3 of the step, a
            // byte 8 r per channel; the dword of channel i is 1 << 8 r
            const uint32_t r32 = *reinterpret_cast<const uint32_t*>(lds + rec + 8 * cx.m + 4 * cx.h);
            const uint32_t ph = *reinterpret_cast<const uint32_t*>(lds + rec + L::RL.phase + 4 * cx.h);
            const i32x4 B = {static_cast<int32_t>(1u << (r32 & 31u)), static_cast<int32_t>(1u << ((r32 >> 8) & 31u)),
                             static_cast<int32_t>(1u << ((r32 >> 16) & 31u)), static_cast<int32_t>(1u << ((r32 >> 24) & 31u))};
            // data A: lane (row m, half h) reads 4-byte windows of channels 4h .. 4h+3
            int w[4];
            uint32_t u[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ai = base + i * L::ROW + static_cast<int>((ph >> (8 * i)) & 0xFFu);
                w[i] = ai & ~3;
                u[i] = static_cast<uint32_t>(ai & 3);
            }
            uint32_t x[NT][4][2];
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t* pi = reinterpret_cast<const uint32_t*>(lds + w[i] + 32 * W * j);
                    x[j][i][0] = pi[0];
                    x[j][i][1] = pi[1];
                }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const i32x4 Av = {static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][0][1], x[j][0][0], u[0]) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][1][1], x[j][1][0], u[1]) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][2][1], x[j][2][0], u[2]) ^ 0x80808080u),
                                  static_cast<int32_t>(__builtin_amdgcn_alignbyte(x[j][3][1], x[j][3][0], u[3]) ^ 0x80808080u)};
                acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Av, B, FIRST ? i32x16{} : acc[j], 0, 0, 0);
            }
        }
        slot = slot + 1 == DEPTH ? 0 : slot + 1;
    };
    step(k0, BoolTag<true>{});
#pragma unroll 1
    for (int k = k0 + 1; k < k1; ++k) {
        mfma_wait<DEPTH>(cx, k);
        step(k, BoolTag<false>{});
    }
    // flush: accumulator register i of lane (m, h) holds row 8 (i / 4) + 4 h + i % 4
    // of the tile and trial m, which goes to t = row - e[m]. The adds are issued as
    // inline ds_add_u32 so that the compiler does not wait for the staging loads in
    // flight (they write other LDS bytes); the barrier after the tile's last block
    // orders them before the final read. A tile whose rows land in [0, TILE) for every
    // e in [0, max e] adds with immediate offsets and no checks. (e[m] and max e are the
    // same in every record of the block; the caller reads them from its first step.)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int q = cx.wave + W * j;
        if (32 * q >= emax && 32 * q + 32 <= TILE) {
            const uint32_t tb = acc_base + 4u * static_cast<uint32_t>(cx.m + 32 * (32 * q + 4 * cx.h - e));
#define AA_FLUSH(I) \
    asm volatile("ds_add_u32 %0, %1 offset:%2" ::"v"(tb), "v"(acc[j][I]), "n"(128 * (8 * ((I) >> 2) + ((I) & 3))) : "memory");
            AA_FLUSH(0) AA_FLUSH(1) AA_FLUSH(2) AA_FLUSH(3) AA_FLUSH(4) AA_FLUSH(5) AA_FLUSH(6) AA_FLUSH(7)
            AA_FLUSH(8) AA_FLUSH(9) AA_FLUSH(10) AA_FLUSH(11) AA_FLUSH(12) AA_FLUSH(13) AA_FLUSH(14) AA_FLUSH(15)
#undef AA_FLUSH
        } else {
            // rows outside [0, TILE) are clamped to the discarded rows -1 and TILE
            const int tq = 32 * q + 4 * cx.h - e;
            const uint32_t mb = acc_base + 4u * static_cast<uint32_t>(cx.m);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int t = min(max(tq + 8 * (i >> 2) + (i & 3), -1), TILE);
                const uint32_t addr = mb + (static_cast<uint32_t>(t) << 7);   // 32 x 4 bytes per row
                asm volatile("ds_add_u32 %0, %1" ::"v"(addr), "v"(acc[j][i]) : "memory");
            }
        }
    }
}

// Channel-block loop of a wave that owns N tiles (N in [U, TPW]): the hot loop is
// specialised for N. Other values of n cannot occur; their cases are empty.
template <int N, int U, int TPW>
constexpr int clamp_nt() { return N < U ? U : (N > TPW ? TPW : N); }

template <int W, int TILE, int DEPTH, int MAXT, int CPS>
__device__ __forceinline__ void dedisp_mfma_tile(const DedispArgs& A, int blk, int64_t t0) {
    // wave w owns the tiles w + W j (j < TPW); a channel block has at least TILE / 32
    // tiles, so each wave owns at least U of them
    constexpr int TPW = (MAXT + W - 1) / W, U = TILE / (32 * W);
    using L = MfmaLayout<TILE, DEPTH, MAXT, CPS>;
    static_assert((W == 8 || W == 16) && TILE % 32 == 0 && U >= 1 && U <= TPW && TPW <= 8 && DEPTH >= 3 &&
                  DEPTH <= 13 && (MAXT == 31 || MAXT == 63) && 32 * MAXT >= TILE && (CPS == 4 || CPS == 8) &&
                  L::SW <= W, "waves / tile / depth / span / channels per step");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    int32_t* acc_lds = reinterpret_cast<int32_t*>(lds + L::ACC0);   // row 0 of the accumulator tile
    MfmaCtx cx;
    cx.A = &A;
    cx.t0 = t0;
    cx.last16 = A.n_in16 - 16;
    cx.K = A.nchan_pad / CPS;
    cx.recg = reinterpret_cast<const uint8_t*>(A.offs) + static_cast<int64_t>(load_block(A.blocks, blk).rec256) * 256;
    const int tid = threadIdx.x;
    cx.wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    cx.lane = tid & 63;
    cx.m = cx.lane & 31;
    cx.h = cx.lane >> 5;
    // staging waves: their row; the others read row 0's entries
    cx.row = cx.wave < L::SW ? cx.wave / L::SPLIT : 0;
    cx.part0 = cx.wave < L::SW ? (cx.wave % L::SPLIT) * L::LPW : 0;
    // loads this wave issues per step: its row's parts, and wave 0 the record
    cx.ps = (cx.wave < L::SW ? L::LPW : 0) + (cx.wave == 0 ? 1 : 0);
    const int32_t* rsv = A.base + static_cast<int64_t>(blk) * A.nchan_pad;
    {
        const DmBlock bk = load_block(A.blocks, blk);
        cx.interior = t0 + bk.rs_lo >= 0 && t0 + bk.rs_hi + L::ROW <= A.n_in16;
    }
    const int64_t step_bytes = CPS * A.in_pitch;
    MfmaNext<CPS> nx{cx.row, A.in + static_cast<int64_t>(cx.row) * A.in_pitch + t0, cx.recg};

    for (int i = tid; i < L::ACC / 16; i += 64 * W) reinterpret_cast<u32x4*>(lds)[i] = u32x4{0u, 0u, 0u, 0u};
    int rs_pro[DEPTH - 1];
#pragma unroll
    for (int j = 0; j < DEPTH - 1; ++j)
        rs_pro[j] = j < cx.K ? __builtin_amdgcn_readfirstlane(rsv[CPS * j + cx.row]) : 0;
#pragma unroll
    for (int j = 0; j < DEPTH - 1; ++j) {
        if (j < cx.K) mfma_issue<TILE, DEPTH, MAXT, CPS>(cx, lds, nx, j, rs_pro[j], L::ROW / 16);
        nx.advance(step_bytes);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");

    const uint32_t acc_base =
        static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) int32_t*)acc_lds));
    int slot = 0;
    for (int k0 = 0; k0 < cx.K;) {
        mfma_wait<DEPTH>(cx, k0);
        const int rec0 = L::RECS + slot * L::RL.size;
        const int nr = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int32_t*>(lds + rec0 + L::RL.tiles));
        const int k1 = k0 + __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int32_t*>(lds + rec0 + L::RL.left));
        const int e = *reinterpret_cast<const int16_t*>(lds + rec0 + L::RL.e + 2 * cx.m);
        const int emax = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const int32_t*>(lds + rec0 + L::RL.max_e));
        const int nt = (nr - cx.wave + W - 1) / W;      // tiles of this wave, U .. TPW
        // one inlined loop per value in [U, TPW] (nt = 1 only reaches the default case)
        switch (nt) {
#define AA_NT(N)                                                                                           \
    case N:                                                                                                \
        if constexpr (N >= U && N <= TPW)                                                                  \
            mfma_block<clamp_nt<N, U, TPW>(), W, TILE, DEPTH, MAXT, CPS>(cx, lds, k0, k1, slot, nx, step_bytes, \
                                                                         acc_base, e, emax);                \
        break;
            AA_NT(8) AA_NT(7) AA_NT(6) AA_NT(5) AA_NT(4) AA_NT(3) AA_NT(2)
#undef AA_NT
            default:
                if constexpr (U == 1)
                    mfma_block<1, W, TILE, DEPTH, MAXT, CPS>(cx, lds, k0, k1, slot, nx, step_bytes, acc_base, e,
                                                             emax);
                break;
        }
        k0 = k1;
    }
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();

    const DmBlock b = load_block(A.blocks, blk);
    const int32_t corr = 128 * A.nchan;
#pragma unroll 1
    for (int idx = tid; idx < TILE * 8; idx += 64 * W) {   // 4 samples x 1 trial per item
        const int d = idx & 31, tq = idx >> 5;
        int32_t v[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) v[jj] = acc_lds[(4 * tq + jj) * 32 + d] + corr;
        if (d < b.count) {
            int32_t* orow = A.out + static_cast<int64_t>(b.first + d) * A.out_pitch;
            const int64_t t = t0 + 4 * tq;
            if (t + 4 <= A.n_out) {
                *reinterpret_cast<u32x4*>(orow + t) = u32x4{static_cast<uint32_t>(v[0]), static_cast<uint32_t>(v[1]),
                                                           static_cast<uint32_t>(v[2]), static_cast<uint32_t>(v[3])};
            } else {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    if (t + jj < A.n_out) orow[t + jj] = v[jj];
            }
        }
    }
}

// Layout 7: shift-and-add on the vector ALUs with one v_sad_u8 per 4 byte-adds (step
// records in aa_internal.h). Thread i owns output samples t0 + i + 64 W j, j < J, of
// all 32 trials of the block. Per step (a quad of channels):
//  * the chunks of the next step are loaded from the input rows into registers (two
//    aligned dwords per channel and unit, raw buffer loads), then the current step is
//    summed, then the loaded rows are aligned (v_alignbyte_b32), transposed 4x4 bytes
//    (8 v_perm_b32) into four sample dwords and written to the other LDS buffer;
//  * summing one trial: J dwords one 64 W stride apart (ds_read2st64_b32) at the
//    trial's recorded offset go through v_sad_u8 into 32-bit accumulators. Consecutive
//    lanes read consecutive dwords: no bank conflicts.
// Records are read with scalar loads; each chunk's four row offsets come precomputed,
// so staging a chunk costs four scalar ops. Each channel row has its own buffer
// resource spanning [0, n_in16) (empty for channels past nchan): the range check of raw
// buffer loads returns zero for the dwords outside it.
// Sums of eight trials, one dword each (one sample per lane): the eight window addresses
// (lane dword plus the u16 halves of four record pairs), the eight LDS reads in flight
// together, then the v_sad_u8 adds as the reads land. The block waits for its own reads
// before it ends; the reads are the youngest LDS/scalar-memory operations in flight, so
// the partial waits are exact or conservative.
__device__ __forceinline__ void sad_group8(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t& c4,
                                           uint32_t& c5, uint32_t& c6, uint32_t& c7, uint32_t base, uint32_t p0,
                                           uint32_t p1, uint32_t p2, uint32_t p3) {
    uint32_t a0, a1, a2, a3, a4, a5, a6, a7;
    asm volatile(
        "v_mad_u32_u16 %[a0], %[p0], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a1], %[p0], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a2], %[p1], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a3], %[p1], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a4], %[p2], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a5], %[p2], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a6], %[p3], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a7], %[p3], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "ds_read_b32 %[a0], %[a0]\n\t"
        "ds_read_b32 %[a1], %[a1]\n\t"
        "ds_read_b32 %[a2], %[a2]\n\t"
        "ds_read_b32 %[a3], %[a3]\n\t"
        "ds_read_b32 %[a4], %[a4]\n\t"
        "ds_read_b32 %[a5], %[a5]\n\t"
        "ds_read_b32 %[a6], %[a6]\n\t"
        "ds_read_b32 %[a7], %[a7]\n\t"
        "s_waitcnt lgkmcnt(7)\n\t"
        "v_sad_u8 %[c0], %[a0], 0, %[c0]\n\t"
        "s_waitcnt lgkmcnt(6)\n\t"
        "v_sad_u8 %[c1], %[a1], 0, %[c1]\n\t"
        "s_waitcnt lgkmcnt(5)\n\t"
        "v_sad_u8 %[c2], %[a2], 0, %[c2]\n\t"
        "s_waitcnt lgkmcnt(4)\n\t"
        "v_sad_u8 %[c3], %[a3], 0, %[c3]\n\t"
        "s_waitcnt lgkmcnt(3)\n\t"
        "v_sad_u8 %[c4], %[a4], 0, %[c4]\n\t"
        "s_waitcnt lgkmcnt(2)\n\t"
        "v_sad_u8 %[c5], %[a5], 0, %[c5]\n\t"
        "s_waitcnt lgkmcnt(1)\n\t"
        "v_sad_u8 %[c6], %[a6], 0, %[c6]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_sad_u8 %[c7], %[a7], 0, %[c7]"
        : [c0] "+v"(c0), [c1] "+v"(c1), [c2] "+v"(c2), [c3] "+v"(c3), [c4] "+v"(c4), [c5] "+v"(c5), [c6] "+v"(c6),
          [c7] "+v"(c7), [a0] "=&v"(a0), [a1] "=&v"(a1), [a2] "=&v"(a2), [a3] "=&v"(a3), [a4] "=&v"(a4),
          [a5] "=&v"(a5), [a6] "=&v"(a6), [a7] "=&v"(a7)
        : [b] "v"(base), [p0] "s"(p0), [p1] "s"(p1), [p2] "s"(p2), [p3] "s"(p3));
}

// Reads of eight trials, two dwords each (two samples per lane, 64 W dwords apart, one
// ds_read2st64_b32): addresses as in sad_group8, the eight reads in flight together,
// and a wait for them before the block ends.
template <int W>
__device__ __forceinline__ void read_group8_st64(uint64_t (&r)[8], uint32_t base, uint32_t p0, uint32_t p1,
                                                 uint32_t p2, uint32_t p3) {
    uint32_t a0, a1, a2, a3, a4, a5, a6, a7;
    asm volatile(
        "v_mad_u32_u16 %[a0], %[p0], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a1], %[p0], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a2], %[p1], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a3], %[p1], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a4], %[p2], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a5], %[p2], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "v_mad_u32_u16 %[a6], %[p3], 1, %[b]\n\t"
        "v_mad_u32_u16 %[a7], %[p3], 1, %[b] op_sel:[1,0,0,0]\n\t"
        "ds_read2st64_b32 %[r0], %[a0] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r1], %[a1] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r2], %[a2] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r3], %[a3] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r4], %[a4] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r5], %[a5] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r6], %[a6] offset1:%[st]\n\t"
        "ds_read2st64_b32 %[r7], %[a7] offset1:%[st]\n\t"
        "s_waitcnt lgkmcnt(0)"
        : [r0] "=&v"(r[0]), [r1] "=&v"(r[1]), [r2] "=&v"(r[2]), [r3] "=&v"(r[3]), [r4] "=&v"(r[4]),
          [r5] "=&v"(r[5]), [r6] "=&v"(r[6]), [r7] "=&v"(r[7]), [a0] "=&v"(a0), [a1] "=&v"(a1), [a2] "=&v"(a2),
          [a3] "=&v"(a3), [a4] "=&v"(a4), [a5] "=&v"(a5), [a6] "=&v"(a6), [a7] "=&v"(a7)
        : [b] "v"(base), [p0] "s"(p0), [p1] "s"(p1), [p2] "s"(p2), [p3] "s"(p3), [st] "n"(W));
}

__device__ __forceinline__ void lds_step_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

constexpr int kRawBufferFlags = 0x00020000;   // word 3 of a gfx9 buffer resource: raw 32-bit data

template <int W, int J, int CPW>
__device__ __forceinline__ void dedisp_quad_tile(const DedispArgs& A, int blk, int64_t t0) {
    constexpr int NT = 64 * W, CH = W * CPW, BUFB = CH * 1024, RD = quad_rec_dwords(CH);
    constexpr int NTR = kQuadTrials;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const DmBlock b = load_block(A.blocks, blk);
    const int nq = A.nchan_pad >> 2, count = b.count;
    const int64_t pitch = A.in_pitch;
    const int32_t n_in16 = static_cast<int32_t>(A.n_in16);
    // records are read-only for the launch: the constant address space makes their
    // (uniform) reads scalar loads
    typedef const __attribute__((address_space(4))) int32_t* rec_ptr;
    const rec_ptr R = (rec_ptr)(A.offs) + static_cast<int64_t>(b.rec256) * 64;
    const uint32_t lane_t0 = 4u * static_cast<uint32_t>(lane) + static_cast<uint32_t>(t0);
    uint8_t* const wdst = lds + 16 * lane + 1024 * wave;   // this lane's unit in chunk `wave`

    uint32_t acc[NTR][J];
#pragma unroll
    for (int d = 0; d < NTR; ++d)
#pragma unroll
        for (int j = 0; j < J; ++j) acc[d][j] = 0;

    // staging registers of one step: per chunk slot, two aligned dwords per channel
    uint32_t sw[CPW][4][2];
    // the current record, in scalar registers: trial offsets of the step being summed,
    // and the chunk count and this wave's chunk row offsets of the step being staged.
    // The next record is read at the end of each step, so that the barrier's wait covers
    // its latency and no scalar load is in flight while the sums wait for LDS reads.
    uint32_t toff[NTR / 2];   // two u16 trial offsets per dword
    int32_t co[CPW][4];
    int nch = 0;
    auto load_rec = [&](rec_ptr E) {
#pragma unroll
        for (int d = 0; d < NTR / 2; ++d) toff[d] = static_cast<uint32_t>(E[d]);
        nch = E[32];
#pragma unroll
        for (int m = 0; m < CPW; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) co[m][i] = E[64 + 4 * (wave + W * m) + i];
    };

    // One buffer resource per quad, based at its first row; row i is reached through the
    // scalar offset i * pitch, which the range check counts. The range ends where the
    // quad's last existing row ends (n_in16 past its start): a row's loads past its own
    // n_in16 read the next row's bytes, which only reach samples at or past n_out (never
    // stored), and nothing past the last row is read. Rows past nchan carry the row
    // offset kQuadNoRow, at or beyond every range (pitches are at most 2^28), and read zero.
    const uint32_t soff[4] = {0u, static_cast<uint32_t>(pitch), static_cast<uint32_t>(2 * pitch),
                              static_cast<uint32_t>(3 * pitch)};
    const int full_quads = A.nchan >> 2;
    const int32_t range_full = static_cast<int32_t>(3 * pitch) + n_in16;
    const int32_t range_last = static_cast<int32_t>((A.nchan - 1 - 4 * full_quads) * pitch) + n_in16;
    const uint8_t* quad_row = A.in;
    int next_q = 0;
    auto issue = [&]() {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t*>(quad_row), 0, next_q < full_quads ? range_full : range_last, kRawBufferFlags);
#pragma unroll
        for (int m = 0; m < CPW; ++m) {
            if (wave + W * m < nch) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // the lane's part in the vector offset, the row's in the scalar one
                    const uint32_t so = soff[i] + static_cast<uint32_t>(co[m][i] & ~3);
                    const auto w2 = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_t0, so, 0);
                    sw[m][i][0] = w2[0];
                    sw[m][i][1] = w2[1];
                }
            }
        }
        quad_row += 4 * pitch;
        ++next_q;
    };

    auto write = [&](int buf) {
#pragma unroll
        for (int m = 0; m < CPW; ++m) {
            if (wave + W * m < nch) {
                uint32_t v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    v[i] = __builtin_amdgcn_alignbyte(sw[m][i][1], sw[m][i][0], static_cast<uint32_t>(co[m][i]));
                // 4x4 byte transpose: o[k] = (v0.byte k, v1.byte k, v2.byte k, v3.byte k)
                const uint32_t t0l = __builtin_amdgcn_perm(v[1], v[0], 0x05010400u);
                const uint32_t t0h = __builtin_amdgcn_perm(v[1], v[0], 0x07030602u);
                const uint32_t t1l = __builtin_amdgcn_perm(v[3], v[2], 0x05010400u);
                const uint32_t t1h = __builtin_amdgcn_perm(v[3], v[2], 0x07030602u);
                const u32x4 o = {__builtin_amdgcn_perm(t1l, t0l, 0x05040100u), __builtin_amdgcn_perm(t1l, t0l, 0x07060302u),
                                 __builtin_amdgcn_perm(t1h, t0h, 0x05040100u), __builtin_amdgcn_perm(t1h, t0h, 0x07060302u)};
                *reinterpret_cast<u32x4*>(wdst + buf * BUFB + 1024 * W * m) = o;
            }
        }
    };

    typedef const __attribute__((address_space(3))) uint32_t* lds_u32;

    load_rec(R);
    issue();
    write(0);
    load_rec(R + RD);
    lds_step_barrier();
    for (int k = 0; k < nq; ++k) {
        const bool more = k + 1 < nq;
        if (more) issue();
        const uint32_t y = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_u32)(const void*)lds)) +
                           static_cast<uint32_t>((k & 1) * BUFB + 4 * tid);
        // trials in groups of 8; a block's absent trials (short blocks) are skipped per group
#pragma unroll
        for (int g = 0; g < NTR / 8; ++g) {
            if (8 * g < count) {
                if constexpr (J == 1) {
                    sad_group8(acc[8 * g][0], acc[8 * g + 1][0], acc[8 * g + 2][0], acc[8 * g + 3][0], acc[8 * g + 4][0],
                               acc[8 * g + 5][0], acc[8 * g + 6][0], acc[8 * g + 7][0], y, toff[4 * g], toff[4 * g + 1],
                               toff[4 * g + 2], toff[4 * g + 3]);
                } else {
                    static_assert(J == 2, "one or two dwords per lane");
                    uint64_t r[8];
                    read_group8_st64<W>(r, y, toff[4 * g], toff[4 * g + 1], toff[4 * g + 2], toff[4 * g + 3]);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        acc[8 * g + i][0] = __builtin_amdgcn_sad_u8(static_cast<uint32_t>(r[i]), 0u, acc[8 * g + i][0]);
                        acc[8 * g + i][1] = __builtin_amdgcn_sad_u8(static_cast<uint32_t>(r[i] >> 32), 0u, acc[8 * g + i][1]);
                    }
                }
            }
        }
        if (more) {
            write((k + 1) & 1);
            asm volatile("" ::: "memory");
            load_rec(R + static_cast<int64_t>(k + 2) * RD);   // offsets of step k + 1, chunks of step k + 2
        }
        lds_step_barrier();
    }

#pragma unroll
    for (int d = 0; d < NTR; ++d) {
        if (d < count) {
            int32_t* orow = A.out + static_cast<int64_t>(b.first + d) * A.out_pitch;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int64_t t = t0 + tid + NT * j;
                if (t < A.n_out) orow[t] = static_cast<int32_t>(acc[d][j]);
            }
        }
    }
}

// Layout 6: the DM block's own step shape (the whole work-group takes one branch).
template <int W, int TILE, int DEPTH, int MAXT>
__device__ __forceinline__ void dedisp_mfma_mixed(const DedispArgs& A, int blk, int64_t t0) {
    if (__builtin_amdgcn_readfirstlane(load_block(A.blocks, blk).cps) == 8)
        dedisp_mfma_tile<W, TILE, DEPTH, MAXT, 8>(A, blk, t0);
    else
        dedisp_mfma_tile<W, TILE, DEPTH, MAXT, 4>(A, blk, t0);
}

// WPE: waves per SIMD the register allocation must allow (2 work-groups per CU for the
// 80 KB matrix-core variants).
template <int DPW, int W, int LAYOUT, int TILE = kTimeTile, int DEPTH = 2, int MAXT = 63, int WPE = 1>
__global__ __launch_bounds__(64 * W, WPE) void dedisp_kernel(DedispArgs a) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    if constexpr (LAYOUT == 7)
        dedisp_quad_tile<W, DPW, DEPTH>(a, bid % a.nblk, static_cast<int64_t>(bid / a.nblk) * TILE);
    else if constexpr (LAYOUT == 6)
        dedisp_mfma_mixed<W, TILE, DEPTH, MAXT>(a, bid % a.nblk, static_cast<int64_t>(bid / a.nblk) * TILE);
    else if constexpr (LAYOUT == 4 || LAYOUT == 5)
        dedisp_mfma_tile<W, TILE, DEPTH, MAXT, mfma_cps(LAYOUT)>(a, bid % a.nblk, static_cast<int64_t>(bid / a.nblk) * TILE);
    else
        dedisp_tile<DPW, W, LAYOUT>(a, bid % a.nblk, static_cast<int64_t>(bid / a.nblk) * kTimeTile);
}

// Batched persistent launch: a grid of resident work-groups pulls (beam, DM block,
// time tile) items from one device counter until the items run out, so beams of any
// shape share one launch. Consecutive items are adjacent DM blocks of the same tile
// of the same beam (their input rows overlap). A work-group reads the item index from
// the counter, finds its beam by binary search over item_begin, and exits when the
// index passes the total: every work-group reaches that exit.
template <int DPW, int W, int LAYOUT, int TILE = kTimeTile, int DEPTH = 2, int MAXT = 63, int WPE = 1>
__global__ __launch_bounds__(64 * W, WPE) void dedisp_batch_kernel(const DedispArgs* __restrict__ args,
                                                              const int64_t* __restrict__ item_begin, int nbeams,
                                                              int64_t total, unsigned long long* counter) {
    __shared__ int64_t item;
    for (;;) {
        if (threadIdx.x == 0) item = static_cast<int64_t>(atomicAdd(counter, 1ull));
        __syncthreads();
        // the item index is the same in every lane: keep it in scalar registers
        const uint64_t itu = static_cast<uint64_t>(item);
        const int64_t it = static_cast<int64_t>(
            (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(itu >> 32))) << 32) |
            static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(itu))));
        __syncthreads();
        if (it >= total) break;
        int lo = 0, hi = nbeams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_begin[mid] <= it) lo = mid; else hi = mid - 1;
        }
        // the beam is the same in every lane; stating it keeps the beam's arguments and
        // the tile's step records in scalar registers
        lo = __builtin_amdgcn_readfirstlane(lo);
        const DedispArgs a = args[lo];
        const int64_t local = it - item_begin[lo];
        if constexpr (LAYOUT == 7)
            dedisp_quad_tile<W, DPW, DEPTH>(a, static_cast<int>(local % a.nblk), (local / a.nblk) * TILE);
        else if constexpr (LAYOUT == 6)
            dedisp_mfma_mixed<W, TILE, DEPTH, MAXT>(a, static_cast<int>(local % a.nblk), (local / a.nblk) * TILE);
        else if constexpr (LAYOUT == 4 || LAYOUT == 5)
            dedisp_mfma_tile<W, TILE, DEPTH, MAXT, mfma_cps(LAYOUT)>(a, static_cast<int>(local % a.nblk),
                                                                     (local / a.nblk) * TILE);
        else
            dedisp_tile<DPW, W, LAYOUT>(a, static_cast<int>(local % a.nblk), (local / a.nblk) * kTimeTile);
        __syncthreads();   // the next item restages LDS buffer 0
    }
}

__global__ void reset_counter_kernel(unsigned long long* c) { *c = 0ull; }

typedef void (*DedispFn)(DedispArgs);
typedef void (*DedispBatchFn)(const DedispArgs*, const int64_t*, int, int64_t, unsigned long long*);

// Indexed by DedispVariant::id (tiling.cpp); layout 4-6 entries repeat the variant's
// time tile, depth and channel-block span; layout 7 entries are <samples per lane, waves,
// 7, tile, chunks per wave, 0, waves per SIMD>.
#define AA_VARIANTS(K)                                                                           \
    K<4, 4, 1>, K<2, 8, 1>, K<4, 8, 1>, K<2, 16, 1>, K<2, 8, 0>, K<4, 4, 0>, K<2, 8, 3>, K<4, 4, 3>, \
        K<2, 8, 2>, K<4, 8, 2>, K<4, 4, 2>, K<4, 8, 4, 1024, 3>, K<2, 16, 4, 1024, 3>, K<2, 16, 4, 768, 7>, \
        K<4, 8, 4, 512, 3, 31, 4>, K<2, 16, 4, 512, 3, 31, 8>, K<4, 8, 4, 480, 4, 31, 4>, K<2, 16, 5, 864, 3, 63>, \
        K<2, 16, 4, 960, 4, 63>, K<2, 16, 4, 896, 5, 63>, K<2, 16, 6, 864, 3, 63>, K<2, 4, 7, 512, 4, 0, 4>, \
        K<2, 8, 7, 1024, 4, 0, 4>, K<1, 16, 7, 1024, 2, 0, 8>, K<1, 8, 7, 512, 2, 0, 8>
const DedispFn kKernels[kNumDedispVariants] = {AA_VARIANTS(dedisp_kernel)};
const DedispBatchFn kBatchKernels[kNumDedispVariants] = {AA_VARIANTS(dedisp_batch_kernel)};
#undef AA_VARIANTS

}  // namespace

DedispArgs dedisp_args(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                       int32_t* d_out, int64_t out_pitch) {
    const DedispTables& T = p->tables[variant];
    DedispArgs a{};
    a.in = d_in;
    a.in_pitch = in_pitch;
    // Staged reads stop at n_in rounded up to 16 bytes (<= in_pitch): nothing past a row's
    // valid samples is needed for a stored output, and the bound keeps every load inside
    // [d_in + c * in_pitch, + round_up(n_in, 16)) even when d_in points into a larger buffer.
    a.n_in16 = (n_in + 15) & ~int64_t{15};
    a.base = T.d_base;
    a.offs = T.d_offs;
    a.blocks = T.d_blocks;
    a.nblk = static_cast<int>(T.blocks.size());
    a.nchan = p->nchan;
    a.nchan_pad = T.nchan_pad;
    a.out = d_out;
    a.out_pitch = out_pitch;
    a.n_out = n_in - p->maxshift;
    a.row = T.max_row;
    const int tile = kDedispVariants[variant].tile;
    a.tile = tile;
    a.ntile = (a.n_out + tile - 1) / tile;
    a.pad = T.d_pad;
    return a;
}

int launch_dedisperse(const aa_plan_s* p, int variant, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                      int32_t* d_out, int64_t out_pitch, hipStream_t stream) {
    const DedispTables& T = p->tables[variant];
    if (T.variant != variant || !T.d_offs) return fail(AA_EINVAL, "aa_dedisperse: variant tables not prepared");
    const DedispVariant& V = kDedispVariants[variant];
    const DedispArgs a = dedisp_args(p, variant, d_in, in_pitch, n_in, d_out, out_pitch);
    if (!variant_takes_pitch(variant, in_pitch))
        return fail(AA_EINVAL, "aa_dedisperse: the quad variants take row pitches of at most 2^28 bytes");
    const int64_t grid = a.ntile * a.nblk;
    if (grid > 0x7fffffff) return fail(AA_EINVAL, "aa_dedisperse: too many tiles for one launch");
    const size_t lds = V.layout >= 4 ? static_cast<size_t>(V.lds_bytes) : static_cast<size_t>(2 * kChanPerPass) * T.max_row;
    hipLaunchKernelGGL(kKernels[variant], dim3(static_cast<unsigned>(grid)), dim3(64 * V.waves), lds, stream, a);
    AA_HIP(hipGetLastError());
    return AA_OK;
}

int launch_dedisperse_batch(int variant, const DedispArgs* d_args, const int64_t* d_item_begin, int nbeams,
                            int64_t total, unsigned long long* d_counter, int max_row, hipStream_t stream) {
    const DedispVariant& V = kDedispVariants[variant];
    const size_t lds = V.layout >= 4 ? static_cast<size_t>(V.lds_bytes) : static_cast<size_t>(2 * kChanPerPass) * max_row;
    int dev = 0, cus = 0, per_cu = 0;
    AA_HIP(hipGetDevice(&dev));
    AA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    AA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kBatchKernels[variant], 64 * V.waves, lds));
    if (per_cu < 1) return fail(AA_EINVAL, "batched dedispersion: the kernel does not fit on a CU");
    const int64_t grid = std::min<int64_t>(static_cast<int64_t>(cus) * per_cu, std::max<int64_t>(total, 1));
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, d_counter);
    AA_HIP(hipGetLastError());
    hipLaunchKernelGGL(kBatchKernels[variant], dim3(static_cast<unsigned>(grid)), dim3(64 * V.waves), lds, stream,
                       d_args, d_item_begin, nbeams, total, d_counter);
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
    return launch_dedisperse(p, p->variant, d_in, in_pitch, n_in, d_out, out_pitch, static_cast<hipStream_t>(stream));
}
