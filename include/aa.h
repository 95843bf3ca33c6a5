/*
 * aa.h - C ABI of the MI355X (gfx950) dedispersion + single-pulse-search library.
 *
 * The library implements the GPU phase of the pipeline studied in Novotny, Adamek
 * and Armour, "Implementing CUDA Streams into AstroAccelerate - A Case Study":
 * the dedispersion phase (section 2.1) and the single-pulse search (section 2.2).
 * Both run over time chunks that are split across streams (section 1, Fig. 2).
 * The five-step streams recipe of section 2 shapes the pipeline calls: create
 * streams, pin host memory, use asynchronous copies, tag kernels and copies with
 * a stream, and take every synchronisation off the hot loop.
 *
 * Conventions for every call:
 *  - The return value is a status code (AA_OK, or one of the codes below). No
 *    C++ exception crosses this boundary. aa_last_error() returns a message for
 *    the last failing call on the calling thread.
 *  - "d_" pointers are device (HBM) pointers and "h_" pointers are host pointers.
 *    A stream argument is a hipStream_t passed as void*. NULL means the null stream.
 *  - Compute calls are asynchronous on the given stream. The caller owns every
 *    buffer it passes and must keep it alive until the stream has finished with it.
 *  - Numeric definitions (shift rounding, statistics, S/N rounding points, the peak
 *    rule) are those stated for aa_plan and aa_single_pulse below.
 */
#ifndef AA_H
#define AA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define AA_OK         0
#define AA_EAGAIN     1    /* nothing ready yet (aa_poll)                         */
#define AA_EINVAL    (-1)  /* invalid argument or descriptor                      */
#define AA_ESHORT    (-2)  /* too few samples for maxshift + widest boxcar        */
#define AA_ENOMEM    (-3)  /* host or device allocation failed                    */
#define AA_EHIP      (-4)  /* a HIP runtime call failed (message in aa_last_error) */
#define AA_EOVERFLOW (-5)  /* more candidates than capacity; the true count is kept */
#define AA_EBUSY     (-6)  /* admission refused: no free slot or HBM budget       */

const char* aa_last_error(void);
const char* aa_version(void);

/* ---- plan (A0) ------------------------------------------------------------
 * Section 1 places "mapping tasks to resources and allocation of all necessary
 * memory" before the search, and section 2.2 moves the search's allocations
 * there. A plan fixes everything that does not depend on the data:
 *   f_c      = f_top - c * foff                  (channel 0 is the highest)
 *   s[d][c]  = floor(((K * dm[d]) * (1/(f_c*f_c) - 1/(f_top*f_top))) / tsamp + 0.5)
 *              K = 4.148808e3 MHz^2 s pc^-1 cm^3. Each step is one IEEE float64
 *              operation in this order, with no fused multiply-add, on the host.
 *   maxshift M = max s;  N_dd = nsamp - M;  T = N_dd - wmax + 1 boxcar starts.
 * On success the plan holds host and device copies of s (int32 [ndm][nchan]).
 * The device copy is uploaded once, to the device current at aa_plan time,
 * unless AA_PLAN_HOST_ONLY is set. A plan is immutable and may be shared between
 * threads.
 * Errors: AA_EINVAL for nchan < 1, ndm < 1, DMs that are negative or not
 * ascending, f_top - (nchan-1)*foff <= 0, foff <= 0, tsamp <= 0, widths that are
 * not ascending, unique and >= 1, wmax > AA_MAX_WIDTH, nchan*255*wmax >= 2^32
 * (boxcar sums are exact 32-bit integers), a stat block that is not a positive
 * multiple of 256 or that could overflow int64 moments, or a threshold that is not
 * finite, a clip_sigma that is negative or not finite, clip_iters outside 0..16, or a
 * boxcar_full_width that is negative or below the first width.
 * AA_ESHORT if T < 1. AA_EHIP or AA_ENOMEM if the upload fails.
 */
#define AA_PLAN_HOST_ONLY 1u
#define AA_MAX_WIDTH      1024
#define AA_MAX_NCHAN      65535

typedef struct aa_plan_s* aa_plan_t;

typedef struct {
    int32_t       nchan;          /* channels (rows of the filterbank)               */
    int64_t       nsamp;          /* samples per channel of a whole-signal call      */
    double        f_top_mhz;      /* centre frequency of channel 0 (highest), MHz   */
    double        foff_mhz;       /* channel width, MHz, > 0                         */
    double        tsamp_s;        /* sampling time, s                                */
    const double* dm;             /* ndm trials, pc cm^-3, ascending, >= 0 (copied)  */
    int32_t       ndm;
    const int32_t* widths;        /* boxcar widths in samples, ascending (copied)    */
    int32_t       nwidths;
    float         snr_threshold;  /* candidates need best S/N >= threshold           */
    int32_t       stat_block;     /* starts per statistics block; 0 means 32768      */
    uint32_t      flags;          /* AA_PLAN_HOST_ONLY                               */
    float         clip_sigma;     /* outlier clipping of the block statistics, in sigma;
                                     0 = off (see aa_single_pulse)                   */
    int32_t       clip_iters;     /* clipping rounds, 0..16; 0 = off                 */
    int32_t       boxcar_full_width; /* decimated boxcar hierarchy: widths above this are
                                     tried on a coarser start grid (see aa_single_pulse);
                                     0 = off, else >= widths[0]                        */
} aa_plan_desc_t;

typedef struct {
    int32_t nchan, ndm, nwidths, wmax;
    int64_t nsamp, maxshift, n_dd, n_start, stat_block, nblocks;
    int64_t in_pitch;       /* recommended input row pitch (bytes): nsamp rounded up to 256 */
    int64_t out_pitch;      /* recommended plane row pitch (elements): n_dd rounded to 64   */
    size_t  work_bytes;     /* aa_single_pulse scratch for a whole-signal call             */
    int32_t device;         /* device of the uploaded shift table, -1 for host-only         */
} aa_plan_info_t;

int aa_plan(const aa_plan_desc_t* desc, aa_plan_t* out);
int aa_plan_info(aa_plan_t plan, aa_plan_info_t* out);
/* Copies the int32 shift table, ndm*nchan entries, row-major [d][c], to h_out. */
int aa_plan_shifts(aa_plan_t plan, int32_t* h_out);
void aa_plan_destroy(aa_plan_t plan);

/* ---- dedispersion (A2) -----------------------------------------------------
 * Section 2.1 (dedispersion phase). Brute-force incoherent dedispersion:
 *   d_out[d * out_pitch + t] = sum over c < nchan of d_in[c * in_pitch + t + s[d][c]]
 * for 0 <= d < ndm and 0 <= t < n_in - maxshift. Sums are exact int32: at most
 * 65535 * 255 < 2^31.
 * d_in:  uint8 [nchan][in_pitch]. Samples 0..n_in-1 of each row are read.
 *        d_in and in_pitch must be multiples of 16 bytes.
 * n_in:  valid samples per row. maxshift + 1 <= n_in <= in_pitch.
 * d_out: int32 [ndm][out_pitch], out_pitch >= n_in - maxshift, 16-byte aligned rows.
 *        Columns >= n_in - maxshift are not written.
 * Errors: AA_EINVAL on a host-only plan, bad sizes or misaligned pointers, or
 * in_pitch above 2^28 bytes with a quad variant (layout 7) in use.
 * AA_EHIP if the launch fails.
 */
int aa_dedisperse(aa_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t n_in,
                  int32_t* d_out, int64_t out_pitch, void* stream);

/* ---- dedispersion kernel variants and autotuner -----------------------------
 * aa_dedisperse has several kernel variants. They differ in work-group shape:
 * waves per work-group, trials per wave (so trials per DM block), LDS budget, and
 * the lane-to-sample layout.
 * All variants compute the same bit-exact result. Preparing a variant builds its
 * tables on the host and uploads them once. That is plan-time work, like aa_plan,
 * and must not run concurrently with compute calls on the same plan.
 *   aa_variant_count()            number of variants
 *   aa_variant_info(v, out)       shape of variant v
 *   aa_plan_set_variant(plan, v)  prepare v and use it for aa_dedisperse (a new plan uses
 *                                 variant 12, the 16-wave i8 matrix-core kernel)
 *   aa_plan_get_variant(plan, v)  variant in use
 *   aa_autotune(...)              time every variant on the caller's buffers (reps runs
 *                                 each, HIP events on `stream`), select the fastest,
 *                                 and write the per-variant mean ms to ms_out
 *                                 [aa_variant_count()]; variants that cannot take the
 *                                 input (quad variants with in_pitch above 2^28) are
 *                                 skipped (-1). For the mixed-shape variant (layout 6)
 *                                 it also times the trial where the 4-channel blocks
 *                                 start at 128 and 256 trials either side of the host's
 *                                 estimate and keeps the fastest (ms_out holds that
 *                                 time). If AA_TUNE_CACHE names a file,
 *                                 the choice is read from and written to that JSON
 *                                 cache, keyed by device arch and plan shape.
 * d_out receives the dedispersed plane of the last run.
 */
typedef struct {
    int32_t id, waves, dm_per_wave, trials_per_block, lds_bytes;
    int32_t layout;   /* 0, 3: a lane owns 16 contiguous samples; 1, 2: four groups of 4, 256 apart
                         (2 reuses a window when the next trial has the same offset);
                         4, 5: i8 matrix-core contraction over an exact split of the shift table
                         (4 or 8 channels per step); 6: both, chosen per block of trials */
    int32_t time_tile;   /* output samples per work-group */
    int32_t depth;       /* staging buffers per work-group (loads run depth - 1 passes ahead) */
    int32_t max_tiles;   /* layouts 4-6: a channel block spans at most 32 * max_tiles rows of the
                            shifted time axis (31 or 63); 0 for the other layouts */
} aa_variant_t;

int aa_variant_count(void);
int aa_variant_info(int32_t v, aa_variant_t* out);
int aa_plan_set_variant(aa_plan_t plan, int32_t v);
int aa_plan_get_variant(aa_plan_t plan, int32_t* v);
int aa_autotune(aa_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, int32_t* d_out,
                int64_t out_pitch, int32_t reps, void* stream, float* ms_out);

/* ---- single-pulse search (A3-A5) -------------------------------------------
 * Section 2.2 (single-pulse search phase). Input: a dedispersed plane whose column
 * j holds absolute start dd_t0 + j, valid for j < dd_n. Output: the candidates
 * among the starts [t_begin, t_end).
 *   - Statistics per DM row and per block of stat_block starts, aligned to absolute
 *     start 0. n, S1 and S2 are exact. mu = S1/n.
 *     var = double(n*S2 - S1^2) / double(n*n), where the integer is exact and is
 *     rounded once. sigma = sqrt(var).
 *     With the plan's clip_sigma c > 0 and clip_iters k > 0 (robust statistics; the
 *     paper defers its search to the single-pulse work it cites): k rounds, each
 *     keeping the block's values D with |double(D) - mu| <= double(c) * sigma and
 *     recomputing exact n, S1, S2, mu and sigma over the kept values; a round that
 *     would keep nothing ends the clipping. Window sums still use every value.
 *     wmu_w = w*mu. r_w = 1/(sigma*sqrt(w)), or 0 if sigma == 0.
 *   - S/N(d,t,w) = (double(sum_{i<w} D[d][t+i]) - wmu_w) * r_w. best = max over w,
 *     and wbest is the smallest width that attains it.
 *     With the plan's boxcar_full_width w0 > 0 (the decimated boxcar hierarchy of the
 *     single-pulse work the paper cites: a boxcar over data decimated by 2^l is a wide
 *     boxcar at a start that is a multiple of 2^l), width w is tried only at starts t
 *     that are multiples of its stride, the smallest power of two s with w0 * s >= w;
 *     best and wbest are over the widths tried at t.
 *   - (d,t) is a candidate iff best >= threshold and best is a 3x3 maximum in
 *     (d, t): strictly greater than the neighbours earlier in row-major order, and
 *     >= the later ones. Neighbours outside [0,ndm) x [0,t_total) are ignored. The
 *     whole window uses the statistics of the centre's block.
 * t_begin must be a multiple of stat_block. t_end - t_begin >= 1.
 * t_total is the T of the whole signal, or -1 if it is not known yet. The plane
 * must hold the column t_begin-1 (if t_begin > 0) and every column up to
 * right + wmax - 2, where right = t_end if t_end == t_total, else t_end + 1.
 * d_work:  scratch of at least aa_single_pulse_work_bytes(plan, t_end - t_begin).
 * d_cand:  aa_candidate_t [cap], written in (dm_idx, t) order with beam = 0.
 * d_count: one int32. It receives the true number of candidates. If that exceeds
 *          cap, only the first cap are written (AA_EOVERFLOW is seen by the caller
 *          when it reads *d_count > cap).
 * d_best:  optional float [ndm][best_pitch] of float(best) for t in [t_begin, t_end).
 */
typedef struct {
    int32_t dm_idx;
    int32_t width;
    int64_t t;        /* absolute start sample of the boxcar */
    float   snr;
    int32_t beam;
} aa_candidate_t;

int aa_single_pulse_work_bytes(aa_plan_t plan, int64_t n_starts, size_t* out);
int aa_single_pulse(aa_plan_t plan, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0,
                    int64_t dd_n, int64_t t_begin, int64_t t_end, int64_t t_total,
                    void* d_work, size_t work_bytes, aa_candidate_t* d_cand, int32_t cap,
                    int32_t* d_count, float* d_best, int64_t best_pitch, void* stream);

/* ---- single-pulse search without allocation ----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, and harnesses that forbid hipMalloc. The same search as
 * aa_single_pulse, with the same arguments, results and errors, minus d_work: its
 * scratch is a fixed array of AA_NOALLOC_SCRATCH_BYTES in the library's device
 * memory, one per GPU, held until the process ends. The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); on its first call on a device it
 * looks up that device's copy of the array once.
 * Limit: aa_single_pulse_work_bytes(plan, t_end - t_begin) must not exceed
 * AA_NOALLOC_SCRATCH_BYTES, else AA_EINVAL (search fewer starts per call, or use
 * aa_single_pulse).
 * Every call on one GPU uses that GPU's one scratch array, so calls that overlap in
 * time on one GPU (other streams, other threads) race: serialise them, e.g. on one
 * stream. Scratch contents left by the last call are never read by the next.
 */
#define AA_NOALLOC_SCRATCH_BYTES (64u << 20)

int aa_single_pulse_noalloc(aa_plan_t plan, const int32_t* d_dd, int64_t dd_pitch, int64_t dd_t0, int64_t dd_n,
                            int64_t t_begin, int64_t t_end, int64_t t_total, aa_candidate_t* d_cand, int32_t cap,
                            int32_t* d_count, float* d_best, int64_t best_pitch, void* stream);

/* ---- per-range time decimation --------------------------------------------------
 * Beyond the paper, whose dedispersion phase (section 2.1) is brute force at the input
 * resolution. The trials are split into consecutive ranges; range r (first trial
 * first[r], first[0] = 0) is dedispersed and searched on the input decimated by
 * factor[r] = 2^k: k halvings, each the rounding average of adjacent samples,
 *   y[c][j] = (x[c][2j] + x[c][2j+1] + 1) >> 1,  0 <= j < floor(n / 2),
 * at sampling time factor[r] * tsamp. Each range is an ordinary plan (aa_plan with the
 * range's trials, nsamp >> k, tsamp * factor[r] and stat_block / factor[r]; the same
 * widths, in the range's samples, and threshold): its own maxshift, N_dd and T, and a
 * 3x3 peak test that does not look across the range's edges. Candidates are reported in
 * input samples: dm_idx is the global trial index, t = factor[r] * (range start) and
 * width = factor[r] * (range width), sorted by (dm_idx, t).
 *   aa_decimate2       one halving of nchan rows (16-byte aligned buffers and pitches,
 *                      out_pitch >= n_in / 2), asynchronous on `stream`.
 *   aa_range_plan      validates the ranges (1..16; first[] ascending below ndm; factors
 *                      powers of two, non-decreasing, dividing the stat block) and builds
 *                      the per-range plans. AA_EINVAL otherwise; AA_ESHORT if a range is
 *                      too short for its maxshift and widest boxcar at desc->nsamp.
 *   aa_range_plan_get  the plan of range r (owned by the range plan: set its variant or
 *                      autotune it; do not destroy it), its first trial and factor.
 *   aa_range_work_bytes  scratch for aa_range_run on n_in input samples and capacity cap:
 *                      the decimated inputs, one plane and one search scratch shared by
 *                      the ranges in turn, and the ranges' candidate lists.
 *   aa_range_run       all ranges over d_in (uint8 [nchan][in_pitch], n_in samples) on
 *                      `stream`: *d_count receives the true total, d_cand the first cap
 *                      candidates. AA_ESHORT if a range is too short at n_in.
 *   aa_range_autotune  decimates d_in into d_work and runs aa_autotune on each range's plan
 *                      with its own decimated input (reps runs per variant), so each range
 *                      gets its fastest variant; ms_out, if not null, receives
 *                      [nranges][aa_variant_count()] mean times. Synchronises `stream`.
 */
typedef struct aa_range_plan_s* aa_range_plan_t;

int aa_decimate2(const uint8_t* d_in, int64_t in_pitch, int64_t n_in, int32_t nchan, uint8_t* d_out,
                 int64_t out_pitch, void* stream);
int aa_range_plan(const aa_plan_desc_t* desc, const int32_t* first, const int32_t* factor, int32_t nranges,
                  aa_range_plan_t* out);
int aa_range_plan_get(aa_range_plan_t rp, int32_t r, aa_plan_t* plan, int32_t* first, int32_t* factor);
int aa_range_work_bytes(aa_range_plan_t rp, int64_t n_in, int32_t cap, size_t* out);
int aa_range_run(aa_range_plan_t rp, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, void* d_work,
                 size_t work_bytes, aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, void* stream);
int aa_range_autotune(aa_range_plan_t rp, const uint8_t* d_in, int64_t in_pitch, int64_t n_in, void* d_work,
                      size_t work_bytes, int32_t reps, void* stream, float* ms_out);
void aa_range_plan_destroy(aa_range_plan_t rp);

/* ---- cross-DM candidate clustering (host) -------------------------------------
 * Beyond the paper (its search, section 2.2, defers to the single-pulse work it cites,
 * which merges the detections of one pulse over neighbouring trials and starts).
 * Friends of friends: two candidates of the same beam are linked iff their dm_idx differ
 * by at most dm_radius and their t by at most t_radius; a cluster is a connected
 * component. Each cluster reports its peak (the member with the highest snr; among equal
 * snr the smallest (dm_idx, t)), its member count and the trial and start ranges of its
 * members. Clusters are written in (beam, peak dm_idx, peak t) order.
 * h_cand: host candidates, any order. h_out: host [cap]. *n_clusters: the true count.
 * Errors: AA_EINVAL for negative sizes or radii; AA_EOVERFLOW if more than cap clusters
 * (the first cap are written); AA_ENOMEM if host memory runs out.
 */
typedef struct {
    aa_candidate_t peak;
    int32_t members;
    int32_t dm_lo, dm_hi;
    int64_t t_lo, t_hi;
} aa_cluster_t;

int aa_cluster(const aa_candidate_t* h_cand, int64_t n, int32_t dm_radius, int64_t t_radius, aa_cluster_t* h_out,
               int64_t cap, int64_t* n_clusters);

/* ---- batched beams in one persistent launch ---------------------------------------
 * Many independent beams of uneven shape (nchan, nsamp, DM plan) are searched together.
 * The dedispersion of every beam in a group is ONE persistent launch: resident
 * work-groups pull (beam, DM block, time tile) items from a device counter. Each beam's
 * single-pulse search follows on the same stream. Beams are packed into groups whose
 * planes and search scratch fit d_work. Results equal per-beam aa_dedisperse +
 * aa_single_pulse runs over the whole input (t_begin 0, t_end = t_total = T).
 * variant: the dedispersion kernel variant for all beams. -1 runs aa_autotune on the
 * beam with the most work and uses its choice.
 * d_cand: [nbeams][cap] candidates; beam i writes its list at d_cand + i*cap, with
 * beam = i. d_count: [nbeams] true counts.
 * The call is ordered on `stream` and returns after the work has completed.
 * Errors: AA_EINVAL for bad beams; AA_ENOMEM if one beam's plane does not fit d_work.
 */
#define AA_BATCH_STATIC 1u   /* one work-group per item instead of the persistent grid */

typedef struct {
    aa_plan_t      plan;
    const uint8_t* d_in;       /* uint8 [nchan][in_pitch], 16-byte aligned */
    int64_t        in_pitch;
    int64_t        n_in;       /* samples per channel */
} aa_batch_beam_t;

#define AA_MAX_VARIANTS 32   /* upper bound of aa_variant_count() */

typedef struct {
    int32_t groups;            /* persistent launches used */
    int32_t variant;           /* dedispersion variant used */
    int64_t items;             /* (beam, DM block, time tile) items over all groups */
    float   ms_dedisp;         /* HIP-event time of the dedispersion launches */
    float   ms_search;         /* HIP-event time of the single-pulse searches */
    int32_t tuned_beam;        /* beam the autotuner timed (variant -1), else -1 */
    float   tune_ms[AA_MAX_VARIANTS];  /* its per-variant mean ms (-1: not timed or from cache) */
} aa_batch_info_t;

int aa_batch_run(const aa_batch_beam_t* beams, int32_t nbeams, int32_t variant, void* d_work, size_t work_bytes,
                 aa_candidate_t* d_cand, int32_t cap, int32_t* d_count, uint32_t flags, aa_batch_info_t* info,
                 void* stream);

/* ---- streamed pipeline and serving loop (A1, A6, A7) ---------------------------
 * Section 1 (Fig. 2) of the paper splits the signal into time chunks and splits each
 * chunk again, once per stream, with every piece tagged with its stream. Section 2
 * gives the recipe: create the streams up front, pin host memory, use asynchronous
 * copies tagged with a stream, and make every synchronisation non-blocking. Section
 * 2.2 moves the search's allocations out of the loop. So does this pipeline: all
 * device memory comes from one arena of `hbm_budget` bytes, allocated at create.
 *
 * A pipeline serves one or more beams. A beam is an independent signal with its own
 * plan. A submit appends `nsamp` new samples to a beam. Only the new samples cross
 * PCIe. The pipeline keeps each beam's overlap tail (maxshift + wmax + stat_block
 * samples at most) on the device, and copies it device-to-device ahead of the next
 * chunk. A submit covers the starts [e, e') that have become computable:
 * e' = floor((R - wmax - maxshift) / stat_block) * stat_block, where R is the number of
 * samples received so far. With AA_SUBMIT_LAST, e' = T = R - maxshift - wmax + 1 and
 * the beam is finished. [e, e') is split into up to `nstreams` block-aligned
 * sub-chunks on the compute streams. H2D and D2D copies run on a copy stream.
 * Concatenated over a beam's chunks, the candidates equal those of a single
 * whole-signal aa_dedisperse + aa_single_pulse run.
 *
 * Requests queue on the host. A scheduler thread admits them in arrival order, and
 * in order per beam, when arena memory and a result slot are free. Chunks of
 * different beams therefore overlap on the GPU. aa_poll returns finished chunks.
 * h_chunk must stay untouched until its tag has been returned by aa_poll. Pinned
 * memory (hipHostMalloc, or torch pin_memory) takes the fast paths below. Pageable
 * memory also works: by default the runtime stages each copy itself (slow, and the
 * copies stop overlapping); with AA_PIPE_STAGED the pipeline stages it through a ring
 * of small pinned bounce buffers (2 * nstreams of about nchan * max_chunk / nstreams
 * bytes, pinned when a beam is added), filled by one host thread per compute stream;
 * the scheduler performs those host copies, so submit and poll calls may wait for
 * them. submit, poll and release are thread-safe. destroy drains all work in flight.
 * H2D: when h_chunk, pitch and the destination column are 16-byte aligned, a row-gather
 * kernel reads the mapped pinned rows directly. Otherwise, or with AA_PIPE_SDMA_COPY,
 * hipMemcpy2DAsync is used.
 * Flags: AA_PIPE_SERIAL puts copies and kernels on one stream, with no overlap (the
 * plain single-stream baseline). AA_PIPE_TIMING records HIP-event times for copies
 * and kernels; aa_pipeline_stats reports them. AA_PIPE_STAGED: staged pageable
 * input, as above (section 2's pinned bounce buffers and per-stream host threads).
 * Errors inside the scheduler: a copy, wait, launch or event call that fails for a
 * chunk does not stop the pipeline. The chunk completes with status AA_EHIP, aa_poll
 * sets the calling thread's aa_last_error() to the failure's message, and the chunk's
 * arena block and result slot are released once its stream has passed them. Other
 * chunks and beams are not affected.
 * Environment, read at create:
 *   AA_LOG=path     appends one JSON line per finished chunk (tag, beam, starts, sub-chunks,
 *                   candidates, status, queue and total latency in seconds).
 *   AA_FAULT=unit:N test hook: the N-th sub-chunk issued (counting from 0) is not launched
 *                   and its chunk completes with AA_EHIP, as if its launch had failed.
 */
#define AA_PIPE_SERIAL 1u
#define AA_PIPE_TIMING 2u
#define AA_PIPE_SDMA_COPY 4u
#define AA_PIPE_STAGED 8u
#define AA_SUBMIT_LAST 1u

typedef struct aa_pipeline_s* aa_pipeline_t;

typedef struct {
    int32_t  nstreams;      /* compute streams, 1..16 (sub-chunks per chunk)                   */
    int32_t  max_beams;     /* beams that can be added                                         */
    int64_t  max_chunk;     /* largest nsamp of one submit                                     */
    int32_t  cand_cap;      /* candidate capacity per sub-chunk (0 means 65536)                */
    int32_t  result_slots;  /* sub-chunks in flight at once (0 means 4 * nstreams)            */
    int64_t  hbm_budget;    /* arena bytes (0: size for one chunk per stream + all histories) */
    uint32_t flags;         /* AA_PIPE_SERIAL | AA_PIPE_TIMING | AA_PIPE_SDMA_COPY | AA_PIPE_STAGED */
    int64_t  min_piece_work;/* smallest sub-chunk in DM-trial x channel x start units: a chunk is
                               split into min(nstreams, work / min_piece_work) sub-chunks, at least
                               one. 0 means 2^33; < 0 always splits into nstreams sub-chunks    */
} aa_pipeline_opts_t;

typedef struct {
    uint64_t tag;
    int32_t  beam;
    int32_t  status;        /* AA_OK, AA_EOVERFLOW (a sub-chunk exceeded cand_cap) or AA_EHIP */
    int64_t  t_begin, t_end;/* absolute starts covered (t_end == t_begin: none yet)         */
    int64_t  n_true;        /* true number of candidates                                     */
    int64_t  n;             /* candidates in cand[] (less than n_true only on overflow)      */
    const aa_candidate_t* cand;  /* sorted (dm_idx, t), beam set; valid until aa_release(tag) */
    double   latency_s;     /* submit call to completion seen by the scheduler (host clock) */
    double   queue_s;       /* submit call to admission                                      */
} aa_result_t;

typedef struct {
    int64_t submitted, completed, in_flight, queued;
    int64_t arena_bytes, arena_used, arena_peak;
    /* with AA_PIPE_TIMING: union lengths (ms) of copy intervals, kernel intervals and
     * their intersection, plus the first-to-last span; hidden = overlap / copy */
    double  copy_ms, kernel_ms, overlap_ms, span_ms, copy_sum_ms, kernel_sum_ms;
} aa_pipeline_stats_t;

int aa_pipeline_create(const aa_pipeline_opts_t* opts, aa_pipeline_t* out);
/* Registers a beam with its plan (created on the pipeline's device). Plan-time call:
 * allocates the beam's history from the arena. Returns the beam id in *beam. */
int aa_pipeline_add_beam(aa_pipeline_t pipe, aa_plan_t plan, int32_t* beam);
/* Resume (checkpoint/restart; the paper has no such passage, this serves restarting a
 * stream after a pipeline was torn down). Registers a beam whose search continues at the
 * absolute start t_resume, a multiple of the plan's stat_block: the t_end of the beam's
 * last result is such a checkpoint. The beam's first submitted sample must be the
 * absolute sample h = (t_resume - 1) rounded down to a multiple of 16 (0 if t_resume is
 * 0), so the submits re-send the samples [h, ...) that the old beam's device tail held.
 * Candidates then carry absolute starts and equal those of an uninterrupted run.
 * Errors: AA_EINVAL for a t_resume that is negative or not block-aligned. */
int aa_pipeline_add_beam_at(aa_pipeline_t pipe, aa_plan_t plan, int64_t t_resume, int32_t* beam);
int aa_stream_submit(aa_pipeline_t pipe, int32_t beam, const uint8_t* h_chunk, int64_t nsamp, int64_t pitch,
                     uint64_t tag, uint32_t flags);
/* Waits up to timeout_us (0: no wait, <0: forever) for a finished chunk. AA_EAGAIN if none. */
int aa_poll(aa_pipeline_t pipe, aa_result_t* out, int32_t timeout_us);
int aa_release(aa_pipeline_t pipe, uint64_t tag);
int aa_pipeline_stats(aa_pipeline_t pipe, aa_pipeline_stats_t* out);
int aa_pipeline_destroy(aa_pipeline_t pipe);

#ifdef __cplusplus
}
#endif
#endif /* AA_H */
