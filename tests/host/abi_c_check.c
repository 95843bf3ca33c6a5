/* A plain C caller of the library's C ABI (no Python, no torch): host-only plan, sizes,
 * shift table, validation errors, the variant table and host clustering. Compiled with a
 * C compiler against include/aa.h and linked to libaa_mi355x.so; needs no GPU. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "aa.h"

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            printf("FAIL line %d: %s (%s)\n", __LINE__, #c, aa_last_error()); \
            ++fails;                                                \
        }                                                           \
    } while (0)

int main(void) {
    double dm[100];
    for (int i = 0; i < 100; ++i) dm[i] = (double)i;
    int32_t widths[6] = {1, 2, 4, 8, 16, 32};
    aa_plan_desc_t d;
    memset(&d, 0, sizeof d);
    d.nchan = 128;
    d.nsamp = 32768;
    d.f_top_mhz = 1500.0;
    d.foff_mhz = 0.78125;
    d.tsamp_s = 64e-6;
    d.dm = dm;
    d.ndm = 100;
    d.widths = widths;
    d.nwidths = 6;
    d.snr_threshold = 6.0f;
    d.flags = AA_PLAN_HOST_ONLY;
    aa_plan_t p = NULL;
    CHECK(aa_plan(&d, &p) == AA_OK && p != NULL);
    aa_plan_info_t info;
    CHECK(aa_plan_info(p, &info) == AA_OK);
    /* the small workload's closed values: maxshift 418, N_dd 32350, T 32319 */
    CHECK(info.maxshift == 418 && info.n_dd == 32350 && info.n_start == 32319 && info.device == -1);
    int32_t* s = (int32_t*)malloc(sizeof(int32_t) * 100 * 128);
    CHECK(aa_plan_shifts(p, s) == AA_OK);
    CHECK(s[50 * 128 + 127] == 211 && s[1 * 128 + 127] == 4 && s[50 * 128 + 64] == 101 && s[0] == 0);
    free(s);
    /* a host-only plan cannot run on the device */
    CHECK(aa_dedisperse(p, (const uint8_t*)16, 32768, 32768, (int32_t*)16, 32768, NULL) == AA_EINVAL);
    aa_plan_destroy(p);
    /* validation: descending DMs, too short */
    dm[5] = 1.0;
    CHECK(aa_plan(&d, &p) == AA_EINVAL);
    dm[5] = 5.0;
    d.nsamp = 400;
    CHECK(aa_plan(&d, &p) == AA_ESHORT);
    /* variants */
    const int nv = aa_variant_count();
    CHECK(nv > 0 && nv <= AA_MAX_VARIANTS);
    for (int v = 0; v < nv; ++v) {
        aa_variant_t vi;
        CHECK(aa_variant_info(v, &vi) == AA_OK && vi.id == v && vi.waves > 0);
    }
    /* clustering: two separate groups and one singleton */
    aa_candidate_t c[5];
    memset(c, 0, sizeof c);
    c[0].dm_idx = 10; c[0].t = 100; c[0].snr = 7.0f; c[0].width = 1;
    c[1].dm_idx = 11; c[1].t = 102; c[1].snr = 9.0f; c[1].width = 2;
    c[2].dm_idx = 12; c[2].t = 104; c[2].snr = 8.0f; c[2].width = 4;
    c[3].dm_idx = 50; c[3].t = 5000; c[3].snr = 6.5f; c[3].width = 1;
    c[4].dm_idx = 51; c[4].t = 5003; c[4].snr = 6.6f; c[4].width = 1;
    aa_cluster_t out[5];
    int64_t n = 0;
    CHECK(aa_cluster(c, 5, 1, 3, out, 5, &n) == AA_OK && n == 2);
    CHECK(out[0].members == 3 && out[0].peak.dm_idx == 11 && out[0].dm_lo == 10 && out[0].dm_hi == 12);
    CHECK(out[1].members == 2 && out[1].peak.dm_idx == 51);
    CHECK(aa_cluster(c, 5, 0, 0, out, 2, &n) == AA_EOVERFLOW && n == 5);
    printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
