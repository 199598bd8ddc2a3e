/* Drives every path of the serial oracle (square lattices of several
 * partitions, the ring, the time-slice variant, the palindrome, given and
 * all-up starts, the score with its magnitudes, the bookkeeping check, the
 * generators) for a build under AddressSanitizer and UndefinedBehavior-
 * Sanitizer; exits non-zero on any inconsistency. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "kmco.h"

static int run_case(kmco_desc d, int32_t flags, int sweeps, int every)
{
    int8_t given[128 * 128];
    for (int i = 0; i < 128 * 128; ++i) given[i] = (i * 7 + 3) % 5 < 2 ? 1 : -1;
    kmco_state *s = kmco_create(&d, 0x1234ABCDull, 3, given);
    if (!s) return 1;
    int n_rec = (sweeps + every - 1) / every;
    kmco_record *rec = calloc((size_t)n_rec + 1, sizeof *rec);
    double *score = calloc(2 * ((size_t)n_rec + 1), sizeof(double));
    double *mag = calloc(2 * ((size_t)n_rec + 1), sizeof(double));
    int64_t n = kmco_run(s, sweeps, every, flags, rec, n_rec, score, mag);
    int bad = n < 0 && !((flags & KMCO_F_SCORE) && d.time_slice > 0.0);
    if (flags & KMCO_F_CHECK) bad |= kmco_check_failures(s) != 0;
    int64_t rt, rd;
    kmco_get_retries(s, &rt, &rd);
    int8_t *sp = malloc((size_t)d.L * d.L);
    kmco_get_spins(s, sp);
    double cs[1 << 12], cc[1 << 12];
    int64_t ev[1 << 12];
    kmco_get_domain_clocks(s, cs, cc);
    kmco_get_domain_events(s, ev);
    int32_t col[1 << 12], ncol;
    kmco_get_partition(s, col, &ncol);
    free(sp);
    free(rec);
    free(score);
    free(mag);
    kmco_destroy(s);
    return bad;
}

int main(void)
{
    int bad = 0;
    kmco_desc d;
    memset(&d, 0, sizeof d);
    d.J = 1.0; d.h = 0.1; d.T = 2.3;
    const struct { int L, tile, rows, dims, sched, init, ni; double tau; } cases[] = {
        {16, 8, 0, 2, 0, 0, 64, 0.0},   {24, 12, 0, 2, 1, 1, 0, 0.0},
        {20, 4, 20, 2, 0, 2, 30, 0.0},  {12, 12, 0, 2, 0, 0, 0, 0.0},
        {15, 5, 0, 2, 1, 0, 9, 0.0},    {8, 2, 4, 2, 0, 0, 3, 0.0},
        {64, 8, 0, 1, 0, 0, 5, 0.0},    {8, 8, 0, 1, 1, 2, 8, 0.0},
        {9, 3, 0, 1, 0, 0, 2, 0.0},     {16, 4, 0, 2, 0, 0, 0, 0.6},
        {12, 12, 0, 2, 1, 0, 0, 1.5},   {30, 10, 0, 1, 0, 0, 0, 0.8},
        {122, 61, 0, 2, 0, 0, 200, 0.0},
    };
    for (size_t k = 0; k < sizeof cases / sizeof cases[0]; ++k) {
        d.L = cases[k].L; d.tile = cases[k].tile; d.tile_rows = cases[k].rows;
        d.dims = cases[k].dims; d.schedule = cases[k].sched; d.init = cases[k].init;
        d.steps_per_visit = cases[k].ni; d.time_slice = cases[k].tau;
        for (int model = 0; model < 2; ++model) {
            d.rate_model = model;
            bad |= run_case(d, KMCO_F_CHECK, 6, 2);
            bad |= run_case(d, KMCO_F_SCORE, 5, 2);
        }
    }
    /* generators and helpers */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    kmco_philox(ctr, key, out);
    int32_t perm[9];
    for (int n = 1; n <= 9; ++n) kmco_perm_from_index_n(0, n, perm);
    int32_t r;
    for (uint32_t t = 0; t < 1000; ++t) (void)kmco_tick_slot(7, 1, 2, 3, 0, t, 144, &r);
    bad |= kmco_count_retry_ticks(7, 1, 2, 3, 0, 1000, 2147483649u) <= 0;
    for (double u = 1.0; u > 1e-300; u *= 0.37) bad |= !(kmco_slice_log(u) <= 0.0);
    /* rejected descriptors */
    d.L = 10; d.tile = 3; d.dims = 2; d.time_slice = 0.0;
    bad |= kmco_create(&d, 1, 0, NULL) != NULL;
    d.tile = 5; d.time_slice = -1.0;
    bad |= kmco_create(&d, 1, 0, NULL) != NULL;
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
