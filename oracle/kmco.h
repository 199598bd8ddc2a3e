/*
 * kmco.h -- serial CPU oracle for domain-decomposed sequential-update kMC.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never calls it, and the two share
 * no code: the Philox generator, the rate table, the schedule draw, the
 * event selection and the clocks are all written out again here.
 *
 * What it computes (Nilmeier & Marian, "A rigorous sequential update strategy
 * for parallel kinetic Monte Carlo simulation"):
 *   - periodic 2D Ising energy, Appendix A, Eq. (Hamiltonian Definition),
 *     extended by a uniform field h:  H = -J sum_<ij> s_i s_j - h sum_i s_i;
 *     or the same energy on a periodic ring (the paper's 1D system, Sec. 3.1);
 *   - single-site kernel with self-loops, Appendix A, Eq. (Glauber_TM):
 *     selection probability 1/n_d inside a domain, acceptance w (Barker form
 *     as printed, or Metropolis min(1, exp(-dE/T)));
 *   - equal, fixed rectangular domains with a frozen halo, each run for N_I
 *     steps, Sec. 2.2 and Fig. 1 (checkerboards, stripes, one domain);
 *   - a schedule drawn uniformly each sweep, Eq. (schedule) and
 *     Eq. (sum of sequential tms); non-interacting domains (one colour of a
 *     proper colouring of the domain grid) run in one phase, Sec. 2.2;
 *   - n-fold-way residence time tau = 1/R per event, Eq. (Poisson
 *     Distribution) and the text after it;
 *   - integer step count s += N_I * N_D per sweep, Eq. (CK_parallel in s);
 *   - statistics only at domain-process endpoints (sweep ends), Sec. 2.3.
 * The readings taken where the paper is silent are listed in the header
 * comment of kmco.c.
 */
#ifndef KMCO_H
#define KMCO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { KMCO_METROPOLIS = 0, KMCO_BARKER = 1 };
enum { KMCO_SCHED_RANDOM_PERM = 0, KMCO_SCHED_PALINDROME = 1 };
enum { KMCO_INIT_RANDOM = 0, KMCO_INIT_ALL_UP = 1, KMCO_INIT_GIVEN = 2 };
enum { KMCO_F_SCORE = 1, KMCO_F_CHECK = 2 };

typedef struct {
    double J, h, T;
    int32_t L;               /* periodic L x L lattice                    */
    int32_t tile;            /* Bx: domain width, L % Bx == 0              */
    int32_t steps_per_visit; /* N_I ticks per domain visit; 0 means B*B    */
    int32_t rate_model;      /* KMCO_METROPOLIS or KMCO_BARKER             */
    int32_t schedule;        /* KMCO_SCHED_*                                */
    int32_t init;            /* KMCO_INIT_*                                 */
    int32_t tile_rows;       /* By: domain height, L % By == 0; 0 means Bx  */
    int32_t dims;            /* 0 or 2: periodic L x L lattice; 1: periodic
                                ring of L sites (Sec. 3.1), domains of
                                `tile` sites, tile_rows 0 or 1              */
    double time_slice;       /* > 0: the rejection-free variant with fixed
                                time slices (see kmco.c, R7): each domain
                                process runs its continuous-time kinetics
                                for this long instead of N_I ticks; 0: the
                                tick chain                                 */
} kmco_desc;

typedef struct {
    int64_t sweep;   /* sweeps completed since creation                   */
    int64_t M;       /* sum of spins                                      */
    int64_t B;       /* sum over right and down bonds of s_i s_j          */
    int64_t events;  /* accepted flips since creation                     */
    int64_t steps;   /* ticks since creation (N_I per visit)              */
    double  t;       /* mean over domains of the per-domain event clocks  */
} kmco_record;

typedef struct kmco_state kmco_state;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void kmco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Per-class rate table: class c = 5*[s=+1] + k, k = up-neighbour count,
 * on the square lattice (4 neighbours).  kmco_rates_z is the same table for
 * z neighbours (z = 2: the ring; classes with k > z are never occupied). */
int kmco_rates(double J, double h, double T, int32_t model,
               uint64_t r[10], double w[10], double gJ[10], double gh[10]);
int kmco_rates_z(double J, double h, double T, int32_t model, int32_t z,
                 uint64_t r[10], double w[10], double gJ[10], double gh[10]);

/* Index in [0, n_perm) of the colour permutation for (seed, replica, sweep);
 * n_perm = n_colours!.  kmco_schedule_index is the 4-colour case (24). */
int32_t kmco_schedule_index_n(uint64_t seed, int32_t replica, int64_t sweep,
                              int32_t n_perm);
int32_t kmco_schedule_index(uint64_t seed, int32_t replica, int64_t sweep);
/* Lexicographic permutation of {0..n-1} of rank idx (n <= 9). */
void kmco_perm_from_index_n(int32_t idx, int32_t n, int32_t *perm);
void kmco_perm_from_index(int32_t idx, int32_t perm[4]);

/* Colour of each domain (row-major over the domain grid) and the number of
 * colours: per axis 1 colour for a single domain, 2 for an even count
 * (t mod 2), 3 for an odd count (t mod 2, the last domain 2); the domain's
 * colour is ax + cx * ay. */
int kmco_get_partition(const kmco_state *s, int32_t *colour, int32_t *n_colours);

/* Natural logarithm of u in (0, 1] by the atanh series (R7): the same
 * sequence of IEEE double operations as the GPU library's, so both take
 * identical time-slice decisions.  Within 2 ulp of the correctly rounded
 * value (tested against libm). */
double kmco_slice_log(double u);

/* Uniform slot in [0, n) for one tick, with rejection and retries. */
uint32_t kmco_tick_slot(uint64_t seed, int32_t replica, int64_t sweep,
                        int32_t domain, int32_t visit, uint32_t tick,
                        uint32_t n, int32_t *retries);

kmco_state *kmco_create(const kmco_desc *d, uint64_t seed, int32_t replica,
                        const int8_t *given);
/* Runs n_sweeps sweeps.  After the i-th sweep of this call (1-based) a record
 * is written when i % record_every == 0.  With KMCO_F_SCORE the likelihood-
 * ratio score (d/dJ, d/dh) of every tick is added to score[2*k], score[2*k+1]
 * where k is the record that closes the interval holding the tick; when
 * score_abs is not NULL it receives, in the same layout, the sum of the
 * absolute values of the terms making up that score (|d ln w_c/d theta| per
 * event; per run of m null ticks m sum_c n_c |w_c d ln w_c/d theta| /
 * (n_d - R_w)), the scale against which rounding differences of the score
 * are judged.
 * Returns the number of records written, or a negative error code. */
int64_t kmco_run(kmco_state *s, int64_t n_sweeps, int32_t record_every,
                 int32_t flags, kmco_record *rec, int64_t rec_cap,
                 double *score, double *score_abs);
int kmco_get_spins(const kmco_state *s, int8_t *out);
int kmco_get_domain_clocks(const kmco_state *s, double *sum, double *comp);
int kmco_get_domain_events(const kmco_state *s, int64_t *events);
int64_t kmco_check_failures(const kmco_state *s);
/* Ticks of all runs so far whose slot was rejected at least once by the
 * exact 1/n_d selection (Lemire rejection, App. A Eq. (Glauber_TM)) and
 * redrawn on the retry streams, and the number of redraws. */
int kmco_get_retries(const kmco_state *s, int64_t *ticks, int64_t *draws);
/* Ticks t < n_ticks of one visit (seed, replica, sweep, domain, visit) whose
 * slot in [0, n) needs a redraw.  Depends only on the counters and n, not on
 * any lattice. */
int64_t kmco_count_retry_ticks(uint64_t seed, int32_t replica, int64_t sweep,
                               int32_t domain, int32_t visit, uint32_t n_ticks,
                               uint32_t n);
void kmco_destroy(kmco_state *s);

#ifdef __cplusplus
}
#endif
#endif
