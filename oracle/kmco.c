/*
 * kmco.c -- serial CPU oracle (test infrastructure, see kmco.h).
 *
 * Plain serial C: one replica, one domain at a time, one tick at a time.
 * Nothing here is blocked, fused or vectorised; every tick is drawn, tested
 * and applied in the order the method defines.  Build with
 * -ffp-contract=off so that the clock and score sums round as written.
 *
 * Readings of the paper (each is also listed in the design notes):
 *  R1  One of the N_I "independent time steps" of a domain process
 *      (Sec. 2.2) is one tick of the single-site kernel of Eq. (Glauber_TM):
 *      a site of the domain is selected with probability 1/n_d and flipped
 *      with probability w; otherwise the tick is a null (self-loop) step.
 *      The kernel is written in n-fold-way form: with integer rates
 *      r = round(w 2^32), a tick draws x uniform on [0, n_d 2^32); x >= R
 *      (R = sum of the domain's rates) is a null tick, otherwise x picks a
 *      rate class by its prefix and a member of that class.  Each site then
 *      flips with probability r/(n_d 2^32), the printed kernel.
 *  R2  Rates: Barker 1/(1+e^{dE/T}) as printed, or Metropolis
 *      min(1, e^{-dE/T}).  dE = 2 s (J n + h), n = sum of the 4 neighbours;
 *      the field h extends Eq. (Hamiltonian Definition).
 *  R3  Domains are Bx wide and By high (checkerboards, vertical stripes with
 *      By = L, a single domain).  The domain grid is coloured per axis: one
 *      colour for a single domain, t mod 2 for an even count, t mod 2 with
 *      the last domain given colour 2 for an odd count; the colour is
 *      ax + cx ay.  Domains of one colour never touch, so the paper's remark
 *      that the order of non-interacting domains is irrelevant (Sec. 2.2)
 *      lets the schedule be a permutation of the n colours, drawn uniformly
 *      each sweep (w(L) = 1/n!, closed under reversal, Eq. (sum of
 *      sequential tms)), or the self-reverse palindrome 0 1 .. n-1 n-1 .. 1 0.
 *      Domains of a colour run in ascending index order; they commute.
 *  R4  Clock: the residence time of Eq. (Poisson Distribution) is drawn per
 *      accepted event as -ln(u)/R_w with R_w = R / 2^32 the domain's total
 *      rate before the event (the paper advances by the mean; it states both
 *      are equivalent).  Each domain sums its own clock (compensated sum);
 *      the replica time is the mean over domains.  The integer step count
 *      of Eq. (CK_parallel in s) is kept as well.
 *  R5  Score: d log P(path)/d theta for theta in (J, h) of the tick chain:
 *      an event at class c adds d ln w_c/d theta, a null tick adds
 *      d ln(1 - R_w/n_d)/d theta = -R'_w/(n_d - R_w), R'_w = sum_c n_c w_c g_c,
 *      using the unquantised w.  The paper has no score; this is the
 *      likelihood ratio of the chain it defines.
 *  R3b The paper's 1D system (Sec. 3.1, Eq. (1D partitions)) is a periodic
 *      ring of L sites cut into domains of B consecutive sites; a site has
 *      the two neighbours left and right, so its class is 5*[s=+1] + k with
 *      k in 0..2 and dE = 2 s (J (2k - 2) + h).  The domains along the ring
 *      are coloured like one axis of the square lattice.
 *  R6  Random numbers: Philox4x32-10, key = (seed low, seed high),
 *      counter = (tick, domain | visit<<20 | stream<<24, sweep, replica).
 *      Word 1 gives the slot (Lemire multiply with rejection, retried on
 *      streams 3..14), word 0 the low 32 bits of x, words 3:2 the 53-bit
 *      uniform for the clock.
 *  R7  The rejection-free variant with fixed time slices (the synchronous
 *      time-horizon approaches the paper contrasts itself with, Sec. 1): a
 *      domain process runs the continuous-time kinetics of its domain, halo
 *      frozen, for a fixed time tau instead of N_I ticks.  Event k of a visit
 *      draws one Philox call, counter (k, domain | visit<<20 | 16<<24, sweep,
 *      replica): words 3:2 give u = (m53 + 1) 2^-53 and the waiting time
 *      dt = (-ln(u) 2^32) / R (R = sum of the Q32 rates); if t + dt > tau the
 *      visit ends (the process is still in its state at tau: memoryless);
 *      otherwise t += dt and words 1:0 give x uniform on [0, R) (Lemire's
 *      64-bit multiply with rejection, redrawn on streams 17..28), which
 *      picks the class and member exactly as in R1 -- every draw is an
 *      event, none is null.  The domain clock advances by tau per visit and
 *      the step count stays 0.  The stop decision compares FP64 times, so
 *      the logarithm is one written here from the atanh series
 *      ln m = 2 atanh((m-1)/(m+1)) after splitting off the binary exponent
 *      (the GPU library evaluates the same series in the same order):
 *      both sides then take identical decisions.  With R = 0 (no possible
 *      event) the visit ends at once.  Each domain process is the
 *      continuous-time chain observed at a fixed time, whose transition
 *      matrix exp(Q tau) is reversible with respect to the conditional
 *      Boltzmann distribution, so Eq. (replica detailed balance) holds for
 *      it and the reversible schedule keeps the equilibrium exact.
 */
#include "kmco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define STREAM_TICK 0u
#define STREAM_INIT 1u
#define STREAM_SCHED 2u
#define STREAM_RETRY0 3u
#define MAX_RETRY 12
#define STREAM_SLICE 16u
#define STREAM_SLICE_RETRY0 17u

/* ---------------------------------------------------------------- Philox */

void kmco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* Philox4x32: per round two 32x32->64 products of counter words 0 and 2
     * with the multipliers; the high halves are mixed with words 1, 3 and the
     * round key, the low halves pass through.  The key advances by the Weyl
     * constants between rounds. */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                 uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    kmco_philox(ctr, key, out);
}

/* ------------------------------------------------------------ rate table */

int kmco_rates_z(double J, double h, double T, int32_t model, int32_t z,
                 uint64_t r[10], double w[10], double gJ[10], double gh[10])
{
    if (!(T > 0.0) || !isfinite(T) || !isfinite(J) || !isfinite(h)) return -1;
    if (model != KMCO_METROPOLIS && model != KMCO_BARKER) return -1;
    if (z != 2 && z != 4) return -1;
    for (int c = 0; c < 10; ++c) {
        int up = c / 5;                 /* 1 if the site spin is +1      */
        int k = c % 5;                  /* number of up neighbours       */
        double s = up ? 1.0 : -1.0;
        double n = (double)(2 * k - z); /* neighbour sum                 */
        double dE = 2.0 * s * (J * n + h);
        double dEdJ = 2.0 * s * n;
        double dEdh = 2.0 * s;
        double wc, dlogw_ddE;
        if (model == KMCO_METROPOLIS) {
            if (dE <= 0.0) {
                wc = 1.0;
                dlogw_ddE = 0.0;
            } else {
                wc = exp(-dE / T);
                dlogw_ddE = -1.0 / T;
            }
        } else {
            wc = 1.0 / (1.0 + exp(dE / T));
            dlogw_ddE = -(1.0 - wc) / T;
        }
        double q = floor(wc * 4294967296.0 + 0.5);
        if (q > 4294967296.0) q = 4294967296.0;
        r[c] = (uint64_t)q;
        w[c] = wc;
        gJ[c] = dlogw_ddE * dEdJ;
        gh[c] = dlogw_ddE * dEdh;
    }
    return 0;
}

int kmco_rates(double J, double h, double T, int32_t model,
               uint64_t r[10], double w[10], double gJ[10], double gh[10])
{
    return kmco_rates_z(J, h, T, model, 4, r, w, gJ, gh);
}

/* -------------------------------------------------------------- schedule */

static int32_t factorial(int32_t n)
{
    int32_t f = 1;
    for (int32_t i = 2; i <= n; ++i) f *= i;
    return f;
}

void kmco_perm_from_index_n(int32_t idx, int32_t n, int32_t *perm)
{
    /* lexicographic rank -> permutation of {0..n-1}: digit i of the rank in
     * the factorial number system picks among the values still unused */
    int avail[9];
    int navail = n;
    for (int i = 0; i < n; ++i) avail[i] = i;
    for (int i = 0; i < n; ++i) {
        int32_t radix = factorial(n - 1 - i);
        int a = idx / radix;
        idx %= radix;
        perm[i] = avail[a];
        for (int j = a; j < navail - 1; ++j) avail[j] = avail[j + 1];
        --navail;
    }
}

void kmco_perm_from_index(int32_t idx, int32_t perm[4])
{
    kmco_perm_from_index_n(idx, 4, perm);
}

int32_t kmco_schedule_index_n(uint64_t seed, int32_t replica, int64_t sweep,
                              int32_t n_perm)
{
    /* Uniform on [0,n): Lemire multiply-high with rejection of the
     * (2^32 mod n) smallest low halves, words taken in order. */
    const uint32_t n = (uint32_t)n_perm;
    const uint32_t thr = (uint32_t)(0u - n) % n;
    for (uint32_t call = 0;; ++call) {
        uint32_t o[4];
        draw(seed, call, STREAM_SCHED << 24, (uint32_t)sweep,
             (uint32_t)replica, o);
        for (int i = 0; i < 4; ++i) {
            uint64_t m = (uint64_t)o[i] * n;
            if ((uint32_t)m >= thr) return (int32_t)(m >> 32);
        }
    }
}

int32_t kmco_schedule_index(uint64_t seed, int32_t replica, int64_t sweep)
{
    return kmco_schedule_index_n(seed, replica, sweep, 24);
}

uint32_t kmco_tick_slot(uint64_t seed, int32_t replica, int64_t sweep,
                        int32_t domain, int32_t visit, uint32_t tick,
                        uint32_t n, int32_t *retries)
{
    uint32_t thr = (uint32_t)(0u - n) % n;  /* 2^32 mod n */
    uint32_t word1;
    uint32_t o[4];
    uint32_t c1 = (uint32_t)domain | ((uint32_t)visit << 20);
    draw(seed, tick, c1 | (STREAM_TICK << 24), (uint32_t)sweep,
         (uint32_t)replica, o);
    word1 = o[1];
    int k = 0;
    for (;;) {
        uint64_t m = (uint64_t)word1 * n;
        if ((uint32_t)m >= thr || k == MAX_RETRY) {
            if (retries) *retries = k;
            return (uint32_t)(m >> 32);
        }
        ++k;
        draw(seed, tick, c1 | ((STREAM_RETRY0 + (uint32_t)(k - 1)) << 24),
             (uint32_t)sweep, (uint32_t)replica, o);
        word1 = o[1];
    }
}

/* ---------------------------------------------------- time-slice variant */

double kmco_slice_log(double u)
{
    /* u = m 2^e with m in [sqrt(1/2), sqrt(2)); f = m - 1 is exact
     * (Sterbenz); s = f / (2 + f); ln m = 2 s (1 + z/3 + z^2/5 + ...),
     * z = s^2 <= 0.0295, twelve terms; ln u = e ln2_hi + (ln m + e ln2_lo)
     * with ln2_hi holding 32 significant bits, so e ln2_hi is exact. */
    const double ln2_hi = 0x1.62e42ffp-1;
    const double ln2_lo = -0x1.718432a1b0e26p-35;
    uint64_t bits;
    memcpy(&bits, &u, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    bits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull; /* m in [1, 2) */
    double m;
    memcpy(&m, &bits, sizeof m);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double sv = f / (2.0 + f);
    double z = sv * sv;
    double q = 1.0 / 25.0;
    q = 1.0 / 23.0 + z * q;
    q = 1.0 / 21.0 + z * q;
    q = 1.0 / 19.0 + z * q;
    q = 1.0 / 17.0 + z * q;
    q = 1.0 / 15.0 + z * q;
    q = 1.0 / 13.0 + z * q;
    q = 1.0 / 11.0 + z * q;
    q = 1.0 / 9.0 + z * q;
    q = 1.0 / 7.0 + z * q;
    q = 1.0 / 5.0 + z * q;
    q = 1.0 / 3.0 + z * q;
    double two_s = sv + sv;
    double lm = two_s + (two_s * z) * q;
    double de = (double)e;
    return de * ln2_hi + (lm + de * ln2_lo);
}

/* x uniform on [0, R), R > 0, from the 64-bit word w1:w0 of event k:
 * Lemire's multiply-high with rejection of the (2^64 mod R) smallest low
 * products, redrawn from the retry streams (words 1:0 of each call). */
static uint64_t slice_select(uint64_t seed, int32_t replica, int64_t sweep,
                             uint32_t c1, uint32_t k, uint64_t R,
                             uint32_t w1, uint32_t w0)
{
    uint64_t word = ((uint64_t)w1 << 32) | w0;
    for (int r = 0;; ++r) {
        unsigned __int128 m = (unsigned __int128)word * R;
        uint64_t lo = (uint64_t)m;
        if (lo >= R || lo >= (0 - R) % R || r == MAX_RETRY)
            return (uint64_t)(m >> 64);
        uint32_t o[4];
        draw(seed, k, c1 | ((STREAM_SLICE_RETRY0 + (uint32_t)r) << 24), (uint32_t)sweep,
             (uint32_t)replica, o);
        word = ((uint64_t)o[1] << 32) | o[0];
    }
}

/* ---------------------------------------------------------------- state */

struct kmco_state {
    int L, Bx, By, NTx, NTy, ND, nd, NI, sched, model;
    int Ly;                /* lattice rows: L, or 1 for the ring          */
    double tau;            /* time slice per visit; 0: N_I ticks (R7)     */
    int z;                 /* neighbours per site: 4, or 2 on the ring    */
    int ncol;              /* colours of the domain grid                  */
    int32_t *colour;       /* [ND]                                        */
    double J, h, T;
    uint64_t seed;
    int replica;
    int8_t *spin;          /* L*L, row-major, +1 / -1                     */
    uint64_t r[10];
    double w[10], gJ[10], gh[10];
    double *clk_sum, *clk_comp; /* per domain                             */
    int64_t *dom_events;
    int64_t sweep, events, steps;
    /* per-visit scratch */
    int nw;                /* words per class bitset                      */
    uint64_t *bits;        /* [10][nw]                                    */
    int8_t *cls;           /* [nd]                                        */
    int64_t check_fail;
    int64_t retry_ticks;   /* ticks whose slot needed at least one redraw */
    int64_t retry_draws;   /* redraws on the retry streams, in total      */
};

static inline int wrap(int a, int L) { a %= L; return a < 0 ? a + L : a; }

static inline int8_t spin_at(const kmco_state *s, int y, int x)
{
    return s->spin[wrap(y, s->Ly) * s->L + wrap(x, s->L)];
}

/* Class of lattice site (y, x): 5*[spin up] + number of up neighbours (4 on
 * the square lattice; left and right on the ring). */
static int site_class(const kmco_state *s, int y, int x)
{
    int up = spin_at(s, y, x) > 0;
    int k = (spin_at(s, y, x - 1) > 0) + (spin_at(s, y, x + 1) > 0);
    if (s->z == 4)
        k += (spin_at(s, y - 1, x) > 0) + (spin_at(s, y + 1, x) > 0);
    return 5 * up + k;
}

/* Colour of position t on an axis of n domains, and the axis's colours. */
static int axis_colour(int t, int n) { return n == 1 ? 0 : (n % 2 && t == n - 1) ? 2 : t % 2; }
static int axis_colours(int n) { return n == 1 ? 1 : n % 2 ? 3 : 2; }

kmco_state *kmco_create(const kmco_desc *d, uint64_t seed, int32_t replica,
                        const int8_t *given)
{
    if (!d || d->L < 1 || d->tile < 1 || d->L % d->tile) return NULL;
    const int ring = d->dims == 1;
    if (d->dims != 0 && d->dims != 1 && d->dims != 2) return NULL;
    if (ring && d->tile_rows > 1) return NULL;
    const int By = ring ? 1 : (d->tile_rows ? d->tile_rows : d->tile);
    if (By < 1 || d->L % By) return NULL;
    if (d->steps_per_visit < 0) return NULL;
    if (d->schedule != KMCO_SCHED_RANDOM_PERM &&
        d->schedule != KMCO_SCHED_PALINDROME) return NULL;
    kmco_state *s = (kmco_state *)calloc(1, sizeof(*s));
    if (!s) return NULL;
    s->L = d->L; s->Bx = d->tile; s->By = By;
    s->Ly = ring ? 1 : d->L;
    s->z = ring ? 2 : 4;
    s->NTx = d->L / d->tile; s->NTy = s->Ly / By;
    s->ND = s->NTx * s->NTy;
    s->nd = s->Bx * s->By;
    s->NI = d->steps_per_visit ? d->steps_per_visit : s->nd;
    if (!(d->time_slice >= 0.0) || !isfinite(d->time_slice)) {
        free(s);
        return NULL;
    }
    s->tau = d->time_slice;
    if (s->tau > 0.0) s->NI = 0; /* no ticks: the step count stays 0 */
    s->sched = d->schedule; s->model = d->rate_model;
    s->J = d->J; s->h = d->h; s->T = d->T;
    s->seed = seed; s->replica = replica;
    if (kmco_rates_z(s->J, s->h, s->T, s->model, s->z, s->r, s->w, s->gJ, s->gh)) {
        free(s);
        return NULL;
    }
    size_t N = (size_t)s->L * s->Ly;
    s->spin = (int8_t *)malloc(N);
    s->clk_sum = (double *)calloc(s->ND, sizeof(double));
    s->clk_comp = (double *)calloc(s->ND, sizeof(double));
    s->dom_events = (int64_t *)calloc(s->ND, sizeof(int64_t));
    s->nw = (s->nd + 63) / 64;
    s->bits = (uint64_t *)calloc((size_t)10 * s->nw, sizeof(uint64_t));
    s->cls = (int8_t *)malloc(s->nd);
    s->colour = (int32_t *)malloc(sizeof(int32_t) * s->ND);
    if (!s->spin || !s->clk_sum || !s->clk_comp || !s->dom_events ||
        !s->bits || !s->cls || !s->colour) {
        kmco_destroy(s);
        return NULL;
    }
    const int cx = axis_colours(s->NTx);
    s->ncol = cx * axis_colours(s->NTy);
    for (int q = 0; q < s->ND; ++q)
        s->colour[q] = axis_colour(q % s->NTx, s->NTx) + cx * axis_colour(q / s->NTx, s->NTy);
    for (size_t i = 0; i < N; ++i) {
        if (d->init == KMCO_INIT_ALL_UP) {
            s->spin[i] = 1;
        } else if (d->init == KMCO_INIT_GIVEN) {
            if (!given || (given[i] != 1 && given[i] != -1)) {
                kmco_destroy(s);
                return NULL;
            }
            s->spin[i] = given[i];
        } else {
            /* bit i of the INIT stream: call i/128, word (i/32)%4, bit i%32 */
            uint32_t o[4];
            draw(seed, (uint32_t)(i >> 7), STREAM_INIT << 24, 0u,
                 (uint32_t)replica, o);
            uint32_t bit = (o[(i >> 5) & 3] >> (i & 31)) & 1u;
            s->spin[i] = bit ? 1 : -1;
        }
    }
    return s;
}

void kmco_destroy(kmco_state *s)
{
    if (!s) return;
    free(s->spin); free(s->clk_sum); free(s->clk_comp); free(s->dom_events);
    free(s->bits); free(s->cls); free(s->colour);
    free(s);
}

/* -------------------------------------------------------- domain process */

static void set_class(kmco_state *s, int k, int c, int64_t n[10])
{
    s->cls[k] = (int8_t)c;
    s->bits[(size_t)c * s->nw + (k >> 6)] |= (uint64_t)1 << (k & 63);
    n[c] += 1;
}

static void clear_class(kmco_state *s, int k, int64_t n[10])
{
    int c = s->cls[k];
    s->bits[(size_t)c * s->nw + (k >> 6)] &= ~((uint64_t)1 << (k & 63));
    n[c] -= 1;
}

/* Local index of the j-th member (0-based, ascending local index) of class c. */
static int select_member(const kmco_state *s, int c, uint64_t j)
{
    const uint64_t *b = s->bits + (size_t)c * s->nw;
    for (int q = 0; q < s->nw; ++q) {
        uint64_t cnt = (uint64_t)__builtin_popcountll(b[q]);
        if (j < cnt) {
            uint64_t word = b[q];
            for (int bit = 0; bit < 64; ++bit) {
                if ((word >> bit) & 1u) {
                    if (j == 0) return q * 64 + bit;
                    --j;
                }
            }
        }
        j -= cnt;
    }
    return -1;
}

static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/* nu_theta = d ln(1 - R_w/n_d)/d theta for the current class counts. */
static void null_score(const kmco_state *s, const int64_t n[10], double nu[2])
{
    double Rw = 0.0, RJ = 0.0, Rh = 0.0;
    for (int c = 0; c < 10; ++c) {
        double nc = (double)n[c];
        Rw += nc * s->w[c];
        RJ += nc * (s->w[c] * s->gJ[c]);
        Rh += nc * (s->w[c] * s->gh[c]);
    }
    double den = (double)s->nd - Rw;
    if (den > 0.0) {
        nu[0] = -RJ / den;
        nu[1] = -Rh / den;
    } else {
        nu[0] = 0.0;
        nu[1] = 0.0;
    }
}

/* Magnitude of the same null term before cancellation:
 * sum_c n_c |w_c g_c| / (n_d - R_w) per theta, the sum of the absolute values
 * of the per-class terms that make up nu_theta. */
static void null_abs(const kmco_state *s, const int64_t n[10], double mag[2])
{
    double Rw = 0.0, AJ = 0.0, Ah = 0.0;
    for (int c = 0; c < 10; ++c) {
        double nc = (double)n[c];
        Rw += nc * s->w[c];
        AJ += nc * fabs(s->w[c] * s->gJ[c]);
        Ah += nc * fabs(s->w[c] * s->gh[c]);
    }
    double den = (double)s->nd - Rw;
    if (den > 0.0) {
        mag[0] = AJ / den;
        mag[1] = Ah / den;
    } else {
        mag[0] = 0.0;
        mag[1] = 0.0;
    }
}

static void check_classes(kmco_state *s, int oy, int ox, const int64_t n[10])
{
    int64_t cnt[10] = {0};
    for (int k = 0; k < s->nd; ++k) {
        int c = site_class(s, oy + k / s->Bx, ox + k % s->Bx);
        cnt[c]++;
        if (c != s->cls[k]) s->check_fail++;
        if (!((s->bits[(size_t)c * s->nw + (k >> 6)] >> (k & 63)) & 1u))
            s->check_fail++;
    }
    for (int c = 0; c < 10; ++c)
        if (cnt[c] != n[c]) s->check_fail++;
}

/* The site an event at x < R picks (R1): the rate class c is the first
 * whose prefix sum exceeds x, the member the j-th of that class in ascending
 * local index, j = floor((x - P_{c-1}) / r_c).  Returns the local index. */
static int pick_site(const kmco_state *s, const int64_t n[10], uint64_t x, int *cls)
{
    int c = 0;
    uint64_t P = 0;
    while (x >= P + (uint64_t)n[c] * s->r[c]) {
        P += (uint64_t)n[c] * s->r[c];
        ++c;
    }
    uint64_t j = (x - P) / s->r[c];
    *cls = c;
    return select_member(s, c, j);
}

/* Flips local site k of domain d (origin oy, ox) and moves it and its
 * neighbours inside the domain to their new classes; halo sites stay. */
static void flip_site(kmco_state *s, int d, int oy, int ox, int k, int64_t n[10], int flags)
{
    const int Bx = s->Bx, By = s->By, L = s->L;
    int gy = oy + k / Bx, gx = ox + k % Bx;
    int aff[5], na = 0;
    const int dy[5] = {0, 0, 0, -1, 1}, dx[5] = {0, -1, 1, 0, 0};
    for (int a = 0; a < 1 + s->z; ++a) {
        int yy = wrap(gy + dy[a], s->Ly), xx = wrap(gx + dx[a], L);
        int ry = wrap(yy - oy, s->Ly), rx = wrap(xx - ox, L);
        if (ry >= By || rx >= Bx) continue; /* halo site: frozen */
        int kk = ry * Bx + rx, dup = 0;
        for (int b = 0; b < na; ++b) dup |= aff[b] == kk;
        if (!dup) aff[na++] = kk;
    }
    for (int a = 0; a < na; ++a) clear_class(s, aff[a], n);
    s->spin[gy * L + gx] = (int8_t)-s->spin[gy * L + gx];
    for (int a = 0; a < na; ++a)
        set_class(s, aff[a], site_class(s, oy + aff[a] / Bx, ox + aff[a] % Bx), n);
    s->events++;
    s->dom_events[d]++;
    if (flags & KMCO_F_CHECK) check_classes(s, oy, ox, n);
}

/* Runs one domain process: N_I ticks of domain d with everything outside the
 * domain held fixed (the halo is read from the lattice, which no other
 * domain changes during the visit). */
static void visit_domain(kmco_state *s, int d, int visit, int64_t w,
                         int flags, double *score, double *score_abs)
{
    const int Bx = s->Bx, By = s->By;
    const int oy = (d / s->NTx) * By, ox = (d % s->NTx) * Bx;
    int64_t n[10] = {0};
    memset(s->bits, 0, sizeof(uint64_t) * 10 * (size_t)s->nw);
    for (int k = 0; k < s->nd; ++k)
        set_class(s, k, site_class(s, oy + k / Bx, ox + k % Bx), n);

    uint64_t m_null = 0; /* null ticks since the last event (score) */
    for (int t = 0; t < s->NI; ++t) {
        uint64_t R = 0;
        for (int c = 0; c < 10; ++c) R += (uint64_t)n[c] * s->r[c];

        uint32_t o[4];
        draw(s->seed, (uint32_t)t,
             (uint32_t)d | ((uint32_t)visit << 20) | (STREAM_TICK << 24),
             (uint32_t)w, (uint32_t)s->replica, o);
        int32_t redraws = 0;
        uint32_t slot = kmco_tick_slot(s->seed, s->replica, w, d, visit,
                                       (uint32_t)t, (uint32_t)s->nd, &redraws);
        if (redraws) {
            s->retry_ticks++;
            s->retry_draws += redraws;
        }
        uint64_t x = ((uint64_t)slot << 32) | o[0];
        if (x >= R) { /* null tick: the selected site is not flipped */
            ++m_null;
            continue;
        }
        /* event: rate class by prefix, then member j of that class */
        int c;
        int k = pick_site(s, n, x, &c);

        if (flags & KMCO_F_SCORE) {
            if (m_null) {
                double nu[2];
                null_score(s, n, nu);
                score[0] += (double)m_null * nu[0];
                score[1] += (double)m_null * nu[1];
                if (score_abs) {
                    double mag[2];
                    null_abs(s, n, mag);
                    score_abs[0] += (double)m_null * mag[0];
                    score_abs[1] += (double)m_null * mag[1];
                }
            }
            score[0] += s->gJ[c];
            score[1] += s->gh[c];
            if (score_abs) {
                score_abs[0] += fabs(s->gJ[c]);
                score_abs[1] += fabs(s->gh[c]);
            }
        }
        m_null = 0;

        /* residence time -ln(u)/R_w, u in (0, 1] from 53 bits of words 3:2 */
        uint64_t u53 = ((uint64_t)o[3] << 21) | (o[2] >> 11);
        double u = (double)(u53 + 1) * 0x1p-53;
        double dt = -log(u) * 4294967296.0 / (double)R;
        neumaier_add(&s->clk_sum[d], &s->clk_comp[d], dt);

        /* the flipped site and its neighbours inside the domain change class */
        flip_site(s, d, oy, ox, k, n, flags);
    }
    if ((flags & KMCO_F_SCORE) && m_null) {
        double nu[2];
        null_score(s, n, nu);
        score[0] += (double)m_null * nu[0];
        score[1] += (double)m_null * nu[1];
        if (score_abs) {
            double mag[2];
            null_abs(s, n, mag);
            score_abs[0] += (double)m_null * mag[0];
            score_abs[1] += (double)m_null * mag[1];
        }
    }
    s->steps += s->NI;
}

/* The time-slice form of a domain process (R7): rejection-free events of
 * domain d until its clock would pass tau. */
static void visit_slice(kmco_state *s, int d, int visit, int64_t w, int flags)
{
    const int Bx = s->Bx, By = s->By;
    const int oy = (d / s->NTx) * By, ox = (d % s->NTx) * Bx;
    const uint32_t c1 = (uint32_t)d | ((uint32_t)visit << 20);
    int64_t n[10] = {0};
    memset(s->bits, 0, sizeof(uint64_t) * 10 * (size_t)s->nw);
    for (int k = 0; k < s->nd; ++k)
        set_class(s, k, site_class(s, oy + k / Bx, ox + k % Bx), n);
    double t = 0.0;
    for (uint32_t ev = 0;; ++ev) {
        uint64_t R = 0;
        for (int c = 0; c < 10; ++c) R += (uint64_t)n[c] * s->r[c];
        if (R == 0) break; /* no event can happen: the state holds to tau */
        uint32_t o[4];
        draw(s->seed, ev, c1 | (STREAM_SLICE << 24), (uint32_t)w, (uint32_t)s->replica, o);
        uint64_t u53 = ((uint64_t)o[3] << 21) | (o[2] >> 11);
        double u = (double)(u53 + 1) * 0x1p-53;
        double dt = (-kmco_slice_log(u) * 4294967296.0) / (double)R;
        double tn = t + dt;
        if (tn > s->tau) break; /* the next event falls after the slice */
        t = tn;
        uint64_t x = slice_select(s->seed, s->replica, w, c1, ev, R, o[1], o[0]);
        int c;
        int k = pick_site(s, n, x, &c);
        flip_site(s, d, oy, ox, k, n, flags);
    }
    neumaier_add(&s->clk_sum[d], &s->clk_comp[d], s->tau);
}

static void observe(const kmco_state *s, kmco_record *r)
{
    int64_t M = 0, Bs = 0;
    for (int y = 0; y < s->Ly; ++y)
        for (int x = 0; x < s->L; ++x) {
            int8_t v = spin_at(s, y, x);
            M += v;
            Bs += v * spin_at(s, y, x + 1);
            if (s->z == 4) Bs += v * spin_at(s, y + 1, x);
        }
    double tot = 0.0;
    for (int d = 0; d < s->ND; ++d) tot += s->clk_sum[d] + s->clk_comp[d];
    r->sweep = s->sweep;
    r->M = M;
    r->B = Bs;
    r->events = s->events;
    r->steps = s->steps;
    r->t = tot / (double)s->ND;
}

int64_t kmco_run(kmco_state *s, int64_t n_sweeps, int32_t record_every,
                 int32_t flags, kmco_record *rec, int64_t rec_cap,
                 double *score, double *score_abs)
{
    if (!s || n_sweeps < 0 || record_every < 1) return -1;
    if ((flags & KMCO_F_SCORE) && !score) return -1;
    if ((flags & KMCO_F_SCORE) && s->tau > 0.0) return -1; /* no score for R7 */
    const int nc = s->ncol;
    int64_t nrec = 0;
    double dummy[2], dummy_abs[2];
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const int64_t w = s->sweep;
        int order[18], visit[18], nphase;
        if (s->sched == KMCO_SCHED_PALINDROME) {
            /* 0 1 .. n-1, then the same colours backwards (second visits) */
            nphase = 2 * nc;
            for (int p = 0; p < nc; ++p) {
                order[p] = p;
                visit[p] = 0;
                order[nphase - 1 - p] = p;
                visit[nphase - 1 - p] = 1;
            }
        } else {
            int32_t perm[9];
            kmco_perm_from_index_n(
                kmco_schedule_index_n(s->seed, s->replica, w, factorial(nc)), nc, perm);
            nphase = nc;
            for (int p = 0; p < nc; ++p) {
                order[p] = perm[p];
                visit[p] = 0;
            }
        }
        double *sc = (flags & KMCO_F_SCORE)
                         ? (nrec < rec_cap ? score + 2 * nrec : dummy)
                         : NULL;
        double *sa = (flags & KMCO_F_SCORE) && score_abs
                         ? (nrec < rec_cap ? score_abs + 2 * nrec : dummy_abs)
                         : NULL;
        for (int p = 0; p < nphase; ++p) {
            for (int d = 0; d < s->ND; ++d)
                if (s->colour[d] == order[p]) {
                    if (s->tau > 0.0)
                        visit_slice(s, d, visit[p], w, flags);
                    else
                        visit_domain(s, d, visit[p], w, flags, sc, sa);
                }
        }
        s->sweep++;
        if ((i + 1) % record_every == 0) {
            if (nrec < rec_cap && rec) observe(s, &rec[nrec]);
            ++nrec;
        }
    }
    return nrec;
}

int kmco_get_spins(const kmco_state *s, int8_t *out)
{
    if (!s || !out) return -1;
    memcpy(out, s->spin, (size_t)s->L * s->Ly);
    return 0;
}

int kmco_get_domain_clocks(const kmco_state *s, double *sum, double *comp)
{
    if (!s) return -1;
    if (sum) memcpy(sum, s->clk_sum, sizeof(double) * s->ND);
    if (comp) memcpy(comp, s->clk_comp, sizeof(double) * s->ND);
    return 0;
}

int kmco_get_domain_events(const kmco_state *s, int64_t *events)
{
    if (!s || !events) return -1;
    memcpy(events, s->dom_events, sizeof(int64_t) * s->ND);
    return 0;
}

int64_t kmco_check_failures(const kmco_state *s) { return s ? s->check_fail : -1; }

int kmco_get_retries(const kmco_state *s, int64_t *ticks, int64_t *draws)
{
    if (!s) return -1;
    if (ticks) *ticks = s->retry_ticks;
    if (draws) *draws = s->retry_draws;
    return 0;
}

int64_t kmco_count_retry_ticks(uint64_t seed, int32_t replica, int64_t sweep,
                               int32_t domain, int32_t visit, uint32_t n_ticks,
                               uint32_t n)
{
    int64_t k = 0;
    for (uint32_t t = 0; t < n_ticks; ++t) {
        int32_t r = 0;
        (void)kmco_tick_slot(seed, replica, sweep, domain, visit, t, n, &r);
        k += r > 0;
    }
    return k;
}

int kmco_get_partition(const kmco_state *s, int32_t *colour, int32_t *n_colours)
{
    if (!s) return -1;
    if (colour) memcpy(colour, s->colour, sizeof(int32_t) * s->ND);
    if (n_colours) *n_colours = s->ncol;
    return 0;
}
