/*
 * kmc.h -- C-ABI of libkmc, the MI355X (gfx950) implementation of
 * domain-decomposed sequential-update kinetic Monte Carlo
 * (Nilmeier & Marian, "A rigorous sequential update strategy for parallel
 * kinetic Monte Carlo simulation").
 *
 * The model (Appendix A): a periodic L x L Ising lattice with energy
 *   H = -J sum_<ij> s_i s_j - h sum_i s_i        (Eq. (Hamiltonian Definition),
 *                                                 extended by the field h),
 * single-spin-flip rates w = Barker 1/(1+e^{dE/T}) as in Eq. (Glauber_TM),
 * or Metropolis min(1, e^{-dE/T}).
 *
 * The method (Sec. 2.2): the lattice is cut into equal square domains of
 * side B (fixed for the run, Fig. 1).  A domain process runs N_I ticks of the
 * single-site kernel with the neighbouring spins (the halo) frozen.  Domains
 * are coloured by a 4-colour checkerboard; domains of one colour do not
 * interact and run concurrently.  Each sweep visits the colours in a
 * schedule drawn uniformly from the 4! orders (Eq. (schedule), Eq. (sum of
 * sequential tms)) or in the self-reverse palindrome ABCDDCBA, so detailed
 * balance holds at sweep endpoints (Eq. (general reversibility condition)).
 * Within a tick, event choice is n-fold way over 10 rate classes with Q32
 * integer rates; each accepted event advances the domain clock by -ln(u)/R
 * (Eq. (Poisson Distribution) and the residence time tau_S = 1/R).
 *
 * Conventions for every call:
 *  - Every call returns a kmc_status; nothing is thrown or aborted across
 *    the ABI.  On failure the context (when there is one) keeps a message
 *    readable with kmc_last_error().
 *  - A context is bound to one device and one HIP stream and is not
 *    thread-safe.  Calls that launch work are asynchronous on that stream
 *    unless stated otherwise.
 *  - Inputs are copied; outputs are caller-owned memory.
 *  - Lattices passed in and out are row-major int8 with values +1 / -1
 *    (the device copy is held domain by domain, which no call exposes).
 */
#ifndef KMC_H
#define KMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kmc_ctx kmc_ctx;

typedef enum {
    KMC_OK = 0,
    KMC_EINVAL = -1,        /* invalid argument or descriptor               */
    KMC_ENOMEM = -2,        /* device or host allocation failed             */
    KMC_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed   */
    KMC_ESTATE = -4,        /* call not valid in the context's state        */
    KMC_EUNSUPPORTED = -5   /* valid for the method, not for this library   */
} kmc_status;

/* values of the descriptor fields rate_model, schedule and init (held there
 * as int32_t) */
typedef enum { KMC_RATE_METROPOLIS = 0, KMC_RATE_BARKER = 1 } kmc_rate_model;
typedef enum { KMC_SCHED_RANDOM_PERM = 0, KMC_SCHED_PALINDROME = 1 } kmc_schedule;
typedef enum { KMC_INIT_RANDOM = 0, KMC_INIT_ALL_UP = 1, KMC_INIT_GIVEN = 2 } kmc_init;

/* flags of kmc_run_schedule */
#define KMC_F_CHECKPOINT 0x1u  /* save the start state for kmc_backward_score */
#define KMC_F_PERSISTENT 0x2u  /* one persistent launch: one wavefront owns a
                                  replica and runs all of its sweeps          */
#define KMC_F_GRAPH 0x4u       /* replay from a captured hipGraph: alone, G
                                  phase-by-phase sweeps per graph; with
                                  KMC_F_PERSISTENT, one persistent launch of
                                  record_every sweeps per graph                */
#define KMC_F_NO_MULTI 0x8u    /* with KMC_F_PERSISTENT: never run four domain
                                  processes per wavefront                      */
#define KMC_F_MULTI 0x20u      /* with KMC_F_PERSISTENT: run replicas with
                                  domains of at most 16x16 four domain
                                  processes per wavefront even in small batches
                                  (default: only when the batch is large)      */
#define KMC_F_SCORE 0x40u      /* accumulate the likelihood-ratio score of
                                  every tick while the run proceeds (the
                                  backward call then only copies it out)      */
#define KMC_F_FLOW 0x100u      /* phase-by-phase form as dataflow launches of
                                  up to 64 sweeps: each domain visit starts as
                                  soon as the visits of its neighbouring
                                  domains that precede it in the sequential
                                  order (Eq. (schedule)) have finished, so
                                  non-adjacent colours and consecutive sweeps
                                  overlap; results equal
                                  the phase launches bit for bit.  Not with
                                  KMC_F_PERSISTENT (KMC_EINVAL).  A wait that
                                  never ends is cut off and reported as
                                  KMC_EDEVICE by kmc_observables              */
#define KMC_F_TIMING 0x80u     /* record HIP events around every launch of the
                                  hot kernel (the phase kernel, or the
                                  persistent kernels), read by kmc_get_timing */
#define KMC_F_RESIDENT 0x200u  /* resident form: one workgroup per replica keeps
                                  the whole lattice, its class codes and
                                  per-row class counts in LDS for every sweep
                                  of the call (one launch; no staging per
                                  visit).  Needs 3 <= L <= 128 and at most 16
                                  domains along x for every replica; the only
                                  form for domains wider or taller than 64
                                  sites (the others return
                                  KMC_EUNSUPPORTED for them).  Not with
                                  KMC_F_PERSISTENT, KMC_F_FLOW or KMC_F_GRAPH
                                  (KMC_EINVAL)                                */
/* flags of kmc_backward_score and kmc_observables */
#define KMC_F_DEVICE_OUT 0x10u /* output pointer is device memory; the copy is
                                  enqueued on the context stream, no sync     */

/* One replica.  Domains are `tile` = Bx sites wide and `tile_rows` = By high
 * (0: By = Bx), the paper's fixed equal partition (Sec. 2.2, Fig. 1):
 * 1 <= Bx, By <= 128, L % Bx == 0, L % By == 0.  Square domains with L/B even
 * give the 4-colour checkerboard, By = L gives vertical stripes, Bx = By = L
 * the unpartitioned lattice as one periodic domain (N_D = 1, the paper's
 * reference dynamics); odd domain counts are allowed too.  The domain grid is
 * coloured per axis (1 colour for one domain, 2 for an even count, 3 for an
 * odd count) and the schedule runs its colours in a uniformly drawn order
 * (Eq. (schedule)) or as a palindrome.  An axis with a single domain wraps
 * inside the domain and needs a side >= 3.  Domains of 65 to 128 sites a
 * side (L <= 128) run in the resident form only (KMC_F_RESIDENT).  steps_per_visit = N_I ticks per
 * domain process (Sec. 2.2); 0 selects Bx*By (one Monte Carlo step per site
 * per visit). */
typedef struct {
    double J, h, T;            /* coupling, field, k_B T (> 0)              */
    int32_t L;                 /* lattice side                              */
    int32_t tile;              /* domain width Bx                           */
    int32_t steps_per_visit;   /* N_I, >= 0                                 */
    int32_t rate_model;        /* KMC_RATE_*                                */
    int32_t schedule;          /* KMC_SCHED_*                               */
    int32_t init;              /* KMC_INIT_*                                */
    int32_t tile_rows;         /* domain height By; 0 means By = Bx         */
    int32_t dims;              /* 0 or 2: the periodic L x L lattice; 1: the
                                  periodic ring of L sites (the paper's 1D
                                  system, Sec. 3.1, Eq. (1D partitions)),
                                  cut into L / tile domains of `tile`
                                  consecutive sites (1 <= tile <= 64,
                                  tile_rows 0 or 1); a site's class counts
                                  its up neighbours among left and right and
                                  dE = 2 s (J (2k - 2) + h).  Rings run in
                                  the phase, dataflow and persistent forms
                                  (the resident form: KMC_EUNSUPPORTED)     */
    double time_slice;         /* > 0: the rejection-free variant with fixed
                                  time slices (the synchronous time-horizon
                                  methods the paper contrasts its own with,
                                  Sec. 1): each domain process runs its
                                  continuous-time kinetics (site flip rates
                                  w, residence times -ln(u)/R, every event
                                  real) for this long instead of N_I ticks;
                                  the domain clocks advance by time_slice
                                  per visit and `steps` stays 0.  Event k
                                  of a visit draws Philox counter (k, domain
                                  | visit<<20 | 16<<24, sweep, replica):
                                  words 3:2 the waiting time, words 1:0 the
                                  event by Lemire's 64-bit multiply with
                                  rejection (redraws on streams 17..28).
                                  All replicas of a context use it or none
                                  (KMC_EINVAL); phase, dataflow and
                                  one-domain-per-wavefront persistent forms
                                  only; no score, checkpoint or resident form
                                  (KMC_EUNSUPPORTED).  0: the tick chain   */
} kmc_replica_desc;

/* Observables at a sweep endpoint, the only points where statistics are
 * valid (Sec. 2.3). */
typedef struct {
    int64_t sweep;   /* sweeps completed since kmc_init_lattice            */
    int64_t M;       /* sum of spins                                        */
    int64_t B;       /* sum over right and down bonds of s_i s_j            */
    int64_t events;  /* accepted flips since kmc_init_lattice               */
    int64_t steps;   /* ticks since kmc_init_lattice: N_I per domain visit,
                        the integer time of Eq. (CK_parallel in s)          */
    double t;        /* mean over domains of the per-domain event clocks    */
} kmc_record;

/* Routes the library's device allocations through a caller allocator (for
 * instance a framework's caching allocator).  NULL restores hipMalloc /
 * hipFree.  Applies to contexts created afterwards. */
typedef void *(*kmc_alloc_fn)(size_t bytes, void *user);
typedef void (*kmc_free_fn)(void *ptr, void *user);
kmc_status kmc_set_device_allocator(kmc_alloc_fn alloc, kmc_free_fn free_fn,
                                    void *user);

/* Bound, in polls, of each wait of the dataflow sweeps (KMC_F_FLOW) of this
 * context; default 2^24 (a poll every few microseconds: about a minute).
 * For callers that test the failure path:
 * a wait that exceeds it gives up, the run is reported as failed
 * (KMC_EDEVICE from kmc_observables, or from kmc_backward_score for a replay
 * with host output), and the context's results stay void from then on.
 * max_polls < 0: KMC_EINVAL. */
kmc_status kmc_set_wait_limit(kmc_ctx *c, int64_t max_polls);

/* Exact propagation (Sec. 3.1: reference values from evolving the
 * probability vector with Eq. (CK_parallel in s)) of one replica's
 * distribution over all 2^N spin configurations (N = L*L, or L for a ring)
 * through n_sweeps sweeps of the parallel transition matrix T_PAR: the
 * uniform mixture over all orders of the colours (Eq. (sum of sequential
 * tms); at most 4 colours, else KMC_EUNSUPPORTED), or the palindrome.  State
 * index s: bit y*L + x set when spin (y, x) is +1.  p: device array of 2^N
 * doubles, the start distribution in, the result out; work: device array of
 * 3 * 2^N doubles (caller-owned scratch; the call allocates nothing).  p and
 * work must not overlap.  N <= 26, else KMC_EINVAL;
 * the descriptor's init and seed play no part.  Flags: KMC_EXACT_QUANTISED
 * uses the Q32 rates the kMC path flips with (else the real w).  Enqueued on
 * hip_stream (NULL: the null stream); asynchronous.  A verification tool:
 * state histograms of many replicas can be compared with it. */
#define KMC_EXACT_QUANTISED 0x1u
kmc_status kmc_exact_sweeps(const kmc_replica_desc *d, double *p, double *work,
                            int64_t n_sweeps, uint32_t flags, void *hip_stream);

/* kmc_exact_sweeps for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same propagation, with the three work vectors
 * in a buffer inside the library, 3 * 2^16 doubles (1.5 MiB), which every
 * device the library runs on holds until the process ends.  So N <= 16:
 * larger systems return KMC_EINVAL before anything is enqueued.  p, flags,
 * hip_stream and the errors are those of kmc_exact_sweeps; the call
 * allocates nothing.  Every call on one device shares that device's buffer:
 * calls whose work overlaps on one device (on different streams, or from
 * different threads, before the previous one has finished) race and give
 * undefined results.  Each call writes every entry of the buffer it reads,
 * so nothing carries over from the previous call. */
kmc_status kmc_exact_sweeps_static(const kmc_replica_desc *d, double *p, int64_t n_sweeps,
                                   uint32_t flags, void *hip_stream);

/* Per-class rate table of one replica (Appendix A, Eq. (Glauber_TM)).
 * Class c = 5*[s=+1] + k, k = number of up neighbours (0..4), flip energy
 * dE = 2 s (J (2k-4) + h).  r[c] = min(2^32, floor(w 2^32 + 1/2)) is the Q32
 * rate used for every decision; w, gJ = d ln w/dJ, gh = d ln w/dh are FP64.
 * Host-only, no device needed.  Returns KMC_EINVAL for T <= 0, a non-finite
 * parameter or an unknown model. */
kmc_status kmc_rate_table(double J, double h, double T, int32_t rate_model,
                          uint64_t r[10], double w[10], double gJ[10],
                          double gh[10]);

/* Creates a context holding n_rep replicas on the current HIP device and
 * initialises their lattices (Sec. 3: the paper's systems are periodic
 * square lattices with a given start configuration).
 *   d           host array of n_rep descriptors (copied)
 *   seed        64-bit key of the counter-based generator; every random
 *               number is Philox4x32-10(key = seed, counter = (tick,
 *               domain | visit<<20 | stream<<24, sweep, replica))
 *   given_spins host int8 array with sum over replicas of L*L values (L for
 *               a ring), replicas concatenated in order; read only for
 *               replicas whose init is KMC_INIT_GIVEN, may be NULL otherwise
 *   hip_stream  hipStream_t for all work of this context; NULL = null stream
 * Validation failures return KMC_EINVAL and create nothing; *out is set only
 * on success.  Synchronises the stream before returning. */
kmc_status kmc_init_lattice(kmc_ctx **out, const kmc_replica_desc *d,
                            int32_t n_rep, uint64_t seed,
                            const int8_t *given_spins, void *hip_stream);

/* Runs n_sweeps schedule sweeps of every replica (Eq. (schedule): each sweep
 * visits every domain once, twice for the palindrome, with a new schedule
 * per sweep).  After the i-th sweep of this call (1-based) a record is
 * appended for every replica when i % record_every == 0.  Asynchronous.
 * Flags: KMC_F_CHECKPOINT keeps the start state so that kmc_backward_score
 * can replay this call; KMC_F_PERSISTENT selects the one-launch batched
 * kernel; KMC_F_GRAPH replays the phase-by-phase launches from a hipGraph.
 * All paths produce bit-identical lattices, events and records.
 * Errors: KMC_EINVAL (n_sweeps < 0, record_every < 1), KMC_ENOMEM, KMC_EDEVICE. */
kmc_status kmc_run_schedule(kmc_ctx *c, int64_t n_sweeps, int32_t record_every,
                            uint32_t flags);
/* All execution forms give bit-identical results; KMC_F_MULTI and
 * KMC_F_NO_MULTI only change how the work is laid out on the GPU. */

/* Endpoint statistics (Sec. 2.3: samples are valid only at the end of
 * domain processes, here the ends of whole sweeps; the paper's ensemble
 * averages, Eq. (time dependent averages), are formed from them over
 * replicas).  Copies all records so far: out[rep * capacity + k] for replica
 * rep and record k < min(capacity, *n_rec_out).  *n_rec_out receives the
 * number of records per replica.  out may be NULL to query the count.  Host
 * output synchronises the stream and returns KMC_EDEVICE when a dataflow
 * wait of an earlier run gave up (the results are void); with
 * KMC_F_DEVICE_OUT out is device memory and the copy is only enqueued. */
kmc_status kmc_observables(kmc_ctx *c, kmc_record *out, int64_t capacity,
                           int64_t *n_rec_out, uint32_t flags);

/* Likelihood-ratio path score of the last kmc_run_schedule call made with
 * KMC_F_CHECKPOINT or KMC_F_SCORE.  This extends the paper, which has no
 * derivatives: it is d ln P(path)/d(J, h) of the tick chain the paper
 * defines (Sec. 2.2, App. A Eq. (Glauber_TM)), whose average against an
 * observable gives the gradient of that observable's expectation.  With KMC_F_SCORE the run accumulated the
 * score itself and this call copies it out.  Otherwise the call replays the
 * run from its saved start state with a dedicated kernel (bit-exact: every
 * decision is integer) and accumulates, for every tick, d ln P/d(J, h) of the
 * tick chain (an event of class c adds d ln w_c/d theta; a null tick adds
 * d ln(1 - R_w/n_d)/d theta with R_w the domain's total FP64 rate).  Output
 * score[(rep * capacity + k) * 2 + {0: J, 1: h}] for interval k: the ticks of
 * sweeps (k*record_every, (k+1)*record_every] of that call; the number of
 * intervals is ceil(n_sweeps / record_every) and must be <= capacity.
 * The live state of the context is not changed.  KMC_ESTATE without a
 * checkpoint or score.  Host output synchronises; KMC_F_DEVICE_OUT enqueues
 * only. */
kmc_status kmc_backward_score(kmc_ctx *c, double *score, int64_t capacity,
                              uint32_t flags);

/* Copies replica `replica`'s lattice (L*L int8, row-major; L for a ring) to
 * host memory.
 * Synchronises; KMC_EDEVICE when a dataflow wait of an earlier run gave up. */
kmc_status kmc_get_spins(kmc_ctx *c, int32_t replica, int8_t *out);

/* Copies the per-domain clock sums and their compensation terms (N_D
 * doubles each, domain d = ty*(L/B) + tx) and per-domain event counts
 * (N_D int64) of one replica to host memory; any pointer may be NULL.
 * Synchronises; KMC_EDEVICE when a dataflow wait of an earlier run gave up. */
kmc_status kmc_get_domain_state(kmc_ctx *c, int32_t replica, double *clk_sum,
                                double *clk_comp, int64_t *events);

/* The per-domain clocks alone (each domain advances its own clock by the
 * residence times of its events, Eq. (Poisson Distribution); the replica
 * time is their mean): t and comp receive N_D doubles each, the compensated
 * clock sums and their compensation terms, as kmc_get_domain_state with no
 * event counts; either may be NULL.  Errors as kmc_get_domain_state.
 * Synchronises. */
kmc_status kmc_get_domain_clocks(kmc_ctx *c, int32_t replica, double *t, double *comp);

/* Number of replicas, and the number of domains of one replica. */
kmc_status kmc_get_info(kmc_ctx *c, int32_t replica, int32_t *n_rep,
                        int32_t *n_domains);

/* Instrumentation for measuring the method's kernels, not part of it: the
 * summed duration in milliseconds of the hot-kernel launches recorded since
 * the last call (runs made with KMC_F_TIMING) and their number.  Events are
 * recorded on the context stream around the launches; synchronises. */
kmc_status kmc_get_timing(kmc_ctx *c, double *ms_total, int64_t *n_launches);

/* Message of the last failed call on c (never NULL). */
const char *kmc_last_error(const kmc_ctx *c);

/* Releases every device buffer of c after synchronising its stream. */
void kmc_destroy(kmc_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
