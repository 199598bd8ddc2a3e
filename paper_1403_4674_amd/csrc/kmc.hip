// kmc.hip -- host side of libkmc: the C-ABI declared in include/kmc.h.
//
// Owns the device buffers of a context, validates descriptors, builds the
// per-replica Q32 rate tables on the host (the GPU never evaluates exp for a
// decision), and enqueues the kernels of kmc_device.h on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "kmc.h"
#include "kmc_device.h"
#include "kmc_multi.h"
#include "kmc_resident.h"
#include "kmc_exact.h"

using kmcdev::Ctl;
using kmcdev::MItem;
using kmcdev::Dom;
using kmcdev::KParams;
using kmcdev::Rates;
using kmcdev::Record;
using kmcdev::Rep;
using kmcdev::RepAcc;

static_assert(sizeof(kmc_record) == sizeof(Record), "record layout");

// ------------------------------------------------------------ allocation

static kmc_alloc_fn g_alloc = nullptr;
static kmc_free_fn g_free = nullptr;
static void *g_alloc_user = nullptr;

extern "C" kmc_status kmc_set_device_allocator(kmc_alloc_fn alloc, kmc_free_fn free_fn,
                                               void *user) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return KMC_EINVAL;
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_user = user;
    return KMC_OK;
}

struct kmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;       // caller's stream, NULL = null stream
    hipStream_t graph_stream = nullptr; // owned, for graph replay on the null stream
    kmc_alloc_fn alloc = nullptr;
    kmc_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;

    int32_t n_rep = 0;
    uint64_t seed = 0;
    std::vector<kmc_replica_desc> desc;
    std::vector<Rep> reps;
    std::vector<Rates> rates;
    int64_t spin_bytes = 0;
    int32_t n_dom = 0;
    int32_t n_tasks = 0, n_tasks32 = 0;
    // persistent queues per row-mask width: [team..., solo...]
    int32_t n_team[2] = {0, 0}, n_solo[2] = {0, 0};
    // multi-slot items (domains <= 16x16): [workgroup items..., wavefront items...]
    std::vector<MItem> m_items;
    int32_t n_m_wg = 0, n_m_wave = 0;
    MItem *d_items = nullptr;
    // the same replicas without the multi-slot form (KMC_F_NO_MULTI)
    int32_t nm_team[2] = {0, 0}, nm_solo[2] = {0, 0};
    int32_t *d_order_nm = nullptr;
    bool multi_auto = false;  // the multi-slot items keep >= 2 wavefronts per SIMD
    // per row-mask width (B <= 32, B > 32): some replica is one periodic
    // domain, so the launches of that width take the wrap-around kernels
    bool wrap[2] = {false, false};
    // every replica runs the time-slice variant (time_slice > 0)
    bool slice = false;
    int n_phase = 1;  // colour phases per sweep, the largest over the replicas

    Rep *d_reps = nullptr;
    Rates *d_rates = nullptr;
    int8_t *d_spins = nullptr;   // every replica's lattice, domain by domain
    uint64_t *d_edges = nullptr; // edge columns of every domain [n_dom][2]
    int8_t *d_stage = nullptr;   // one row-major lattice (given starts, copies out)
    Dom *d_dom = nullptr;
    RepAcc *d_acc = nullptr;
    Record *d_rec = nullptr;
    Ctl *d_ctl = nullptr;
    int64_t *d_done = nullptr;  // per-domain visit counters of the one-launch sweeps
    // per-sweep slots of a dataflow launch (allocated on first use)
    int64_t flow_max_polls = kmcdev::kFlowMaxPolls;  // bound of each dataflow wait
    int64_t *d_flow_acc = nullptr;  // [flow_window][n_rep][3]
    double *d_flow_clk = nullptr;   // [flow_window][n_dom][2]
    bool graph_flow = false;    // the cached phase graph was captured with flow
    bool flow = false;          // phase-by-phase sweeps as one dataflow launch
    int32_t *d_task_rep = nullptr;
    int32_t *d_order = nullptr;
    int64_t rec_cap = 0, n_rec = 0;
    int64_t sweep = 0;

    // checkpoint of the last run made with KMC_F_CHECKPOINT
    bool have_ckpt = false;
    int8_t *c_spins = nullptr;
    Dom *c_dom = nullptr;
    RepAcc *c_acc = nullptr;
    int64_t ck_sweep = 0, ck_n_sweeps = 0;
    int32_t ck_rec_every = 1;
    uint32_t ck_flags = 0;
    // the score of the last run with KMC_F_SCORE, accumulated while it ran
    bool fused_score = false;
    int64_t fused_bins = 0;

    // replay buffers of kmc_backward_score
    int8_t *r_spins = nullptr;
    uint64_t *r_edges = nullptr;
    Dom *r_dom = nullptr;
    RepAcc *r_acc = nullptr;
    Ctl *r_ctl = nullptr;
    double *d_bins = nullptr;
    int64_t bins_cap = 0;
    Record *d_tmp_rec = nullptr;
    int64_t tmp_rec_cap = 0;

    // captured phase-by-phase sweeps, and captured persistent chunks
    hipGraphExec_t graph = nullptr;
    int graph_sweeps = 0;
    hipGraphExec_t pgraph = nullptr;
    int64_t pgraph_chunk = 0;
    uint32_t pgraph_key = 0;

    // KMC_F_TIMING: event pairs around each hot-kernel launch
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
    std::vector<hipEvent_t> ev_pool;

    std::string err;
};

namespace {

struct Fail {
    kmc_status st;
};

void *dev_alloc(kmc_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void *p = nullptr;
    if (c->alloc) {
        p = c->alloc(bytes, c->alloc_user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) {
        c->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
        throw Fail{KMC_ENOMEM};
    }
    return p;
}

void dev_free(kmc_ctx *c, void *p) {
    if (!p) return;
    if (c->free_fn)
        c->free_fn(p, c->alloc_user);
    else
        (void)hipFree(p);
}

template <typename T>
T *alloc_n(kmc_ctx *c, int64_t n) {
    return static_cast<T *>(dev_alloc(c, sizeof(T) * (size_t)std::max<int64_t>(n, 1)));
}

void hip_check(kmc_ctx *c, hipError_t e, const char *what) {
    if (e != hipSuccess) {
        c->err = std::string(what) + ": " + hipGetErrorString(e);
        throw Fail{KMC_EDEVICE};
    }
}

void launch_check(kmc_ctx *c, const char *what) { hip_check(c, hipGetLastError(), what); }

void fail(kmc_ctx *c, kmc_status st, const std::string &msg) {
    if (c) c->err = msg;
    throw Fail{st};
}

// Per-class rates (Appendix A, Eq. (Glauber_TM)); classes c = 5*[s=+1] + k
// with k the up neighbours among z (4 on the square lattice, 2 on the ring;
// classes with k > z stay empty).
kmc_status rate_table(double J, double h, double T, int32_t model, uint64_t r[10],
                      double w[10], double gJ[10], double gh[10], int z = 4) {
    if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(J) || !std::isfinite(h))
        return KMC_EINVAL;
    if (model != KMC_RATE_METROPOLIS && model != KMC_RATE_BARKER) return KMC_EINVAL;
    for (int c = 0; c < 10; ++c) {
        const int up = c / 5, k = c % 5;
        const double s = up ? 1.0 : -1.0;
        const double n = (double)(2 * k - z);
        const double dE = 2.0 * s * (J * n + h);
        double wc, dlw;  // w and d ln w / d dE
        if (model == KMC_RATE_METROPOLIS) {
            if (dE <= 0.0) {
                wc = 1.0;
                dlw = 0.0;
            } else {
                wc = std::exp(-dE / T);
                dlw = -1.0 / T;
            }
        } else {
            wc = 1.0 / (1.0 + std::exp(dE / T));
            dlw = -(1.0 - wc) / T;
        }
        double q = std::floor(wc * 4294967296.0 + 0.5);
        if (q > 4294967296.0) q = 4294967296.0;
        r[c] = (uint64_t)q;
        w[c] = wc;
        gJ[c] = dlw * (2.0 * s * n);
        gh[c] = dlw * (2.0 * s);
    }
    return KMC_OK;
}

// Expected work of one sweep of a replica, for ordering the persistent
// queues (longest first); results do not depend on it.  Events cost about
// six null ticks; the event fraction grows with T (piecewise linear fit of
// equilibrium Metropolis runs at h = 0).
double sweep_cost(const Rep &rp, const kmc_replica_desc &d) {
    static const double Tk[] = {1.0, 1.5, 2.269, 2.5, 3.0, 3.5, 5.0};
    static const double pk[] = {0.001, 0.013, 0.20, 0.32, 0.46, 0.55, 0.70};
    double p = pk[6];
    if (d.T <= Tk[0]) {
        p = pk[0];
    } else {
        for (int i = 1; i < 7; ++i)
            if (d.T <= Tk[i]) {
                p = pk[i - 1] + (pk[i] - pk[i - 1]) * (d.T - Tk[i - 1]) / (Tk[i] - Tk[i - 1]);
                break;
            }
    }
    return (double)rp.NI * rp.ND * rp.visits * (1.0 + 6.0 * p);
}

// The periodic ring of L sites (the paper's 1D system), one row.
bool is_ring(const kmc_replica_desc &d) { return d.dims == 1; }

// Domain height By (tile_rows 0: square domains; 1 on the ring).
int tile_rows_of(const kmc_replica_desc &d) {
    return is_ring(d) ? 1 : (d.tile_rows ? d.tile_rows : d.tile);
}

// Rows of the lattice: L, or 1 on the ring.
int rows_of(const kmc_replica_desc &d) { return is_ring(d) ? 1 : d.L; }

// Colours along an axis of n domains (1, 2 for an even count, 3 for odd),
// and the most domains any one colour holds on it.
int axis_colours(int n) { return n == 1 ? 1 : (n % 2 ? 3 : 2); }
int axis_most(int n) { return n == 1 ? 1 : n / 2; }

// Domains of the largest colour class (phase tasks of the replica).
int max_per_colour(const Rep &rp) { return axis_most(rp.NT) * axis_most(rp.NTy); }

// Replicas the multi-slot kernel runs: square domains of at most 16 x 16 on a
// 4-colour checkerboard.
bool multi_ok(const Rep &rp) {
    return rp.z == 4 && rp.tau == 0.0 && rp.B <= 16 && rp.By == rp.B && rp.NT >= 2 && rp.NT % 2 == 0 &&
           rp.NTy == rp.NT;
}

// Row masks of 64 bits (and 64-lane row scans) when a domain is wider or
// taller than 32.
bool wide(const Rep &rp) { return rp.B > 32 || rp.By > 32; }

// Domains over 64 sites a side: only the resident form holds them.
bool big(const Rep &rp) { return rp.B > 64 || rp.By > 64; }

// Replicas the resident form can hold in one workgroup's LDS.
bool resident_ok(const Rep &rp) {
    return rp.z == 4 && rp.L >= 3 && rp.L <= kmcdev::kResMaxL && rp.NT <= kmcdev::kResMaxNTx;
}

void validate(kmc_ctx *c, const kmc_replica_desc &d, int rho) {
    auto bad = [&](const char *why) {
        fail(c, KMC_EINVAL, "replica " + std::to_string(rho) + ": " + why);
    };
    if (!std::isfinite(d.J) || !std::isfinite(d.h) || !std::isfinite(d.T) || !(d.T > 0))
        bad("J, h must be finite and T > 0");
    if (d.dims != 0 && d.dims != 1 && d.dims != 2) bad("dims must be 0, 1 or 2");
    if (!std::isfinite(d.time_slice) || !(d.time_slice >= 0.0))
        bad("time_slice must be finite and >= 0");
    if (is_ring(d)) {
        if (d.tile_rows != 0 && d.tile_rows != 1) bad("a ring's tile_rows must be 0 or 1");
        if (d.tile < 1 || d.tile > 64) bad("a ring's tile must be in [1, 64]");
        if (d.L < d.tile || d.L % d.tile) bad("L must be a multiple of tile");
        if (d.L == d.tile && d.tile < 3)
            bad("a domain as long as the ring needs tile >= 3 (distinct left and right "
                "neighbours)");
        if (d.L / d.tile > (1 << 20)) bad("more than 2^20 domains");
    }
    const int by = tile_rows_of(d);
    if (d.tile < 1 || d.tile > 128) bad("tile must be in [1, 128]");
    if (by < 1 || by > 128) bad("tile_rows must be 0 or in [1, 128]");
    if ((d.tile > 64 || by > 64) && d.L > kmcdev::kResMaxL)
        bad("domains over 64 sites a side need L <= 128 (resident form)");
    if (d.L < d.tile || d.L % d.tile) bad("L must be a multiple of tile");
    if (rows_of(d) < by || rows_of(d) % by) bad("L must be a multiple of tile_rows");
    if (d.L == d.tile && d.tile < 3)
        bad("a domain as wide as the lattice needs tile >= 3 (distinct left and right "
            "neighbours)");
    if (!is_ring(d) && d.L == by && by < 3)
        bad("a domain as high as the lattice needs tile_rows >= 3 (distinct up and down "
            "neighbours)");
    if ((int64_t)(d.L / d.tile) * (rows_of(d) / by) > (1 << 20)) bad("more than 2^20 domains");
    if (d.steps_per_visit < 0) bad("steps_per_visit must be >= 0");
    if (d.rate_model != KMC_RATE_METROPOLIS && d.rate_model != KMC_RATE_BARKER)
        bad("unknown rate model");
    if (d.schedule != KMC_SCHED_RANDOM_PERM && d.schedule != KMC_SCHED_PALINDROME)
        bad("unknown schedule");
    if (d.init < KMC_INIT_RANDOM || d.init > KMC_INIT_GIVEN) bad("unknown init");
}

KParams params(kmc_ctx *c) {
    KParams K;
    K.reps = c->d_reps;
    K.rates = c->d_rates;
    K.spins = c->d_spins;
    K.dom = c->d_dom;
    K.acc = c->d_acc;
    K.rec = c->d_rec;
    K.ctl = c->d_ctl;
    K.task_rep = c->d_task_rep;
    K.order = c->d_order;
    K.bins = nullptr;
    K.n_rep = c->n_rep;
    K.n_team = 0;
    K.n_solo = 0;
    K.n_bins = 0;
    K.seed = c->seed;
    K.write_records = 1;
    K.task_begin = 0;
    K.flow_acc = c->d_flow_acc;
    K.flow_clk = c->d_flow_clk;
    K.n_dom_total = c->n_dom;
    K.flow_max_polls = c->flow_max_polls;
    K.edges = c->d_edges;
    return K;
}

hipEvent_t pool_event(kmc_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(c, hipEventCreate(&e), "event create");
    return e;
}

// Brackets the launches made by fn with timing events when KMC_F_TIMING is on.
template <typename F>
void timed_launch(kmc_ctx *c, F fn) {
    if (!c->timing) {
        fn();
        return;
    }
    hipEvent_t a = pool_event(c), b = pool_event(c);
    hip_check(c, hipEventRecord(a, c->stream), "event record");
    fn();
    hip_check(c, hipEventRecord(b, c->stream), "event record");
    c->tev.emplace_back(a, b);
}

// Calls f with std::true_type when replicas of row-mask width g include a
// lattice that is one periodic domain, std::false_type otherwise.
template <typename F>
void with_wrap(const kmc_ctx *c, int g, F f) {
    if (c->wrap[g])
        f(std::true_type{});
    else
        f(std::false_type{});
}

// Calls f(wrap, slice) with the context's wrap-around and time-slice kinds
// as std::true_type / std::false_type (the time-slice kernels exist without
// the score only).
template <bool SCORE, typename F>
void with_kind(const kmc_ctx *c, int g, F f) {
    with_wrap(c, g, [&](auto W) {
        if (!SCORE && c->slice)
            f(W, std::true_type{});
        else
            f(W, std::false_type{});
    });
}

template <bool SCORE>
void launch_sweep(kmc_ctx *c, KParams K);

// A launch of 64-lane blocks covers fewer than 2^32 work-items (the grid
// size of a dispatch is a 32-bit count of work-items).
constexpr int64_t kMaxBlocks = ((int64_t)1 << 32) / 64 - 1;

// Device memory the per-sweep clock snapshots of one dataflow launch may use.
constexpr int64_t kFlowClockBytes = (int64_t)256 << 20;

// Sweeps one dataflow launch may hold: kFlowMaxSweeps, fewer when the grid
// of G sweeps x phases x tasks would not fit one dispatch (0: not even one)
// or the domains' clock snapshots of G sweeps would exceed kFlowClockBytes
// (at least one sweep).
int flow_window(const kmc_ctx *c) {
    const int64_t per_sweep = (int64_t)c->n_phase * std::max(c->n_tasks32, c->n_tasks - c->n_tasks32);
    const int64_t by_grid = kMaxBlocks / std::max<int64_t>(per_sweep, 1);
    const int64_t by_mem =
        std::max<int64_t>(1, kFlowClockBytes / (16 * (int64_t)std::max(c->n_dom, 1)));
    return (int)std::min<int64_t>({(int64_t)kmcdev::kFlowMaxSweeps, by_grid, by_mem});
}

unsigned flow_blocks(kmc_ctx *c, int G, int n_tasks) {
    const int64_t b = (int64_t)G * c->n_phase * n_tasks;
    if (b > kMaxBlocks) fail(c, KMC_EUNSUPPORTED, "dataflow grid too large");
    return (unsigned)b;
}

// G sweeps (G <= kFlowMaxSweeps) as one dataflow launch per row-mask width
// (replicas of the two widths never interact), then the records.
template <bool SCORE>
void launch_flow(kmc_ctx *c, KParams K, int G) {
    const int64_t slots = (int64_t)G * c->n_rep * 3;
    hipLaunchKernelGGL(kmcdev::k_fill_i64, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0,
                       c->stream, c->d_flow_acc, slots, (int64_t)0);
    timed_launch(c, [&] {
        if (c->n_tasks32) {
            K.task_begin = 0;
            with_kind<SCORE>(c, 0, [&](auto W, auto S) {
                hipLaunchKernelGGL((kmcdev::k_flow<uint32_t, SCORE, decltype(W)::value,
                                                   decltype(S)::value && !SCORE>),
                                   dim3(flow_blocks(c, G, c->n_tasks32)), dim3(64), 0,
                                   c->stream, K, c->n_tasks32, c->n_phase, c->d_done);
            });
            launch_check(c, "flow launch");
        }
        if (c->n_tasks > c->n_tasks32) {
            const int nt = c->n_tasks - c->n_tasks32;
            K.task_begin = c->n_tasks32;
            with_kind<SCORE>(c, 1, [&](auto W, auto S) {
                hipLaunchKernelGGL((kmcdev::k_flow<uint64_t, SCORE, decltype(W)::value,
                                                   decltype(S)::value && !SCORE>),
                                   dim3(flow_blocks(c, G, nt)), dim3(64), 0, c->stream, K, nt,
                                   c->n_phase, c->d_done);
            });
            launch_check(c, "flow launch");
        }
    });
    hipLaunchKernelGGL(kmcdev::k_flow_close, dim3(c->n_rep), dim3(64 * kmcdev::kFlowCloseWaves),
                       0, c->stream, K, G);
    hipLaunchKernelGGL(kmcdev::k_advance, dim3(1), dim3(1), 0, c->stream, K.ctl, (int64_t)G);
    launch_check(c, "flow launch");
}

// n sweeps of the phase-by-phase form (dataflow launches of up to
// kFlowMaxSweeps sweeps when c->flow).
template <bool SCORE>
void run_sweeps(kmc_ctx *c, KParams K, int64_t n) {
    if (c->flow) {
        const int G = flow_window(c);
        for (int64_t i = 0; i < n; i += G)
            launch_flow<SCORE>(c, K, (int)std::min<int64_t>(G, n - i));
        return;
    }
    for (int64_t i = 0; i < n; ++i) launch_sweep<SCORE>(c, K);
}

template <bool SCORE>
void launch_sweep(kmc_ctx *c, KParams K) {
    if (c->flow) {
        launch_flow<SCORE>(c, K, 1);
        return;
    }
    for (int p = 0; p < c->n_phase; ++p) {
        timed_launch(c, [&] {
        if (c->n_tasks32) {
            K.task_begin = 0;
            with_kind<SCORE>(c, 0, [&](auto W, auto S) {
                hipLaunchKernelGGL((kmcdev::k_phase<uint32_t, SCORE, decltype(W)::value,
                                                    decltype(S)::value && !SCORE>),
                                   dim3(c->n_tasks32), dim3(64), 0, c->stream, K, p);
            });
        }
        if (c->n_tasks > c->n_tasks32) {
            K.task_begin = c->n_tasks32;
            with_kind<SCORE>(c, 1, [&](auto W, auto S) {
                hipLaunchKernelGGL((kmcdev::k_phase<uint64_t, SCORE, decltype(W)::value,
                                                    decltype(S)::value && !SCORE>),
                                   dim3(c->n_tasks - c->n_tasks32), dim3(64), 0, c->stream, K,
                                   p);
            });
        }
        });
    }
    hipLaunchKernelGGL(kmcdev::k_sweep_end, dim3(c->n_rep), dim3(64), 0, c->stream, K);
    hipLaunchKernelGGL(kmcdev::k_advance, dim3(1), dim3(1), 0, c->stream, K.ctl, (int64_t)1);
    launch_check(c, "phase launch");
}

template <bool SCORE>
void launch_persistent(kmc_ctx *c, KParams K, int64_t n_sweeps, uint32_t flags) {
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    const int waves = kmcdev::kWavesPerPersistentGroup;
    const bool multi = !(flags & KMC_F_NO_MULTI) && (c->n_m_wg + c->n_m_wave) > 0 &&
                       ((flags & KMC_F_MULTI) || c->multi_auto);
    const int32_t *order = multi ? c->d_order : c->d_order_nm;
    const int32_t *nt = multi ? c->n_team : c->nm_team;
    const int32_t *ns = multi ? c->n_solo : c->nm_solo;
    int32_t off = 0;
    for (int g = 0; g < 2; ++g) {
        if (!nt[g] && !ns[g]) continue;
        K.order = order + off;
        K.n_team = nt[g];
        K.n_solo = ns[g];
        off += nt[g] + ns[g];
        const int groups = std::max(1, std::min(nt[g] + (ns[g] + waves - 1) / waves, cus * 8));
        hipLaunchKernelGGL(kmcdev::k_reset_queue, dim3(1), dim3(1), 0, c->stream, K.ctl);
        timed_launch(c, [&] {
            with_kind<SCORE>(c, g, [&](auto W, auto S) {
                constexpr bool SL = decltype(S)::value && !SCORE;
                if (g == 0)
                    hipLaunchKernelGGL(
                        (kmcdev::k_persistent<uint32_t, SCORE, decltype(W)::value, SL>),
                        dim3(groups), dim3(64 * waves), 0, c->stream, K, n_sweeps);
                else
                    hipLaunchKernelGGL(
                        (kmcdev::k_persistent<uint64_t, SCORE, decltype(W)::value, SL>),
                        dim3(groups), dim3(64 * waves), 0, c->stream, K, n_sweeps);
            });
        });
    }
    if (multi) {
        const int groups = std::max(
            1, std::min(c->n_m_wg + (c->n_m_wave + waves - 1) / waves, cus * 8));
        hipLaunchKernelGGL(kmcdev::k_reset_queue, dim3(1), dim3(1), 0, c->stream, K.ctl);
        timed_launch(c, [&] {
            hipLaunchKernelGGL((kmcdev::k_persistent_multi<SCORE>), dim3(groups),
                               dim3(64 * waves), 0, c->stream, K, c->d_items, c->n_m_wg,
                               c->n_m_wave, n_sweeps);
        });
    }
    hipLaunchKernelGGL(kmcdev::k_advance, dim3(1), dim3(1), 0, c->stream, K.ctl, n_sweeps);
    launch_check(c, "persistent launch");
}

// Resident form: one workgroup per replica, as many wavefronts as the
// largest colour class has domains (at most 16).
template <bool SCORE>
void launch_resident(kmc_ctx *c, KParams K, int64_t n_sweeps) {
    int waves = 1, lds = 0;
    for (const Rep &rp : c->reps) {
        waves = std::max(waves, std::min(max_per_colour(rp), kmcdev::kResMaxWaves));
        lds = std::max(lds, kmcdev::resident_lds_bytes(rp.L, rp.NT));
    }
    timed_launch(c, [&] {
        hipLaunchKernelGGL((kmcdev::k_resident<SCORE>), dim3(c->n_rep), dim3(64 * waves),
                           (unsigned)lds, c->stream, K, n_sweeps);
    });
    hipLaunchKernelGGL(kmcdev::k_advance, dim3(1), dim3(1), 0, c->stream, K.ctl, n_sweeps);
    launch_check(c, "resident launch");
}

// Per-sweep slots of the dataflow launches, allocated once (captured graphs
// keep their addresses).
// (Each buffer is checked on its own: after a failed allocation the next
// call allocates what is still missing.)
void ensure_flow_slots(kmc_ctx *c) {
    const int64_t G = std::max(flow_window(c), 1);
    if (!c->d_flow_acc) c->d_flow_acc = alloc_n<int64_t>(c, G * c->n_rep * 3);
    if (!c->d_flow_clk) c->d_flow_clk = alloc_n<double>(c, G * std::max(c->n_dom, 1) * 2);
}

void ensure_records(kmc_ctx *c, int64_t need) {
    if (need <= c->rec_cap) return;
    const int64_t cap = std::max<int64_t>(need, c->rec_cap * 2);
    Record *p = alloc_n<Record>(c, cap * c->n_rep);
    if (c->n_rec)
        hip_check(c, hipMemcpyAsync(p, c->d_rec, sizeof(Record) * c->n_rec * c->n_rep,
                                    hipMemcpyDeviceToDevice, c->stream),
                  "record copy");
    hip_check(c, hipStreamSynchronize(c->stream), "record copy");
    dev_free(c, c->d_rec);
    c->d_rec = p;
    c->rec_cap = cap;
    if (c->graph) {  // the captured graphs hold the old record pointer
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    if (c->pgraph) {
        (void)hipGraphExecDestroy(c->pgraph);
        c->pgraph = nullptr;
    }
}

void ensure_bins(kmc_ctx *c, int64_t n_bins) {
    if (n_bins <= c->bins_cap && c->d_bins) return;
    hip_check(c, hipStreamSynchronize(c->stream), "bins sync");
    dev_free(c, c->d_bins);
    c->d_bins = nullptr;
    c->bins_cap = 0;  // stays 0 if the allocation below fails
    c->d_bins = alloc_n<double>(c, n_bins * c->n_rep * 2);
    c->bins_cap = n_bins;
}

void run_graph(kmc_ctx *c, int64_t n_sweeps) {
    const int G = 16;
    // The null stream cannot be captured: replay on a private blocking stream,
    // which the null stream orders implicitly.
    if (!c->stream && !c->graph_stream) {
        hip_check(c, hipStreamCreate(&c->graph_stream), "stream create");
    }
    hipStream_t gs = c->stream ? c->stream : c->graph_stream;
    hipStream_t saved = c->stream;
    if (c->graph && c->graph_flow != c->flow) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    if (!c->graph) {
        c->graph_flow = c->flow;
        hipGraph_t g;
        c->stream = gs;
        hip_check(c, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal),
                  "begin capture");
        for (int i = 0; i < G; ++i) launch_sweep<false>(c, params(c));
        c->stream = saved;
        hip_check(c, hipStreamEndCapture(gs, &g), "end capture");
        hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hip_check(c, e, "graph instantiate");
        c->graph_sweeps = G;
    }
    int64_t i = 0;
    for (; i + c->graph_sweeps <= n_sweeps; i += c->graph_sweeps)
        hip_check(c, hipGraphLaunch(c->graph, gs), "graph launch");
    for (; i < n_sweeps; ++i) launch_sweep<false>(c, params(c));
}

// Persistent form replayed from a captured graph: one graph holds one
// chunk (queue reset, persistent launch(es) of `chunk` sweeps, counter
// advance); the kernels read the sweep counters from device memory, so
// every replay continues where the previous one stopped.
void run_persistent_graph(kmc_ctx *c, KParams K, int64_t n_sweeps, int32_t record_every,
                          uint32_t flags) {
    const int64_t chunk = std::min<int64_t>(record_every, n_sweeps);
    const uint32_t key = flags & (KMC_F_MULTI | KMC_F_NO_MULTI);
    if (!c->pgraph || c->pgraph_chunk != chunk || c->pgraph_key != key) {
        if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
        c->pgraph = nullptr;
        if (!c->stream && !c->graph_stream)
            hip_check(c, hipStreamCreate(&c->graph_stream), "stream create");
        hipStream_t gs = c->stream ? c->stream : c->graph_stream;
        hipStream_t saved = c->stream;
        hipGraph_t g;
        c->stream = gs;
        hip_check(c, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal),
                  "begin capture");
        launch_persistent<false>(c, K, chunk, flags);
        c->stream = saved;
        hip_check(c, hipStreamEndCapture(gs, &g), "end capture");
        hipError_t e = hipGraphInstantiate(&c->pgraph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hip_check(c, e, "graph instantiate");
        c->pgraph_chunk = chunk;
        c->pgraph_key = key;
    }
    hipStream_t gs = c->stream ? c->stream : c->graph_stream;
    int64_t i = 0;
    for (; i + chunk <= n_sweeps; i += chunk)
        hip_check(c, hipGraphLaunch(c->pgraph, gs), "graph launch");
    if (i < n_sweeps) launch_persistent<false>(c, K, n_sweeps - i, flags);
}

int64_t bytes_of_spins(const kmc_replica_desc &d) { return (int64_t)d.L * rows_of(d); }

// A one-launch sweep whose bounded wait gave up leaves ctl->err set (a
// dependency never satisfied): the results of the run are not valid.
// A dataflow wait that gave up leaves the flag set for good: visits after
// it may have read a halo out of order, so the context's results are void.
// Rebuild the edge columns of every domain of K.spins into K.edges (before a
// run of the staged visits, which read and keep them).
void rebuild_edges(kmc_ctx *c, const KParams &K) {
    int most = 1;
    for (const Rep &rp : c->reps) most = std::max(most, rp.ND);
    hipLaunchKernelGGL(kmcdev::k_edges, dim3((unsigned)((most + 255) / 256), c->n_rep),
                       dim3(256), 0, c->stream, K);
    launch_check(c, "edge columns");
}

void check_flow_error(kmc_ctx *c, const Ctl *ctl) {
    Ctl h;
    hip_check(c, hipMemcpy(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost), "ctl copy");
    if (h.err) fail(c, KMC_EDEVICE, "a dataflow sweep timed out waiting for a neighbour");
}

void destroy_buffers(kmc_ctx *c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
    c->pgraph = nullptr;
    void *bufs[] = {c->d_reps,  c->d_rates, c->d_spins, c->d_dom,   c->d_acc,
                    c->d_rec,   c->d_ctl,   c->d_task_rep, c->d_order, c->c_spins,
                    c->c_dom,   c->c_acc,   c->r_spins, c->r_dom,   c->r_acc,
                    c->r_ctl,   c->d_bins,  c->d_tmp_rec, c->d_order_nm, c->d_items,
                    c->d_done, c->d_flow_acc, c->d_flow_clk, c->d_edges, c->d_stage,
                    c->r_edges};
    for (void *p : bufs) dev_free(c, p);
}

}  // namespace

// ------------------------------------------------------------------- ABI

extern "C" kmc_status kmc_rate_table(double J, double h, double T, int32_t rate_model,
                                     uint64_t r[10], double w[10], double gJ[10],
                                     double gh[10]) {
    if (!r || !w || !gJ || !gh) return KMC_EINVAL;
    return rate_table(J, h, T, rate_model, r, w, gJ, gh);
}

extern "C" kmc_status kmc_set_wait_limit(kmc_ctx *c, int64_t max_polls) {
    if (!c) return KMC_EINVAL;
    if (max_polls < 0) {
        c->err = "max_polls must be >= 0";
        return KMC_EINVAL;
    }
    c->flow_max_polls = max_polls;
    // captured graphs hold the old bound in their kernel arguments
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
    c->pgraph = nullptr;
    return KMC_OK;
}

namespace {

// Everything one exact propagation needs, built on the stack (no heap, no
// device allocation): the domains with their colours, and the colour orders
// the sweep mixes (all n! orders of at most 4 colours, or the palindrome).
struct ExactPlan {
    kmcdev::ExactDomain dom[kmcdev::kExactMaxSites];
    int col[kmcdev::kExactMaxSites];
    bool two_pass[kmcdev::kExactMaxSites];  // a site at state bit 14 or above
    int n_dom = 0;
    int orders[24][18];
    int n_orders = 0, order_len = 0;
    kmcdev::ExactRates R;
    int NI = 0;
    double inv_nd = 0.0;
};

// Validates d and fills the plan; KMC_OK, KMC_EINVAL or KMC_EUNSUPPORTED.
kmc_status exact_plan(const kmc_replica_desc *d, uint32_t flags, int max_sites, ExactPlan &P) {
    validate(nullptr, *d, 0);  // throws Fail{KMC_EINVAL}
    if (d->time_slice > 0.0) return KMC_EUNSUPPORTED;  // propagates the tick chain only
    const bool ring = is_ring(*d);
    const int L = d->L, Ly = rows_of(*d), N = L * Ly;
    if (N > max_sites) return KMC_EINVAL;
    const int Bx = d->tile, By = tile_rows_of(*d), NTx = L / Bx, NTy = Ly / By;
    const int cx = axis_colours(NTx), ncol = cx * axis_colours(NTy);
    const bool pal = d->schedule == KMC_SCHED_PALINDROME;
    if (!pal && ncol > 4) return KMC_EUNSUPPORTED;  // more than 4! orders to mix
    uint64_t r[10];
    double w[10], gJ[10], gh[10];
    if (rate_table(d->J, d->h, d->T, d->rate_model, r, w, gJ, gh, ring ? 2 : 4) != KMC_OK)
        return KMC_EINVAL;
    for (int c = 0; c < 10; ++c)
        P.R.w[c] = (flags & KMC_EXACT_QUANTISED) ? (double)r[c] * 0x1p-32 : w[c];
    // domains (row-major over the grid, sites row-major inside)
    auto axis_colour = [](int t, int n) { return n == 1 ? 0 : (n % 2 && t == n - 1) ? 2 : t % 2; };
    P.n_dom = 0;
    for (int ty = 0; ty < NTy; ++ty)
        for (int tx = 0; tx < NTx; ++tx) {
            kmcdev::ExactDomain &D = P.dom[P.n_dom];
            std::memset(&D, 0, sizeof(D));
            D.n = Bx * By;
            for (int ly = 0; ly < By; ++ly)
                for (int lx = 0; lx < Bx; ++lx) {
                    const int a = ly * Bx + lx, y = ty * By + ly, x = tx * Bx + lx;
                    D.site[a] = y * L + x;
                    // the ring has no up and down neighbours; on a side of 2
                    // the two neighbours along an axis are one site, counted
                    // twice
                    int nb[4] = {y * L + (x + L - 1) % L, y * L + (x + 1) % L, -1, -1};
                    if (!ring) {
                        nb[2] = ((y + L - 1) % L) * L + x;
                        nb[3] = ((y + 1) % L) * L + x;
                    }
                    for (int q = 0; q < 4; ++q) {
                        if (nb[q] < 0) continue;
                        const uint32_t bit = 1u << nb[q];
                        if (D.nb1[a] & bit)
                            D.nb2[a] |= bit;
                        else
                            D.nb1[a] |= bit;
                    }
                }
            P.two_pass[P.n_dom] = false;
            for (int a = 0; a < D.n; ++a) {
                P.two_pass[P.n_dom] |= D.site[a] >= kmcdev::kExactLoBits;
                // state j of a thread differs from its state 0 in the bits
                // J_j (contiguous pass: j << 9; strided pass: tile bits
                // 10..13 of j placed as the pass spreads them); its class
                // moves by the neighbours and the site itself among them
                const int c = kmcdev::kExactHiBits + kmcdev::kExactLoBits - N;
                for (int j = 0; j < kmcdev::kExactPerThread; ++j) {
                    const uint32_t l = (uint32_t)j << (kmcdev::kExactLoBits - 4);
                    const uint32_t lh = (uint32_t)j << (kmcdev::kExactHiBits - 4);
                    uint32_t Jh = 0;
                    if (N > kmcdev::kExactLoBits)
                        Jh = (lh & ((1u << c) - 1u)) | ((lh >> c) << kmcdev::kExactLoBits);
                    auto delta = [&](uint32_t J) {
                        return (uint64_t)(__builtin_popcount(J & D.nb1[a]) +
                                          __builtin_popcount(J & D.nb2[a]) +
                                          (((J >> D.site[a]) & 1u) << 3));
                    };
                    D.dlo[a] |= delta(l) << (4 * j);
                    D.dhi[a] |= delta(Jh) << (4 * j);
                }
            }
            P.col[P.n_dom++] = axis_colour(tx, NTx) + cx * axis_colour(ty, NTy);
        }
    // colour orders: all of them (mixed uniformly) or the palindrome
    P.n_orders = 0;
    if (pal) {
        P.order_len = 2 * ncol;
        for (int k = 0; k < ncol; ++k) {
            P.orders[0][k] = k;
            P.orders[0][2 * ncol - 1 - k] = k;
        }
        P.n_orders = 1;
    } else {
        int o[4];
        for (int k = 0; k < ncol; ++k) o[k] = k;
        P.order_len = ncol;
        do {
            for (int k = 0; k < ncol; ++k) P.orders[P.n_orders][k] = o[k];
            ++P.n_orders;
        } while (std::next_permutation(o, o + ncol));
    }
    P.NI = d->steps_per_visit ? d->steps_per_visit : Bx * By;
    P.inv_nd = 1.0 / (double)(Bx * By);
    return KMC_OK;
}

// Enqueues n_sweeps sweeps of the plan on st: p in and out, work holds three
// vectors of 2^N doubles (the mixture's accumulator and two tick buffers);
// every entry of work is written before it is read.  An order's first tick
// reads p itself.  With one order its last tick writes p (in place when it
// is also the first: each tile of a tick pass is read whole before any of it
// is written, and no other workgroup reads it); with several the orders'
// results are mixed in the accumulator.
void exact_enqueue(const ExactPlan &P, int N, double *p, double *work, int64_t n_sweeps,
                   hipStream_t st) {
    const int64_t n = (int64_t)1 << N;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    const unsigned lo_tiles = N >= kmcdev::kExactLoBits ? 1u << (N - kmcdev::kExactLoBits) : 1u;
    const unsigned hi_tiles = N > kmcdev::kExactHiBits ? 1u << (N - kmcdev::kExactHiBits) : 1u;
    double *acc = work, *b0 = work + n, *b1 = work + 2 * n;
    auto tick = [&](int i, const double *in, double *out, double *part) {
        if (N < kmcdev::kExactLoBits) {
            hipLaunchKernelGGL(kmcdev::k_exact_small, dim3(1), dim3(1024), 0, st, in, out, N,
                               P.dom[i], P.R, P.inv_nd);
        } else if (!P.two_pass[i]) {
            hipLaunchKernelGGL(kmcdev::k_exact_lo<false>, dim3(lo_tiles),
                               dim3(kmcdev::kExactLoBlock), 0, st, in, nullptr, out, N, P.dom[i],
                               P.R, P.inv_nd);
        } else {  // part holds the high sites' terms between the passes
            hipLaunchKernelGGL(kmcdev::k_exact_hi, dim3(hi_tiles), dim3(kmcdev::kExactHiBlock),
                               0, st, in, part, N, P.dom[i], P.R);
            hipLaunchKernelGGL(kmcdev::k_exact_lo<true>, dim3(lo_tiles),
                               dim3(kmcdev::kExactLoBlock), 0, st, in, part, out, N, P.dom[i],
                               P.R, P.inv_nd);
        }
    };
    // the domains of one order, visit by visit
    int seq[2 * kmcdev::kExactMaxSites];
    for (int64_t sw = 0; sw < n_sweeps; ++sw) {
        for (int k = 0; k < P.n_orders; ++k) {
            int n_seq = 0;
            for (int q = 0; q < P.order_len; ++q)
                for (int i = 0; i < P.n_dom; ++i)
                    if (P.col[i] == P.orders[k][q]) seq[n_seq++] = i;
            const int n_ticks = n_seq * P.NI;
            const double *cur = p;
            double *nxt = b0;
            for (int v = 0, tk = 0; v < n_seq; ++v)
                for (int t = 0; t < P.NI; ++t, ++tk) {
                    const bool last = tk == n_ticks - 1 && P.n_orders == 1;
                    double *out = last ? p : nxt;
                    // the high sites' terms: out itself, or any vector but cur
                    double *part = out != p ? out : (cur == b0 ? b1 : b0);
                    tick(seq[v], cur, out, part);
                    cur = out;
                    nxt = nxt == b0 ? b1 : b0;
                }
            if (P.n_orders > 1)
                hipLaunchKernelGGL(kmcdev::k_exact_axpy, dim3(grid), dim3(256), 0, st, acc, cur,
                                   1.0 / (double)P.n_orders, n, k == 0 ? 1 : 0);
        }
        if (P.n_orders > 1)
            hipLaunchKernelGGL(kmcdev::k_exact_copy, dim3(grid), dim3(256), 0, st, acc, p, n);
    }
}

}  // namespace

extern "C" kmc_status kmc_exact_sweeps(const kmc_replica_desc *d, double *p, double *work,
                                       int64_t n_sweeps, uint32_t flags, void *hip_stream) {
    if (!d || !p || !work || n_sweeps < 0) return KMC_EINVAL;
    try {
        ExactPlan P;
        const kmc_status st = exact_plan(d, flags, kmcdev::kExactMaxSites, P);
        if (st != KMC_OK) return st;
        exact_enqueue(P, d->L * rows_of(*d), p, work, n_sweeps, (hipStream_t)hip_stream);
        if (hipGetLastError() != hipSuccess) return KMC_EDEVICE;
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

// ------------------------------------------- exact propagation, no allocation
//
// The work vectors of kmc_exact_sweeps_static live in this file-scope device
// array: 3 * 2^16 doubles (1.5 MiB), held by every device the library runs
// on until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): its device
// address is taken once per device with hipGetSymbolAddress, with that
// device current, and kept here.
constexpr int kExactStaticMaxSites = 16;
static __device__ __align__(256) double scratch[3 * ((size_t)1 << kExactStaticMaxSites)];

namespace {

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up on the
// first call there).
kmc_status scratch_address(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KMC_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return KMC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return KMC_EDEVICE;
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return KMC_OK;
}

}  // namespace

extern "C" kmc_status kmc_exact_sweeps_static(const kmc_replica_desc *d, double *p,
                                              int64_t n_sweeps, uint32_t flags,
                                              void *hip_stream) {
    if (!d || !p || n_sweeps < 0) return KMC_EINVAL;
    try {
        ExactPlan P;
        const kmc_status st = exact_plan(d, flags, kExactStaticMaxSites, P);
        if (st != KMC_OK) return st;
        double *work = nullptr;
        const kmc_status sa = scratch_address(&work);
        if (sa != KMC_OK) return sa;
        exact_enqueue(P, d->L * rows_of(*d), p, work, n_sweeps, (hipStream_t)hip_stream);
        if (hipGetLastError() != hipSuccess) return KMC_EDEVICE;
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_init_lattice(kmc_ctx **out, const kmc_replica_desc *d,
                                       int32_t n_rep, uint64_t seed,
                                       const int8_t *given_spins, void *hip_stream) {
    if (!out || !d || n_rep < 1) return KMC_EINVAL;
    kmc_ctx *c = new (std::nothrow) kmc_ctx;
    if (!c) return KMC_ENOMEM;
    try {  // descriptors are checked before any device call
        for (int rho = 0; rho < n_rep; ++rho) validate(c, d[rho], rho);
    } catch (const Fail &f) {
        std::fprintf(stderr, "kmc_init_lattice: %s\n", c->err.c_str());
        delete c;
        return f.st;
    }
    try {
        c->alloc = g_alloc;
        c->free_fn = g_free;
        c->alloc_user = g_alloc_user;
        hip_check(c, hipGetDevice(&c->device), "hipGetDevice");
        c->stream = (hipStream_t)hip_stream;  // NULL: the null stream
        c->n_rep = n_rep;
        c->seed = seed;
        c->desc.assign(d, d + n_rep);
        c->reps.resize(n_rep);
        c->rates.resize(n_rep);
        int64_t off = 0;
        int32_t dom = 0;
        bool any_given = false;
        for (int rho = 0; rho < n_rep; ++rho) {
            const kmc_replica_desc &q = d[rho];
            Rep &rp = c->reps[rho];
            rp.L = q.L;
            rp.B = q.tile;
            rp.By = tile_rows_of(q);
            rp.NT = q.L / q.tile;
            rp.NTy = rows_of(q) / rp.By;
            rp.z = is_ring(q) ? 2 : 4;
            rp.cx = axis_colours(rp.NT);
            rp.ncol = rp.cx * axis_colours(rp.NTy);
            rp.nperm = 1;
            for (int k = 2; k <= rp.ncol; ++k) rp.nperm *= k;
            rp.NI = q.steps_per_visit ? q.steps_per_visit : q.tile * rp.By;
            rp.tau = q.time_slice;
            if (rp.tau > 0.0) rp.NI = 0;  // no ticks: the step count stays 0
            rp.sched = q.schedule;
            rp.ND = rp.NT * rp.NTy;
            rp.nd = (uint32_t)(q.tile * rp.By);
            rp.thr = (uint32_t)(0u - rp.nd) % rp.nd;
            rp.spin_off = off;
            off += (bytes_of_spins(q) + 255) / 256 * 256;
            rp.dom_off = dom;
            dom += rp.ND;
            rp.visits = q.schedule == KMC_SCHED_PALINDROME ? 2 : 1;
            rp.init = q.init;
            c->n_phase = std::max(c->n_phase,
                                  (q.schedule == KMC_SCHED_PALINDROME ? 2 : 1) * rp.ncol);
            if (q.init == KMC_INIT_GIVEN) any_given = true;
            Rates &R = c->rates[rho];
            std::memset(&R, 0, sizeof(R));
            double gJ[10], gh[10];
            if (rate_table(q.J, q.h, q.T, q.rate_model, R.r, R.w, gJ, gh, rp.z) != KMC_OK)
                fail(c, KMC_EINVAL, "replica " + std::to_string(rho) + ": rate table");
            for (int k = 0; k < 10; ++k) {
                R.rd[k] = (double)R.r[k];
                R.inv_rd[k] = R.r[k] ? 1.0 / (double)R.r[k] : 0.0;
                R.gJ[k] = gJ[k];
                R.gh[k] = gh[k];
                R.aJ[k] = R.w[k] * gJ[k];
                R.ah[k] = R.w[k] * gh[k];
            }
        }
        if (any_given && !given_spins) fail(c, KMC_EINVAL, "KMC_INIT_GIVEN needs given_spins");
        c->slice = d[0].time_slice > 0.0;
        for (int rho = 1; rho < n_rep; ++rho)
            if ((d[rho].time_slice > 0.0) != c->slice)
                fail(c, KMC_EINVAL,
                     "all replicas of a context run time slices (time_slice > 0) or none");
        c->spin_bytes = off;
        c->n_dom = dom;

        // phase tasks (as many per replica as its largest colour class has
        // domains): replicas with domains of at most 32 x 32 first (32-bit
        // row masks)
        std::vector<int32_t> task_rep;
        for (int pass = 0; pass < 2; ++pass)
            for (int rho = 0; rho < n_rep; ++rho) {
                Rep &rp = c->reps[rho];
                if (wide(rp) != (pass == 1)) continue;
                if (rp.NT == 1 || rp.NTy == 1) c->wrap[pass] = true;
                rp.task_off = (int32_t)task_rep.size();
                for (int i = 0; i < max_per_colour(rp); ++i) task_rep.push_back(rho);
                if (pass == 0) c->n_tasks32 = (int32_t)task_rep.size();
            }
        c->n_tasks = (int32_t)task_rep.size();
        // persistent queues.  Replicas with domains of at most 16x16 may run
        // in the multi-slot kernel (four domain processes per wavefront):
        // one replica split over the slots of a workgroup (>= 16 domains per
        // colour) or of a wavefront (>= 4), or four replicas of one shape per
        // wavefront.  It is used when its items keep at least two wavefronts
        // per SIMD busy.  The others, and every replica when the multi-slot
        // form is not used, go to the one-domain-per-wavefront kernel: a
        // workgroup team when the replica has >= 4 domains per colour and a
        // large sweep (or the batch is small), else one wavefront.
        int n_simd = 1024;
        {
            int dev = 0;
            hipDeviceProp_t prop;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                n_simd = 4 * prop.multiProcessorCount;
        }
        const bool few = n_rep < 4 * n_simd;
        auto by_cost = [&](int a, int b) {
            return sweep_cost(c->reps[a], c->desc[a]) > sweep_cost(c->reps[b], c->desc[b]);
        };
        std::vector<int32_t> mrep;  // multi-slot candidates
        for (int rho = 0; rho < n_rep; ++rho)
            if (multi_ok(c->reps[rho])) mrep.push_back(rho);
        {
            std::stable_sort(mrep.begin(), mrep.end(), by_cost);
            std::vector<MItem> wg, wv;
            std::vector<std::vector<int32_t>> pending;  // inter groups by shape
            auto same_shape = [&](int a, int b) {
                const Rep &x = c->reps[a], &y = c->reps[b];
                return x.L == y.L && x.B == y.B && x.NI == y.NI && x.sched == y.sched;
            };
            for (int rho : mrep) {
                const int per_colour = c->reps[rho].ND / 4;
                if (per_colour >= 4) {
                    MItem it{1, per_colour >= 16 ? 4 : 1, {rho, -1, -1, -1}};
                    (it.nw == 4 ? wg : wv).push_back(it);
                    continue;
                }
                bool placed = false;
                for (auto &grp : pending)
                    if (grp.size() < 4 && same_shape(grp[0], rho)) {
                        grp.push_back(rho);
                        placed = true;
                        if (grp.size() == 4) {
                            wv.push_back(MItem{0, 1, {grp[0], grp[1], grp[2], grp[3]}});
                            grp.clear();
                        }
                        break;
                    }
                if (!placed) pending.push_back({rho});
            }
            for (auto &grp : pending)
                if (!grp.empty()) {
                    MItem it{0, 1, {-1, -1, -1, -1}};
                    for (size_t q = 0; q < grp.size(); ++q) it.rho[q] = grp[q];
                    wv.push_back(it);
                }
            // A launch lasts as long as its longest item: start the items
            // whose busiest slot has the most work per sweep first.  (A
            // group of four small replicas runs one replica per slot, so
            // its length is one replica's whole sweep; a replica split over
            // the slots of a wavefront or workgroup divides its sweep.)
            auto chain = [&](const MItem &it) {
                auto per_slot = [&](int rho, int slots) {
                    const Rep &r = c->reps[rho];
                    const int passes = (r.ND / 4 + slots - 1) / slots;
                    return sweep_cost(r, c->desc[rho]) / r.ND * 4.0 * passes;
                };
                if (it.kind == 1) return per_slot(it.rho[0], kmcdev::kSlots * it.nw);
                double m = 0.0;
                for (int q = 0; q < kmcdev::kSlots; ++q)
                    if (it.rho[q] >= 0) m = std::max(m, per_slot(it.rho[q], 1));
                return m;
            };
            auto longer = [&](const MItem &a, const MItem &b) { return chain(a) > chain(b); };
            std::stable_sort(wg.begin(), wg.end(), longer);
            std::stable_sort(wv.begin(), wv.end(), longer);
            const int64_t m_waves = 4 * (int64_t)wg.size() + (int64_t)wv.size();
            c->m_items = wg;
            c->m_items.insert(c->m_items.end(), wv.begin(), wv.end());
            c->n_m_wg = (int32_t)wg.size();
            c->n_m_wave = (int32_t)wv.size();
            c->multi_auto = !mrep.empty() && m_waves >= 2 * n_simd;
        }
        auto build_queue = [&](bool use_multi, int32_t *n_team, int32_t *n_solo) {
            std::vector<int32_t> order;
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<int32_t> team, solo;
                for (int rho = 0; rho < n_rep; ++rho) {
                    const Rep &rp = c->reps[rho];
                    if (wide(rp) != (pass == 1)) continue;
                    if (use_multi && multi_ok(rp)) continue;
                    const int64_t ticks = (int64_t)rp.NI * rp.ND * rp.visits;
                    const bool split = max_per_colour(rp) >= 4 && (ticks >= 8192 || few);
                    (split ? team : solo).push_back(rho);
                }
                std::stable_sort(team.begin(), team.end(), by_cost);
                std::stable_sort(solo.begin(), solo.end(), by_cost);
                n_team[pass] = (int32_t)team.size();
                n_solo[pass] = (int32_t)solo.size();
                order.insert(order.end(), team.begin(), team.end());
                order.insert(order.end(), solo.begin(), solo.end());
            }
            return order;
        };
        std::vector<int32_t> order = build_queue(!c->m_items.empty(), c->n_team, c->n_solo);
        std::vector<int32_t> order_nm = build_queue(false, c->nm_team, c->nm_solo);

        c->d_reps = alloc_n<Rep>(c, n_rep);
        c->d_rates = alloc_n<Rates>(c, n_rep);
        c->d_spins = alloc_n<int8_t>(c, off);
        c->d_edges = alloc_n<uint64_t>(c, 2 * (int64_t)std::max(dom, 1));
        {
            int64_t most = 1;
            for (auto &q : c->desc) most = std::max(most, bytes_of_spins(q));
            c->d_stage = alloc_n<int8_t>(c, most);
        }
        c->d_dom = alloc_n<Dom>(c, dom);
        c->d_acc = alloc_n<RepAcc>(c, n_rep);
        c->d_ctl = alloc_n<Ctl>(c, 1);
        c->d_done = alloc_n<int64_t>(c, std::max(dom, 1));
        c->d_task_rep = alloc_n<int32_t>(c, c->n_tasks);
        c->d_order = alloc_n<int32_t>(c, n_rep);
        c->d_order_nm = alloc_n<int32_t>(c, n_rep);
        c->d_items = alloc_n<MItem>(c, (int64_t)c->m_items.size());
        hipStream_t s = c->stream;
        hip_check(c, hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(Rep) * n_rep,
                                    hipMemcpyHostToDevice, s), "copy reps");
        hip_check(c, hipMemcpyAsync(c->d_rates, c->rates.data(), sizeof(Rates) * n_rep,
                                    hipMemcpyHostToDevice, s), "copy rates");
        hip_check(c, hipMemcpyAsync(c->d_task_rep, task_rep.data(),
                                    sizeof(int32_t) * std::max<size_t>(task_rep.size(), 1),
                                    hipMemcpyHostToDevice, s), "copy tasks");
        hip_check(c, hipMemcpyAsync(c->d_order, order.data(), sizeof(int32_t) * order.size(),
                                    hipMemcpyHostToDevice, s), "copy order");
        hip_check(c, hipMemcpyAsync(c->d_order_nm, order_nm.data(), sizeof(int32_t) * n_rep,
                                    hipMemcpyHostToDevice, s), "copy order");
        if (!c->m_items.empty())
            hip_check(c, hipMemcpyAsync(c->d_items, c->m_items.data(),
                                        sizeof(MItem) * c->m_items.size(),
                                        hipMemcpyHostToDevice, s), "copy items");
        hip_check(c, hipMemsetAsync(c->d_dom, 0, sizeof(Dom) * std::max(dom, 1), s), "zero");
        hip_check(c, hipMemsetAsync(c->d_acc, 0, sizeof(RepAcc) * n_rep, s), "zero");
        hip_check(c, hipMemsetAsync(c->d_ctl, 0, sizeof(Ctl), s), "zero");
        hip_check(c, hipMemsetAsync(c->d_done, 0, sizeof(int64_t) * std::max(dom, 1), s),
                  "zero");
        KParams K = params(c);
        if (any_given) {
            // row-major in, domain by domain on the device (the staging
            // lattice is reused in stream order)
            int64_t src = 0;
            for (int rho = 0; rho < n_rep; ++rho) {
                const int64_t nb = bytes_of_spins(d[rho]);
                if (d[rho].init == KMC_INIT_GIVEN) {
                    for (int64_t i = 0; i < nb; ++i)
                        if (given_spins[src + i] != 1 && given_spins[src + i] != -1)
                            fail(c, KMC_EINVAL, "given spins must be +1 or -1");
                    hip_check(c, hipMemcpyAsync(c->d_stage, given_spins + src, nb,
                                                hipMemcpyHostToDevice, s),
                              "copy given spins");
                    hipLaunchKernelGGL(kmcdev::k_spins_layout<true>,
                                       dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, K,
                                       rho, c->d_stage);
                    launch_check(c, "given spins");
                }
                src += nb;
            }
        }
        int maxL = 0;
        for (auto &q : c->desc) maxL = std::max(maxL, q.L);
        const int64_t maxN = (int64_t)maxL * maxL;
        hipLaunchKernelGGL(kmcdev::k_init_spins,
                           dim3((unsigned)((maxN / 128 + 255) / 256 + 1), n_rep), dim3(256),
                           0, s, K);
        hipLaunchKernelGGL(kmcdev::k_init_obs, dim3((unsigned)((maxN + 255) / 256), n_rep),
                           dim3(256), 0, s, K);
        hipLaunchKernelGGL(kmcdev::k_set_ctl, dim3(1), dim3(1), 0, s, c->d_ctl, (int64_t)0,
                           (int64_t)0, (int64_t)1, (int64_t)0);
        launch_check(c, "init launch");
        hip_check(c, hipStreamSynchronize(s), "init sync");
    } catch (const Fail &f) {
        // the message is lost with the context; report it on stderr
        std::fprintf(stderr, "kmc_init_lattice: %s\n", c->err.c_str());
        destroy_buffers(c);
        delete c;
        return f.st;
    }
    *out = c;
    return KMC_OK;
}

extern "C" kmc_status kmc_run_schedule(kmc_ctx *c, int64_t n_sweeps, int32_t record_every,
                                       uint32_t flags) {
    if (!c) return KMC_EINVAL;
    try {
        if (n_sweeps < 0 || record_every < 1)
            fail(c, KMC_EINVAL, "n_sweeps must be >= 0 and record_every >= 1");
        if (c->sweep + n_sweeps > 0xFFFFFFFFll)
            fail(c, KMC_EINVAL, "sweep counter would exceed 2^32 - 1");
        if ((flags & KMC_F_SCORE) && (flags & KMC_F_GRAPH))
            fail(c, KMC_EINVAL, "KMC_F_SCORE is not available with KMC_F_GRAPH");
        if (c->slice && (flags & (KMC_F_SCORE | KMC_F_CHECKPOINT | KMC_F_RESIDENT)))
            fail(c, KMC_EUNSUPPORTED,
                 "the time-slice variant runs without score, checkpoint or the resident form");
        if ((flags & KMC_F_TIMING) && (flags & KMC_F_GRAPH))
            fail(c, KMC_EINVAL, "KMC_F_TIMING is not available with KMC_F_GRAPH");
        if ((flags & KMC_F_FLOW) && (flags & KMC_F_PERSISTENT))
            fail(c, KMC_EINVAL, "KMC_F_FLOW applies to the phase-by-phase form only");
        if (flags & KMC_F_RESIDENT) {
            if (flags & (KMC_F_PERSISTENT | KMC_F_FLOW | KMC_F_GRAPH))
                fail(c, KMC_EINVAL,
                     "KMC_F_RESIDENT is not available with KMC_F_PERSISTENT, KMC_F_FLOW or "
                     "KMC_F_GRAPH");
            for (int rho = 0; rho < c->n_rep; ++rho)
                if (c->reps[rho].z == 2)
                    fail(c, KMC_EUNSUPPORTED,
                         "replica " + std::to_string(rho) +
                             ": the resident form holds square lattices only");
            for (int rho = 0; rho < c->n_rep; ++rho)
                if (!resident_ok(c->reps[rho]))
                    fail(c, KMC_EINVAL,
                         "replica " + std::to_string(rho) +
                             ": the resident form needs 3 <= L <= 128 and at most 16 domains "
                             "along x");
        } else {
            for (int rho = 0; rho < c->n_rep; ++rho)
                if (big(c->reps[rho]))
                    fail(c, KMC_EUNSUPPORTED,
                         "replica " + std::to_string(rho) +
                             ": domains over 64 sites a side run only with KMC_F_RESIDENT");
        }
        if (!(flags & (KMC_F_PERSISTENT | KMC_F_RESIDENT))) {
            // one block per phase task: the phase launches need the task
            // count below the dispatch limit, the dataflow launches one
            // sweep of tasks per phase
            if (c->n_tasks > kMaxBlocks)
                fail(c, KMC_EUNSUPPORTED, "more phase tasks than one launch can hold");
            if ((flags & KMC_F_FLOW) && flow_window(c) < 1)
                fail(c, KMC_EUNSUPPORTED, "one dataflow sweep exceeds the launch grid limit");
        }
        if (n_sweeps == 0) return KMC_OK;
        // every buffer the run needs is allocated before anything is
        // enqueued or any state changes: a failed allocation (KMC_ENOMEM)
        // leaves the context as it was
        const bool score = (flags & KMC_F_SCORE) != 0;
        const int64_t n_bins = (n_sweeps + record_every - 1) / record_every;
        ensure_records(c, c->n_rec + n_sweeps / record_every);
        if (flags & KMC_F_CHECKPOINT) {
            if (!c->c_spins) c->c_spins = alloc_n<int8_t>(c, c->spin_bytes);
            if (!c->c_dom) c->c_dom = alloc_n<Dom>(c, c->n_dom);
            if (!c->c_acc) c->c_acc = alloc_n<RepAcc>(c, c->n_rep);
        }
        if (flags & KMC_F_FLOW) ensure_flow_slots(c);
        if (score) ensure_bins(c, n_bins);
        if (flags & KMC_F_CHECKPOINT) {
            hip_check(c, hipMemcpyAsync(c->c_spins, c->d_spins, c->spin_bytes,
                                        hipMemcpyDeviceToDevice, c->stream), "checkpoint");
            hip_check(c, hipMemcpyAsync(c->c_dom, c->d_dom, sizeof(Dom) * c->n_dom,
                                        hipMemcpyDeviceToDevice, c->stream), "checkpoint");
            hip_check(c, hipMemcpyAsync(c->c_acc, c->d_acc, sizeof(RepAcc) * c->n_rep,
                                        hipMemcpyDeviceToDevice, c->stream), "checkpoint");
            c->have_ckpt = true;
            c->ck_sweep = c->sweep;
            c->ck_n_sweeps = n_sweeps;
            c->ck_rec_every = record_every;
            c->ck_flags = flags;
        }
        c->timing = (flags & KMC_F_TIMING) != 0;
        c->flow = (flags & KMC_F_FLOW) != 0;
        if (c->flow) {
            // counters restart with every run (a replay may go back in sweeps)
            hipLaunchKernelGGL(kmcdev::k_fill_i64, dim3((unsigned)((c->n_dom + 255) / 256)),
                               dim3(256), 0, c->stream, c->d_done, (int64_t)c->n_dom,
                               (int64_t)0);
        }
        KParams K = params(c);
        if (score || (flags & KMC_F_CHECKPOINT)) c->fused_score = false;
        if (score) {
            const int64_t nb = n_bins * c->n_rep * 2;
            hipLaunchKernelGGL(kmcdev::k_fill_f64, dim3((unsigned)((nb + 255) / 256)),
                               dim3(256), 0, c->stream, c->d_bins, nb, 0.0);
            K.bins = c->d_bins;
            K.n_bins = (int32_t)n_bins;
        }
        hipLaunchKernelGGL(kmcdev::k_set_ctl, dim3(1), dim3(1), 0, c->stream, c->d_ctl,
                           (int64_t)0, c->n_rec, (int64_t)record_every, c->sweep);
        if (!(flags & KMC_F_RESIDENT)) rebuild_edges(c, K);
        if (flags & KMC_F_RESIDENT) {
            if (score)
                launch_resident<true>(c, K, n_sweeps);
            else
                launch_resident<false>(c, K, n_sweeps);
        } else if (flags & KMC_F_PERSISTENT) {
            if (score)
                launch_persistent<true>(c, K, n_sweeps, flags);
            else if (flags & KMC_F_GRAPH)
                run_persistent_graph(c, K, n_sweeps, record_every, flags);
            else
                launch_persistent<false>(c, K, n_sweeps, flags);
        } else if (flags & KMC_F_GRAPH) {
            run_graph(c, n_sweeps);
        } else {
            if (score)
                run_sweeps<true>(c, K, n_sweeps);
            else
                run_sweeps<false>(c, K, n_sweeps);
        }
        if (score) {
            c->fused_score = true;
            c->fused_bins = (n_sweeps + record_every - 1) / record_every;
        }
        c->timing = false;
        c->n_rec += n_sweeps / record_every;
        c->sweep += n_sweeps;
    } catch (const Fail &f) {
        c->timing = false;
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_observables(kmc_ctx *c, kmc_record *out, int64_t capacity,
                                      int64_t *n_rec_out, uint32_t flags) {
    if (!c) return KMC_EINVAL;
    try {
        if (n_rec_out) *n_rec_out = c->n_rec;
        if (!out) return KMC_OK;
        if (capacity < 0) fail(c, KMC_EINVAL, "capacity must be >= 0");
        const int64_t n = std::min(capacity, c->n_rec);
        if (n == 0) return KMC_OK;
        if (flags & KMC_F_DEVICE_OUT) {
            const int64_t tot = (int64_t)c->n_rep * c->n_rec;
            hipLaunchKernelGGL(kmcdev::k_transpose_records, dim3((unsigned)((tot + 255) / 256)),
                               dim3(256), 0, c->stream, c->d_rec,
                               reinterpret_cast<Record *>(out), c->n_rep, c->n_rec, capacity);
            launch_check(c, "record transpose");
            return KMC_OK;
        }
        std::vector<Record> h((size_t)c->n_rec * c->n_rep);
        hip_check(c, hipMemcpyAsync(h.data(), c->d_rec, sizeof(Record) * h.size(),
                                    hipMemcpyDeviceToHost, c->stream), "record copy");
        hip_check(c, hipStreamSynchronize(c->stream), "record sync");
        check_flow_error(c, c->d_ctl);
        for (int rho = 0; rho < c->n_rep; ++rho)
            for (int64_t k = 0; k < n; ++k)
                std::memcpy(&out[rho * capacity + k], &h[k * c->n_rep + rho], sizeof(Record));
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_backward_score(kmc_ctx *c, double *score, int64_t capacity,
                                         uint32_t flags) {
    if (!c) return KMC_EINVAL;
    try {
        const hipMemcpyKind kind =
            (flags & KMC_F_DEVICE_OUT) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (c->fused_score) {  // accumulated by the run itself
            const int64_t n_bins = c->fused_bins;
            if (!score || capacity < n_bins)
                fail(c, KMC_EINVAL, "score buffer smaller than the number of intervals");
            hip_check(c, hipMemcpy2DAsync(score, (size_t)capacity * 2 * sizeof(double),
                                          c->d_bins, (size_t)n_bins * 2 * sizeof(double),
                                          (size_t)n_bins * 2 * sizeof(double), c->n_rep, kind,
                                          c->stream),
                      "score copy");
            if (!(flags & KMC_F_DEVICE_OUT)) {
                hip_check(c, hipStreamSynchronize(c->stream), "score sync");
                check_flow_error(c, c->d_ctl);
            }
            return KMC_OK;
        }
        if (!c->have_ckpt)
            fail(c, KMC_ESTATE, "no run with KMC_F_CHECKPOINT or KMC_F_SCORE");
        const int64_t n_bins = (c->ck_n_sweeps + c->ck_rec_every - 1) / c->ck_rec_every;
        if (!score || capacity < n_bins)
            fail(c, KMC_EINVAL, "score buffer smaller than the number of intervals");
        if (!c->r_spins) c->r_spins = alloc_n<int8_t>(c, c->spin_bytes);
        if (!c->r_edges) c->r_edges = alloc_n<uint64_t>(c, 2 * (int64_t)std::max(c->n_dom, 1));
        if (!c->r_dom) c->r_dom = alloc_n<Dom>(c, c->n_dom);
        if (!c->r_acc) c->r_acc = alloc_n<RepAcc>(c, c->n_rep);
        if (!c->r_ctl) c->r_ctl = alloc_n<Ctl>(c, 1);
        ensure_bins(c, n_bins);
        if (c->ck_flags & KMC_F_FLOW) ensure_flow_slots(c);
        hipStream_t s = c->stream;
        hip_check(c, hipMemcpyAsync(c->r_spins, c->c_spins, c->spin_bytes,
                                    hipMemcpyDeviceToDevice, s), "replay copy");
        hip_check(c, hipMemcpyAsync(c->r_dom, c->c_dom, sizeof(Dom) * c->n_dom,
                                    hipMemcpyDeviceToDevice, s), "replay copy");
        hip_check(c, hipMemcpyAsync(c->r_acc, c->c_acc, sizeof(RepAcc) * c->n_rep,
                                    hipMemcpyDeviceToDevice, s), "replay copy");
        const int64_t nb = n_bins * c->n_rep * 2;
        hipLaunchKernelGGL(kmcdev::k_fill_f64, dim3((unsigned)((nb + 255) / 256)), dim3(256),
                           0, s, c->d_bins, nb, 0.0);
        KParams K = params(c);
        K.spins = c->r_spins;
        K.edges = c->r_edges;
        K.dom = c->r_dom;
        K.acc = c->r_acc;
        K.ctl = c->r_ctl;
        K.bins = c->d_bins;
        K.n_bins = (int32_t)n_bins;
        K.write_records = 0;
        // each replay starts from the checkpoint with a clear error flag
        hip_check(c, hipMemsetAsync(c->r_ctl, 0, sizeof(Ctl), s), "replay ctl");
        hipLaunchKernelGGL(kmcdev::k_set_ctl, dim3(1), dim3(1), 0, s, c->r_ctl, (int64_t)0,
                           (int64_t)0, (int64_t)c->ck_rec_every, c->ck_sweep);
        if (!(c->ck_flags & KMC_F_RESIDENT)) rebuild_edges(c, K);
        if (c->ck_flags & KMC_F_RESIDENT) {
            launch_resident<true>(c, K, c->ck_n_sweeps);
        } else if (c->ck_flags & KMC_F_PERSISTENT) {
            launch_persistent<true>(c, K, c->ck_n_sweeps, c->ck_flags);
        } else {
            c->flow = (c->ck_flags & KMC_F_FLOW) != 0;
            if (c->flow)
                hipLaunchKernelGGL(kmcdev::k_fill_i64, dim3((unsigned)((c->n_dom + 255) / 256)),
                                   dim3(256), 0, s, c->d_done, (int64_t)c->n_dom, (int64_t)0);
            if (c->flow) ensure_flow_slots(c);
            K.flow_acc = c->d_flow_acc;
            K.flow_clk = c->d_flow_clk;
            run_sweeps<true>(c, K, c->ck_n_sweeps);
        }
        hip_check(c, hipMemcpy2DAsync(score, (size_t)capacity * 2 * sizeof(double), c->d_bins,
                                      (size_t)n_bins * 2 * sizeof(double),
                                      (size_t)n_bins * 2 * sizeof(double), c->n_rep, kind, s),
                  "score copy");
        if (!(flags & KMC_F_DEVICE_OUT)) {
            hip_check(c, hipStreamSynchronize(s), "score sync");
            if (c->ck_flags & KMC_F_FLOW) check_flow_error(c, c->r_ctl);
        }
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_get_spins(kmc_ctx *c, int32_t replica, int8_t *out) {
    if (!c || !out || replica < 0 || replica >= c->n_rep) {
        if (c) c->err = "kmc_get_spins: bad replica or output";
        return KMC_EINVAL;
    }
    try {
        const Rep &rp = c->reps[replica];
        const int64_t n = kmcdev::lattice_sites(rp);
        // domain by domain on the device, row-major out
        hipLaunchKernelGGL(kmcdev::k_spins_layout<false>, dim3((unsigned)((n + 255) / 256)),
                           dim3(256), 0, c->stream, params(c), replica, c->d_stage);
        launch_check(c, "spin layout");
        hip_check(c, hipMemcpyAsync(out, c->d_stage, (size_t)n, hipMemcpyDeviceToHost,
                                    c->stream), "spin copy");
        hip_check(c, hipStreamSynchronize(c->stream), "spin sync");
        check_flow_error(c, c->d_ctl);
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_get_domain_state(kmc_ctx *c, int32_t replica, double *clk_sum,
                                           double *clk_comp, int64_t *events) {
    if (!c || replica < 0 || replica >= c->n_rep) {
        if (c) c->err = "kmc_get_domain_state: bad replica";
        return KMC_EINVAL;
    }
    try {
        const Rep &rp = c->reps[replica];
        std::vector<Dom> h(rp.ND);
        hip_check(c, hipMemcpyAsync(h.data(), c->d_dom + rp.dom_off, sizeof(Dom) * rp.ND,
                                    hipMemcpyDeviceToHost, c->stream), "domain copy");
        hip_check(c, hipStreamSynchronize(c->stream), "domain sync");
        check_flow_error(c, c->d_ctl);
        for (int i = 0; i < rp.ND; ++i) {
            if (clk_sum) clk_sum[i] = h[i].clk_sum;
            if (clk_comp) clk_comp[i] = h[i].clk_comp;
            if (events) events[i] = h[i].events;
        }
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_get_domain_clocks(kmc_ctx *c, int32_t replica, double *t,
                                            double *comp) {
    return kmc_get_domain_state(c, replica, t, comp, nullptr);
}

extern "C" kmc_status kmc_get_info(kmc_ctx *c, int32_t replica, int32_t *n_rep,
                                   int32_t *n_domains) {
    if (!c) return KMC_EINVAL;
    if (n_rep) *n_rep = c->n_rep;
    if (n_domains) {
        if (replica < 0 || replica >= c->n_rep) return KMC_EINVAL;
        *n_domains = c->reps[replica].ND;
    }
    return KMC_OK;
}

extern "C" kmc_status kmc_get_timing(kmc_ctx *c, double *ms_total, int64_t *n_launches) {
    if (!c) return KMC_EINVAL;
    try {
        hip_check(c, hipStreamSynchronize(c->stream), "timing sync");
        double tot = 0.0;
        for (auto &pr : c->tev) {
            float ms = 0.0f;
            hip_check(c, hipEventElapsedTime(&ms, pr.first, pr.second), "elapsed time");
            tot += ms;
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        if (ms_total) *ms_total = tot;
        if (n_launches) *n_launches = (int64_t)c->tev.size();
        c->tev.clear();
    } catch (const Fail &f) {
        return f.st;
    }
    return KMC_OK;
}

extern "C" const char *kmc_last_error(const kmc_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

extern "C" void kmc_destroy(kmc_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph_stream) (void)hipStreamSynchronize(c->graph_stream);
    destroy_buffers(c);
    if (c->graph_stream) (void)hipStreamDestroy(c->graph_stream);
    for (auto &pr : c->tev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}
