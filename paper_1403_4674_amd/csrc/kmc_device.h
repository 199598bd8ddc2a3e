// kmc_device.h -- gfx950 kernels of libkmc.
//
// One 64-lane wavefront runs one domain process (Sec. 2.2: N_I ticks of a
// domain with its halo frozen).  Domains of one checkerboard colour never
// touch, so they run as independent wavefronts; colours follow the sweep's
// schedule (Eq. (schedule), Eq. (sum of sequential tms)).
//
// Wavefront layout of a B x B domain (4 <= B <= 64):
//   * lane y < B holds row y of the domain as a bit mask (bit x = spin up),
//     in a 32-bit word when B <= 32 and a 64-bit word otherwise;
//   * the top and bottom halo rows are wave-uniform masks and the left and
//     right halo columns one bit per lane; all are staged through LDS;
//   * per-site class c = 5*[s=+1] + k (k = up neighbours) is never stored:
//     three bit planes (k in binary) are rebuilt with two lane shuffles and
//     ~15 bitwise ops after each flip;
//   * lanes 0..9 hold the class counts n_c, the Q32 class weights
//     W_c = n_c r_c and their inclusive prefix (a 16-lane scan); R = P_9;
//   * ticks are drawn 64 at a time, one per lane, and one ballot finds the
//     first tick whose x falls below R: every earlier tick is a null tick,
//     exactly as if the ticks were tested one by one.
// Event selection (n-fold way): class = first c with x < P_c (ballot over
// lanes 0..9); member j = floor((x - P_{c-1}) / r_c) (exact integer, FP64
// quotient corrected by integer multiplies); the j-th member in ascending
// row-major order is found by a 64-lane prefix scan of per-row popcounts and
// a ballot, then a binary search inside the row's mask.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmcdev {

// Philox4x32-10 constants (Salmon et al., SC'11).
constexpr uint32_t kMulA = 0xD2511F53u;
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kKeyIncA = 0x9E3779B9u;
constexpr uint32_t kKeyIncB = 0xBB67AE85u;

// counter word 1 = domain | visit << 20 | stream << 24
constexpr uint32_t kStreamTick = 0;
constexpr uint32_t kStreamInit = 1;
constexpr uint32_t kStreamSched = 2;
constexpr uint32_t kStreamRetry0 = 3;
constexpr int kMaxRetry = 12;
// the time-slice variant: one call per event, redraws of its 64-bit
// selection word on streams 17 .. 28
constexpr uint32_t kStreamSlice = 16;
constexpr uint32_t kStreamSliceRetry0 = 17;

constexpr int kLdsPerWave = 64 * 64 + 2 * 64;  // tile + top/bottom halo rows
constexpr int kWavesPerPersistentGroup = 4;

struct Rates {
    uint64_t r[10];                       // Q32 rates
    double rd[10];                        // r as a double (exact: r <= 2^32)
    double inv_rd[10];                    // fl(1/r) (0 for r = 0)
    double w[10], aJ[10], ah[10];         // w, w*dlnw/dJ, w*dlnw/dh
    double gJ[10], gh[10];                // dlnw/dJ, dlnw/dh
};

struct Rep {
    int32_t L, B, NT, NI;   // lattice side, domain width Bx, L/Bx, ticks per visit
    int32_t By, NTy;        // domain height, L/By
    int32_t ncol, cx;       // colours of the domain grid, colours along x
    int32_t nperm;          // ncol! (orders of the random schedule)
    int32_t sched, ND;      // schedule kind, number of domains
    uint32_t nd, thr;       // sites per domain, 2^32 mod nd
    int64_t spin_off;       // byte offset of the lattice
    int32_t dom_off;        // first domain record
    int32_t task_off;       // first phase task
    int32_t visits;         // visits of each domain per sweep (1 or 2)
    int32_t init;           // kmc_init kind
    int32_t z;              // neighbours per site: 4 (L x L lattice) or 2 (ring
                            // of L sites: one row, By = NTy = 1)
    double tau;             // time slice of a domain process (> 0: the
                            // rejection-free variant; NI = 0 then)
};

// Sites of a replica's lattice: L^2, or L on the ring.
__device__ __host__ __forceinline__ int64_t lattice_sites(const Rep &rp) {
    return rp.z == 2 ? (int64_t)rp.L : (int64_t)rp.L * rp.L;
}

// Spins in HBM are held domain by domain: domain d = ty NT + tx owns the
// bytes [d n_d, (d + 1) n_d) of its replica's block, its By rows of Bx sites
// in order.  A visit's tile is then one contiguous run of whole memory
// sectors, and so is the row of a neighbouring domain that forms a halo row.
// (On the ring, and with one domain across, this is the plain row-major
// order.)  Only the kernels see this order: spins enter and leave the
// library row-major.
__device__ __host__ __forceinline__ int64_t site_offset(const Rep &rp, int y, int x) {
    const int ty = y / rp.By, tx = x / rp.B;
    return ((int64_t)(ty * rp.NT + tx) * rp.By + (y - ty * rp.By)) * rp.B + (x - tx * rp.B);
}

// The inverse: row-major index y L + x of the site at byte j of the block.
__device__ __host__ __forceinline__ int64_t row_major_of(const Rep &rp, int64_t j) {
    const int nd = (int)rp.nd;
    const int dd = (int)(j / nd), k = (int)(j - (int64_t)dd * nd);
    const int r = k / rp.B, c = k - r * rp.B;
    const int ty = dd / rp.NT, tx = dd - ty * rp.NT;
    return (int64_t)(ty * rp.By + r) * rp.L + tx * rp.B + c;
}

struct Dom {
    double clk_sum, clk_comp;  // compensated event clock
    int64_t events;
    int64_t pad;
};

struct RepAcc {
    int64_t M, B, events, pad;  // running totals (M, B include the start state)
};

struct Record {
    int64_t sweep, M, B, events, steps;
    double t;
};

struct Ctl {
    int64_t sweep;      // absolute index of the next sweep
    int64_t run_done;   // sweeps done in the current run
    int64_t rec_base;   // records written before the current run
    int64_t rec_every;  // record interval of the current run
    int64_t queue;      // persistent team-queue head
    int64_t queue2;     // persistent solo-queue head
    int64_t err;        // nonzero: a bounded wait of k_flow gave up
    int64_t pad;
};

struct KParams {
    const Rep *reps;
    const Rates *rates;
    int8_t *spins;
    Dom *dom;
    RepAcc *acc;
    Record *rec;
    Ctl *ctl;
    const int32_t *task_rep;  // phase task -> replica
    const int32_t *order;     // persistent queue: team replicas, then solo ones
    double *bins;             // score bins [n_rep][n_bins][2]
    int32_t n_rep;
    int32_t n_team;           // persistent queue: replicas run by a workgroup
    int32_t n_solo;           // persistent queue: replicas run by a wavefront
    int32_t n_bins;
    uint64_t seed;
    int32_t write_records;
    int32_t task_begin;       // first phase task of this launch
    // one-launch sweeps: per-sweep changes of M, B, events [sweep][replica][3]
    // and each domain's clock after the sweep [sweep][domain] (sum, comp)
    int64_t *flow_acc;
    double *flow_clk;
    int32_t n_dom_total;      // domain records of all replicas
    int64_t flow_max_polls;   // bound of each wait of the dataflow sweeps
    // edge columns of every domain as row bit masks [domain record][2]: its
    // first (x = ox) and last (x = ox + Bx - 1) column, bit r = row r.
    // Rebuilt from the spins before each run of the staged visits and kept
    // by them, so a visit reads its left and right halo as two words.
    uint64_t *edges;
};

// ------------------------------------------------------------------ Philox

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += kKeyIncA;
            k1 += kKeyIncB;
        }
        // one 32x32->64 product per word pair (v_mad_u64_u32): ~1.3x the
        // throughput of separate low and high multiplies on gfx950
        const uint64_t p0 = (uint64_t)kMulA * c0, p1 = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform index in [0, n) of the colour order of (replica, sweep), n = ncol!:
// Lemire multiply-high with rejection of the 2^32 mod n smallest low halves.
__device__ inline int schedule_index(uint64_t seed, uint32_t rho, uint32_t w, uint32_t n) {
    const uint32_t thr = (0u - n) % n;  // 2^32 mod n
    for (uint32_t call = 0;; ++call) {
        const uint4 o = philox(call, kStreamSched << 24, w, rho, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
        const uint32_t v[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t m = (uint64_t)v[i] * n;
            if ((uint32_t)m >= thr) return (int)(m >> 32);
        }
    }
}

// Positions of the permutation of {0..N-1} with lexicographic rank idx, as
// 4-bit fields: field e holds the position of element e.  Digit i of the
// rank in the factorial number system (radix (N-1-i)!, a constant once the
// loop is unrolled) picks among the unused values.
constexpr int cfact(int n) { return n <= 1 ? 1 : n * cfact(n - 1); }

template <int N>
__device__ __forceinline__ uint64_t perm_positions_n(int idx) {
    uint32_t avail = (1u << N) - 1u;
    uint64_t pos = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int f = cfact(N - 1 - i);
        const int a = idx / f;
        idx -= a * f;
        uint32_t m = avail;
        for (int k = 0; k < a; ++k) m &= m - 1u;  // drop the a smallest
        const int pick = __builtin_ctz(m);
        avail &= ~(1u << pick);
        pos |= (uint64_t)i << (4 * pick);
    }
    return pos;
}

// The colour counts a grid can have: 1, 2, 3 colours per axis.
__device__ inline uint64_t perm_positions(int idx, int n) {
    switch (n) {
    case 2: return perm_positions_n<2>(idx);
    case 3: return perm_positions_n<3>(idx);
    case 4: return perm_positions_n<4>(idx);
    case 6: return perm_positions_n<6>(idx);
    case 9: return perm_positions_n<9>(idx);
    default: return 0;  // one colour
    }
}

// Element at position p of that permutation.
__device__ inline int perm_element(int idx, int p, int n) {
    const uint64_t pos = perm_positions(idx, n);
    int out = 0;
    for (int e = 0; e < n; ++e)
        if ((int)((pos >> (4 * e)) & 15u) == p) out = e;
    return out;
}

// Colouring of the domain grid, per axis of n domains: one colour for a
// single domain, t mod 2 for an even count, t mod 2 with the last domain
// given colour 2 for an odd count (an odd cycle needs three colours).  The
// colour of domain (ty, tx) is ax + cx ay; domains of one colour never share
// an edge, so they commute (Sec. 2.2).
__device__ __forceinline__ int axis_colour(int t, int n) {
    return n == 1 ? 0 : ((n & 1) && t == n - 1) ? 2 : (t & 1);
}
// Number of domains of axis colour a, and the position of the i-th of them.
__device__ __forceinline__ int axis_count(int a, int n) {
    return n == 1 ? (a == 0 ? 1 : 0) : (n & 1) ? (a == 2 ? 1 : (n - 1) >> 1) : (a < 2 ? n >> 1 : 0);
}
__device__ __forceinline__ int axis_pos(int i, int a, int n) {
    return ((n & 1) && a == 2) ? n - 1 : 2 * i + a;
}
__device__ __forceinline__ int dom_colour(const Rep &rp, int ty, int tx) {
    return axis_colour(tx, rp.NT) + rp.cx * axis_colour(ty, rp.NTy);
}
// Axis colours (ax, ay) of colour col (cx is 1, 2 or 3; col < 9).
__device__ __forceinline__ void split_colour(const Rep &rp, int col, int *ax, int *ay) {
    const int y = rp.cx == 2 ? col >> 1 : rp.cx == 1 ? col : (col * 11) >> 5;  // col / 3
    *ay = y;
    *ax = col - rp.cx * y;
}

// Colour and visit index of phase p of sweep w (p < ncol for the random
// order, p < 2 ncol for the palindrome); -1 when the phase is empty.
__device__ inline int phase_colour(const Rep &rp, uint64_t seed, uint32_t rho,
                                   uint32_t w, int p, int *visit) {
    const int n = rp.ncol;
    if (rp.sched == 1) {  // 0 1 .. n-1 n-1 .. 1 0, second visits on the way back
        *visit = p < n ? 0 : 1;
        if (p >= 2 * n) return -1;
        return p < n ? p : 2 * n - 1 - p;
    }
    *visit = 0;
    if (p >= n) return -1;
    return perm_element(schedule_index(seed, rho, w, (uint32_t)rp.nperm), p, n);
}

// phase_colour for a replica known to be a 4-colour checkerboard (the
// multi-slot kernel's replicas): the same colours and visits.
__device__ inline int phase_colour4(uint32_t sched, uint64_t seed, uint32_t rho, uint32_t w,
                                    int p, int *visit) {
    if (sched == 1) {
        *visit = p < 4 ? 0 : 1;
        return p < 8 ? (p < 4 ? p : 7 - p) : -1;
    }
    *visit = 0;
    if (p >= 4) return -1;
    const uint64_t pos = perm_positions_n<4>(schedule_index(seed, rho, w, 24u));
    int out = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if ((int)((pos >> (4 * e)) & 15u) == p) out = e;
    return out;
}

// ------------------------------------------------------------ wave helpers
//
// Lane-to-lane moves inside the event chain use DPP (data-parallel
// primitives: a VALU operand modifier, no LDS round trip).  Out-of-range
// source lanes and rows excluded by the row mask read 0.

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// DPP move with bound control: lanes whose source is out of range read 0
// (all rows and banks written, so no previous value is needed).
template <int CTRL>
__device__ __forceinline__ uint32_t dppz(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// sched_barrier mask: scalar instructions may be moved across, vector ones not
constexpr int kSchedScalarMayCross = 0x4;

constexpr int kWaveShr1 = 0x138;   // lane i <- lane i-1
constexpr int kWaveShl1 = 0x130;   // lane i <- lane i+1
constexpr int kRowShr = 0x110;     // + n: lane i <- lane i-n inside a row of 16
constexpr int kRowBcast15 = 0x142; // lane 15 of each row -> the next row
constexpr int kRowBcast31 = 0x143; // lane 31 -> rows 2 and 3

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_any(T v) {
    if constexpr (sizeof(T) == 8) {
        const uint32_t lo = dpp<CTRL>((uint32_t)v);
        const uint32_t hi = dpp<CTRL>((uint32_t)(v >> 32));
        return ((T)hi << 32) | lo;
    } else {
        return (T)dpp<CTRL>((uint32_t)v);
    }
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t scan64(uint32_t v) {
    v += dppz<kRowShr + 1>(v);
    v += dppz<kRowShr + 2>(v);
    v += dppz<kRowShr + 4>(v);
    v += dppz<kRowShr + 8>(v);
    v += dpp<kRowBcast15, 0xA>(v);
    v += dpp<kRowBcast31, 0xC>(v);
    return v;
}

// Inclusive prefix sum over lanes 0..15 (64-bit values).
__device__ __forceinline__ uint64_t scan16_dpp(uint64_t v) {
    v += dpp_any<kRowShr + 1>(v);
    v += dpp_any<kRowShr + 2>(v);
    v += dpp_any<kRowShr + 4>(v);
    v += dpp_any<kRowShr + 8>(v);
    return v;
}

// Sum over lanes 0..15 of a double, returned in every lane.
__device__ __forceinline__ double rowsum16_f64(double v, int lane);

__device__ __forceinline__ uint32_t rdl32(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint64_t rdl64(uint64_t v, int lane) {
    const uint32_t lo = rdl32((uint32_t)v, lane);
    const uint32_t hi = rdl32((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double rdl_f64(double v, int lane) {
    return __longlong_as_double((long long)rdl64((uint64_t)__double_as_longlong(v), lane));
}

template <int CTRL>
__device__ __forceinline__ double dppz_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = dppz<CTRL>((uint32_t)b), hi = dppz<CTRL>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Inclusive prefix sum over each 16-lane row of doubles.  Used for integer
// rate sums below 2^53, where every addition is exact.
__device__ __forceinline__ double scan16_f64(double v) {
    v += dppz_f64<kRowShr + 1>(v);
    v += dppz_f64<kRowShr + 2>(v);
    v += dppz_f64<kRowShr + 4>(v);
    v += dppz_f64<kRowShr + 8>(v);
    return v;
}

// Inclusive prefix sum over lanes 0..31 (lanes 32..63 get sums of their own).
__device__ __forceinline__ uint32_t scan32(uint32_t v) {
    v += dppz<kRowShr + 1>(v);
    v += dppz<kRowShr + 2>(v);
    v += dppz<kRowShr + 4>(v);
    v += dppz<kRowShr + 8>(v);
    v += dpp<kRowBcast15, 0xA>(v);
    return v;
}

// Total of lanes 0..15 (the last element of the row scan; the multi-slot
// kernel sums in the same order, so the two agree bit for bit).
__device__ __forceinline__ double rowsum16_f64(double v, int lane) {
    (void)lane;
    return rdl_f64(scan16_f64(v), 15);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t scan16(uint64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        const uint64_t t = __shfl_up(v, o);
        if ((lane & 15) >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double sum16_f64(double v) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void neumaier_add(double &sum, double &comp, double x) {
    const double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

template <typename MT>
__device__ __forceinline__ int popc(MT m) {
    if constexpr (sizeof(MT) == 8)
        return __popcll(m);
    else
        return __popc(m);
}

// Number of set bits of the wave-uniform mask m below this lane.
__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Position of the n-th (0-based) set bit of m; n < popc(m).
template <typename MT>
__device__ __forceinline__ int nth_set_bit(MT m, int n) {
    int pos = 0;
    if constexpr (sizeof(MT) == 8) {
        const int pc = __popc((uint32_t)m);
        if (n >= pc) {
            n -= pc;
            m >>= 32;
            pos += 32;
        }
    }
    uint32_t v = (uint32_t)m;
#pragma unroll
    for (int width = 16; width >= 1; width >>= 1) {
        const int pc = __popc(v & ((1u << width) - 1u));
        if (n >= pc) {
            n -= pc;
            v >>= width;
            pos += width;
        }
    }
    return pos;
}

// Four row bytes (+1 / -1) -> four bits (1 = up).
__device__ __forceinline__ uint32_t bytes_to_bits(uint32_t v) {
    const uint32_t b = (~v >> 7) & 0x01010101u;
    return (b | (b >> 7) | (b >> 14) | (b >> 21)) & 0xFu;
}

__device__ __forceinline__ uint32_t bits_to_bytes(uint32_t nib) {
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) v |= (((nib >> i) & 1u) ? 0x01u : 0xFFu) << (8 * i);
    return v;
}

// Bit planes of the up-neighbour count k (k = s0 + 2 s1 + 4 s2) of every site
// of this lane's row.
template <typename MT>
struct Planes {
    MT s0, s1, s2;
};

template <typename MT>
__device__ __forceinline__ Planes<MT> neighbour_planes(MT S, MT top, MT bot,
                                                      MT hl, MT hr, int Bx, int By,
                                                      MT VM, int lane) {
    MT U = dpp_any<kWaveShr1>(S);
    if (lane == 0) U = top;
    MT D = dpp_any<kWaveShl1>(S);
    if (lane == By - 1) D = bot;
    const MT Lf = ((S << 1) | hl) & VM;
    const MT Rt = ((S >> 1) | (hr << (Bx - 1))) & VM;
    U &= VM;
    D &= VM;
    const MT p1 = U ^ D, q1 = U & D;
    const MT p2 = Lf ^ Rt, q2 = Lf & Rt;
    const MT c0 = p1 & p2;
    Planes<MT> P;
    P.s0 = p1 ^ p2;
    P.s1 = q1 ^ q2 ^ c0;
    P.s2 = (q1 & q2) | (c0 & (q1 ^ q2));
    return P;
}

// Sites of class c = 5 [s=+1] + k among this lane's row.  Each plane is
// taken as is or complemented; bit c of these tables says "complement"
// (s = -1 for c < 5; k0, k1, k2 = 0), expanded to all ones by 0 - bit.
// (The signed bit-field builtin is avoided: the compiler takes its result
// for non-negative and drops the upper word of a 64-bit extension.)
constexpr uint32_t kInvS = 0x01F, kInvK0 = 0x2B5, kInvK1 = 0x273, kInvK2 = 0x1EF;

template <typename MT>
__device__ __forceinline__ MT class_mask(int c, MT S, const Planes<MT> &P, MT VM) {
    const MT xS = (MT)0 - (MT)__builtin_amdgcn_ubfe(kInvS, c, 1);
    const MT x0 = (MT)0 - (MT)__builtin_amdgcn_ubfe(kInvK0, c, 1);
    const MT x1 = (MT)0 - (MT)__builtin_amdgcn_ubfe(kInvK1, c, 1);
    const MT x2 = (MT)0 - (MT)__builtin_amdgcn_ubfe(kInvK2, c, 1);
    return (S ^ xS) & (P.s0 ^ x0) & (P.s1 ^ x1) & (P.s2 ^ x2) & VM;
}

// The same selection for a class c held in a scalar register, as in the
// event chain: the four complement masks are sign-extended table bits taken
// by the scalar unit (s_bfe_i32 with width 1 gives 0 or all ones), and the
// mask is a chain of t & (plane ^ x) steps, one 3-input bit operation each
// (truth table 0x60 = src0 & (src1 ^ src2)).
struct ClassSel {
    uint32_t xS, x0, x1, x2;
};

// The table is an immediate of the instruction (a literal, or an inline
// constant), so no register is spent on it in the chain.
template <uint32_t TABLE>
__device__ __forceinline__ uint32_t sgpr_sign_bit(uint32_t c) {
    uint32_t r;
    asm("s_bfe_i32 %0, %1, %2" : "=s"(r) : "i"(TABLE), "s"(c | 0x10000u) : "scc");
    return r;
}

__device__ __forceinline__ ClassSel class_sel(int c) {
    return ClassSel{sgpr_sign_bit<kInvS>((uint32_t)c), sgpr_sign_bit<kInvK0>((uint32_t)c),
                    sgpr_sign_bit<kInvK1>((uint32_t)c), sgpr_sign_bit<kInvK2>((uint32_t)c)};
}

__device__ __forceinline__ uint32_t and_xor(uint32_t t, uint32_t v, uint32_t x) {
    return __builtin_amdgcn_bitop3_b32(t, v, x, 0x60);
}

template <typename MT>
__device__ __forceinline__ MT class_mask(const ClassSel &q, MT S, const Planes<MT> &P, MT VM) {
    if constexpr (sizeof(MT) == 8) {
        auto half = [&](int h) {
            const uint32_t sh = 32 * h;
            uint32_t t = and_xor((uint32_t)(VM >> sh), (uint32_t)(S >> sh), q.xS);
            t = and_xor(t, (uint32_t)(P.s0 >> sh), q.x0);
            t = and_xor(t, (uint32_t)(P.s1 >> sh), q.x1);
            return and_xor(t, (uint32_t)(P.s2 >> sh), q.x2);
        };
        return (MT)half(0) | ((MT)half(1) << 32);
    } else {
        uint32_t t = and_xor(VM, S, q.xS);
        t = and_xor(t, P.s0, q.x0);
        t = and_xor(t, P.s1, q.x1);
        return and_xor(t, P.s2, q.x2);
    }
}

// Per-lane form (the class differs between the slots of a wavefront): the
// vector signed bit-field extract gives 0 or all ones per lane.
__device__ __forceinline__ uint32_t vgpr_sign_bit(uint32_t table, uint32_t c) {
    uint32_t r;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "s"(table), "v"(c));
    return r;
}

__device__ __forceinline__ ClassSel class_sel_lane(uint32_t c) {
    return ClassSel{vgpr_sign_bit(kInvS, c), vgpr_sign_bit(kInvK0, c), vgpr_sign_bit(kInvK1, c),
                    vgpr_sign_bit(kInvK2, c)};
}

template <typename MT>
__device__ __forceinline__ int class_at(MT S, const Planes<MT> &P, int b) {
    return 5 * (int)((S >> b) & 1) + (int)((P.s0 >> b) & 1) +
           2 * (int)((P.s1 >> b) & 1) + 4 * (int)((P.s2 >> b) & 1);
}

// 3 * class of site b of this lane's row (the bit offset of the class's
// field in a packed 3-bit tally word).
template <typename MT>
__device__ __forceinline__ uint32_t class_pos3(MT S, const Planes<MT> &P, int b) {
    uint32_t s, p0, p1, p2;
    if constexpr (sizeof(MT) == 8) {
        s = (uint32_t)(S >> b);
        p0 = (uint32_t)(P.s0 >> b);
        p1 = (uint32_t)(P.s1 >> b);
        p2 = (uint32_t)(P.s2 >> b);
        b = 0;
    } else {
        s = S;
        p0 = P.s0;
        p1 = P.s1;
        p2 = P.s2;
    }
    // k = k0 + 2 k1 + 4 k2, then 3 (k + 5 s)
    const uint32_t k = __builtin_amdgcn_ubfe(p0, b, 1) | (__builtin_amdgcn_ubfe(p1, b, 1) << 1) |
                       (__builtin_amdgcn_ubfe(p2, b, 1) << 2);
    const uint32_t q = k + 5u * __builtin_amdgcn_ubfe(s, b, 1);
    return q + 2u * q;
}

// Adds one (inv = 0) or subtracts one (inv = all ones) from the
// up-neighbour count k of the sites in m, on the bit planes; no site
// overflows (k stays in 0..4).
template <typename MT>
__device__ __forceinline__ void planes_step_inv(Planes<MT> &P, MT m, MT inv) {
    const MT c1 = (P.s0 ^ inv) & m;
    const MT c2 = (P.s1 ^ inv) & c1;
    P.s0 ^= m;
    P.s1 ^= c1;
    P.s2 ^= c2;
}

template <typename MT>
__device__ __forceinline__ void planes_step(Planes<MT> &P, MT m, bool inc) {
    planes_step_inv<MT>(P, m, inc ? (MT)0 : ~(MT)0);
}

// Natural logarithm of u in (0, 1] for the stop decisions of the time-slice
// variant, by the atanh series: u = m 2^e with m in [sqrt(1/2), sqrt(2)),
// f = m - 1 (exact), s = f / (2 + f), ln m = 2 s (1 + z/3 + z^2/5 + ...) with
// z = s^2 <= 0.0295 (twelve terms), ln u = e ln2_hi + (ln m + e ln2_lo) where
// ln2_hi holds 32 significant bits (e ln2_hi is exact).  Only IEEE additions,
// multiplications and correctly rounded divisions, in a fixed order and
// without contraction, so the value is reproducible bit for bit by any
// implementation of the same steps; within 2 ulp of ln u.
__device__ __forceinline__ double slice_log(double u) {
    const double ln2_hi = 0x1.62e42ffp-1;
    const double ln2_lo = -0x1.718432a1b0e26p-35;
    const uint64_t bits = (uint64_t)__double_as_longlong(u);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    double m = __longlong_as_double(
        (long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double sv = f / (2.0 + f);
    const double z = sv * sv;
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
    const double two_s = sv + sv;
    const double lm = two_s + (two_s * z) * q;
    const double de = (double)e;
    return de * ln2_hi + (lm + de * ln2_lo);
}

// m / den for the score of a run of m null ticks (den > 0): the hardware
// reciprocal refined by two Newton steps (within an ulp of 1/den), times m.
// Cheaper than the correctly rounded quotient.  Every form of the score
// uses it, so where the visits' scores are summed in a fixed order (the
// persistent and resident forms) fused and replayed scores agree bit for
// bit; the phase and dataflow forms add them with atomics, in no fixed
// order, so there the bins agree to rounding.
__device__ __forceinline__ double null_quot(uint32_t m, double den) {
    double r = __builtin_amdgcn_rcp(den);
    double e = __builtin_fma(-den, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-den, r, 1.0);
    r = __builtin_fma(r, e, r);
    return (double)m * r;
}

struct VisitOut {
    int64_t events;
    int64_t dM, dB;
    double sJ, sh;
};

// One domain process: N_I ticks of domain d (origin oy, ox) of the lattice
// `lat` (side L, domains Bx x By, held domain by domain).  Executed by one
// full wavefront; `lds` points at this wavefront's kLdsPerWave bytes.
// `edges` is the replica's edge-column table (two row masks per domain): the
// left and right halo are read from the neighbours' entries, and the
// domain's own entry is rewritten with the tile.  The domain's compensated
// clock in *dom is advanced; the changes of M, B and the event count are
// returned (and the score when SCORE).  WRAP admits replicas whose lattice
// is a single periodic domain; without it the wrap-around bookkeeping is
// compiled out of the event chain (every instruction of the chain costs an
// issue slot when a wavefront runs alone on its SIMD).
template <typename MT, bool SCORE, bool WRAP, bool SLICE = false>
__device__ VisitOut visit_domain(int8_t *__restrict__ lat, const Rep &rp,
                                 const Rates *__restrict__ rt, int oy, int ox,
                                 uint32_t d, uint32_t vis, uint32_t w,
                                 uint32_t rho, uint64_t seed, Dom *dom,
                                 uint64_t *edges, uint8_t *lds) {
    const int lane = __lane_id();
    // B: row width (bits of a row mask), By: rows (lanes)
    const int B = rp.B, By = rp.By, NI = rp.NI;
    const int B4 = B >> 2;
    const uint32_t nd = rp.nd, thr = rp.thr;

    // neighbouring domains (periodic), from the origin: no division
    const int NT = rp.NT, NTy = rp.NTy;
    const int dd = (int)d;
    const int d_up = oy == 0 ? dd + (NTy - 1) * NT : dd - NT;
    const int d_dn = oy + By == By * NTy ? dd - (NTy - 1) * NT : dd + NT;
    const int d_lf = ox == 0 ? dd + NT - 1 : dd - 1;
    const int d_rt = ox + B == B * NT ? dd - (NT - 1) : dd + 1;

    // ---- stage the tile and the top/bottom halo rows through LDS.  LDS rows
    // are padded to whole dwords (stride SB).  With widths that are multiples
    // of 4 the LDS tile is the HBM tile byte for byte and moves in 16-byte
    // (else 4-byte) pieces; other widths move byte by byte.  Every load of
    // the visit (tile, halo rows, edge words, rate tables, domain record) is
    // issued before the first one is waited for: one memory round trip
    // instead of one per kind.
    const int SB = (B + 3) & ~3, SB4 = SB >> 2;
    uint8_t *tile = lds;
    uint8_t *hrow = lds + 64 * 64;  // [0, B): top halo, [64, 64 + B): bottom
    const int8_t *blk = lat + (int64_t)dd * (int)nd;
    const int8_t *up_row = lat + (int64_t)d_up * (int)nd + (By - 1) * B;  // its last row
    const int8_t *dn_row = lat + (int64_t)d_dn * (int)nd;                 // its first row
    // the ring (one row of L sites) has no rows above and below: its domains
    // have no top and bottom halo, and those neighbours count as down
    const bool ring = rp.z == 2;
    const bool vec4 = (B & 3) == 0, vec16 = vec4 && (nd & 15u) == 0;
    const int n16 = vec16 ? (int)(nd >> 4) : 0;  // at most 64 * 64 / 16 = 4 per lane
    // (every lane of a row of pieces loads, the last lanes clamped to the
    // last piece, so the loads carry no lane mask and nothing waits for them
    // here)
    const uint4 *blk16 = reinterpret_cast<const uint4 *>(blk);
    uint4 tv0 = {0, 0, 0, 0}, tv1 = tv0, tv2 = tv0, tv3 = tv0;
    if (n16 > 0) tv0 = blk16[min(lane, n16 - 1)];
    if (n16 > 64) tv1 = blk16[min(lane + 64, n16 - 1)];
    if (n16 > 128) tv2 = blk16[min(lane + 128, n16 - 1)];
    if (n16 > 192) tv3 = blk16[min(lane + 192, n16 - 1)];
    const bool hlane = vec4 && lane < 2 * B4 && !ring;
    const int hwhich = hlane ? lane / B4 : 0, hc4 = hlane ? lane - hwhich * B4 : 0;
    uint32_t hv = 0;
    if (hlane) hv = *reinterpret_cast<const uint32_t *>((hwhich ? dn_row : up_row) + 4 * hc4);
    // left halo: the left neighbour's last column; right: the right one's first
    const uint64_t e_lf = edges[2 * d_lf + 1], e_rt = edges[2 * d_rt];
    const double rd_lane = lane < 10 ? rt->rd[lane] : 0.0;
    const double inv_lane = lane < 10 ? rt->inv_rd[lane] : 0.0;
    double w_lane = 0.0;  // score: w_c in the class lanes (the other tables at the end)
    if constexpr (SCORE) {
        if (lane < 10) w_lane = rt->w[lane];
    }
    // the domain record (only this domain's visits write it), updated at the end
    double dom_sum = 0.0, dom_comp = 0.0;
    int64_t dom_ev = 0;
    if (lane == 0) {
        dom_sum = dom->clk_sum;
        dom_comp = dom->clk_comp;
        dom_ev = dom->events;
    }
    if (vec16) {
        uint4 *tile16 = reinterpret_cast<uint4 *>(tile);
        if (lane < n16) tile16[lane] = tv0;
        if (lane + 64 < n16) tile16[lane + 64] = tv1;
        if (lane + 128 < n16) tile16[lane + 128] = tv2;
        if (lane + 192 < n16) tile16[lane + 192] = tv3;
    } else if (vec4) {
        for (int q = lane; q < (int)(nd >> 2); q += 64)
            *reinterpret_cast<uint32_t *>(tile + 4 * q) =
                *reinterpret_cast<const uint32_t *>(blk + 4 * q);
    } else {
        for (int q = lane; q < By * B; q += 64) {
            const int row = q / B, col = q - row * B;
            tile[row * SB + col] = (uint8_t)blk[q];
        }
        for (int q = lane; q < 2 * B && !ring; q += 64) {
            const int which = q / B, col = q - which * B;
            hrow[which * 64 + col] = (uint8_t)(which ? dn_row : up_row)[col];
        }
    }
    if (hlane) *reinterpret_cast<uint32_t *>(hrow + hwhich * 64 + 4 * hc4) = hv;
    const MT hl = lane < By ? (MT)((e_lf >> lane) & 1u) : (MT)0;
    const MT hr = lane < By ? (MT)((e_rt >> lane) & 1u) : (MT)0;
    wave_sync_lds();

    const MT vm_row = B == 8 * (int)sizeof(MT) ? ~(MT)0 : (((MT)1 << B) - 1);
    const MT VM = lane < By ? vm_row : (MT)0;
    MT S = 0, top = 0, bot = 0;
    for (int q = 0; q < SB4; ++q) {
        if (lane < By)
            S |= (MT)bytes_to_bits(
                     *reinterpret_cast<const uint32_t *>(tile + lane * SB + 4 * q))
                 << (4 * q);
        top |= (MT)bytes_to_bits(*reinterpret_cast<const uint32_t *>(hrow + 4 * q))
               << (4 * q);
        bot |= (MT)bytes_to_bits(*reinterpret_cast<const uint32_t *>(hrow + 64 + 4 * q))
               << (4 * q);
    }
    S &= VM;  // padding bytes decode to set bits: clear them
    top = ring ? (MT)0 : top & vm_row;
    bot = ring ? (MT)0 : bot & vm_row;
    Planes<MT> P = neighbour_planes<MT>(S, top, bot, hl, hr, B, By, VM, lane);

    // ---- class counts: per-row popcounts, two classes per 32-bit word
    uint32_t n_lane = 0;  // lanes 0..9: n_c
#pragma unroll
    for (int c = 0; c < 10; c += 2) {
        const uint32_t a = popc(class_mask<MT>(c, S, P, VM));
        const uint32_t b = popc(class_mask<MT>(c + 1, S, P, VM));
        const uint32_t tot = rdl32(scan64(a | (b << 16)), 63);
        if (lane == c) n_lane = tot & 0xFFFFu;
        if (lane == c + 1) n_lane = tot >> 16;
    }
    // Rate sums are integers below n_d 2^32 <= 2^44, held in doubles: every
    // sum, difference, product n_c * r_c and comparison below is exact.
    const uint32_t lane3 = lane < 10 ? 3u * lane : 30u;  // tally field (30: always 0)
    double W = (double)n_lane * rd_lane;
    double Pinc = scan16_f64(W);
    double R = rdl_f64(Pinc, 9);

    VisitOut out{0, 0, 0, 0.0, 0.0};
    uint32_t ev_lane = 0;                  // lanes 0..9: events of class c = lane
    double clk_sum = 0.0, clk_comp = 0.0;  // this lane's events' residence times
    uint32_t m_null = 0;                   // null ticks since the last event (score)
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = d | (vis << 20) | (kStreamTick << 24);
    // along an axis with a single domain (one domain, or a stripe) the
    // domain is periodic in itself: its boundary neighbours on that axis are
    // its own sites and change during the visit
    const int wrapY = WRAP && rp.NTy == 1 && !ring ? By : 0;
    const int wrapX = WRAP && rp.NT == 1 ? B : 0;

    // Score.  A run of m null ticks adds m d ln(1 - R_w/n_d)/d theta =
    // -m sum_c n_c a_c / (n_d - R_w) (a_c = w_c d ln w_c/d theta), linear in
    // the counts: class lane c accumulates A_c = sum over runs of
    // m n_c / (n_d - R_w), and the visit's score is
    // sum_c (events_c g_c - a_c A_c), formed once at the end.
    double A_lane = 0.0;
    auto null_run = [&](uint32_t m) {
        const double nl = (double)n_lane;
        const double Rw = rowsum16_f64(nl * w_lane, lane);
        const double den = (double)nd - Rw;
        if (den > 0.0) A_lane += null_quot(m, den) * nl;
    };

    // One event at x_e (held as x_e + 1/2): rate class, member, flip and the
    // class bookkeeping of the flipped site and its in-tile neighbours.
    auto event = [&](const double xe) {
        // rate class: first c with x_e < P_c (lane 9 holds R > x_e).
        // Member index j = floor((x_e - P_{c-1}) / r_c), formed in every
        // class lane at once as trunc((x_e + 1/2 - P_{c-1}) fl(1/r_c)): the
        // quotient lies at least 1/(2 r_c) >= 2^-33 from an integer and
        // the product is within 2^-39 of it (quotient < 2^13), so the
        // truncation is exact.  Only lane c's quotient is read, then
        // converted.
        const int c = __builtin_ctzll(__ballot(xe < Pinc));
        const double q = (xe - (Pinc - W)) * inv_lane;
        const uint32_t j = (uint32_t)rdl_f64(q, c);

        if constexpr (SCORE) {
            if (m_null) null_run(m_null);
        }
        m_null = 0;

        // member j of class c in ascending row-major order: the row by a
        // scan of per-row counts, the column by counting the row's
        // members below each lane (mbcnt)
        const MT cm = class_mask<MT>(class_sel(c), S, P, VM);
        const uint32_t cnt = (uint32_t)popc(cm);
        const uint32_t incl = sizeof(MT) == 4 ? scan32(cnt) : scan64(cnt);
        const int ys = __builtin_ctzll(__ballot(incl > j));
        const uint32_t jr = j - rdl32(incl - cnt, ys);
        int xs;
        if constexpr (sizeof(MT) == 8) {
            const uint64_t row = rdl64(cm, ys);
            xs = __builtin_ctzll(__ballot(bits_below_lane(row) == jr) & row);
        } else {
            const uint32_t row = rdl32(cm, ys);
            xs = __builtin_ctzll(
                __ballot(__builtin_amdgcn_mbcnt_lo(row, 0u) == jr) & (uint64_t)row);
        }

        // class changes of the flipped site and its in-tile neighbours as
        // packed 3-bit per-class tallies (10 classes in 30 bits): row ys
        // holds the sites at columns xs -/+ 1, rows ys -/+ 1 the site at
        // column xs; the three rows are summed into row ys by DPP
        // neighbour rows and columns; outside the tile (-1 or B) they are
        // halo and frozen, unless the lattice is one periodic domain
        // upm: all ones when the flipped spin is +1 (c >= 5), whose
        // neighbours then lose an up neighbour; the flipped site moves
        // to class c -/+ 5 (tally field 3 c -/+ 15)
        const uint32_t upm = sgpr_sign_bit<0x3E0>((uint32_t)c);
        const int c3 = 3 * c;
        const int c3_new = c3 + 15 - (int)(upm & 30u);
        const bool on_row = lane == ys;
        constexpr int NB = 8 * (int)sizeof(MT);
        int ym = ys - 1, yp = ys + 1, xm = xs - 1, xp = xs + 1;
        bool adj;
        MT nm = 0;    // this lane's neighbours of the flipped site
        uint32_t nb;  // their classes as tallies
        if constexpr (!WRAP) {
            // row ys: columns xs -/+ 1 inside the tile; rows ys -/+ 1:
            // column xs.  Each lane reads its sites at xa (xs - 1 on row
            // ys, else xs) and xb = xs + 1; a column outside the tile, or
            // not this lane's, is a clear bit of nm
            const MT bx = (MT)1 << xs;
            const MT mrow = ((bx << 1) | (bx >> 1)) & vm_row;
            adj = (lane == ym || lane == yp) && lane < By;
            nm = on_row ? mrow : (adj ? bx : (MT)0);
            const int xa = (xs - (on_row ? 1 : 0)) & (NB - 1), xb = (xs + 1) & (NB - 1);
            const uint32_t va = (uint32_t)(nm >> xa) & 1u, vb = (uint32_t)(nm >> xb) & 1u;
            nb = (va << class_pos3<MT>(S, P, xa)) + (vb << class_pos3<MT>(S, P, xb));
            // the old classes are read: move the neighbours' up-counts on
            // the bit planes, sum the tallies, flip.  The barriers pin this
            // vector order (scalar work may cross them): the plane update
            // and the flip then sit in the waits of the DPP sum and of its
            // read-back.  (Measured: 3 % off the dataflow sweep.)
            planes_step_inv<MT>(P, nm, (MT)(int64_t)(int32_t)upm);
            __builtin_amdgcn_sched_barrier(kSchedScalarMayCross);
            nb += dppz<kWaveShr1>(nb) + dppz<kWaveShl1>(nb);
            __builtin_amdgcn_sched_barrier(kSchedScalarMayCross);
            if (on_row) S ^= bx;
            __builtin_amdgcn_sched_barrier(kSchedScalarMayCross);
        } else {
            ym += ys == 0 ? wrapY : 0;
            yp -= ys == By - 1 ? wrapY : 0;
            xm += xs == 0 ? wrapX : 0;
            xp -= xs == B - 1 ? wrapX : 0;
            adj = (lane == ym || lane == yp) && lane < By;
            const int ca = on_row ? xm : xs;
            const bool va = on_row ? xm >= 0 : adj;
            const bool vb = on_row && xp < B;
            const uint32_t pa = class_pos3<MT>(S, P, ca & (NB - 1));
            const uint32_t pb = class_pos3<MT>(S, P, xp & (NB - 1));
            nb = ((va ? 1u : 0u) << pa) + ((vb ? 1u : 0u) << pb);
        }
        uint32_t nb_s;
        if (wrapY == 0) {  // rows ys -/+ 1 are the neighbouring lanes
            if constexpr (WRAP) nb += dppz<kWaveShr1>(nb) + dppz<kWaveShl1>(nb);
            nb_s = rdl32(nb, ys);
        } else {
            nb_s = rdl32(nb, ys) + rdl32(nb, ym) + rdl32(nb, yp);
        }
        // every neighbour moves one class up (flip to +1) or down: the
        // whole tally shifts by one field (no class leaves its spin's range)
        const uint32_t sub_s = nb_s + (1u << c3);
        const uint32_t add_s =
            (uint32_t)(((uint64_t)nb_s << 3) >> (upm & 6u)) + (1u << c3_new);
        n_lane = n_lane + ((add_s >> lane3) & 7u) - ((sub_s >> lane3) & 7u);
        ev_lane += lane == c ? 1u : 0u;
        W = (double)n_lane * rd_lane;
        Pinc = scan16_f64(W);
        R = rdl_f64(Pinc, 9);

        if constexpr (WRAP) {
            // flip, and move the neighbours' up-counts on the bit planes
            const MT bx = (MT)1 << xs;
            const MT mrow = (xm >= 0 ? (MT)1 << xm : (MT)0) | (xp < B ? (MT)1 << xp : (MT)0);
            nm = on_row ? mrow : (adj ? bx : (MT)0);
            if (on_row) S ^= bx;
            planes_step_inv<MT>(P, nm, (MT)(int64_t)(int32_t)upm);
        }
    };

    if constexpr (SLICE) {
        // The rejection-free variant with fixed time slices: the domain's
        // continuous-time kinetics run for rp.tau.  Event k takes Philox call
        // (k, d | vis << 20 | kStreamSlice << 24, w, rho): words 3:2 give u
        // and the waiting time dt = (-ln(u) 2^32) / R, words 1:0 a 64-bit
        // word whose Lemire multiply by R (with rejection, redrawn on the
        // slice retry streams) is x uniform on [0, R).  The visit ends at
        // the first event whose time would pass tau, or at once when no
        // event is possible (R = 0).  The calls of 64 events are drawn a
        // batch at a time, one per lane; the logarithm is slice_log, whose
        // sequence of IEEE operations is fixed, so every stop decision is
        // reproducible.
        const double tau = rp.tau;
        const uint32_t cs = d | (vis << 20);
        double tt = 0.0;
        bool done = false;
        for (uint32_t kb = 0; !done; kb += 64) {
            const uint4 o = philox(kb + (uint32_t)lane, cs | (kStreamSlice << 24), w, rho, key0,
                                   key1);
            const uint64_t u53 = ((uint64_t)o.w << 21) | (o.z >> 11);
            const double nl = -slice_log((double)(u53 + 1) * 0x1p-53) * 4294967296.0;
            const uint64_t word = ((uint64_t)o.y << 32) | o.x;
            for (int l = 0; l < 64; ++l) {
                if (R == 0.0) {
                    done = true;
                    break;
                }
                const double tn = tt + rdl_f64(nl, l) / R;
                if (tn > tau) {
                    done = true;
                    break;
                }
                tt = tn;
                const uint64_t Ru = (uint64_t)R;
                uint64_t U = rdl64(word, l);
                uint64_t lo = U * Ru;
                if (lo < Ru) {  // rare: Lemire's threshold 2^64 mod R
                    const uint64_t thr64 = (0 - Ru) % Ru;
                    for (int r = 0; r < kMaxRetry && lo < thr64; ++r) {
                        const uint4 o2 =
                            philox(kb + (uint32_t)l, cs | ((kStreamSliceRetry0 + r) << 24), w,
                                   rho, key0, key1);
                        U = ((uint64_t)o2.y << 32) | o2.x;
                        lo = U * Ru;
                    }
                }
                event((double)__umul64hi(U, Ru) + 0.5);
            }
        }
    } else {
        for (int base = 0; base < NI; base += 64) {
            const uint32_t t = (uint32_t)(base + lane);
            const bool valid = base + lane < NI;
            const uint4 o = philox(t, c1, w, rho, key0, key1);
            uint64_t mm = (uint64_t)o.y * nd;
            bool rej = valid && (uint32_t)mm < thr;
            if (__ballot(rej)) {  // rare: redraw the slot on the retry streams
                for (int k = 1; rej && k <= kMaxRetry; ++k) {
                    const uint4 o2 =
                        philox(t, d | (vis << 20) | ((kStreamRetry0 + k - 1) << 24), w,
                               rho, key0, key1);
                    mm = (uint64_t)o2.y * nd;
                    rej = (uint32_t)mm < thr;
                }
            }
            // x = slot 2^32 + w0, exact in a double, held as xh = x + 1/2: the
            // comparisons with the integer sums R and P_c are unchanged by the
            // half, and the member quotient below starts from it
            const double xh = (double)(uint32_t)(mm >> 32) * 4294967296.0 + (double)o.x + 0.5;
            uint64_t left = __ballot(valid);  // ticks of the batch not yet decided
            double Rb = 0.0;                  // this lane's R before its event (0: none)
            int pos = 0;
            // the first undecided tick below R is the next event; the ticks
            // before it are nulls
            uint64_t cand = __ballot(xh < R) & left;
            while (cand) {
                const int e = __builtin_ctzll(cand);
                left &= ~1ull << e;  // drop the ticks up to and including e
                m_null += (uint32_t)(e - pos);
                const double xe = rdl_f64(xh, e);  // x_e + 1/2
                if (lane == e) Rb = R;

                event(xe);
                pos = e + 1;
                cand = __ballot(xh < R) & left;
            }
            m_null += (uint32_t)__popcll(left);  // the batch's trailing nulls
            // residence times -ln(u)/R of this batch's events, kept per lane
            if (Rb != 0.0) {
                const uint64_t u53 = ((uint64_t)o.w << 21) | (o.z >> 11);
                const double u = (double)(u53 + 1) * 0x1p-53;
                neumaier_add(clk_sum, clk_comp, -log(u) * 4294967296.0 / Rb);
            }
        }
    }
    if constexpr (SCORE) {
        if (m_null) null_run(m_null);
        const double ev = (double)ev_lane;
        const int cl = lane < 10 ? lane : 0;
        const double gJ = lane < 10 ? rt->gJ[cl] : 0.0, gh = lane < 10 ? rt->gh[cl] : 0.0;
        const double aJ = lane < 10 ? rt->aJ[cl] : 0.0, ah = lane < 10 ? rt->ah[cl] : 0.0;
        out.sJ = rowsum16_f64(gJ * ev - aJ * A_lane, lane);
        out.sh = rowsum16_f64(gh * ev - ah * A_lane, lane);
    }
    {
        // events, dM and dB from the per-class event counts: a flip of class
        // c = 5 [s=+1] + k changes M by -2s and the bond sum by -2s (2k - 4)
#pragma unroll
        for (int cc = 0; cc < 10; ++cc) {
            const int64_t n = (int64_t)rdl32(ev_lane, cc);
            const int64_t m2 = cc >= 5 ? -2 : 2;
            out.events += n;
            out.dM += m2 * n;
            out.dB += m2 * (2 * (cc % 5) - rp.z) * n;
        }
    }
    {
        double cs = clk_sum, cc = clk_comp;
        cs = wave_sum_f64(cs);
        cc = wave_sum_f64(cc);
        if (lane == 0) {
            double ds = dom_sum, dc = dom_comp;
            if constexpr (SLICE) {
                neumaier_add(ds, dc, rp.tau);  // the domain's clock: one slice
            } else {
                neumaier_add(ds, dc, cs);
                neumaier_add(ds, dc, cc);
            }
            dom->clk_sum = ds;
            dom->clk_comp = dc;
            dom->events = dom_ev + out.events;
        }
    }

    // ---- write the tile back through LDS, and the domain's edge columns
    if (lane < By) {
        for (int q = 0; q < SB4; ++q)
            *reinterpret_cast<uint32_t *>(tile + lane * SB + 4 * q) =
                bits_to_bytes((uint32_t)(S >> (4 * q)) & 0xFu);
    }
    {
        // S is clear in lanes >= By
        const uint64_t first = __ballot((uint32_t)S & 1u);
        const uint64_t last = __ballot((uint32_t)(S >> (B - 1)) & 1u);
        if (lane == 0)
            *reinterpret_cast<ulonglong2 *>(edges + 2 * dd) =
                make_ulonglong2((unsigned long long)first, (unsigned long long)last);
    }
    wave_sync_lds();
    int8_t *wblk = lat + (int64_t)dd * (int)nd;
    if ((B & 3) == 0) {
        if ((nd & 15u) == 0) {
            for (int q = lane; q < (int)(nd >> 4); q += 64)
                *reinterpret_cast<uint4 *>(wblk + 16 * q) =
                    *reinterpret_cast<const uint4 *>(tile + 16 * q);
        } else {
            for (int q = lane; q < (int)(nd >> 2); q += 64)
                *reinterpret_cast<uint32_t *>(wblk + 4 * q) =
                    *reinterpret_cast<const uint32_t *>(tile + 4 * q);
        }
    } else {
        for (int q = lane; q < By * B; q += 64) {
            const int row = q / B, col = q - row * B;
            wblk[q] = (int8_t)tile[row * SB + col];
        }
    }
    wave_sync_lds();  // LDS reads of the write-back finish before reuse
    return out;
}

// Number of domains of colour `col` (N_D / 4 on a 4-colour checkerboard).
__device__ __forceinline__ int domains_of_colour(const Rep &rp, int col) {
    if (col < 0 || col >= rp.ncol) return 0;
    int ax, ay;
    split_colour(rp, col, &ax, &ay);
    return axis_count(ax, rp.NT) * axis_count(ay, rp.NTy);
}

// Index and origin of the i-th domain of colour `col` (ascending index).
__device__ __forceinline__ void colour_domain(const Rep &rp, int col, int i,
                                              int *d, int *oy, int *ox) {
    int ax, ay;
    split_colour(rp, col, &ax, &ay);
    const int nx = axis_count(ax, rp.NT);
    const int tx = axis_pos(i % nx, ax, rp.NT);
    const int ty = axis_pos(i / nx, ay, rp.NTy);
    *d = ty * rp.NT + tx;
    *oy = ty * rp.By;
    *ox = tx * rp.B;
}

// Mean of the replica's domain clocks (wave-parallel, fixed order).
__device__ inline double replica_time(const KParams &K, const Rep &rp, int lane) {
    double s = 0.0, cpen = 0.0;
    for (int dd = lane; dd < rp.ND; dd += 64) {
        const Dom &dm = K.dom[rp.dom_off + dd];
        neumaier_add(s, cpen, dm.clk_sum + dm.clk_comp);
    }
    return wave_sum_f64(s + cpen) / (double)rp.ND;
}

// ---------------------------------------------------------------- kernels

// Phase p of the current sweep: one wavefront per (replica, domain of the
// phase's colour).  Launched once per phase; domains of a colour commute.
template <typename MT, bool SCORE, bool WRAP, bool SLICE = false>
__global__ __launch_bounds__(64) void k_phase(KParams K, int p) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsPerWave];
    const int task = K.task_begin + (int)blockIdx.x;
    const int rho = K.task_rep[task];
    const Rep rp = K.reps[rho];
    const uint32_t w = (uint32_t)K.ctl->sweep;
    int vis;
    const int col = phase_colour(rp, K.seed, (uint32_t)rho, w, p, &vis);
    if (col < 0 || task - rp.task_off >= domains_of_colour(rp, col)) return;
    int d, oy, ox;
    colour_domain(rp, col, task - rp.task_off, &d, &oy, &ox);
    const VisitOut o = visit_domain<MT, SCORE, WRAP, SLICE>(
        K.spins + rp.spin_off, rp, K.rates + rho, oy, ox, (uint32_t)d,
        (uint32_t)vis, w, (uint32_t)rho, K.seed, K.dom + rp.dom_off + d,
        K.edges + 2 * (int64_t)rp.dom_off, lds);
    if (__lane_id() == 0) {
        if (o.events) {
            atomicAdd((unsigned long long *)&K.acc[rho].M, (unsigned long long)o.dM);
            atomicAdd((unsigned long long *)&K.acc[rho].B, (unsigned long long)o.dB);
            atomicAdd((unsigned long long *)&K.acc[rho].events,
                      (unsigned long long)o.events);
        }
        if constexpr (SCORE) {
            const int64_t bin = K.ctl->run_done / K.ctl->rec_every;
            double *b = K.bins + ((int64_t)rho * K.n_bins + bin) * 2;
            atomicAdd(b, o.sJ);
            atomicAdd(b + 1, o.sh);
        }
    }
}

// End of a sweep: one wavefront per replica writes the record when due.
// Number of visits of colour `col` at positions before p in the sweep's
// schedule (random order: one visit per sweep, at the position held in the
// 4-bit field col of pos_of; palindrome 0 1 .. n-1 n-1 .. 1 0: two).
__device__ inline int visits_before(const Rep &rp, uint64_t pos_of, int col, int p) {
    if (rp.sched == 1) return (col < p ? 1 : 0) + (2 * rp.ncol - 1 - col < p ? 1 : 0);
    return (int)((pos_of >> (4 * col)) & 15u) < p ? 1 : 0;
}

constexpr int64_t kFlowMaxPolls = int64_t(1) << 24;  // default bound of a wait
constexpr int kFlowMaxSweeps = 64;  // sweeps of one dataflow launch

// G whole sweeps of the phase-by-phase form in one launch.  Block b runs
// sweep g = b / (P n_tasks), phase p = (b / n_tasks) mod P, task
// b mod n_tasks (P phases per sweep).  A visit starts once every visit that
// precedes it in the sequential order and touches its halo or its tile has
// finished: the visits of its four neighbouring domains earlier in this
// sweep's schedule, the neighbours' visits of the previous sweep (all of
// them: sweeps are sequential), and its own previous visit.  Each domain
// publishes 4 w + (its visits so far in sweep w) with a device-scope release
// after writing its tile back; waiters poll it with relaxed device-scope
// loads and then take one device-scope acquire fence.  A visit that follows
// ours waits for ours the same way, so no visit reads a
// halo a later visit has already changed.  The halo every visit reads is
// therefore exactly the one of the sequential order, and results equal the
// phase-by-phase launches bit for bit, while domains of non-adjacent
// colours, domains whose neighbours finished early, and the next sweep's
// early visits run ahead.  Blocks are numbered sweep- and phase-major, so a
// block only waits on blocks numbered before it.  A wait that exceeds
// K.flow_max_polls polls (kFlowMaxPolls unless the host sets another bound)
// sets ctl->err and gives up (the host reports the run as failed), so no wave
// can hang.  Sweeps overlap, so a visit adds its
// changes of M, B and events to its sweep's slot and stores its domain's
// clock after the sweep's last visit; k_flow_close forms the records.
template <typename MT, bool SCORE, bool WRAP, bool SLICE = false>
__global__ __launch_bounds__(64) void k_flow(KParams K, int n_tasks, int n_phase,
                                             int64_t *done) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsPerWave];
    const int per_sweep = n_phase * n_tasks;
    const int g = (int)blockIdx.x / per_sweep;
    const int b = (int)blockIdx.x - g * per_sweep;
    const int p = b / n_tasks;
    const int task = K.task_begin + b % n_tasks;
    const int rho = K.task_rep[task];
    const Rep rp = K.reps[rho];
    const int64_t run_done = K.ctl->run_done + g;  // sweeps of the run before this one
    const uint32_t w = (uint32_t)(K.ctl->sweep + g);
    int vis;
    const int col = phase_colour(rp, K.seed, (uint32_t)rho, w, p, &vis);
    if (col < 0 || task - rp.task_off >= domains_of_colour(rp, col)) return;
    int d, oy, ox;
    colour_domain(rp, col, task - rp.task_off, &d, &oy, &ox);
    int64_t *dn = done + rp.dom_off;
    const int64_t base = 4 * (int64_t)w;
    // every visit of the previous sweep (counters restart with each run, and
    // a run's first sweep follows complete sweeps)
    const int64_t prev = run_done > 0 ? base - 4 + rp.visits : 0;
    if (__lane_id() == 0) {
        uint64_t pos_of = 0;  // 4-bit position of each colour in this sweep's order
        if (rp.sched != 1)
            pos_of = perm_positions(
                schedule_index(K.seed, (uint32_t)rho, w, (uint32_t)rp.nperm), rp.ncol);
        const int NT = rp.NT, NTy = rp.NTy, ty = d / NT, tx = d - ty * NT;
        auto wait_for = [&](int ey, int ex) {
            const int need = visits_before(rp, pos_of, dom_colour(rp, ey, ex), p);
            const int64_t target = need ? base + need : prev;
            if (target == 0) return;
            const int64_t *cnt = dn + ey * NT + ex;
            int64_t polls = 0;
            // relaxed polls (no cache invalidation per poll); one acquire
            // fence once every wait is over.  Thousands of wavefronts wait
            // at a time; a long sleep between polls (64 x 64 cycles) keeps
            // them from crowding the memory system.  (Measured on the 1024^2
            // lattice: 5 % off a sweep of one-tick visits against a 128-cycle
            // sleep, none on the full visits; a twice longer sleep is slower.)
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(64);
                if (++polls > K.flow_max_polls) {
                    __hip_atomic_store(&K.ctl->err, (int64_t)1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    return;
                }
            }
        };
        wait_for((ty + NTy - 1) % NTy, tx);
        wait_for((ty + 1) % NTy, tx);
        wait_for(ty, (tx + NT - 1) % NT);
        wait_for(ty, (tx + 1) % NT);
        wait_for(ty, tx);  // its own previous visit
        // the values the polls observed were published by release stores:
        // this fence orders the visit's reads after those visits' writes
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __builtin_amdgcn_wave_barrier();
    Dom *dm = K.dom + rp.dom_off + d;
    const VisitOut o = visit_domain<MT, SCORE, WRAP, SLICE>(
        K.spins + rp.spin_off, rp, K.rates + rho, oy, ox, (uint32_t)d,
        (uint32_t)vis, w, (uint32_t)rho, K.seed, dm,
        K.edges + 2 * (int64_t)rp.dom_off, lds);
    if (__lane_id() == 0) {
        // this domain's visits so far in sweep w (the palindrome's second
        // visit has vis = 1), published first: the visits waiting on it need
        // only the tile and the domain record, both written above
        __hip_atomic_store(dn + d, base + (int64_t)vis + 1,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // what only k_flow_close reads, after the launch
        if (o.events) {
            int64_t *a = K.flow_acc + ((int64_t)g * K.n_rep + rho) * 3;
            atomicAdd((unsigned long long *)&a[0], (unsigned long long)o.dM);
            atomicAdd((unsigned long long *)&a[1], (unsigned long long)o.dB);
            atomicAdd((unsigned long long *)&a[2], (unsigned long long)o.events);
        }
        if (vis + 1 == rp.visits) {  // the domain's clock at the end of sweep w
            double *ck = K.flow_clk + ((int64_t)g * K.n_dom_total + rp.dom_off + d) * 2;
            ck[0] = dm->clk_sum;
            ck[1] = dm->clk_comp;
        }
        if constexpr (SCORE) {
            const int64_t bin = run_done / K.ctl->rec_every;
            double *bb = K.bins + ((int64_t)rho * K.n_bins + bin) * 2;
            atomicAdd(bb, o.sJ);
            atomicAdd(bb + 1, o.sh);
        }
    }
}

// After a dataflow launch of G sweeps: one workgroup per replica.  Its first
// thread adds the sweeps' changes to the running totals in sweep order; its
// wavefronts then write the records that fall due, one sweep each at a
// time, with the replica time from the clock snapshots (the same fixed-order
// mean as replica_time).
constexpr int kFlowCloseWaves = 16;

__global__ __launch_bounds__(64 * kFlowCloseWaves) void k_flow_close(KParams K, int G) {
    __shared__ int64_t tot[kFlowMaxSweeps][3];  // running totals after sweep g
    const int rho = blockIdx.x;
    const Ctl c = *K.ctl;
    const Rep rp = K.reps[rho];
    const int lane = __lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) {
        RepAcc acc = K.acc[rho];
        for (int g = 0; g < G; ++g) {
            const int64_t *a = K.flow_acc + ((int64_t)g * K.n_rep + rho) * 3;
            acc.M += a[0];
            acc.B += a[1];
            acc.events += a[2];
            tot[g][0] = acc.M;
            tot[g][1] = acc.B;
            tot[g][2] = acc.events;
        }
        K.acc[rho] = acc;
    }
    __syncthreads();
    if (!K.write_records) return;
    // the records due, one sweep per wavefront at a time
    for (int g = wave; g < G; g += kFlowCloseWaves) {
        const int64_t done = c.run_done + g + 1;
        if (done % c.rec_every) continue;
        double s = 0.0, cpen = 0.0;
        for (int dd = lane; dd < rp.ND; dd += 64) {
            const double *ck = K.flow_clk + ((int64_t)g * K.n_dom_total + rp.dom_off + dd) * 2;
            neumaier_add(s, cpen, ck[0] + ck[1]);
        }
        const double t = wave_sum_f64(s + cpen) / (double)rp.ND;
        if (lane == 0) {
            const int64_t k = c.rec_base + done / c.rec_every - 1;
            Record r;
            r.sweep = c.sweep + g + 1;
            r.M = tot[g][0];
            r.B = tot[g][1];
            r.events = tot[g][2];
            r.steps = (c.sweep + g + 1) * (int64_t)rp.NI * rp.ND * rp.visits;
            r.t = t;
            K.rec[k * K.n_rep + rho] = r;
        }
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(64) void k_sweep_end(KParams K) {
    const int rho = blockIdx.x;
    const Ctl c = *K.ctl;
    const int64_t done = c.run_done + 1;
    if (!K.write_records || done % c.rec_every) return;
    const Rep rp = K.reps[rho];
    const int lane = __lane_id();
    const double t = replica_time(K, rp, lane);
    if (lane == 0) {
        const int64_t k = c.rec_base + done / c.rec_every - 1;
        Record r;
        r.sweep = c.sweep + 1;
        r.M = K.acc[rho].M;
        r.B = K.acc[rho].B;
        r.events = K.acc[rho].events;
        r.steps = (c.sweep + 1) * (int64_t)rp.NI * rp.ND * rp.visits;
        r.t = t;
        K.rec[k * K.n_rep + rho] = r;
    }
}

__global__ void k_advance(Ctl *ctl, int64_t n) {
    ctl->sweep += n;
    ctl->run_done += n;
}

__global__ void k_reset_queue(Ctl *ctl) {
    ctl->queue = 0;
    ctl->queue2 = 0;
}

__global__ void k_set_ctl(Ctl *ctl, int64_t run_done, int64_t rec_base,
                          int64_t rec_every, int64_t sweep) {
    ctl->run_done = run_done;
    ctl->rec_base = rec_base;
    ctl->rec_every = rec_every;
    ctl->queue = 0;
    ctl->queue2 = 0;
    ctl->sweep = sweep;
}

// Closes a record interval of replica rho after sweep w: adds the score to
// its bin and writes the record when due (lane 0 writes).
template <bool SCORE>
__device__ inline void close_interval(const KParams &K, const Rep &rp, int rho, uint32_t w,
                                      int64_t done, int64_t rec_every, int64_t rec_base,
                                      const RepAcc &acc, double sJ, double sh, int lane) {
    __threadfence();
    if constexpr (SCORE) {
        if (lane == 0) {
            const int64_t bin = (done - 1) / rec_every;
            double *b = K.bins + ((int64_t)rho * K.n_bins + bin) * 2;
            b[0] += sJ;
            b[1] += sh;
        }
    }
    if (K.write_records && done % rec_every == 0) {
        const double t = replica_time(K, rp, lane);
        if (lane == 0) {
            const int64_t k = rec_base + done / rec_every - 1;
            Record r;
            r.sweep = (int64_t)w + 1;
            r.M = acc.M;
            r.B = acc.B;
            r.events = acc.events;
            r.steps = ((int64_t)w + 1) * (int64_t)rp.NI * rp.ND * rp.visits;
            r.t = t;
            K.rec[k * K.n_rep + rho] = r;
        }
    }
}

struct TeamShared {
    int64_t dM[kWavesPerPersistentGroup], dB[kWavesPerPersistentGroup],
        ev[kWavesPerPersistentGroup];
    double sJ[kWavesPerPersistentGroup], sh[kWavesPerPersistentGroup];
};

// All n_sweeps sweeps of replica rho, run by `nw` wavefronts (1, or the 4 of
// the workgroup).  In each colour phase wavefront `wave` takes the phase's
// domains wave, wave + nw, ...; with a team a workgroup barrier separates the
// phases (domains of one colour never touch, so the split changes no result).
template <typename MT, bool SCORE, bool WRAP, bool SLICE = false>
__device__ void run_replica(const KParams &K, int rho, int wave, int nw, int lane,
                            uint8_t *lds, TeamShared *ts, int64_t sweep0,
                            int64_t run_done0, int64_t n_sweeps, int64_t rec_every,
                            int64_t rec_base) {
    const Rep rp = K.reps[rho];
    RepAcc acc = K.acc[rho];  // with a team, wavefront 0 keeps the totals
    int64_t dM = 0, dB = 0, ev = 0;
    double sJ = 0.0, sh = 0.0;
    const int nphase = (rp.sched == 1 ? 2 : 1) * rp.ncol;
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t w = (uint32_t)(sweep0 + i);
        for (int p = 0; p < nphase; ++p) {
            int vis;
            const int col = phase_colour(rp, K.seed, (uint32_t)rho, w, p, &vis);
            const int per_colour = domains_of_colour(rp, col);
            for (int i2 = wave; i2 < per_colour; i2 += nw) {
                int d, oy, ox;
                colour_domain(rp, col, i2, &d, &oy, &ox);
                const VisitOut o = visit_domain<MT, SCORE, WRAP, SLICE>(
                    K.spins + rp.spin_off, rp, K.rates + rho, oy, ox, (uint32_t)d,
                    (uint32_t)vis, w, (uint32_t)rho, K.seed, K.dom + rp.dom_off + d,
        K.edges + 2 * (int64_t)rp.dom_off, lds);
                dM += o.dM;
                dB += o.dB;
                ev += o.events;
                sJ += o.sJ;
                sh += o.sh;
            }
            if (nw > 1) __syncthreads();
        }
        const int64_t done = run_done0 + i + 1;
        if (done % rec_every == 0 || i + 1 == n_sweeps) {
            if (nw > 1) {
                if (lane == 0) {
                    ts->dM[wave] = dM;
                    ts->dB[wave] = dB;
                    ts->ev[wave] = ev;
                    ts->sJ[wave] = sJ;
                    ts->sh[wave] = sh;
                }
                __syncthreads();
                if (wave == 0) {
                    dM = dB = ev = 0;
                    sJ = sh = 0.0;
                    for (int q = 0; q < nw; ++q) {
                        dM += ts->dM[q];
                        dB += ts->dB[q];
                        ev += ts->ev[q];
                        sJ += ts->sJ[q];
                        sh += ts->sh[q];
                    }
                }
            }
            if (wave == 0) {
                acc.M += dM;
                acc.B += dB;
                acc.events += ev;
                close_interval<SCORE>(K, rp, rho, w, done, rec_every, rec_base, acc, sJ, sh,
                                      lane);
            }
            dM = dB = ev = 0;
            sJ = sh = 0.0;
            if (nw > 1) __syncthreads();
        }
    }
    if (wave == 0 && lane == 0) K.acc[rho] = acc;
}

// Persistent batched form.  The launch's queue holds n_team replicas run by
// a whole workgroup (costliest first), then n_solo replicas run by single
// wavefronts (costliest first).  Every wavefront leaves once both queues
// are drained.  One call site keeps the domain process inlined once.
template <typename MT, bool SCORE, bool WRAP, bool SLICE = false>
__global__ __launch_bounds__(64 * kWavesPerPersistentGroup) void k_persistent(
    KParams K, int64_t n_sweeps) {
    __shared__ __attribute__((aligned(16)))
    uint8_t lds_all[kWavesPerPersistentGroup][kLdsPerWave];
    // the sweep counters come from device memory, so a captured launch can
    // be replayed: k_advance moves them on after the launch
    const int64_t sweep0 = K.ctl->sweep;
    const int64_t run_done0 = K.ctl->run_done;
    __shared__ TeamShared ts;
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint8_t *lds = lds_all[wave];
    const int lane = __lane_id();
    const int64_t rec_every = K.ctl->rec_every;
    const int64_t rec_base = K.ctl->rec_base;
    bool team_phase = true;
    for (;;) {
        int rho, me, nw;
        if (team_phase) {  // workgroup-uniform branch
            if (threadIdx.x == 0)
                s_item = (int)atomicAdd((unsigned long long *)&K.ctl->queue, 1ull);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            if (it >= K.n_team) {
                team_phase = false;
                continue;
            }
            rho = K.order[it];
            me = wave;
            nw = kWavesPerPersistentGroup;
        } else {
            int idx = 0;
            if (lane == 0)
                idx = (int)atomicAdd((unsigned long long *)&K.ctl->queue2, 1ull);
            idx = (int)rdl32((uint32_t)idx, 0);
            if (idx >= K.n_solo) return;
            rho = K.order[K.n_team + idx];
            me = 0;
            nw = 1;
        }
        // wave-uniform: keep them (and all replica data) in scalar registers
        rho = __builtin_amdgcn_readfirstlane(rho);
        me = __builtin_amdgcn_readfirstlane(me);
        nw = __builtin_amdgcn_readfirstlane(nw);
        run_replica<MT, SCORE, WRAP, SLICE>(K, rho, me, nw, lane, lds, &ts, sweep0, run_done0, n_sweeps,
                               rec_every, rec_base);
    }
}

// ------------------------------------------------------------ init kernels

// Random and all-up starts.  Site i of the row-major order (y = i / L,
// x = i mod L) takes bit i of the INIT stream: call i / 128, word
// (i / 32) mod 4, bit i mod 32.
__global__ void k_init_spins(KParams K) {
    const int rho = blockIdx.y;
    const Rep rp = K.reps[rho];
    const int64_t N = lattice_sites(rp);
    const int64_t call = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (call * 128 >= N || rp.init == 2) return;
    int8_t *lat = K.spins + rp.spin_off;
    const int L = rp.L;
    uint32_t v[4] = {~0u, ~0u, ~0u, ~0u};
    if (rp.init != 1) {
        const uint4 o = philox((uint32_t)call, kStreamInit << 24, 0u, (uint32_t)rho,
                               (uint32_t)K.seed, (uint32_t)(K.seed >> 32));
        v[0] = o.x;
        v[1] = o.y;
        v[2] = o.z;
        v[3] = o.w;
    }
    for (int i = 0; i < 128 && call * 128 + i < N; ++i) {
        const int64_t s = call * 128 + i;
        const int y = (int)(s / L), x = (int)(s - (int64_t)y * L);
        lat[site_offset(rp, y, x)] = ((v[i >> 5] >> (i & 31)) & 1u) ? 1 : -1;
    }
}

// Given starts and copies out: row-major `rm` <-> the replica's
// domain-by-domain block (one thread per site, coalesced on the block).
template <bool TO_BLOCK>
__global__ __launch_bounds__(256) void k_spins_layout(KParams K, int rho, int8_t *rm) {
    const Rep rp = K.reps[rho];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= lattice_sites(rp)) return;
    const int64_t i = row_major_of(rp, j);
    int8_t *lat = K.spins + rp.spin_off;
    if (TO_BLOCK)
        lat[j] = rm[i];
    else
        rm[i] = lat[j];
}

// Rebuild every domain's edge columns from the spins (before a run of the
// staged visits): one thread per domain, bit r = row r.
__global__ __launch_bounds__(256) void k_edges(KParams K) {
    const int rho = blockIdx.y;
    const Rep rp = K.reps[rho];
    const int dd = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (dd >= rp.ND || rp.By > 64) return;
    const int8_t *blk = K.spins + rp.spin_off + (int64_t)dd * (int)rp.nd;
    uint64_t first = 0, last = 0;
    for (int r = 0; r < rp.By; ++r) {
        first |= (uint64_t)(blk[r * rp.B] > 0) << r;
        last |= (uint64_t)(blk[r * rp.B + rp.B - 1] > 0) << r;
    }
    uint64_t *e = K.edges + 2 * ((int64_t)rp.dom_off + dd);
    e[0] = first;
    e[1] = last;
}

// M and B of the start lattice; one thread per site, int64 atomics.
__global__ __launch_bounds__(256) void k_init_obs(KParams K) {
    const int rho = blockIdx.y;
    const Rep rp = K.reps[rho];
    const int L = rp.L;
    const int64_t N = lattice_sites(rp);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int m = 0, b = 0;
    if (i < N) {
        const int8_t *lat = K.spins + rp.spin_off;
        const int y = (int)(i / L), x = (int)(i % L);
        const int s = lat[site_offset(rp, y, x)];
        m = s;
        b = s * lat[site_offset(rp, y, (x + 1) % L)];  // right bond
        if (rp.z == 4) b += s * lat[site_offset(rp, (y + 1) % L, x)];  // down bond
    }
    const uint32_t sm = wave_sum_u32((uint32_t)m);
    const uint32_t sb = wave_sum_u32((uint32_t)b);
    if (__lane_id() == 0 && (sm || sb)) {
        atomicAdd((unsigned long long *)&K.acc[rho].M, (unsigned long long)(int64_t)(int32_t)sm);
        atomicAdd((unsigned long long *)&K.acc[rho].B, (unsigned long long)(int64_t)(int32_t)sb);
    }
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_transpose_records(const Record *in, Record *out, int n_rep,
                                    int64_t n_rec, int64_t capacity) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_rep * n_rec) return;
    const int64_t k = i / n_rep, rho = i % n_rep;
    if (k < capacity) out[rho * capacity + k] = in[i];
}

}  // namespace kmcdev
