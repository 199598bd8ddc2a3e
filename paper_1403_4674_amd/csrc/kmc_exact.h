// kmc_exact.h -- exact propagation of the distribution over all 2^N spin
// configurations of a tiny lattice through the parallel transition matrix
// (Sec. 3.1: the paper's reference values come from evolving the probability
// vector with Eq. (CK_parallel in s); Eq. (sum of sequential tms)).
//
// State index s in [0, 2^N), N = L^2 (or the ring's L): bit y L + x set when
// spin (y, x) is +1.  One tick of a domain process (Eq. (Glauber_TM)): a site
// i of the domain's n_d sites is chosen with probability 1/n_d and flipped
// with probability w_i(s), so the tick maps p to
//   p'(s) = p(s) + (1/n_d) sum_i [ w_i(s ^ 2^i) p(s ^ 2^i) - w_i(s) p(s) ],
// formed here in gather form.  The class of site i in s is 8 [s_i = +1] + k,
// k its up neighbours (a table of 16 entries of which 10 are used); in
// s ^ 2^i the count is the same and the spin is flipped.
//
// The flip partners s ^ 2^i of one state span the whole vector, so a tick is
// two passes over tiles of 2^14 states (128 KiB) held in LDS:
//   * k_exact_hi (N > 14 and a domain site at bit 14 or above) goes first:
//     tiles of the states that share bits c..13, c = 28 - N (bits 0..c-1 and
//     14..N-1 vary: runs of 2^c consecutive states); it writes the entering
//     terms of the sites at bit 14 and above.
//   * k_exact_lo: tiles of consecutive states (bits 0..13 vary).  It reads
//     p and those terms together, adds every site's leaving term and the
//     entering terms of the sites below bit 14, and writes p'.
// The passes move 40 bytes a state, against the 16 of one read and one write
// of the vector.  Each thread holds 16 states, t + 1024 j: the flip partners
// along the four bits j sets are its own registers, and the part of a site's
// class that depends on j is the same in every lane (a table built on the
// host), so a site whose neighbourhood misses those bits reads its rates once
// for all 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmcdev {

constexpr int kExactMaxSites = 26;   // 2^26 doubles = 512 MiB per vector
constexpr int kExactPerThread = 16;  // states a thread holds
// the contiguous pass: tiles of 2^14 states (128 KiB), 1024 threads (tiles
// of 2^13, two workgroups a compute unit, cut this pass by a quarter, but the
// strided pass then reads runs of half the length and loses more)
constexpr int kExactLoBits = 14;
constexpr int kExactLoBlock = (1 << kExactLoBits) / kExactPerThread;
// the strided pass: tiles of 2^14 states (128 KiB), 1024 threads
constexpr int kExactHiBits = 14;
constexpr int kExactHiBlock = (1 << kExactHiBits) / kExactPerThread;

struct ExactDomain {
    int32_t n;                           // sites of the domain
    int32_t site[kExactMaxSites];        // their state bits (y L + x)
    uint32_t nb1[kExactMaxSites];        // bits of their lattice neighbours
    uint32_t nb2[kExactMaxSites];        // neighbours met twice (L = 2: up = down)
    // class change of a thread's state j against its state 0 (4 bits per j),
    // for the thread layouts of the contiguous and the strided pass
    uint64_t dlo[kExactMaxSites];
    uint64_t dhi[kExactMaxSites];
};

struct ExactRates {
    double w[10];  // acceptance per class 5 [s=+1] + k
};

// LDS of a tick pass: the rate table first (its entries then sit at
// immediate offsets), the tile after it.  wt[8 up + k] = (w of the class,
// w of the flipped class).
template <int BITS>
struct ExactLds {
    double2 wt[16];
    double tile[1 << BITS];
};

template <int BITS>
__device__ __forceinline__ void exact_table(ExactLds<BITS> &S, const ExactRates &R, int tid) {
    if (tid < 16) {
        const int up = tid >> 3, k = tid & 7;
        S.wt[tid] = k <= 4 ? double2{R.w[5 * up + k], R.w[5 * (1 - up) + k]} : double2{0.0, 0.0};
    }
}

__device__ __forceinline__ uint32_t exact_class(uint32_t s, int i, uint32_t m1, uint32_t m2) {
    return (uint32_t)(__popc(s & m1) + __popc(s & m2)) + (((s >> i) & 1u) << 3);
}

// The terms of one site for the 16 states a thread of a BLOCK-thread tile
// holds (tile entries t + BLOCK j): acc_j += w(flipped c_j) p(partner_j)
// [ENTER] - w(c_j) p_j [LEAVE], where c_j = c0 + (4-bit field j of dj).  The
// partner of state j is tile entry pt + BLOCK j (RB < 0: the site's tile bit
// is below log2 BLOCK) or the thread's own state j ^ 2^RB.  dj = 0: one class
// for all 16, one table read.
template <bool LEAVE, bool ENTER, int RB, int BITS, int BLOCK>
__device__ __forceinline__ void exact_site(double *acc, const double *ps,
                                           const ExactLds<BITS> &S, uint32_t c0, uint64_t dj,
                                           uint32_t pt) {
    auto partner = [&](int j) { return RB < 0 ? S.tile[pt + BLOCK * j] : ps[j ^ (1 << RB)]; };
    if (dj == 0) {
        const double2 w = S.wt[c0];
#pragma unroll
        for (int j = 0; j < kExactPerThread; ++j) {
            if (LEAVE) acc[j] = fma(-w.x, ps[j], acc[j]);
            if (ENTER) acc[j] = fma(w.y, partner(j), acc[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < kExactPerThread; ++j) {
            const double2 w = S.wt[c0 + (uint32_t)((dj >> (4 * j)) & 15u)];
            if (LEAVE) acc[j] = fma(-w.x, ps[j], acc[j]);
            if (ENTER) acc[j] = fma(w.y, partner(j), acc[j]);
            // groups of four states: their reads in flight together, and
            // the registers of the next group not taken early
            if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// exact_site with the partner kind of tile bit b (JB = log2 BLOCK: tile bits
// JB .. JB + 3 are the bits j sets)
template <bool LEAVE, bool ENTER, int BITS, int BLOCK>
__device__ __forceinline__ void exact_site_at(double *acc, const double *ps,
                                              const ExactLds<BITS> &S, uint32_t c0, uint64_t dj,
                                              int b, int tid) {
    constexpr int JB = BITS - 4;
    switch (b - JB) {
        case 0: exact_site<LEAVE, ENTER, 0, BITS, BLOCK>(acc, ps, S, c0, dj, 0); break;
        case 1: exact_site<LEAVE, ENTER, 1, BITS, BLOCK>(acc, ps, S, c0, dj, 0); break;
        case 2: exact_site<LEAVE, ENTER, 2, BITS, BLOCK>(acc, ps, S, c0, dj, 0); break;
        case 3: exact_site<LEAVE, ENTER, 3, BITS, BLOCK>(acc, ps, S, c0, dj, 0); break;
        default:
            exact_site<LEAVE, ENTER, -1, BITS, BLOCK>(acc, ps, S, c0, dj,
                                                      (uint32_t)tid ^ (1u << b));
    }
}

// One tick, N < 14: the whole vector is one tile, thread t holds the states
// t + 1024 j below 2^N.  out receives p' (out may be in: all of in is read
// before any of out is written).
__global__ __launch_bounds__(1024) void k_exact_small(const double *in, double *out,
                                                     int n_bits,
                                                     ExactDomain D, ExactRates R,
                                                     double inv_nd) {
    __shared__ ExactLds<kExactLoBits> S;
    const int tid = threadIdx.x;
    const uint32_t tn = 1u << n_bits;
    exact_table(S, R, tid);
    for (uint32_t l = tid; l < tn; l += 1024) S.tile[l] = in[l];
    __syncthreads();
    for (uint32_t s = tid; s < tn; s += 1024) {
        const double ps = S.tile[s];
        double acc = 0.0;
        for (int a = 0; a < D.n; ++a) {
            const int i = D.site[a];
            const double2 w = S.wt[exact_class(s, i, D.nb1[a], D.nb2[a])];
            acc = fma(w.y, S.tile[s ^ (1u << i)], fma(-w.x, ps, acc));
        }
        out[s] = ps + acc * inv_nd;
    }
}

// One tick, N >= 14, the pass over tiles of 2^14 consecutive states (tile
// blockIdx.x, thread t holding states t + 1024 j): every site's leaving
// term, and the entering terms of the sites below bit 14.  PART: the sites
// at bit 14 and above have their entering terms in part (from k_exact_hi),
// read here.  part and in may each be out: a tile is read whole before any
// of it is written, each entry by the thread that writes it.
template <bool PART>
__global__ __launch_bounds__(kExactLoBlock) void k_exact_lo(const double *in,
                                                           const double *part, double *out,
                                                           int n_bits, ExactDomain D,
                                                           ExactRates R, double inv_nd) {
    constexpr int BITS = kExactLoBits, BLOCK = kExactLoBlock;
    __shared__ ExactLds<BITS> S;
    const int tid = threadIdx.x;
    const uint32_t t = blockIdx.x;
    exact_table(S, R, tid);
    // state (t << 14) + tid + 1024 j at the uniform address of entry
    // (t << 14) + 1024 j plus the lane's byte offset
    const uint32_t lane_bytes = (uint32_t)tid * 8u;
    auto at = [&](const double *v, int j) {
        return (const double *)((const char *)(v + (t << BITS) + (uint32_t)(BLOCK * j)) +
                                lane_bytes);
    };
    double ps[kExactPerThread], acc[kExactPerThread];
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j) {  // all in flight
        ps[j] = *at(in, j);
        acc[j] = PART ? *at(part, j) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j) S.tile[tid + BLOCK * j] = ps[j];
    __syncthreads();
    const uint32_t s0 = (t << BITS) | (uint32_t)tid;
    for (int a = 0; a < D.n; ++a) {
        const int i = D.site[a];
        const uint32_t c0 = exact_class(s0, i, D.nb1[a], D.nb2[a]);
        if (i < BITS)
            exact_site_at<true, true, BITS, BLOCK>(acc, ps, S, c0, D.dlo[a], i, tid);
        else
            exact_site<true, false, -1, BITS, BLOCK>(acc, ps, S, c0, D.dlo[a], 0);
    }
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j)
        *const_cast<double *>(at(out, j)) = ps[j] + acc[j] * inv_nd;
}

// One tick, 15 <= N <= 26, the pass that goes first when a domain site is at
// bit 14 or above: part receives sum_{i >= 14} w_i(s ^ 2^i) p(s ^ 2^i).
// Tile t holds the states whose bits c..13 are t (c = 28 - N): tile bit b is
// state bit b below c and state bit 14 + b - c from c on, so a tile is
// 2^(14 - c) runs of 2^c consecutive states.  Below c = 4 a run is under the
// 128 bytes HBM is read in, and the 2^(4 - c) tiles that differ in their low
// bits share their lines: they go to workgroups b, b + 8, b + 16, ..., which
// run on one XCD at about the same time, so a line is read once into that
// XCD's L2.
__global__ __launch_bounds__(kExactHiBlock) void k_exact_hi(const double *__restrict__ in,
                                                           double *__restrict__ part,
                                                           int n_bits, ExactDomain D,
                                                           ExactRates R) {
    constexpr int BITS = kExactHiBits, BLOCK = kExactHiBlock;
    __shared__ ExactLds<BITS> S;
    const int tid = threadIdx.x;
    const int c = kExactHiBits + kExactLoBits - n_bits;
    const uint32_t lowm = (1u << c) - 1u;
    auto spread = [=](uint32_t l) { return (l & lowm) | ((l >> c) << kExactLoBits); };
    const uint32_t b = blockIdx.x;
    const int g = c < 4 ? 4 - c : 0;  // tile bits a line spans
    const uint32_t t = (((b >> (3 + g)) << 3 | (b & 7u)) << g) | ((b >> 3) & ((1u << g) - 1u));
    exact_table(S, R, tid);
    const uint32_t s0 = (t << c) | spread((uint32_t)tid);
    const uint32_t lane_bytes = s0 * 8u;  // below 2^29
    auto at = [&](const double *v, int j) {
        return (const double *)((const char *)(v + spread((uint32_t)(BLOCK * j))) + lane_bytes);
    };
    double ps[kExactPerThread], acc[kExactPerThread];
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j) ps[j] = *at(in, j);  // all in flight
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j) {
        S.tile[tid + BLOCK * j] = ps[j];
        acc[j] = 0.0;
    }
    __syncthreads();
    for (int a = 0; a < D.n; ++a) {
        const int i = D.site[a];
        if (i < kExactLoBits) continue;
        const uint32_t c0 = exact_class(s0, i, D.nb1[a], D.nb2[a]);
        exact_site_at<false, true, BITS, BLOCK>(acc, ps, S, c0, D.dhi[a],
                                                i - kExactLoBits + c, tid);
    }
#pragma unroll
    for (int j = 0; j < kExactPerThread; ++j) *const_cast<double *>(at(part, j)) = acc[j];
}

__global__ __launch_bounds__(256) void k_exact_copy(const double *__restrict__ in,
                                                    double *__restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride)
        out[s] = in[s];
}

// acc = (first ? 0 : acc) + a x
__global__ __launch_bounds__(256) void k_exact_axpy(double *__restrict__ acc,
                                                    const double *__restrict__ x, double a,
                                                    int64_t n, int first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride)
        acc[s] = (first ? 0.0 : acc[s]) + a * x[s];
}

}  // namespace kmcdev
