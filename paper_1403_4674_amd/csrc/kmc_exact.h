// kmc_exact.h -- exact propagation of the distribution over all 2^N spin
// configurations of a tiny lattice through the parallel transition matrix
// (Sec. 3.1: the paper's reference values come from evolving the probability
// vector with Eq. (CK_parallel in s); Eq. (sum of sequential tms)).
//
// State index s in [0, 2^N), N = L^2: bit y L + x set when spin (y, x) is +1.
// One tick of a domain process (Eq. (Glauber_TM)): a site i of the domain's
// n_d sites is chosen with probability 1/n_d and flipped with probability
// w_i(s), so the tick maps p to
//   p'(s) = p(s) - (1/n_d) sum_i w_i(s) p(s) + (1/n_d) sum_i w_i(s ^ 2^i) p(s ^ 2^i),
// formed here in gather form, one thread per state.  The class of site i in
// s is 5 [s_i = +1] + (up neighbours), and in s ^ 2^i the same count with the
// spin flipped.  The kernels are memory-bound streams over the vector.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmcdev {

constexpr int kExactMaxSites = 26;  // 2^26 doubles = 512 MiB per vector

struct ExactDomain {
    int32_t n;                          // sites of the domain
    int32_t site[kExactMaxSites];       // lattice sites (y L + x)
    int32_t nb[kExactMaxSites][4];      // their four lattice neighbours
};

struct ExactRates {
    double w[10];  // acceptance per class c = 5 [s=+1] + k
};

__global__ __launch_bounds__(256) void k_exact_tick(const double *__restrict__ in,
                                                    double *__restrict__ out, int64_t n_states,
                                                    ExactDomain D, ExactRates R, double inv_nd) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_states; s += stride) {
        const double ps = in[s];
        double leave = 0.0, enter = 0.0;
        for (int a = 0; a < D.n; ++a) {
            const int i = D.site[a];
            const int up = (int)((s >> i) & 1);
            const int k = (int)((s >> D.nb[a][0]) & 1) + (int)((s >> D.nb[a][1]) & 1) +
                          (int)((s >> D.nb[a][2]) & 1) + (int)((s >> D.nb[a][3]) & 1);
            leave += R.w[5 * up + k];
            enter += R.w[5 * (1 - up) + k] * in[s ^ ((int64_t)1 << i)];
        }
        out[s] = ps + (enter - leave * ps) * inv_nd;
    }
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
