// kmc_resident.h -- resident form: one workgroup keeps one whole replica in
// LDS for every sweep of a call.
//
// Made for small lattices (L <= 128) run with few ticks per visit, and for
// domains wider or taller than 64 sites (the unpartitioned 100 x 100 lattice,
// 100-site stripes), which the one-row-per-lane kernels cannot hold.
//
// LDS holds, for the whole lattice, the class code 5 [s=+1] + k of every site
// (one byte; the spin is code >= 5), and for every domain, row and class the
// number of the row's sites in the class (one byte each, 16 bytes per row).
// Every flip updates the codes and counts of the site and of its four lattice
// neighbours wherever they are, so codes always equal the classes of the
// current lattice: a visit needs no staging, its class totals are summed from
// its rows' counts, and a single-domain axis wraps with no special case.
// Waves of the workgroup take the domains of each colour (wave w: domains
// w, w + nw, ...), with a barrier between colour phases.  Domains of one
// colour never share an edge, so a site inside an active domain is touched by
// that domain's wave only; a halo site may be the neighbour of two active
// domains, so neighbour updates are LDS atomic adds on the byte (codes stay
// in 0..9 and counts in 0..128, so no carry leaves the byte) and the result
// does not depend on their order.
//
// The tick, class and member decisions are those of visit_domain, so results
// are bit-identical to the other forms and to the oracle.
#pragma once

#include "kmc_device.h"

namespace kmcdev {

constexpr int kResMaxL = 128;     // lattice side
constexpr int kResMaxNTx = 16;    // domains along x (bounds the row counts)
constexpr int kResMaxWaves = 16;  // wavefronts per workgroup

// LDS bytes of a replica: codes (L x L, padded to 16) and row counts.
__host__ __device__ inline int resident_lds_bytes(int L, int NTx) {
    return ((L * L + 15) & ~15) + NTx * L * 16;
}

struct ResShared {
    int64_t dM[kResMaxWaves], dB[kResMaxWaves], ev[kResMaxWaves];
    double sJ[kResMaxWaves], sh[kResMaxWaves];
};

// Adds delta (+-1, or +-5 for a flipped site) to the byte at index i of the
// LDS array base; returns the byte's previous value.
__device__ __forceinline__ uint32_t lds_byte_add(uint8_t *base, int i, int delta) {
    uint32_t *w = reinterpret_cast<uint32_t *>(base + (i & ~3));
    const int sh = 8 * (i & 3);
    const uint32_t old = atomicAdd(w, (uint32_t)delta << sh);
    return (old >> sh) & 0xFFu;
}

// One domain process of a resident replica: N_I ticks of domain d (origin
// oy, ox; grid position ty, tx).  `code` is the replica's code array, `rowc`
// its row counts.  One full wavefront.
template <bool SCORE>
__device__ VisitOut visit_resident(const Rep &rp, const Rates *__restrict__ rt, uint8_t *code,
                                   uint8_t *rowc, int d, int ty, int tx, int oy, int ox,
                                   uint32_t vis, uint32_t w, uint32_t rho, uint64_t seed,
                                   Dom *dom) {
    const int lane = __lane_id();
    const int L = rp.L, Bx = rp.B, By = rp.By, NI = rp.NI, NTx = rp.NT, NTy = rp.NTy;
    const uint32_t nd = rp.nd, thr = rp.thr;
    uint8_t *rc = rowc + (size_t)d * By * 16;

    // the four neighbouring domains (the domain itself along an axis with one)
    const int dU = ((ty + NTy - 1) % NTy) * NTx + tx, dD = ((ty + 1) % NTy) * NTx + tx;
    const int dL = ty * NTx + (tx + NTx - 1) % NTx, dR = ty * NTx + (tx + 1) % NTx;

    // ---- class totals from the rows' counts (two classes per 32-bit scan)
    uint32_t n_lane = 0;
#pragma unroll
    for (int c = 0; c < 10; c += 2) {
        uint32_t a = 0, b = 0;
        if (lane < By) {
            a += rc[lane * 16 + c];
            b += rc[lane * 16 + c + 1];
        }
        if (lane + 64 < By) {
            a += rc[(lane + 64) * 16 + c];
            b += rc[(lane + 64) * 16 + c + 1];
        }
        const uint32_t tot = rdl32(scan64(a | (b << 16)), 63);
        if (lane == c) n_lane = tot & 0xFFFFu;
        if (lane == c + 1) n_lane = tot >> 16;
    }
    const double rd_lane = lane < 10 ? rt->rd[lane] : 0.0;
    const double inv_lane = lane < 10 ? rt->inv_rd[lane] : 0.0;
    const uint32_t lane3 = lane < 10 ? 3u * lane : 30u;
    double W = (double)n_lane * rd_lane;
    double Pinc = scan16_f64(W);
    double R = rdl_f64(Pinc, 9);

    double w_lane = 0.0;
    if constexpr (SCORE) {
        if (lane < 10) w_lane = rt->w[lane];
    }
    VisitOut out{0, 0, 0, 0.0, 0.0};
    uint32_t ev_lane = 0;
    double clk_sum = 0.0, clk_comp = 0.0;
    uint32_t m_null = 0;
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = (uint32_t)d | (vis << 20) | (kStreamTick << 24);
    double A_lane = 0.0;
    auto null_run = [&](uint32_t m) {
        const double nl = (double)n_lane;
        const double Rw = rowsum16_f64(nl * w_lane, lane);
        const double den = (double)nd - Rw;
        if (den > 0.0) A_lane += null_quot(m, den) * nl;
    };

    for (int base = 0; base < NI; base += 64) {
        const uint32_t t = (uint32_t)(base + lane);
        const bool valid = base + lane < NI;
        const uint4 o = philox(t, c1, w, rho, key0, key1);
        uint64_t mm = (uint64_t)o.y * nd;
        bool rej = valid && (uint32_t)mm < thr;
        if (__ballot(rej)) {
            for (int k = 1; rej && k <= kMaxRetry; ++k) {
                const uint4 o2 = philox(t, (uint32_t)d | (vis << 20) |
                                               ((kStreamRetry0 + k - 1) << 24),
                                        w, rho, key0, key1);
                mm = (uint64_t)o2.y * nd;
                rej = (uint32_t)mm < thr;
            }
        }
        // x + 1/2, as in visit_domain
        const double xh = (double)(uint32_t)(mm >> 32) * 4294967296.0 + (double)o.x + 0.5;
        uint64_t left = __ballot(valid);
        double Rb = 0.0;
        int pos = 0;
        uint64_t cand = __ballot(xh < R) & left;
        while (cand) {
            const int e = __builtin_ctzll(cand);
            left &= ~1ull << e;
            m_null += (uint32_t)(e - pos);
            const double xe = rdl_f64(xh, e);
            if (lane == e) Rb = R;

            // rate class and member index (exact, as in visit_domain)
            const int c = __builtin_ctzll(__ballot(xe < Pinc));
            const double q = (xe - (Pinc - W)) * inv_lane;
            const uint32_t j = (uint32_t)rdl_f64(q, c);

            if constexpr (SCORE) {
                if (m_null) null_run(m_null);
            }
            m_null = 0;

            // row of member j: scans of the class-c counts of rows l and l + 64
            const uint32_t r0 = lane < By ? rc[lane * 16 + c] : 0u;
            const uint32_t i0 = scan64(r0);
            const uint32_t tot0 = rdl32(i0, 63);
            int ys;
            uint32_t jr;
            if (j < tot0) {
                ys = __builtin_ctzll(__ballot(i0 > j));
                jr = j - rdl32(i0 - r0, ys);
            } else {
                const uint32_t r1 = lane + 64 < By ? rc[(lane + 64) * 16 + c] : 0u;
                const uint32_t i1 = scan64(r1);
                const uint32_t j1 = j - tot0;
                const int q1 = __builtin_ctzll(__ballot(i1 > j1));
                ys = 64 + q1;
                jr = j1 - rdl32(i1 - r1, q1);
            }
            // column: the jr-th class-c site of row ys (columns l and l + 64)
            const uint8_t *row = code + (oy + ys) * L + ox;
            const uint64_t m0 = __ballot(lane < Bx && row[lane < Bx ? lane : 0] == (uint8_t)c);
            const uint32_t k0 = (uint32_t)__popcll(m0);
            int xs;
            if (jr < k0) {
                xs = __builtin_ctzll(__ballot(bits_below_lane(m0) == jr) & m0);
            } else {
                const bool in1 = lane + 64 < Bx;
                const uint64_t m1 = __ballot(in1 && row[in1 ? lane + 64 : 0] == (uint8_t)c);
                xs = 64 + __builtin_ctzll(__ballot(bits_below_lane(m1) == jr - k0) & m1);
            }

            // the flipped site (lane 0) and its four lattice neighbours
            // (lanes 1..4): codes, row counts of their own domains, and the
            // class tallies of this domain's sites
            const bool up = c >= 5;  // the site goes from +1 to -1
            const int c_new = up ? c - 5 : c + 5;
            uint32_t add = 0, sub = 0;
            if (lane < 5) {
                int ly = ys, lx = xs, dd = d;
                if (lane == 1) {
                    if (ys > 0) ly = ys - 1; else { ly = By - 1; dd = dU; }
                } else if (lane == 2) {
                    if (ys < By - 1) ly = ys + 1; else { ly = 0; dd = dD; }
                } else if (lane == 3) {
                    if (xs > 0) lx = xs - 1; else { lx = Bx - 1; dd = dL; }
                } else if (lane == 4) {
                    if (xs < Bx - 1) lx = xs + 1; else { lx = 0; dd = dR; }
                }
                const int gy = (dd / NTx) * By + ly, gx = (dd % NTx) * Bx + lx;
                const int delta = lane == 0 ? c_new - c : (up ? -1 : 1);
                const uint32_t old = lds_byte_add(code, gy * L + gx, delta);
                const uint32_t neu = (uint32_t)((int)old + delta);
                uint8_t *cnt = rowc + ((size_t)dd * By + ly) * 16;
                lds_byte_add(cnt, (int)old, -1);
                lds_byte_add(cnt, (int)neu, 1);
                if (dd == d) {
                    add = 1u << (3 * neu);
                    sub = 1u << (3 * old);
                }
            }
            add += dpp<kRowShr + 1>(add);
            sub += dpp<kRowShr + 1>(sub);
            add += dpp<kRowShr + 2>(add);
            sub += dpp<kRowShr + 2>(sub);
            add += dpp<kRowShr + 4>(add);
            sub += dpp<kRowShr + 4>(sub);
            const uint32_t add_s = rdl32(add, 4), sub_s = rdl32(sub, 4);
            n_lane = n_lane + ((add_s >> lane3) & 7u) - ((sub_s >> lane3) & 7u);
            ev_lane += lane == c ? 1u : 0u;
            W = (double)n_lane * rd_lane;
            Pinc = scan16_f64(W);
            R = rdl_f64(Pinc, 9);
            pos = e + 1;
            cand = __ballot(xh < R) & left;
        }
        m_null += (uint32_t)__popcll(left);
        if (Rb != 0.0) {
            const uint64_t u53 = ((uint64_t)o.w << 21) | (o.z >> 11);
            const double u = (double)(u53 + 1) * 0x1p-53;
            neumaier_add(clk_sum, clk_comp, -log(u) * 4294967296.0 / Rb);
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
#pragma unroll
    for (int cc = 0; cc < 10; ++cc) {
        const int64_t n = (int64_t)rdl32(ev_lane, cc);
        const int64_t m2 = cc >= 5 ? -2 : 2;
        out.events += n;
        out.dM += m2 * n;
        out.dB += m2 * (2 * (cc % 5) - 4) * n;  // square lattices only
    }
    {
        double cs = wave_sum_f64(clk_sum), cc = wave_sum_f64(clk_comp);
        if (lane == 0) {
            double ds = dom->clk_sum, dc = dom->clk_comp;
            neumaier_add(ds, dc, cs);
            neumaier_add(ds, dc, cc);
            dom->clk_sum = ds;
            dom->clk_comp = dc;
            dom->events += out.events;
        }
    }
    return out;
}

// Resident form: workgroup b runs replica b for n_sweeps sweeps with all of
// its state in LDS (dynamic shared memory of resident_lds_bytes for the
// largest replica of the launch), using blockDim.x / 64 wavefronts.
template <bool SCORE>
__global__ __launch_bounds__(64 * kResMaxWaves) void k_resident(KParams K, int64_t n_sweeps) {
    extern __shared__ __attribute__((aligned(16))) uint8_t res_lds[];
    __shared__ ResShared rs;
    const int rho = (int)blockIdx.x;
    const Rep rp = K.reps[rho];
    const int L = rp.L, NTx = rp.NT;
    const int nthr = (int)blockDim.x, tid = (int)threadIdx.x;
    const int nw = nthr >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = __lane_id();
    uint8_t *code = res_lds;
    uint8_t *rowc = res_lds + ((L * L + 15) & ~15);
    int8_t *lat = K.spins + rp.spin_off;
    const int64_t sweep0 = K.ctl->sweep, run_done0 = K.ctl->run_done;
    const int64_t rec_every = K.ctl->rec_every, rec_base = K.ctl->rec_base;

    // ---- codes of the current lattice and the row counts of every domain
    // (HBM holds the lattice domain by domain; LDS row-major)
    for (int j = tid; j < L * L; j += nthr) code[row_major_of(rp, j)] = lat[j] > 0 ? 0x80 : 0;
    for (int i = tid; i < NTx * L * 4; i += nthr) reinterpret_cast<uint32_t *>(rowc)[i] = 0u;
    __syncthreads();
    for (int i = tid; i < L * L; i += nthr) {
        const int y = i / L, x = i - y * L;
        const int k = (code[(y == 0 ? L - 1 : y - 1) * L + x] >> 7) +
                      (code[(y == L - 1 ? 0 : y + 1) * L + x] >> 7) +
                      (code[y * L + (x == 0 ? L - 1 : x - 1)] >> 7) +
                      (code[y * L + (x == L - 1 ? 0 : x + 1)] >> 7);
        code[i] = (uint8_t)((code[i] & 0x80) | (5 * (code[i] >> 7) + k));
    }
    __syncthreads();
    for (int i = tid; i < L * L; i += nthr) {
        const uint32_t cd = code[i] & 0x7Fu;
        code[i] = (uint8_t)cd;
        const int y = i / L, x = i - y * L;
        const int dd = (y / rp.By) * NTx + x / rp.B;
        lds_byte_add(rowc + ((size_t)dd * rp.By + (y % rp.By)) * 16, (int)cd, 1);
    }
    __syncthreads();

    RepAcc acc = K.acc[rho];
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
                const VisitOut o = visit_resident<SCORE>(
                    rp, K.rates + rho, code, rowc, d, d / NTx, d % NTx, oy, ox, (uint32_t)vis,
                    w, (uint32_t)rho, K.seed, K.dom + rp.dom_off + d);
                dM += o.dM;
                dB += o.dB;
                ev += o.events;
                sJ += o.sJ;
                sh += o.sh;
            }
            __syncthreads();
        }
        const int64_t done = run_done0 + i + 1;
        if (done % rec_every == 0 || i + 1 == n_sweeps) {
            if (lane == 0) {
                rs.dM[wave] = dM;
                rs.dB[wave] = dB;
                rs.ev[wave] = ev;
                rs.sJ[wave] = sJ;
                rs.sh[wave] = sh;
            }
            __syncthreads();
            if (wave == 0) {
                dM = dB = ev = 0;
                sJ = sh = 0.0;
                for (int q = 0; q < nw; ++q) {
                    dM += rs.dM[q];
                    dB += rs.dB[q];
                    ev += rs.ev[q];
                    sJ += rs.sJ[q];
                    sh += rs.sh[q];
                }
                acc.M += dM;
                acc.B += dB;
                acc.events += ev;
                close_interval<SCORE>(K, rp, rho, w, done, rec_every, rec_base, acc, sJ, sh,
                                      lane);
            }
            dM = dB = ev = 0;
            sJ = sh = 0.0;
            __syncthreads();
        }
    }
    if (wave == 0 && lane == 0) K.acc[rho] = acc;
    // ---- the lattice back to HBM
    for (int j = tid; j < L * L; j += nthr)
        lat[j] = code[row_major_of(rp, j)] >= 5 ? (int8_t)1 : (int8_t)-1;
}

}  // namespace kmcdev
