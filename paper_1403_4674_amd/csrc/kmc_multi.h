// kmc_multi.h -- multi-slot batched form for domains of side B <= 16.
//
// A 64-lane wavefront runs four independent domain processes side by side,
// one per 16-lane row ("slot").  Every instruction of the event chain then
// serves up to four events, which matters once the machine is full of
// wavefronts and the batched kernel is bound by instruction issue.
// Values that are wave-uniform in visit_domain are slot-uniform here: they
// live in vector registers, shifts and scans stay inside a row (DPP row
// ops), and a slot reads a lane of its own row by ds_bpermute.
//
// Each slot computes exactly what visit_domain computes for its domain (the
// same Philox counters, the same integer decisions), so results are
// bit-identical to the one-domain-per-wavefront kernels and to the oracle.
#pragma once

#include "kmc_device.h"

namespace kmcdev {

constexpr int kSlots = 4;
constexpr int kSlotW = 16;
constexpr int kSlotLds = 16 * 16 + 2 * 16;  // tile + top/bottom halo rows

// Work item of the multi-slot kernel.
//   kind 0: four (or fewer) replicas of one shape, one per slot (rho < 0: idle);
//   kind 1: one replica whose colour phases are split over the slots of
//           nw wavefronts (nw = 1, or 4 with a barrier per phase).
struct MItem {
    int32_t kind, nw;
    int32_t rho[kSlots];
};

__device__ __forceinline__ uint32_t sbc32(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint64_t sbc64(uint64_t v, int src) {
    const uint32_t lo = sbc32((uint32_t)v, src), hi = sbc32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double sbc_f64(double v, int src) {
    return __longlong_as_double((long long)sbc64((uint64_t)__double_as_longlong(v), src));
}

__device__ __forceinline__ uint32_t seg16(uint64_t m, int slot) {
    return (uint32_t)(m >> (16 * slot)) & 0xFFFFu;
}

// Inclusive prefix sum inside each 16-lane row.
// The vector conversion of a double to uint32 saturates (negative and NaN to
// 0, too large to 2^32 - 1).  Lanes other than the class lane of a slot
// convert values outside that range; written as the instruction itself so
// that the conversion is defined for them (only lane c's value is read).
__device__ __forceinline__ uint32_t cvt_u32_sat(double q) {
    uint32_t r;
    asm("v_cvt_u32_f64 %0, %1" : "=v"(r) : "v"(q));
    return r;
}

__device__ __forceinline__ uint32_t scan_row(uint32_t v) {
    v += dppz<kRowShr + 1>(v);
    v += dppz<kRowShr + 2>(v);
    v += dppz<kRowShr + 4>(v);
    v += dppz<kRowShr + 8>(v);
    return v;
}

// Lane N of each 16-lane row copied to the whole row (DPP row_newbcast, a
// VALU operand modifier: no LDS round trip).
constexpr int kRowNewBcast = 0x150;

template <int N>
__device__ __forceinline__ uint32_t rowbcast(uint32_t v) {
    return dpp<kRowNewBcast + N>(v);
}

template <int N>
__device__ __forceinline__ double rowbcast_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = rowbcast<N>((uint32_t)b), hi = rowbcast<N>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double sum_row_f64(double v, int base) {
    (void)base;
    return rowbcast_f64<15>(scan16_f64(v));
}

constexpr int kRowShl1 = 0x101;  // lane i <- lane i+1 inside a row

struct SlotDomain {     // per lane, uniform within a slot
    const int8_t *lat;  // not written through: see visit_multi
    int64_t spin_off;
    int oy, ox;
    uint32_t d, rho;
    bool on;            // the slot has a domain in this step
};

// One step of up to four domain processes (N_I ticks each).  `rp` is the
// common shape (L, B <= 16, N_I); spins, rates and domain records are
// addressed per slot.  Returns the per-slot changes (uniform within a slot).
template <bool SCORE>
__device__ VisitOut visit_multi(int8_t *__restrict__ spins, const Rep &rp,
                                const Rates *__restrict__ rates, Dom *__restrict__ dom_base,
                                int dom_off, const SlotDomain &A, uint32_t vis, uint32_t w,
                                uint64_t seed, uint8_t *lds) {
    const int lane = __lane_id();
    const int slot = lane >> 4, sl = lane & 15, base = lane & ~15;
    const int L = rp.L, B = rp.B, NI = rp.NI;
    const int B4 = B >> 2;
    const uint32_t nd = rp.nd, thr = rp.thr;
    int8_t *lat = spins + A.spin_off;
    const Rates *rt = rates + A.rho;

    // ---- stage the slot's tile and halo rows through LDS (rows padded to
    // whole dwords, stride SB; sides that are not multiples of 4 byte by byte)
    // The lattice is held domain by domain (B x B tiles of B^2 bytes, rows in
    // order): the tile is contiguous, a halo row is a row of the domain above
    // or below, a halo column a column of the tile to the left or right.
    const int SB = (B + 3) & ~3, SB4 = SB >> 2;
    uint8_t *tile = lds + slot * kSlotLds;
    uint8_t *hrow = tile + 16 * 16;  // [0, 16): top, [16, 32): bottom
    const int NT = L / B, n2 = B * B, dd = (int)A.d;
    const int d_up = A.oy == 0 ? dd + (NT - 1) * NT : dd - NT;
    const int d_dn = A.oy + B == L ? dd - (NT - 1) * NT : dd + NT;
    const int d_lf = A.ox == 0 ? dd + NT - 1 : dd - 1;
    const int d_rt = A.ox + B == L ? dd - (NT - 1) : dd + 1;
    const int8_t *blk = lat + (int64_t)dd * n2;
    const int8_t *up_row = lat + (int64_t)d_up * n2 + (B - 1) * B;
    const int8_t *dn_row = lat + (int64_t)d_dn * n2;
    if (A.on) {
        if ((B & 3) == 0) {
            for (int q = sl; q < B * B4; q += kSlotW)
                *reinterpret_cast<uint32_t *>(tile + 4 * q) =
                    *reinterpret_cast<const uint32_t *>(blk + 4 * q);
            if (sl < 2 * B4) {
                const int which = sl / B4, c4 = sl - which * B4;
                *reinterpret_cast<uint32_t *>(hrow + which * 16 + 4 * c4) =
                    *reinterpret_cast<const uint32_t *>((which ? dn_row : up_row) + 4 * c4);
            }
        } else {
            for (int q = sl; q < B * B; q += kSlotW) {
                const int row = q / B, col = q - row * B;
                tile[row * SB + col] = (uint8_t)blk[q];
            }
            for (int q = sl; q < 2 * B; q += kSlotW) {
                const int which = q / B, col = q - which * B;
                hrow[which * 16 + col] = (uint8_t)(which ? dn_row : up_row)[col];
            }
        }
    }
    uint32_t hl = 0, hr = 0;
    if (A.on && sl < B) {
        hl = lat[(int64_t)d_lf * n2 + sl * B + B - 1] > 0 ? 1u : 0u;
        hr = lat[(int64_t)d_rt * n2 + sl * B] > 0 ? 1u : 0u;
    }
    wave_sync_lds();

    const uint32_t VM = (A.on && sl < B) ? ((1u << B) - 1u) : 0u;
    uint32_t S = 0, top = 0, bot = 0;
    if (A.on) {
        for (int q = 0; q < SB4; ++q) {
            if (sl < B)
                S |= bytes_to_bits(*reinterpret_cast<const uint32_t *>(tile + sl * SB + 4 * q))
                     << (4 * q);
            top |= bytes_to_bits(*reinterpret_cast<const uint32_t *>(hrow + 4 * q)) << (4 * q);
            bot |= bytes_to_bits(*reinterpret_cast<const uint32_t *>(hrow + 16 + 4 * q))
                   << (4 * q);
        }
        S &= VM;  // padding bytes decode to set bits: clear them
        top &= (1u << B) - 1u;
        bot &= (1u << B) - 1u;
    }
    auto planes = [&](uint32_t s) {
        uint32_t U = dpp<kRowShr + 1>(s);
        if (sl == 0) U = top;
        uint32_t D = dpp<kRowShl1>(s);
        if (sl == B - 1) D = bot;
        const uint32_t Lf = ((s << 1) | hl) & VM;
        const uint32_t Rt = ((s >> 1) | (hr << (B - 1))) & VM;
        U &= VM;
        D &= VM;
        const uint32_t p1 = U ^ D, q1 = U & D, p2 = Lf ^ Rt, q2 = Lf & Rt, c0 = p1 & p2;
        Planes<uint32_t> P;
        P.s0 = p1 ^ p2;
        P.s1 = q1 ^ q2 ^ c0;
        P.s2 = (q1 & q2) | (c0 & (q1 ^ q2));
        return P;
    };
    Planes<uint32_t> P = planes(S);

    // ---- class counts of each slot
    uint32_t n_lane = 0;
#pragma unroll
    for (int c = 0; c < 10; c += 2) {
        const uint32_t a = popc(class_mask<uint32_t>(c, S, P, VM));
        const uint32_t b = popc(class_mask<uint32_t>(c + 1, S, P, VM));
        const uint32_t tot = rowbcast<15>(scan_row(a | (b << 16)));
        if (sl == c) n_lane = tot & 0xFFFFu;
        if (sl == c + 1) n_lane = tot >> 16;
    }
    // exact FP64 rate sums (integers below 2^44), as in visit_domain
    const double rd_lane = (A.on && sl < 10) ? rt->rd[sl] : 0.0;
    const double inv_lane = (A.on && sl < 10) ? rt->inv_rd[sl] : 0.0;
    const uint32_t sl3 = sl < 10 ? 3u * (uint32_t)sl : 30u;  // tally field (30: always 0)
    // the fields a class lane's count moves from: the class above (the
    // flipped spin was +1, its neighbours lose an up neighbour) or below
    const uint32_t from_up = sl < 9 ? sl3 + 3u : 30u;
    const uint32_t from_dn = sl >= 1 && sl < 10 ? sl3 - 3u : 30u;
    double W = (double)n_lane * rd_lane;
    double Pinc = scan16_f64(W);
    double R = rowbcast_f64<9>(Pinc);
    const uint32_t vm_row = (1u << B) - 1u;
    const uint32_t upto_lane = (2u << sl) - 1u;  // bits 0..sl

    double w_lane = 0.0;  // score: w_c in the class lanes (the other tables at the end)
    if constexpr (SCORE) {
        if (A.on && sl < 10) w_lane = rt->w[sl];
    }

    VisitOut out{0, 0, 0, 0.0, 0.0};
    uint32_t ev_lane = 0;  // lanes 0..9 of a slot: events of class c = lane
    double clk_sum = 0.0, clk_comp = 0.0;
    uint32_t m_null = 0;
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = A.d | (vis << 20) | (kStreamTick << 24);

    // score: per-class accumulation of the null runs, as in visit_domain
    double A_lane = 0.0;
    auto null_run = [&](uint32_t m, bool act) {
        const double nl = (double)n_lane;
        const double Rw = sum_row_f64(nl * w_lane, base);
        const double den = (double)nd - Rw;
        if (act && m && den > 0.0) A_lane += null_quot(m, den) * nl;
    };

    for (int b0 = 0; b0 < NI; b0 += kSlotW) {
        const uint32_t t = (uint32_t)(b0 + sl);
        const bool valid = A.on && b0 + sl < NI;
        const uint4 o = philox(t, c1, w, A.rho, key0, key1);
        uint64_t mm = (uint64_t)o.y * nd;
        bool rej = valid && (uint32_t)mm < thr;
        if (__ballot(rej)) {
            for (int k = 1; rej && k <= kMaxRetry; ++k) {
                const uint4 o2 = philox(t, A.d | (vis << 20) | ((kStreamRetry0 + k - 1) << 24),
                                        w, A.rho, key0, key1);
                mm = (uint64_t)o2.y * nd;
                rej = (uint32_t)mm < thr;
            }
        }
        // x + 1/2, as in visit_domain
        const double xh = (double)(uint32_t)(mm >> 32) * 4294967296.0 + (double)o.x + 0.5;
        uint32_t left = seg16(__ballot(valid), slot);  // the slot's undecided ticks
        double Rb = 0.0;
        int pos = 0;
        for (;;) {
            // a slot without a further event in this batch adds its
            // remaining nulls once: its `left` is cleared below
            const uint32_t cseg = seg16(__ballot(xh < R), slot) & left;
            if (!cseg) m_null += (uint32_t)__popc(left);
            const bool act = cseg != 0;
            if (!__ballot(act)) break;
            const int e = __builtin_ctz(cseg | 0x10000u);  // 16 when idle
            left &= ~(cseg ^ (cseg - 1u));
            if (act) m_null += (uint32_t)(e - pos);
            const double xe = sbc_f64(xh, base + e);
            if (act && sl == e) Rb = R;

            // rate class and member index (class lanes of each slot; the
            // FP64 index is exact, see visit_domain)
            const uint32_t cseg_c = seg16(__ballot(xe < Pinc), slot);
            // an active slot always finds its class at or below lane 9 (lane 9
            // holds R > xe); an idle slot gets 9 too, so every class-indexed
            // shift below stays in range (its results are discarded)
            const int c = __builtin_ctz(cseg_c | 0x200u);
            const double q = (xe - (Pinc - W)) * inv_lane;
            const uint32_t jl = cvt_u32_sat(q);
            const uint32_t j = sbc32(jl, base + c);

            if constexpr (SCORE) {
                if (__ballot(act && m_null)) null_run(m_null, act);
            }
            if (act) m_null = 0;

            // member j: row by a row scan of per-row counts, column by rank
            const uint32_t cm = class_mask<uint32_t>(class_sel_lane((uint32_t)c), S, P, VM);
            const uint32_t cnt = (uint32_t)__popc(cm);
            const uint32_t incl = scan_row(cnt);
            const uint32_t yseg = seg16(__ballot(incl > j), slot);
            const int ys = __builtin_ctz(yseg | 0x10000u);
            const uint32_t jr = j - sbc32(incl - cnt, base + ys);
            const uint32_t rowm = sbc32(cm, base + ys);
            // the column: the first lane whose count of members up to and
            // including it exceeds jr
            const uint32_t rank_incl = (uint32_t)__popc(rowm & upto_lane);
            const uint32_t xseg = seg16(__ballot(rank_incl > jr), slot);
            const int xs = __builtin_ctz(xseg | 0x10000u);

            // packed class tallies of the flipped site's in-tile neighbours,
            // the three rows summed inside the slot by DPP
            const bool up = c >= 5;
            const int c_new = up ? c - 5 : c + 5;
            // this lane's neighbours of the flipped site (nm, as in
            // visit_domain): read at xa and xb, kept where nm has the bit
            const bool on_row = sl == ys;
            const bool near = (uint32_t)(sl - ys + 1) <= 2u && sl < B;  // rows ys - 1 .. ys + 1
            const uint32_t bx = 1u << xs;
            const uint32_t mrow = ((bx << 1) | (bx >> 1)) & vm_row;
            const uint32_t nm = near ? (on_row ? mrow : bx) : 0u;
            const int xa = (xs - (on_row ? 1 : 0)) & 31, xb = (xs + 1) & 31;
            const uint32_t va = (nm >> xa) & 1u, vb = (nm >> xb) & 1u;
            uint32_t nb = (va << class_pos3<uint32_t>(S, P, xa)) +
                          (vb << class_pos3<uint32_t>(S, P, xb));
            nb += dppz<kRowShr + 1>(nb) + dppz<kRowShl1>(nb);
            const uint32_t nb_s = sbc32(nb, base + ys);
            if (act) {
                // every neighbour moves one class up (flip to +1) or down, so
                // class lane l gains the neighbours of class l -/+ 1 and loses
                // its own; the flipped site moves from c to c -/+ 5
                n_lane = n_lane + __builtin_amdgcn_ubfe(nb_s, up ? from_up : from_dn, 3) -
                         __builtin_amdgcn_ubfe(nb_s, sl3, 3) + (sl == c_new ? 1u : 0u) -
                         (sl == c ? 1u : 0u);
                ev_lane += sl == c ? 1u : 0u;
            }
            W = (double)n_lane * rd_lane;
            Pinc = scan16_f64(W);
            R = rowbcast_f64<9>(Pinc);

            if (act && on_row) S ^= bx;
            planes_step<uint32_t>(P, act ? nm : 0u, !up);
            if (act) pos = e + 1;
        }
        if (Rb != 0.0) {
            const uint64_t u53 = ((uint64_t)o.w << 21) | (o.z >> 11);
            const double u = (double)(u53 + 1) * 0x1p-53;
            neumaier_add(clk_sum, clk_comp, -log(u) * 4294967296.0 / Rb);
        }
    }
    if constexpr (SCORE) {
        null_run(m_null, A.on);
        const double ev = (double)ev_lane;
        const bool cl_on = A.on && sl < 10;
        const int cl = cl_on ? sl : 0;
        const double gJ = cl_on ? rt->gJ[cl] : 0.0, gh = cl_on ? rt->gh[cl] : 0.0;
        const double aJ = cl_on ? rt->aJ[cl] : 0.0, ah = cl_on ? rt->ah[cl] : 0.0;
        out.sJ = sum_row_f64(gJ * ev - aJ * A_lane, base);
        out.sh = sum_row_f64(gh * ev - ah * A_lane, base);
    }
    // events, dM and dB of each slot from its per-class event counts
#pragma unroll
    for (int cc = 0; cc < 10; ++cc) {
        const int64_t n = (int64_t)sbc32(ev_lane, base + cc);
        const int64_t m2 = cc >= 5 ? -2 : 2;
        out.events += n;
        out.dM += m2 * n;
        out.dB += m2 * (2 * (cc % 5) - 4) * n;  // square lattices only
    }
    {
        const double cs = sum_row_f64(clk_sum, base);
        const double cc = sum_row_f64(clk_comp, base);
        if (A.on && sl == 0) {
            Dom *dm = dom_base + dom_off + A.d;
            double ds = dm->clk_sum, dc = dm->clk_comp;
            neumaier_add(ds, dc, cs);
            neumaier_add(ds, dc, cc);
            dm->clk_sum = ds;
            dm->clk_comp = dc;
            dm->events += out.events;
        }
    }

    // ---- write the tiles back through LDS
    if (A.on && sl < B) {
        for (int q = 0; q < SB4; ++q)
            *reinterpret_cast<uint32_t *>(tile + sl * SB + 4 * q) =
                bits_to_bytes((S >> (4 * q)) & 0xFu);
    }
    wave_sync_lds();
    if (A.on) {
        int8_t *wblk = lat + (int64_t)dd * n2;
        if ((B & 3) == 0) {
            for (int q = sl; q < B * B4; q += kSlotW)
                *reinterpret_cast<uint32_t *>(wblk + 4 * q) =
                    *reinterpret_cast<const uint32_t *>(tile + 4 * q);
        } else {
            for (int q = sl; q < B * B; q += kSlotW) {
                const int row = q / B, col = q - row * B;
                wblk[q] = (int8_t)tile[row * SB + col];
            }
        }
    }
    wave_sync_lds();
    return out;
}

// Mean of the slot's replica's domain clocks (all lanes of the slot).
__device__ inline double replica_time_slot(const KParams &K, const Rep &rp, int rho_ok,
                                           int dom_off, int sl, int base) {
    double s = 0.0, cpen = 0.0;
    if (rho_ok)
        for (int dd = sl; dd < rp.ND; dd += kSlotW) {
            const Dom &dm = K.dom[dom_off + dd];
            neumaier_add(s, cpen, dm.clk_sum + dm.clk_comp);
        }
    return sum_row_f64(s + cpen, base) / (double)rp.ND;
}

struct MultiShared {
    int64_t dM[kWavesPerPersistentGroup], dB[kWavesPerPersistentGroup],
        ev[kWavesPerPersistentGroup];
    double sJ[kWavesPerPersistentGroup], sh[kWavesPerPersistentGroup];
};

// All n_sweeps sweeps of one work item.
template <bool SCORE>
__device__ void run_item(const KParams &K, const MItem &it, int wave, int lane, uint8_t *lds,
                         MultiShared *ms, int64_t sweep0, int64_t run_done0, int64_t n_sweeps,
                         int64_t rec_every, int64_t rec_base) {
    const int slot = lane >> 4, sl = lane & 15, base = lane & ~15;
    const bool intra = it.kind == 1;
    const int nw = intra ? it.nw : 1;
    const int rho = intra ? it.rho[0] : it.rho[slot];  // per slot
    const bool on_rep = rho >= 0;
    const int rho0 = it.rho[0];
    const Rep shape = K.reps[rho0];  // common to the item's replicas
    // per-slot replica fields (the rest of the descriptor is the shape's)
    const int64_t spin_off = on_rep ? K.reps[rho].spin_off : 0;
    const int32_t dom_off = on_rep ? K.reps[rho].dom_off : 0;
    const Rep &rp = shape;
    RepAcc acc = on_rep ? K.acc[rho] : RepAcc{0, 0, 0, 0};
    int64_t dM = 0, dB = 0, ev = 0;
    double sJ = 0.0, sh = 0.0;
    const int nphase = shape.sched == 1 ? 8 : 4;
    const int per_colour = shape.ND >> 2;
    const int g = intra ? wave * kSlots + slot : 0;  // slot index within the team
    const int stride = intra ? kSlots * nw : 1;
    const int steps = intra ? (per_colour + stride - 1) / stride : per_colour;
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t w = (uint32_t)(sweep0 + i);
        for (int p = 0; p < nphase; ++p) {
            int vis = 0;
            const int col = on_rep ? phase_colour4((uint32_t)rp.sched, K.seed, (uint32_t)rho, w, p, &vis) : 0;
            for (int kk = 0; kk < steps; ++kk) {
                const int i2 = intra ? g + kk * stride : kk;
                SlotDomain A;
                A.on = on_rep && col >= 0 && i2 < per_colour;
                int d = 0, oy = 0, ox = 0;
                if (A.on) colour_domain(rp, col, i2, &d, &oy, &ox);
                A.lat = nullptr;
                A.spin_off = spin_off;
                A.oy = oy;
                A.ox = ox;
                A.d = (uint32_t)d;
                A.rho = (uint32_t)(on_rep ? rho : 0);
                const VisitOut o = visit_multi<SCORE>(K.spins, shape, K.rates, K.dom, dom_off, A,
                                                      (uint32_t)vis, w, K.seed, lds);
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
            if (intra) {
                // sum the slots' parts: first inside the wavefront, then
                // over the team's wavefronts
                int64_t v0 = dM, v1 = dB, v2 = ev;
                double f0 = sJ, f1 = sh;
                int64_t t0 = 0, t1 = 0, t2 = 0;
                double u0 = 0.0, u1 = 0.0;
                for (int s2 = 0; s2 < kSlots; ++s2) {
                    const int src = s2 * kSlotW;
                    t0 += (int64_t)sbc64((uint64_t)v0, src);
                    t1 += (int64_t)sbc64((uint64_t)v1, src);
                    t2 += (int64_t)sbc64((uint64_t)v2, src);
                    u0 += __longlong_as_double((long long)sbc64(__double_as_longlong(f0), src));
                    u1 += __longlong_as_double((long long)sbc64(__double_as_longlong(f1), src));
                }
                if (nw > 1) {
                    if (lane == 0) {
                        ms->dM[wave] = t0;
                        ms->dB[wave] = t1;
                        ms->ev[wave] = t2;
                        ms->sJ[wave] = u0;
                        ms->sh[wave] = u1;
                    }
                    __syncthreads();
                    t0 = t1 = t2 = 0;
                    u0 = u1 = 0.0;
                    for (int q = 0; q < nw; ++q) {
                        t0 += ms->dM[q];
                        t1 += ms->dB[q];
                        t2 += ms->ev[q];
                        u0 += ms->sJ[q];
                        u1 += ms->sh[q];
                    }
                }
                acc.M += t0;
                acc.B += t1;
                acc.events += t2;
                if (wave == 0) {
                    // the replica record: lanes of slot 0 reduce the clocks
                    const double tt = replica_time_slot(K, rp, 1, dom_off, sl, base);
                    if (lane == 0) {
                        if constexpr (SCORE) {
                            const int64_t bin = (done - 1) / rec_every;
                            double *b = K.bins + ((int64_t)rho * K.n_bins + bin) * 2;
                            b[0] += u0;
                            b[1] += u1;
                        }
                        if (K.write_records && done % rec_every == 0) {
                            Record r;
                            r.sweep = (int64_t)w + 1;
                            r.M = acc.M;
                            r.B = acc.B;
                            r.events = acc.events;
                            r.steps = ((int64_t)w + 1) * (int64_t)rp.NI * rp.ND * rp.visits;
                            r.t = tt;
                            K.rec[(rec_base + done / rec_every - 1) * K.n_rep + rho] = r;
                        }
                    }
                }
                if (nw > 1) __syncthreads();
            } else {
                acc.M += dM;
                acc.B += dB;
                acc.events += ev;
                const double tt = replica_time_slot(K, rp, on_rep, dom_off, sl, base);
                if (on_rep && sl == 0) {
                    if constexpr (SCORE) {
                        const int64_t bin = (done - 1) / rec_every;
                        double *b = K.bins + ((int64_t)rho * K.n_bins + bin) * 2;
                        b[0] += sJ;
                        b[1] += sh;
                    }
                    if (K.write_records && done % rec_every == 0) {
                        Record r;
                        r.sweep = (int64_t)w + 1;
                        r.M = acc.M;
                        r.B = acc.B;
                        r.events = acc.events;
                        r.steps = ((int64_t)w + 1) * (int64_t)rp.NI * rp.ND * rp.visits;
                        r.t = tt;
                        K.rec[(rec_base + done / rec_every - 1) * K.n_rep + rho] = r;
                    }
                }
            }
            dM = dB = ev = 0;
            sJ = sh = 0.0;
        }
    }
    if (intra) {
        if (wave == 0 && lane == 0) K.acc[rho] = acc;
    } else if (on_rep && sl == 0) {
        K.acc[rho] = acc;
    }
}

// Multi-slot persistent kernel: workgroup items (teams of four wavefronts)
// first, then wavefront items; every wavefront leaves once both queues are
// drained.  Occupancy: the forward instantiation is held to 168 registers
// (three wavefronts per SIMD), the score one to 128 (four per SIMD: it runs
// ~9% faster than at three on the differentiable batch, while the forward
// one at four loses ~13% on the ragged batch).  Both spill a few values of
// the item and sweep loops, none inside the tick loop.
template <bool SCORE>
__global__ __launch_bounds__(64 * kWavesPerPersistentGroup) __attribute__((amdgpu_waves_per_eu(SCORE ? 4 : 3, 8))) void k_persistent_multi(
    KParams K, const MItem *__restrict__ items, int n_wg_items, int n_wave_items,
    int64_t n_sweeps) {
    const int64_t sweep0 = K.ctl->sweep;  // device counters: replayable launch
    const int64_t run_done0 = K.ctl->run_done;
    __shared__ __attribute__((aligned(16)))
    uint8_t lds_all[kWavesPerPersistentGroup][kSlots * kSlotLds];
    __shared__ MultiShared ms;
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint8_t *lds = lds_all[wave];
    const int lane = __lane_id();
    const int64_t rec_every = K.ctl->rec_every;
    const int64_t rec_base = K.ctl->rec_base;
    bool wg_phase = true;
    for (;;) {
        int idx;
        int me;
        if (wg_phase) {
            if (threadIdx.x == 0)
                s_item = (int)atomicAdd((unsigned long long *)&K.ctl->queue, 1ull);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            if (it >= n_wg_items) {
                wg_phase = false;
                continue;
            }
            idx = it;
            me = wave;
        } else {
            int v = 0;
            if (lane == 0) v = (int)atomicAdd((unsigned long long *)&K.ctl->queue2, 1ull);
            v = (int)rdl32((uint32_t)v, 0);
            if (v >= n_wave_items) return;
            idx = n_wg_items + v;
            me = 0;
        }
        idx = __builtin_amdgcn_readfirstlane(idx);
        me = __builtin_amdgcn_readfirstlane(me);
        const MItem it = items[idx];
        run_item<SCORE>(K, it, me, lane, lds, &ms, sweep0, run_done0, n_sweeps, rec_every,
                        rec_base);
    }
}

}  // namespace kmcdev
