// rewl_lipid.hip -- the amphiphile model with explicit solvent (Vogel, Li,
// Wuest, Landau, J. Phys.: Conf. Ser. (2014), Sec. 3.2, Eqs. (3)-(5) and
// Fig. 5), sampled with the Wang-Landau rule on energy bins (Sec. 2).
//
// Particles: nmol lipids of a polar head P and two hydrophobic tails H
// (P-H-H) and solvent W in a periodic cube.  Non-bonded pairs H-W and H-P
// repel by 4 (1.05 / r)^9 (Eq. 3); the other pairs are Lennard-Jones
// 4 eps (r^-12 - r^-6) (Eq. 4), eps = 1 or eps_ww for W-W, both cut at
// r = 2.5 without shift.  Consecutive beads of a lipid are bonded by FENE
// (K = 30, R = 1.3) plus the WCA repulsion (Eq. 5); a bond at r >= R is
// forbidden.  The FENE logarithm is evaluated from basic IEEE operations
// (log_basic), so every implementation following the same steps agrees to
// the bit.
//
// Moves: with probability rep_thr / 2^32 a reptation (Fig. 5): a lipid and
// one of its ends are drawn, one of the n_c solvent particles within R of
// that end is captured as the new end bead, the beads shift along the chain
// and the far end is released as solvent (positions unchanged); the
// acceptance carries the selection ratio n_c / n_r, n_r counting solvent
// within R of the new end next to the released particle.  Otherwise one
// particle is displaced by 0.1 (2u - 1) per axis.
//
// State of a walker (one row of st.spins): coordinates float[np][3], types
// int8[np] (0 P, 1 H, 2 W; padded to 4 bytes), lipid rows int32[nmol][3]
// (head first), position table int32[np] (3 lipid + bead, -1 solvent).
//
// Energies are fixed point (units of 2^-32): every pair term is rounded once
// and totals and changes are exact integer sums, so the lanes and waves may
// add the partner terms in any order and every implementation agrees to the
// bit.
//
// Mapping: one walker per workgroup (the attempt kernel: up to 16 wavefronts
// sharing the 64-partner chunks; walk-in and set-up: one wavefront), its
// state, ln g and H in LDS.  Attempts are sequential.
#include "rewl_device.h"

namespace rewl_gpu {

namespace {

constexpr double kLipRc2 = 6.25;                       // 2.5^2
constexpr double kLipWcaRc2 = 0x1.428a2f98d728bp+0;    // RN(2^(1/3)) = RN((2^(1/6))^2)
constexpr double kLipR2 = 1.69;                        // FENE R^2, R = 1.3
constexpr double kLipSqrt2 = 0x1.6a09e667f3bcdp+0;     // RN(sqrt 2)
constexpr double kLn2C1 = 0x1.62e42fefa4000p-1;        // ln 2 to 40 bits
constexpr double kLn2C2 = -0x1.8432a1b0e2634p-43;      // RN(ln 2 - C1)
constexpr int kP = 0, kH = 1, kW = 2;

// Natural logarithm of a positive normal x: x = 2^k m with m in
// [sqrt(1/2), sqrt(2)), f = (m - 1) / (m + 1), ln m = 2 f (1 + s/3 + ... +
// s^12/25), s = f^2, by Horner without fused operations; ln x = k C1 +
// (k C2 + ln m).
__device__ __forceinline__ double log_basic(double x) {
#pragma clang fp contract(off)
    int k = 0;
    double m = __builtin_frexp(x, &k);
    m = m * 2.0;
    k -= 1;
    if (m > kLipSqrt2) {
        m = m * 0.5;
        k += 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double s2 = f * f;
    double p = 1.0 / 25.0;
    for (int n = 11; n >= 0; --n) {
        const double t = s2 * p;
        p = 1.0 / (double)(2 * n + 1) + t;
    }
    const double lm = (2.0 * f) * p;
    return (double)k * kLn2C1 + ((double)k * kLn2C2 + lm);
}

__device__ __forceinline__ double lip_min_image(float a, float b, float box, float half) {
#pragma clang fp contract(off)
    float x = b - a;
    if (x > half) x = x - box;
    else if (x < -half) x = x + box;
    return (double)x;
}

__device__ __forceinline__ double lip_r2(const float *a, const float *b, float box, float half) {
#pragma clang fp contract(off)
    const double dx = lip_min_image(a[0], b[0], box, half);
    const double dy = lip_min_image(a[1], b[1], box, half);
    const double dz = lip_min_image(a[2], b[2], box, half);
    return (dx * dx + dy * dy) + dz * dz;
}

// Pair energy of types ti, tj at squared distance r2 (Eqs. 3-5).
__device__ __forceinline__ double lip_pair(int ti, int tj, bool bonded, double r2, double eps_ww) {
#pragma clang fp contract(off)
    if (bonded) {
        if (r2 >= kLipR2) return __builtin_inf();
        const double fene = -(0.5 * 30.0 * 1.69) * log_basic(1.0 - r2 / kLipR2);
        double wca = 0.0;
        if (r2 < kLipWcaRc2) {
            const double s2 = 1.0 / r2;
            const double s6 = (s2 * s2) * s2;
            wca = 4.0 * ((s6 * s6) - s6) + 1.0;
        }
        return fene + wca;
    }
    if (r2 >= kLipRc2) return 0.0;
    const bool rep = (ti == kH && tj != kH) || (tj == kH && ti != kH);
    if (rep) {
        const double q = 1.05 / __builtin_sqrt(r2);
        const double q3 = (q * q) * q;
        return 4.0 * ((q3 * q3) * q3);
    }
    const double s2 = 1.0 / r2;
    const double s6 = (s2 * s2) * s2;
    const double v = 4.0 * ((s6 * s6) - s6);
    return (ti == kW && tj == kW) ? eps_ww * v : v;
}

__device__ __forceinline__ bool lip_bonded(int a, int b) {
    if (a < 0 || b < 0 || a / 3 != b / 3) return false;
    return a - b == 1 || b - a == 1;
}

__device__ __forceinline__ int lip_bin(const DevState &st, int64_t e) { return fx_bin(st.emin_fx, st.binw_fx, st.binw_inv, e); }

// fx(V_new) - fx(V_old) of one pair; false for a hard overlap.
__device__ __forceinline__ bool lip_term(double vn, double vo, int64_t &t) {
    int64_t a = 0, b = 0;
    const bool ok = fx_term(vn, a) & fx_term(vo, b);
    t = a - b;
    return ok;
}

__device__ __forceinline__ float lip_disp(uint32_t r) {
#pragma clang fp contract(off)
    return 0.1f * ((float)(r >> 9) * 0x1p-22f - 1.0f);
}
__device__ __forceinline__ float lip_wrap(float v, float box) {
#pragma clang fp contract(off)
    if (v < 0.0f) v = v + box;
    if (v >= box) v = v - box;
    return v;
}

// One walker's state in LDS.
struct LipView {
    float *x;
    int8_t *type;
    int32_t *lip;
    int32_t *where;
};

__device__ __forceinline__ LipView lip_view(const DevState &st, unsigned char *base) {
    LipView v;
    v.x = (float *)base;
    v.type = (int8_t *)(base + st.lip_off_type);
    v.lip = (int32_t *)(base + st.lip_off_lip);
    v.where = (int32_t *)(base + st.lip_off_where);
    return v;
}

// A proposal: displacement of particle b to xn, or a reptation of `lipid`
// changing the four particles c[] (ascending) to types nt[] and positions
// nwh[] with the new lipid row nl[]; n_c, n_r; energy change de.
struct LipProp {
    bool ok, rep;
    int b;
    float xn[3];
    int lipid, nc, nr;
    int c[4], nt[4], nwh[4], nl[3];
    int64_t de;   // units of 2^-32
};

// Solvent particles within R of particle e under the types `type` except the
// four particles of cs (given types ct); returns the count and, if pick >=
// 0, the pick-th of them in index order.
__device__ __forceinline__ int lip_near(const DevState &st, const LipView &v, int e, const int *cs, const int *ct,
                                        int pick, int *found, int lane) {
    const float box = st.box, half = 0.5f * st.box;
    const float xe[3] = {v.x[3 * e], v.x[3 * e + 1], v.x[3 * e + 2]};
    int n = 0;
    for (int c0 = 0; c0 < st.nb; c0 += 64) {
        const int j = c0 + lane;
        bool hit = false;
        if (j < st.nb && j != e) {
            int tj = v.type[j];
            if (cs) {
                for (int a = 0; a < 4; ++a)
                    if (cs[a] == j) tj = ct[a];
            }
            if (tj == kW) hit = lip_r2(xe, v.x + 3 * j, box, half) < kLipR2;
        }
        const unsigned long long m = __ballot(hit);
        const int cnt = __builtin_popcountll(m);
        if (pick >= 0 && pick >= n && pick < n + cnt) {
            unsigned long long mm = m;
            for (int r = pick - n; r > 0; --r) mm &= mm - 1ull;
            *found = c0 + (int)__builtin_ctzll(mm);
        }
        n += cnt;
    }
    return n;
}

// Build the proposal of one attempt from its Philox blocks (a: particle or
// lipid, displacement; u: acceptance, move type, end, captured particle).
__device__ __forceinline__ void lip_propose(const DevState &st, const LipView &v, const U4 &a, const U4 &u,
                                            LipProp &p, int lane) {
#pragma clang fp contract(off)
    const float box = st.box, half = 0.5f * st.box;
    p.ok = false;
    p.rep = u.y < st.lip_rep_thr;
    int64_t acc = 0;
    bool bad = false;
    if (!p.rep) {
        const int b = (int)mul_shift(a.x, (uint32_t)st.nb);
        p.b = b;
        const float o[3] = {v.x[3 * b], v.x[3 * b + 1], v.x[3 * b + 2]};
        p.xn[0] = lip_wrap(o[0] + lip_disp(a.y), box);
        p.xn[1] = lip_wrap(o[1] + lip_disp(a.z), box);
        p.xn[2] = lip_wrap(o[2] + lip_disp(a.w), box);
        const int tb = v.type[b], wb = v.where[b];
        for (int c0 = 0; c0 < st.nb; c0 += 64) {
            const int j = c0 + lane;
            if (j < st.nb && j != b) {
                const float *xj = v.x + 3 * j;
                const int tj = v.type[j];
                const bool bd = lip_bonded(wb, v.where[j]);
                int64_t t = 0;
                bad |= !lip_term(lip_pair(tb, tj, bd, lip_r2(p.xn, xj, box, half), st.lip_eps_ww),
                                 lip_pair(tb, tj, bd, lip_r2(o, xj, box, half), st.lip_eps_ww), t);
                acc += t;
            }
        }
    } else {
        const int lipid = (int)mul_shift(a.x, (uint32_t)st.nmol);
        p.lipid = lipid;
        const int end = (int)(u.z >> 31);
        const int l0 = v.lip[3 * lipid], l1 = v.lip[3 * lipid + 1], l2 = v.lip[3 * lipid + 2];
        const int e = end == 0 ? l0 : l2;
        int cap = -1;
        const int nc = lip_near(st, v, e, nullptr, nullptr, -1, &cap, lane);
        if (nc == 0) return;
        lip_near(st, v, e, nullptr, nullptr, (int)mul_shift(u.w, (uint32_t)nc), &cap, lane);
        cap = __builtin_amdgcn_readfirstlane(cap);
        int rel;
        if (end == 0) { p.nl[0] = cap; p.nl[1] = l0; p.nl[2] = l1; rel = l2; }
        else { p.nl[0] = l1; p.nl[1] = l2; p.nl[2] = cap; rel = l0; }
        int all[4] = {cap, l0, l1, l2};
        for (int i = 1; i < 4; ++i)
            for (int k = i; k > 0 && all[k - 1] > all[k]; --k) {
                const int t = all[k]; all[k] = all[k - 1]; all[k - 1] = t;
            }
        for (int i = 0; i < 4; ++i) {
            const int q = all[i];
            p.c[i] = q;
            if (q == rel) { p.nt[i] = kW; p.nwh[i] = -1; }
            else {
                const int pos = q == p.nl[0] ? 0 : (q == p.nl[1] ? 1 : 2);
                p.nt[i] = pos == 0 ? kP : kH;
                p.nwh[i] = 3 * lipid + pos;
            }
        }
        p.nc = nc;
        p.nr = lip_near(st, v, l1, p.c, p.nt, -1, &cap, lane);
        // fx(V_new(i, j)) - fx(V_old(i, j)) over the pairs holding a changed
        // particle i (each pair once: i != j, and i < j when j changes too)
        for (int c0 = 0; c0 < st.nb; c0 += 64) {
            const int j = c0 + lane;
            if (j < st.nb) {
                int tjo = v.type[j], wjo = v.where[j], tjn = tjo, wjn = wjo;
                bool jin = false;
                for (int i = 0; i < 4; ++i)
                    if (p.c[i] == j) { jin = true; tjn = p.nt[i]; wjn = p.nwh[i]; }
                for (int i = 0; i < 4; ++i) {
                    const int ci = p.c[i];
                    if (ci == j || (jin && ci > j)) continue;
                    const double r2 = lip_r2(v.x + 3 * ci, v.x + 3 * j, box, half);
                    int64_t t = 0;
                    bad |= !lip_term(lip_pair(p.nt[i], tjn, lip_bonded(p.nwh[i], wjn), r2, st.lip_eps_ww),
                                     lip_pair(v.type[ci], tjo, lip_bonded(v.where[ci], wjo), r2, st.lip_eps_ww), t);
                    acc += t;
                }
            }
        }
    }
    p.de = wave_sum64(acc);
    p.ok = __ballot(bad) == 0ull;
}

__device__ __forceinline__ bool lip_accept(const LipProp &p, double d, uint32_t r) {
#pragma clang fp contract(off)
    if (!p.rep) return accept64(d, r);
    const double uu = (double)r * 0x1p-32;
    if (d >= 0.0) return (uu * (double)p.nr) * exp_neg(-d) < (double)p.nc;
    return uu * (double)p.nr < exp_neg(d) * (double)p.nc;
}

__device__ __forceinline__ void lip_apply(const DevState &st, const LipView &v, const LipProp &p, int lane) {
    if (lane == 0) {
        if (!p.rep) {
            v.x[3 * p.b] = p.xn[0];
            v.x[3 * p.b + 1] = p.xn[1];
            v.x[3 * p.b + 2] = p.xn[2];
        } else {
            for (int i = 0; i < 4; ++i) {
                v.type[p.c[i]] = (int8_t)p.nt[i];
                v.where[p.c[i]] = p.nwh[i];
            }
            for (int i = 0; i < 3; ++i) v.lip[3 * p.lipid + i] = p.nl[i];
        }
    }
    (void)st;
}

__device__ __forceinline__ void lip_words(const DevState &st, uint64_t t, uint32_t w, uint32_t dom, uint32_t dom_u,
                                          U4 &a, U4 &u) {
    a = philox10((uint32_t)t, (uint32_t)(t >> 32), w, st.ctr3 | (dom << 24), st.key0, st.key1);
    u = philox10((uint32_t)t, (uint32_t)(t >> 32), w, st.ctr3 | (dom_u << 24), st.key0, st.key1);
}

// ---------------------------------------------------------------------------
// Energy of every walker's starting configuration: the exact sum of the
// pair terms over i < j, rows i dealt to the lanes, each term's high and low
// 32 bits summed separately (neither sum can overflow); a start with a hard
// overlap (a bond at R or beyond included) or out of range gets the bin
// INT32_MIN, which the host refuses.
__global__ __launch_bounds__(64) void k_lipid_init(DevState st) {
#pragma clang fp contract(off)
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    unsigned char *row = (unsigned char *)(st.spins + (size_t)w * st.Npad);
    const LipView v = lip_view(st, row);
    const float box = st.box, half = 0.5f * st.box;
    int64_t shi = 0, slo = 0;
    bool bad = false;
    for (int i = lane; i < st.nb; i += 64) {
        const int ti = v.type[i], wi = v.where[i];
        for (int j = i + 1; j < st.nb; ++j) {
            int64_t t = 0;
            bad |= !fx_term(lip_pair(ti, v.type[j], lip_bonded(wi, v.where[j]),
                                     lip_r2(v.x + 3 * i, v.x + 3 * j, box, half), st.lip_eps_ww), t);
            shi += t >> 32;
            slo += t & 0xffffffffll;
        }
    }
    shi = wave_sum64(shi);
    slo = wave_sum64(slo);
    bad = __ballot(bad) != 0ull;
    if (lane == 0) {
        int64_t e = 0;
        const bool ok = !bad && shi > -(1ll << 30) && shi < (1ll << 30) && fx_add(shi * 4294967296ll, slo, e);
        st.Efx[w] = ok ? e : 0;
        st.E[w] = ok ? lip_bin(st, e) : INT32_MIN;
    }
}

// Walk-in (the trimer walk-in rule with the lipid moves): Wang-Landau with
// ln f = 1 as visit counts over the B bins (energies outside the range count
// at the nearest end bin), under the lid, until the bin lies in the window.
__global__ __launch_bounds__(64) void k_lipid_walkin(DevState st, int64_t chunk, int64_t budget) {
#pragma clang fp contract(off)
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    if (st.walkin_done[w]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *cnt = (uint32_t *)(smem + st.Npad);
    const uint32_t *gx = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ((uint32_t *)smem)[i] = gx[i];
    const uint32_t *gcnt = st.walkin_cnt + (size_t)w * st.Bpad;
    for (int b = lane; b < st.B; b += 64) cnt[b] = gcnt[b];
    __syncthreads();
    const LipView v = lip_view(st, smem);

    const int k = w / st.m;
    const int lo = st.start[k], hi = lo + st.W - 1;
    const int B = st.B;
    int E = st.E[w];
    int64_t Ef = st.Efx[w];
    int64_t t = st.walkin_att[w];
    const int slack = st.walkin_slack;
    const bool down = E > hi;
    int bound = t == 0 ? (down ? E + slack : E - slack) : st.walkin_bound[w];
    const int64_t end = (t + chunk < budget) ? t + chunk : budget;
    bool done = (E >= lo && E <= hi);
    while (!done && t < end) {
        U4 a, u;
        lip_words(st, (uint64_t)t, (uint32_t)w, kDomWalkin, kDomWalkinU, a, u);
        LipProp p;
        lip_propose(st, v, a, u, p, lane);
        int64_t e_new = 0;
        if (p.ok && fx_add(Ef, p.de, e_new)) {
            const int bn = lip_bin(st, e_new);
            const int co = E < 0 ? 0 : (E >= B ? B - 1 : E);
            const int cn = bn < 0 ? 0 : (bn >= B ? B - 1 : bn);
            const double d = (double)((int64_t)cnt[co] - (int64_t)cnt[cn]);
            const bool inside = slack == 0 || (down ? bn <= bound : bn >= bound);
            if (inside && lip_accept(p, d, u.x)) {
                lip_apply(st, v, p, lane);
                Ef = e_new;
                E = bn;
                if (slack && down && E + slack < bound) bound = E + slack;
                if (slack && !down && E - slack > bound) bound = E - slack;
            }
        }
        if (lane == 0) cnt[E < 0 ? 0 : (E >= B ? B - 1 : E)] += 1u;
        __syncthreads();
        ++t;
        if (E >= lo && E <= hi) done = true;
    }
    __syncthreads();
    uint32_t *ox = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ox[i] = ((uint32_t *)smem)[i];
    uint32_t *ocnt = st.walkin_cnt + (size_t)w * st.Bpad;
    for (int b = lane; b < B; b += 64) ocnt[b] = cnt[b];
    if (lane == 0) {
        st.E[w] = E;
        st.Efx[w] = Ef;
        st.walkin_att[w] = t;
        st.walkin_done[w] = done ? 1 : 0;
        st.walkin_bound[w] = bound;
    }
}

// Main-phase attempts s0 .. s0+n-1 of every walker (Sec. 2): a proposal
// whose new bin leaves the window is rejected, else accepted with
// min[1, g(old)/g(new)] (times n_c / n_r for a reptation); then
// ln g += ln f and H += 1 at the bin after the decision.
//
// One workgroup per walker with up to 16 wavefronts: wave v takes the
// 64-partner chunks c = v, v + nwave, ...; the fixed-point partner terms go
// to LDS (tbuf[c][lane]) and wave 0 adds them up (exact, any order), decides
// and applies the move.  Reptation candidates are
// found with one ballot mask per chunk, written to LDS and read by every
// wave.  All branches that contain a barrier depend only on the attempt's
// random words or on values every wave reads from LDS, so the waves agree.
__global__ __launch_bounds__(1024) void k_lipid_sweep(DevState st, int64_t s0, int64_t n) {
#pragma clang fp contract(off)
    const int w = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nwave = (int)(blockDim.x >> 6);
    if (*st.converged) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = st.W, Wpad = st.Wpad;
    const int nch = (st.nb + 63) / 64;
    double *g = (double *)(smem + st.Npad);
    uint32_t *H = (uint32_t *)(smem + st.Npad + (size_t)Wpad * 8);
    int64_t *tbuf = (int64_t *)(smem + st.Npad + (size_t)Wpad * 12);
    unsigned long long *mask1 = (unsigned long long *)(tbuf + (size_t)nch * 64);
    unsigned long long *mask2 = mask1 + nch;
    const uint32_t *gx = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = threadIdx.x; i < st.Npad / 4; i += blockDim.x) ((uint32_t *)smem)[i] = gx[i];
    const size_t row = (size_t)w * Wpad;
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        g[b] = st.lng[row + b];
        H[b] = st.H[row + b];
    }
    __syncthreads();
    const LipView v = lip_view(st, smem);
    const float box = st.box, half = 0.5f * st.box;
    const int k = w / st.m;
    const int lo = st.start[k], hi = lo + W - 1;
    const double lnf = st.lnf[k];
    int E = st.E[w];
    int64_t Ef = st.Efx[w];
    if (E < lo || E > hi) return;   // not walked in (every wave reads the same E)
    U4 la, lu;   // random words of attempt t0 + lane, drawn 64 attempts at a time
    for (int64_t t = 0; t < n; ++t) {
        const int j64 = (int)(t & 63);
        if (j64 == 0) lip_words(st, (uint64_t)(s0 + t + lane), (uint32_t)w, kDomMove, kDomMoveU, la, lu);
        U4 a, u;
        a.x = __builtin_amdgcn_readlane(la.x, j64); a.y = __builtin_amdgcn_readlane(la.y, j64);
        a.z = __builtin_amdgcn_readlane(la.z, j64); a.w = __builtin_amdgcn_readlane(la.w, j64);
        u.x = __builtin_amdgcn_readlane(lu.x, j64); u.y = __builtin_amdgcn_readlane(lu.y, j64);
        u.z = __builtin_amdgcn_readlane(lu.z, j64); u.w = __builtin_amdgcn_readlane(lu.w, j64);
        LipProp p;
        p.ok = true;
        p.rep = u.y < st.lip_rep_thr;
        if (!p.rep) {
            const int b = (int)mul_shift(a.x, (uint32_t)st.nb);
            p.b = b;
            const float o[3] = {v.x[3 * b], v.x[3 * b + 1], v.x[3 * b + 2]};
            p.xn[0] = lip_wrap(o[0] + lip_disp(a.y), box);
            p.xn[1] = lip_wrap(o[1] + lip_disp(a.z), box);
            p.xn[2] = lip_wrap(o[2] + lip_disp(a.w), box);
            const int tb = v.type[b], wb = v.where[b];
            for (int c = wave; c < nch; c += nwave) {
                const int j = c * 64 + lane;
                int64_t tj = 0;
                if (j < st.nb && j != b) {
                    const float *xj = v.x + 3 * j;
                    const int tjt = v.type[j];
                    const bool bd = lip_bonded(wb, v.where[j]);
                    if (!lip_term(lip_pair(tb, tjt, bd, lip_r2(p.xn, xj, box, half), st.lip_eps_ww),
                                  lip_pair(tb, tjt, bd, lip_r2(o, xj, box, half), st.lip_eps_ww), tj))
                        tj = kFxBad;
                }
                tbuf[c * 64 + lane] = tj;
            }
        } else {
            const int lipid = (int)mul_shift(a.x, (uint32_t)st.nmol);
            p.lipid = lipid;
            const int end = (int)(u.z >> 31);
            const int l0 = v.lip[3 * lipid], l1 = v.lip[3 * lipid + 1], l2 = v.lip[3 * lipid + 2];
            const int e = end == 0 ? l0 : l2;
            const float xe[3] = {v.x[3 * e], v.x[3 * e + 1], v.x[3 * e + 2]};
            for (int c = wave; c < nch; c += nwave) {
                const int j = c * 64 + lane;
                bool hit = false;
                if (j < st.nb && j != e && v.type[j] == kW) hit = lip_r2(xe, v.x + 3 * j, box, half) < kLipR2;
                const unsigned long long m = __ballot(hit);
                if (lane == 0) mask1[c] = m;
            }
            __syncthreads();
            int nc = 0;
            for (int c = 0; c < nch; ++c) nc += __builtin_popcountll(mask1[c]);
            if (nc == 0) {
                p.ok = false;
            } else {
                int pick = (int)mul_shift(u.w, (uint32_t)nc);
                int cap = -1;
                for (int c = 0; c < nch && cap < 0; ++c) {
                    unsigned long long m = mask1[c];
                    const int cnt = __builtin_popcountll(m);
                    if (pick < cnt) {
                        for (int r = pick; r > 0; --r) m &= m - 1ull;
                        cap = c * 64 + (int)__builtin_ctzll(m);
                    } else {
                        pick -= cnt;
                    }
                }
                int rel;
                if (end == 0) { p.nl[0] = cap; p.nl[1] = l0; p.nl[2] = l1; rel = l2; }
                else { p.nl[0] = l1; p.nl[1] = l2; p.nl[2] = cap; rel = l0; }
                int all[4] = {cap, l0, l1, l2};
                for (int i = 1; i < 4; ++i)
                    for (int q = i; q > 0 && all[q - 1] > all[q]; --q) {
                        const int tq = all[q]; all[q] = all[q - 1]; all[q - 1] = tq;
                    }
                for (int i = 0; i < 4; ++i) {
                    const int q = all[i];
                    p.c[i] = q;
                    if (q == rel) { p.nt[i] = kW; p.nwh[i] = -1; }
                    else {
                        const int pos = q == p.nl[0] ? 0 : (q == p.nl[1] ? 1 : 2);
                        p.nt[i] = pos == 0 ? kP : kH;
                        p.nwh[i] = 3 * lipid + pos;
                    }
                }
                p.nc = nc;
                // n_r: solvent within R of l1 under the new types
                const float x1[3] = {v.x[3 * l1], v.x[3 * l1 + 1], v.x[3 * l1 + 2]};
                for (int c = wave; c < nch; c += nwave) {
                    const int j = c * 64 + lane;
                    bool hit = false;
                    if (j < st.nb && j != l1) {
                        int tj = v.type[j];
                        for (int i = 0; i < 4; ++i)
                            if (p.c[i] == j) tj = p.nt[i];
                        if (tj == kW) hit = lip_r2(x1, v.x + 3 * j, box, half) < kLipR2;
                    }
                    const unsigned long long m = __ballot(hit);
                    if (lane == 0) mask2[c] = m;
                }
                // partner terms of the reptation (see lip_propose)
                for (int c = wave; c < nch; c += nwave) {
                    const int j = c * 64 + lane;
                    int64_t tj = 0;
                    bool bad = false;
                    if (j < st.nb) {
                        const int tjo = v.type[j], wjo = v.where[j];
                        int tjn = tjo, wjn = wjo;
                        bool jin = false;
                        for (int i = 0; i < 4; ++i)
                            if (p.c[i] == j) { jin = true; tjn = p.nt[i]; wjn = p.nwh[i]; }
                        for (int i = 0; i < 4; ++i) {
                            const int ci = p.c[i];
                            if (ci == j || (jin && ci > j)) continue;
                            const double r2 = lip_r2(v.x + 3 * ci, v.x + 3 * j, box, half);
                            int64_t d = 0;
                            bad |= !lip_term(lip_pair(p.nt[i], tjn, lip_bonded(p.nwh[i], wjn), r2, st.lip_eps_ww),
                                             lip_pair(v.type[ci], tjo, lip_bonded(v.where[ci], wjo), r2,
                                                      st.lip_eps_ww),
                                             d);
                            tj += d;
                        }
                    }
                    tbuf[c * 64 + lane] = bad ? kFxBad : tj;
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            if (p.ok) {
                int64_t acc = 0;
                bool bad = false;
                for (int c = 0; c < nch; ++c) {
                    const int64_t tj = tbuf[c * 64 + lane];
                    if (tj == kFxBad) bad = true;
                    else acc += tj;
                }
                p.de = wave_sum64(acc);
                p.ok = __ballot(bad) == 0ull;
                if (p.rep) {
                    int nr = 0;
                    for (int c = 0; c < nch; ++c) nr += __builtin_popcountll(mask2[c]);
                    p.nr = nr;
                }
                int64_t e_new = 0;
                if (p.ok && fx_add(Ef, p.de, e_new)) {
                    const int bn = lip_bin(st, e_new);
                    if (bn >= lo && bn <= hi && lip_accept(p, g[E - lo] - g[bn - lo], u.x)) {
                        lip_apply(st, v, p, lane);
                        Ef = e_new;
                        E = bn;
                    }
                }
            }
            if (lane == 0) {
                g[E - lo] = g[E - lo] + lnf;
                H[E - lo] += 1u;
            }
        }
        __syncthreads();
    }
    const uint32_t *sx = (const uint32_t *)smem;
    uint32_t *ox = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = threadIdx.x; i < st.Npad / 4; i += blockDim.x) ox[i] = sx[i];
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        st.lng[row + b] = g[b];
        st.H[row + b] = H[b];
    }
    if (threadIdx.x == 0) {
        st.E[w] = E;
        st.Efx[w] = Ef;
    }
}

hipError_t lip_allow(const void *fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

static int lipid_waves(const DevState &st) {
    const int nch = (st.nb + 63) / 64;
    return nch < 16 ? nch : 16;
}
size_t lipid_sweep_lds_bytes(const DevState &st) {
    const int nch = (st.nb + 63) / 64;
    return (size_t)st.Npad + (size_t)st.Wpad * 12 + (size_t)nch * 64 * 8 + (size_t)nch * 16;
}
size_t lipid_walkin_lds_bytes(const DevState &st) { return (size_t)st.Npad + (size_t)st.Bpad * 4; }

hipError_t launch_lipid_init(const DevState &st, hipStream_t s) {
    hipLaunchKernelGGL(k_lipid_init, dim3(st.nw), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_lipid_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s) {
    const size_t lds = lipid_walkin_lds_bytes(st);
    hipError_t e = lip_allow((const void *)k_lipid_walkin, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lipid_walkin, dim3(st.nw), dim3(64), lds, s, st, chunk, budget);
    return hipGetLastError();
}

hipError_t launch_lipid_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s) {
    const size_t lds = lipid_sweep_lds_bytes(st);
    hipError_t e = lip_allow((const void *)k_lipid_sweep, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lipid_sweep, dim3(st.nw), dim3(64 * lipid_waves(st)), lds, s, st, s0, n);
    return hipGetLastError();
}

}  // namespace rewl_gpu
