// rewl_trimer.hip -- the continuous-move model of the library: amphiphilic
// head-tail-tail trimers in a periodic cube, sampled by single-bead
// displacements with the Wang-Landau rule on energy bins (Vogel, Li, Wuest,
// Landau, J. Phys.: Conf. Ser. (2014): Sec. 2 for the method, Sec. 3.2 for a
// bead-spring amphiphile sampled with local displacement moves).
//
// Force field: bonds head-tail1 and tail1-tail2 are harmonic, k (r - r0)^2
// with k = 100, r0 = 1; every other pair interacts by 4 (r^-12 - r^-6):
// tail-tail pairs cut at r = 2.5 without shift, pairs involving a head cut at
// r = 2^(1/6) and shifted by +1 (Weeks-Chandler-Andersen).  Coordinates are
// binary32 in [0, box); the minimum-image difference per axis is binary32;
// pair energies are binary64 from those differences, the bond length by the
// correctly rounded binary64 square root.
//
// Energies are fixed point (units of 2^-32): every pair term is rounded once
// and totals and changes are exact integer sums, so the lanes may add the
// partner terms in any order and every implementation agrees to the bit.
//
// Mapping: one walker per workgroup.  Its coordinates, ln g and H live in
// LDS.  Attempts are sequential; inside an attempt the lanes evaluate the
// pair terms of the moved bead with 64 partners each and add them up.
#include "rewl_device.h"

namespace rewl_gpu {

namespace {

constexpr double kTriMargin64 = 1e-10;   // log-domain slack of the acceptance test (binary64)
constexpr double kTriMargin32 = 1e-5;    // log-domain slack of the acceptance test (binary32)
constexpr double kBondK = 100.0;
constexpr double kBondR0 = 1.0;
constexpr double kTailCut2 = 6.25;                    // 2.5^2
constexpr double kWcaCut2 = 0x1.428a2f98d728bp+0;     // RN(2^(1/3)) = RN((2^(1/6))^2)

__device__ __forceinline__ double min_image(float a, float b, float box, float half) {
#pragma clang fp contract(off)
    float x = b - a;
    if (x > half) x = x - box;
    else if (x < -half) x = x + box;
    return (double)x;
}

// Energy of beads i (at p) and j (at r).
__device__ __forceinline__ double pair_energy(int i, int j, float p0, float p1, float p2, float r0, float r1,
                                              float r2v, float box, float half) {
#pragma clang fp contract(off)
    const double dx = min_image(p0, r0, box, half);
    const double dy = min_image(p1, r1, box, half);
    const double dz = min_image(p2, r2v, box, half);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const int ti = i % 3, tj = j % 3;
    if (i / 3 == j / 3 && (ti - tj == 1 || tj - ti == 1)) {
        const double x = __builtin_sqrt(r2) - kBondR0;
        return kBondK * (x * x);
    }
    const bool tails = ti > 0 && tj > 0;
    if (r2 >= (tails ? kTailCut2 : kWcaCut2)) return 0.0;
    const double s2 = 1.0 / r2;
    const double s6 = (s2 * s2) * s2;
    const double v = 4.0 * ((s6 * s6) - s6);
    return tails ? v : v + 1.0;
}

// Displacement of one axis: 0.1 (2u - 1), u a 23-bit uniform; periodic wrap.
__device__ __forceinline__ float displacement(uint32_t r) {
#pragma clang fp contract(off)
    return 0.1f * ((float)(r >> 9) * 0x1p-22f - 1.0f);
}
__device__ __forceinline__ float wrap(float v, float box) {
#pragma clang fp contract(off)
    if (v < 0.0f) v = v + box;
    if (v >= box) v = v - box;
    return v;
}

__device__ __forceinline__ double readlane_d_tri(double v, int l) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((unsigned long long)b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Energy change of moving bead b (coordinates in LDS x) to n: the sum over
// partners j of fx(V(b at n, j)) - fx(V(b, j)); false for a hard overlap.
// Every lane returns the same result.
__device__ __forceinline__ bool delta_e(const DevState &st, const float *x, int b, float n0, float n1, float n2,
                                        int lane, int64_t &de) {
#pragma clang fp contract(off)
    const float box = st.box, half = 0.5f * st.box;
    const float o0 = x[3 * b], o1 = x[3 * b + 1], o2 = x[3 * b + 2];
    int64_t acc = 0;
    bool bad = false;
    for (int c = 0; c < st.nb; c += 64) {
        const int j = c + lane;
        if (j < st.nb && j != b) {
            const float r0 = x[3 * j], r1 = x[3 * j + 1], r2 = x[3 * j + 2];
            int64_t tn = 0, to = 0;
            bad |= !fx_term(pair_energy(b, j, n0, n1, n2, r0, r1, r2, box, half), tn);
            bad |= !fx_term(pair_energy(b, j, o0, o1, o2, r0, r1, r2, box, half), to);
            acc += tn - to;
        }
    }
    de = wave_sum64(acc);
    return __ballot(bad) == 0ull;
}

// Bin of a fixed-point energy (also outside [0, B), bounded to +-2^30).
__device__ __forceinline__ int energy_bin(const DevState &st, int64_t e) { return fx_bin(st.emin_fx, st.binw_fx, st.binw_inv, e); }

// ---------------------------------------------------------------------------
// Energy of every walker's starting configuration: the exact sum of the
// pair terms over i < j, rows i dealt to the lanes.  Each term is split into
// its high and low 32 bits, summed separately (neither sum can overflow), and
// the total is checked against the energy range; a start with a hard
// overlap or out of range gets the bin INT32_MIN, which the host refuses.
__global__ __launch_bounds__(64) void k_trimer_init(DevState st) {
#pragma clang fp contract(off)
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const float *x = (const float *)(st.spins + (size_t)w * st.Npad);
    const float box = st.box, half = 0.5f * st.box;
    int64_t shi = 0, slo = 0;
    bool bad = false;
    for (int i = lane; i < st.nb; i += 64) {
        const float p0 = x[3 * i], p1 = x[3 * i + 1], p2 = x[3 * i + 2];
        for (int j = i + 1; j < st.nb; ++j) {
            int64_t t = 0;
            bad |= !fx_term(pair_energy(i, j, p0, p1, p2, x[3 * j], x[3 * j + 1], x[3 * j + 2], box, half), t);
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
        st.E[w] = ok ? energy_bin(st, e) : INT32_MIN;
    }
}

// Random words of 64 attempts, one attempt per lane: bead, displacement,
// uniform word (Philox blocks (t, walker, dom) and (t, walker, dom_u)).
struct Draw {
    int bead;
    float d0, d1, d2;
    uint32_t u;
};

__device__ __forceinline__ Draw draw(const DevState &st, uint32_t dom, uint32_t dom_u, uint64_t t, uint32_t w) {
    const U4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), w, st.ctr3 | (dom << 24), st.key0, st.key1);
    const U4 ru = philox10((uint32_t)t, (uint32_t)(t >> 32), w, st.ctr3 | (dom_u << 24), st.key0, st.key1);
    Draw d;
    d.bead = (int)mul_shift(r.x, (uint32_t)st.nb);
    d.d0 = displacement(r.y);
    d.d1 = displacement(r.z);
    d.d2 = displacement(r.w);
    d.u = ru.x;
    return d;
}

// ---------------------------------------------------------------------------
// Walk-in (the Potts walk-in rule on energy bins): Wang-Landau with ln f = 1
// as uint32 visit counts over the B bins (an energy outside the range counts
// at the nearest end bin), under the lid, until the bin lies in the window.
__global__ __launch_bounds__(64) void k_trimer_walkin(DevState st, int64_t chunk, int64_t budget) {
#pragma clang fp contract(off)
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    if (st.walkin_done[w]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    float *x = (float *)smem;
    uint32_t *cnt = (uint32_t *)(smem + st.Npad);
    const uint32_t *gx = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ((uint32_t *)x)[i] = gx[i];
    const uint32_t *gcnt = st.walkin_cnt + (size_t)w * st.Bpad;
    for (int b = lane; b < st.B; b += 64) cnt[b] = gcnt[b];
    __syncthreads();

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
        const Draw dr = draw(st, kDomWalkin, kDomWalkinU, (uint64_t)(t + lane), (uint32_t)w);
        const int todo = (int)((end - t) < 64 ? (end - t) : 64);
        for (int j = 0; j < todo; ++j) {
            const int b = __builtin_amdgcn_readlane(dr.bead, j);
            const float d0 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d0), j));
            const float d1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d1), j));
            const float d2 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d2), j));
            const uint32_t u = __builtin_amdgcn_readlane(dr.u, j);
            const float n0 = wrap(x[3 * b] + d0, st.box);
            const float n1 = wrap(x[3 * b + 1] + d1, st.box);
            const float n2 = wrap(x[3 * b + 2] + d2, st.box);
            int64_t de = 0, e_new = 0;
            const bool ok = delta_e(st, x, b, n0, n1, n2, lane, de) && fx_add(Ef, de, e_new);
            const int bn = ok ? energy_bin(st, e_new) : 0;
            const int co = E < 0 ? 0 : (E >= B ? B - 1 : E);
            const int cn = bn < 0 ? 0 : (bn >= B ? B - 1 : bn);
            const double d = (double)((int64_t)cnt[co] - (int64_t)cnt[cn]);
            const bool inside = slack == 0 || (down ? bn <= bound : bn >= bound);
            if (ok && inside && accept64(d, u)) {
                if (lane == 0) {
                    x[3 * b] = n0;
                    x[3 * b + 1] = n1;
                    x[3 * b + 2] = n2;
                }
                Ef = e_new;
                E = bn;
                if (slack && down && E + slack < bound) bound = E + slack;
                if (slack && !down && E - slack > bound) bound = E - slack;
            }
            if (lane == 0) cnt[E < 0 ? 0 : (E >= B ? B - 1 : E)] += 1u;
            __syncthreads();
            ++t;
            if (E >= lo && E <= hi) { done = true; break; }
        }
    }
    __syncthreads();
    uint32_t *ox = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ox[i] = ((uint32_t *)x)[i];
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

// ---------------------------------------------------------------------------
// Main-phase attempts s0 .. s0+n-1 of every walker (Sec. 2): propose a bead
// displacement, reject it if the new energy bin leaves the window, else
// accept with min[1, g(bin_old)/g(bin_new)]; then ln g += ln f and H += 1 at
// the bin after the decision.
//
// One workgroup per walker with one wavefront per 64 partner beads: wave c
// evaluates the fixed-point pair terms of partners j = 64c + lane and leaves
// them in LDS; wave 0 adds them up (exact integers, any order) and takes the
// decision.  Every wave draws the same random words.

// Layout of a trimer attempt workgroup: partner chunks of 64 beads; with
// two roles the waves of role 0 evaluate the partners' energies with the bead
// at its new position and those of role 1 at its old one, otherwise one wave
// does both; P waves per role take chunks p, p+P, ... (at most 16 waves).
struct TrimerWaves {
    int chunks, roles, per_role;
};
__host__ __device__ inline TrimerWaves trimer_waves_of(int nb) {
    TrimerWaves t;
    t.chunks = (nb + 63) / 64;
    t.roles = 2 * t.chunks <= 16 ? 2 : 1;
    t.per_role = t.chunks < 16 / t.roles ? t.chunks : 16 / t.roles;
    return t;
}

template <int PREC>
__global__ __launch_bounds__(1024) void k_trimer_sweep(DevState st, int64_t s0, int64_t n) {
#pragma clang fp contract(off)
    if (*st.converged) return;
    const int w = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const TrimerWaves tw = trimer_waves_of(st.nb);
    const int role = wave / tw.per_role, part = wave - role * tw.per_role;
    const int k = w / st.m;
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = st.W, Wpad = st.Wpad;
    float *x = (float *)smem;
    double *g = (double *)(smem + st.Npad);
    float *gh = (float *)(smem + st.Npad);
    float *gl = gh + Wpad;
    uint32_t *H = (uint32_t *)(smem + st.Npad + (size_t)Wpad * 8);
    int64_t *tbuf = (int64_t *)(smem + st.Npad + (size_t)Wpad * 12);   // [roles][chunks][64]
    const uint32_t *gx = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = threadIdx.x; i < st.Npad / 4; i += blockDim.x) ((uint32_t *)x)[i] = gx[i];
    const size_t row = (size_t)w * Wpad;
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        if (PREC == 0) {
            g[b] = st.lng[row + b];
        } else {
            gh[b] = st.lng_hi[row + b];
            gl[b] = st.lng_lo[row + b];
        }
        H[b] = st.H[row + b];
    }
    __syncthreads();
    const int lo = st.start[k], hi = lo + W - 1;
    int E = st.E[w];
    int64_t Ef = st.Efx[w];
    if (E < lo || E > hi) return;   // not walked in: leave the walker untouched
    const double lnf = st.lnf[k];
    const float lnf32 = (float)lnf;
    const float box = st.box, half = 0.5f * st.box;
    for (int64_t base = 0; base < n; base += 64) {
        const int todo = (int)((n - base) < 64 ? (n - base) : 64);
        const Draw dr = draw(st, kDomMove, kDomMoveU, (uint64_t)(s0 + base + lane), (uint32_t)w);
        // ln u of this lane's attempt: the serial step compares it with d and
        // evaluates exp only inside a margin that covers the error of log/exp
        double lnu = 0.0;
        if (wave == 0) {
            if (PREC == 0) lnu = dr.u == 0u ? -64.0 : log((double)dr.u * 0x1p-32);
            else lnu = (dr.u >> 8) == 0u ? -64.0 : log((double)(dr.u >> 8) * 0x1p-24);
        }
        for (int a = 0; a < todo; ++a) {
            const int b = __builtin_amdgcn_readlane(dr.bead, a);
            const float d0 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d0), a));
            const float d1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d1), a));
            const float d2 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(dr.d2), a));
            const float o0 = x[3 * b], o1 = x[3 * b + 1], o2 = x[3 * b + 2];
            const float n0 = wrap(o0 + d0, box);
            const float n1 = wrap(o1 + d1, box);
            const float n2 = wrap(o2 + d2, box);
            for (int c = part; c < tw.chunks; c += tw.per_role) {
                const int j = c * 64 + lane;
                int64_t v = 0;
                if (j < st.nb && j != b) {
                    const float r0 = x[3 * j], r1 = x[3 * j + 1], r2 = x[3 * j + 2];
                    int64_t tn = 0, to = 0;
                    bool ok = true;
                    if (tw.roles == 2) {
                        ok = role == 0 ? fx_term(pair_energy(b, j, n0, n1, n2, r0, r1, r2, box, half), tn)
                                       : fx_term(pair_energy(b, j, o0, o1, o2, r0, r1, r2, box, half), to);
                        v = role == 0 ? tn : to;
                    } else {
                        ok = fx_term(pair_energy(b, j, n0, n1, n2, r0, r1, r2, box, half), tn) &
                             fx_term(pair_energy(b, j, o0, o1, o2, r0, r1, r2, box, half), to);
                        v = tn - to;
                    }
                    if (!ok) v = kFxBad;
                }
                tbuf[(role * tw.chunks + c) * 64 + lane] = v;
            }
            __syncthreads();
            if (wave == 0) {
                // fx(V(new)) - fx(V(old)) per partner, added up exactly
                int64_t sl = 0;
                bool bad = false;
                for (int c = 0; c < tw.chunks; ++c) {
                    const int64_t a0 = tbuf[c * 64 + lane];
                    const int64_t a1 = tw.roles == 2 ? tbuf[(tw.chunks + c) * 64 + lane] : 0;
                    if (a0 == kFxBad || a1 == kFxBad) bad = true;
                    else sl += a0 - a1;
                }
                const int64_t de = wave_sum64(sl);
                int64_t e_new = 0;
                const bool ok = __ballot(bad) == 0ull && fx_add(Ef, de, e_new);
                const int bn = ok ? energy_bin(st, e_new) : 0;
                bool acc = false;
                if (ok && bn >= lo && bn <= hi) {
                    const int io = E - lo, in = bn - lo;
                    const double luj = readlane_d_tri(lnu, a);
                    const uint32_t u = __builtin_amdgcn_readlane(dr.u, a);
                    if (PREC == 0) {
                        const double d = g[io] - g[in];
                        const double t = d - luj;
                        if (fabs(t) > kTriMargin64) acc = t > 0.0;
                        else acc = accept64(d, u);
                    } else {
                        const float d = (gh[io] - gh[in]) + (gl[io] - gl[in]);
                        const double t = (double)d - luj;
                        if (fabs(t) > kTriMargin32) acc = t > 0.0;
                        else acc = accept32(d, u);
                    }
                    acc = __ballot(acc) != 0ull;
                }
                if (acc) {
                    if (lane == 0) {
                        x[3 * b] = n0;
                        x[3 * b + 1] = n1;
                        x[3 * b + 2] = n2;
                    }
                    Ef = e_new;
                    E = bn;
                }
                if (lane == 0) {
                    const int ib = E - lo;
                    if (PREC == 0) {
                        g[ib] = g[ib] + lnf;
                    } else {
                        float hh = gh[ib], ll = gl[ib];
                        two_sum_add(hh, ll, lnf32);
                        gh[ib] = hh;
                        gl[ib] = ll;
                    }
                    H[ib] += 1u;
                }
            }
            __syncthreads();
        }
    }
    uint32_t *ox = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = threadIdx.x; i < st.Npad / 4; i += blockDim.x) ox[i] = ((uint32_t *)x)[i];
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        if (PREC == 0) {
            st.lng[row + b] = g[b];
        } else {
            st.lng_hi[row + b] = gh[b];
            st.lng_lo[row + b] = gl[b];
        }
        st.H[row + b] = H[b];
    }
    if (threadIdx.x == 0) {
        st.E[w] = E;
        st.Efx[w] = Ef;
    }
}

hipError_t allow(const void *fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

static int trimer_threads(const DevState &st) {
    const TrimerWaves t = trimer_waves_of(st.nb);
    return 64 * t.roles * t.per_role;
}
size_t trimer_sweep_lds_bytes(const DevState &st) {
    const TrimerWaves t = trimer_waves_of(st.nb);
    return (size_t)st.Npad + (size_t)st.Wpad * 12 + (size_t)t.roles * t.chunks * 64 * 8;
}
size_t trimer_walkin_lds_bytes(const DevState &st) { return (size_t)st.Npad + (size_t)st.Bpad * 4; }

hipError_t launch_trimer_init(const DevState &st, hipStream_t s) {
    hipLaunchKernelGGL(k_trimer_init, dim3(st.nw), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_trimer_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s) {
    const size_t lds = trimer_walkin_lds_bytes(st);
    hipError_t e = allow((const void *)k_trimer_walkin, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trimer_walkin, dim3(st.nw), dim3(64), lds, s, st, chunk, budget);
    return hipGetLastError();
}

hipError_t launch_trimer_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s) {
    const size_t lds = trimer_sweep_lds_bytes(st);
    if (st.precision == 0) {
        hipError_t e = allow((const void *)k_trimer_sweep<0>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_trimer_sweep<0>, dim3(st.nw), dim3(trimer_threads(st)), lds, s, st, s0, n);
    } else {
        hipError_t e = allow((const void *)k_trimer_sweep<1>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_trimer_sweep<1>, dim3(st.nw), dim3(trimer_threads(st)), lds, s, st, s0, n);
    }
    return hipGetLastError();
}

}  // namespace rewl_gpu
