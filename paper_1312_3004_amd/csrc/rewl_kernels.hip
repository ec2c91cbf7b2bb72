// rewl_kernels.hip -- HIP kernels (gfx950) of the Replica-Exchange Wang-Landau
// walker update and its sync points.
//
// Vogel, Li, Wuest, Landau, J. Phys.: Conf. Ser. (2014):
//   Sec. 2      Wang-Landau acceptance, refinement g -> f g, H(E)++, flatness,
//               averaging within a window, replica exchange (Eq. 1), joining.
//   Sec. 3.1    2D q-state Potts model (Eq. 2), single-spin-flip moves.
//
// Mapping: one walker per 64-lane wavefront (one workgroup).  Its lattice
// (int8), ln g and H live in LDS for the whole launch; global memory is
// touched only at launch start and end.  Attempts of one walker form a strict
// sequence (each decision depends on the previous energy and ln g), so the
// lanes first draw the Philox words and site neighbourhoods of the next 64
// attempts in parallel and then walk through them in order.
#include <type_traits>

#include "rewl_device.h"

namespace rewl_gpu {

namespace {

// v_writelane_b32: lane `lane` of `old` takes the uniform value `v`.
extern "C" __device__ int writelane_i32(int v, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Phase clocks of the attempt loop.  The profiling build (REWL_PHASE_CLOCKS
// defined, librewl_clocks.so) adds per-walker cycle and event counts to
// g_phase_ctr, row w = walker w of a single run, slots kPc*; the product
// build compiles every call below to nothing.
enum {
    kPcLaneCycles = 0,    // lane-parallel phase of a block (proposals, dE, conflicts)
    kPcDecideCycles = 1,  // decision phase of a block (speculative or serial)
    kPcSegments = 2,      // speculative segments
    kPcRounds = 3,        // speculative rounds
    kPcExact = 4,         // attempts through the exact (settling) path
    kPcBlocks = 5,        // blocks of up to 64 attempts
    kPcRoundCycles = 6,   // cycles inside the speculative rounds
    kPcAttempts = 7,
    kPcSetupCycles = 8,   // segment set-up before the first round (margins, cache)
    kPcCommitCycles = 9,  // committing a segment (flips, visit counts, ln g replay)
    kPcExactCycles = 10,  // the exact path after a speculative stop, with the restart
    kPcTailCycles = 11,   // end of a block (pending flips, H increments)
    kPcSlots = 12,
};
#ifdef REWL_PHASE_CLOCKS
constexpr int kPcRows = 4096;
__device__ unsigned long long g_phase_ctr[kPcRows * kPcSlots];
struct PhaseClock {
    unsigned long long v[kPcSlots] = {};
    __device__ __forceinline__ long long now() const { return clock64(); }
    __device__ __forceinline__ void add(int i, long long k) { v[i] += (unsigned long long)k; }
    __device__ __forceinline__ void flush(int w, int lane) {
        if (lane == 0 && w < kPcRows)
            for (int i = 0; i < kPcSlots; ++i) atomicAdd(&g_phase_ctr[(size_t)w * kPcSlots + i], v[i]);
    }
};
#else
struct PhaseClock {
    __device__ __forceinline__ long long now() const { return 0; }
    __device__ __forceinline__ void add(int, long long) {}
    __device__ __forceinline__ void flush(int, int) {}
};
#endif

__device__ __forceinline__ int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double rfl(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float rfl(float x) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

// Proposal of one attempt, computed by one lane: site i uniform in [0, N),
// new value uniform among the q-1 others (offset), u word, and the four
// periodic neighbours of i (Sec. 3.1 single spin flips on the L x L torus).
struct Proposal {
    int site, off, nb0, nb1, nb2, nb3;
    uint32_t u;
};

__device__ __forceinline__ Proposal propose(const DevState &st, uint32_t domain, uint64_t t,
                                            uint32_t walker) {
    const U4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), walker, st.ctr3 | (domain << 24),
                          st.key0, st.key1);
    Proposal p;
    p.site = (int)mul_shift(r.x, (uint32_t)st.N);
    p.off = (int)mul_shift(r.y, (uint32_t)(st.q - 1));
    p.u = r.z;
    const int L = st.L;
    const int y = p.site / L;
    const int x = p.site - y * L;
    const int row = y * L;
    p.nb0 = row + (x + 1 == L ? 0 : x + 1);
    p.nb1 = row + (x == 0 ? L - 1 : x - 1);
    p.nb2 = (y + 1 == L ? 0 : row + L) + x;
    p.nb3 = (y == 0 ? (L - 1) * L : row - L) + x;
    return p;
}

// Energy change of setting site to nv, from the lattice in LDS (Eq. 2).
__device__ __forceinline__ int delta_e(const int8_t *sp, int sc, int nv, int n0, int n1, int n2,
                                       int n3) {
    const int a0 = sp[n0], a1 = sp[n1], a2 = sp[n2], a3 = sp[n3];
    return (int)(sc == a0) + (int)(sc == a1) + (int)(sc == a2) + (int)(sc == a3) -
           (int)(nv == a0) - (int)(nv == a1) - (int)(nv == a2) - (int)(nv == a3);
}

// ---------------------------------------------------------------------------
// Energy of every walker's starting lattice (Eq. 2, each bond once).
__global__ __launch_bounds__(256) void k_init_energy(DevState st) {
    const int w = blockIdx.x;
    const int8_t *s = st.spins + (size_t)w * st.Npad;
    const int L = st.L;
    int e = 0;
    for (int i = threadIdx.x; i < st.N; i += blockDim.x) {
        const int y = i / L, x = i - y * L;
        const int right = y * L + (x + 1 == L ? 0 : x + 1);
        const int down = (y + 1 == L ? 0 : (y + 1) * L) + x;
        e -= (s[i] == s[right]) + (s[i] == s[down]);
    }
    __shared__ int part[256];
    part[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) st.E[w] = part[0];
}

// ---------------------------------------------------------------------------
// Walk-in: a Wang-Landau walk over all 2N+1 energies with ln f = 1, run until
// the walker's energy first lies in its own window (every walker must start
// inside its window, Sec. 3.2).  With ln f = 1 every ln g entry is an integer
// visit count, kept exactly as uint32 in LDS.  A walker above its window
// walks under a lid (moves more than walkin_slack above the lowest energy
// reached are rejected), a walker below it above a floor; the flooded band
// then stays walkin_slack wide instead of spanning the whole way down.  Runs at most `chunk`
// attempts per launch; the host relaunches until every walker is placed.
__device__ __forceinline__ void walkin_walker(const DevState &st, int w, int64_t chunk, int64_t budget,
                                              unsigned char *smem) {
    const int lane = threadIdx.x;
    if (st.walkin_done[w]) return;
    int8_t *sp = (int8_t *)smem;
    uint32_t *cnt = (uint32_t *)(smem + st.Npad);
    const uint32_t *gsp = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ((uint32_t *)sp)[i] = gsp[i];
    const uint32_t *gcnt = st.walkin_cnt + (size_t)w * st.Bpad;
    for (int b = lane; b < st.B; b += 64) cnt[b] = gcnt[b];
    __syncthreads();

    const int k = w / st.m;
    const int lo = st.start[k], hi = lo + st.W - 1;
    const int e_lo = st.e_lo, q = st.q;
    int E = st.E[w];
    int64_t t = st.walkin_att[w];
    const int slack = st.walkin_slack;
    const bool down = E > hi;
    int bound = t == 0 ? (down ? E + slack : E - slack) : st.walkin_bound[w];
    const int64_t end = (t + chunk < budget) ? t + chunk : budget;
    bool done = (E >= lo && E <= hi);
    while (!done && t < end) {
        const Proposal p = propose(st, kDomWalkin, (uint64_t)(t + lane), (uint32_t)w);
        const int todo = (int)((end - t) < 64 ? (end - t) : 64);
        for (int j = 0; j < todo; ++j) {
            const int site = __builtin_amdgcn_readlane(p.site, j);
            const int off = __builtin_amdgcn_readlane(p.off, j);
            const uint32_t u = __builtin_amdgcn_readlane(p.u, j);
            const int n0 = __builtin_amdgcn_readlane(p.nb0, j);
            const int n1 = __builtin_amdgcn_readlane(p.nb1, j);
            const int n2 = __builtin_amdgcn_readlane(p.nb2, j);
            const int n3 = __builtin_amdgcn_readlane(p.nb3, j);
            const int sc = rfl((int)sp[site]);
            int nv = sc + 1 + off;
            if (nv >= q) nv -= q;
            const int En = E + rfl(delta_e(sp, sc, nv, n0, n1, n2, n3));
            const int64_t ci = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(cnt[E - e_lo]);
            const int64_t cn = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(cnt[En - e_lo]);
            const double d = (double)(ci - cn);
            const bool inside = slack == 0 || (down ? En <= bound : En >= bound);
            if (inside && accept64(d, u)) {
                if (lane == 0) sp[site] = (int8_t)nv;
                E = En;
                if (slack && down && E + slack < bound) bound = E + slack;
                if (slack && !down && E - slack > bound) bound = E - slack;
            }
            if (lane == 0) cnt[E - e_lo] += 1u;
            ++t;
            if (E >= lo && E <= hi) { done = true; break; }
        }
    }
    __syncthreads();
    uint32_t *osp = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) osp[i] = ((uint32_t *)sp)[i];
    uint32_t *ocnt = st.walkin_cnt + (size_t)w * st.Bpad;
    for (int b = lane; b < st.B; b += 64) ocnt[b] = cnt[b];
    if (lane == 0) {
        st.E[w] = E;
        st.walkin_att[w] = t;
        st.walkin_done[w] = done ? 1 : 0;
        st.walkin_bound[w] = bound;
    }
}

__global__ __launch_bounds__(64) void k_walkin(DevState st, int64_t chunk, int64_t budget) {
    extern __shared__ __align__(16) unsigned char smem[];
    walkin_walker(st, blockIdx.x, chunk, budget, smem);
}

// ---------------------------------------------------------------------------
// Main-phase Wang-Landau attempts (Sec. 2): n attempts of every walker,
// attempt indices s0 .. s0+n-1.  Per attempt: propose a single spin flip,
// reject it if the new energy leaves the window, else accept with
// min[1, g(E_old)/g(E_new)]; then ln g(E) += ln f and H(E) += 1 at the
// energy after the decision.
//
// The attempts of one walker are a strict sequence.  The kernel processes
// them in blocks of 64 with a lane-parallel phase and a serial phase that
// reproduces the sequential result exactly:
//  * lanes draw the 64 proposals and compute their energy changes from the
//    lattice at block start.  A proposal whose site or neighbours were hit by
//    an earlier proposal of the same block carries a conflict mask (built by
//    OR-ing lane bits into an LDS tag table); if any of those earlier
//    proposals was accepted, its energy change is recomputed from LDS;
//  * lanes compute ln u of their uniform word; u < exp(d) is then settled by
//    comparing d with ln u up to a margin that covers the error of exp_neg
//    and log; attempts inside the margin evaluate exp_neg exactly, as the
//    sequential rule does;
//  * ln g of 64 consecutive energies around the walker sit in VGPRs (lane b
//    holds energy ebase + b; energies outside the window hold +inf, which
//    makes any move there a certain reject).
// The serial phase carries the walker's current ln g through every attempt
// and compares it with the cached ln g of the proposed energy.
// H(E) increments and accepted spins are applied to LDS once per block (no
// two pending spin writes share a site: a repeat hit is a conflict and is
// written at once).
constexpr double kMargin64 = 1e-10;   // log-domain slack of the exact-mode test (binary64)
constexpr double kMargin32 = 1e-5;    // log-domain slack of the exact-mode test (binary32)
// Blocks of a window whose ln f is at most this run the speculative phase:
// the ln g drift inside a block (64 ln f at most) is then small against the
// spread of d - ln u, so few attempts fall inside the decision margin.
constexpr double kSpecLnf = 0x1p-8;


__device__ __forceinline__ uint64_t readlane64(uint64_t v, int j) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, j);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double readlane_d(double v, int j) {
    return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), j));
}
__device__ __forceinline__ float readlane_f(float v, int j) {
    return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), j));
}
// Set bits of m in the lanes below this one.
__device__ __forceinline__ int mbcnt64(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// v of lane src (a different lane per lane) by ds_bpermute; every lane active.
__device__ __forceinline__ double lane_read_d(double v, int src) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float lane_read_f(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
// Orders this wavefront's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// Orders this wavefront's LDS traffic at a phase boundary of a walker.  With
// one walker per workgroup a workgroup barrier; with several independent
// walkers (one per wavefront) in a workgroup a fence of the wave's own memory
// operations (a wave's LDS operations execute in order).
template <bool WAVE>
__device__ __forceinline__ void walker_sync() {
    if (WAVE) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    else __syncthreads();
}

// GLOB: the walker's ln g and H rows stay in device memory (read and written
// only when the register cache moves, H by atomic increments), so a walker
// needs LDS for its lattice and tag table alone and more walkers fit a CU.
template <int PREC, bool WAVE = false, bool GLOB = false>
__device__ __forceinline__ void sweep_walker(const DevState &st, int w, int64_t s0, int64_t n,
                                             unsigned char *smem) {
#pragma clang fp contract(off)
    if (*st.converged) return;
    const int lane = threadIdx.x & 63;
    const int k = w / st.m;
    const int W = st.W, Wpad = st.Wpad;
    const size_t row = (size_t)w * Wpad;
    int8_t *sp = (int8_t *)smem;
    double *g;
    float *gh, *gl;
    uint32_t *H;
    unsigned long long *tag;
    if (GLOB) {
        g = PREC == 0 ? st.lng + row : nullptr;
        gh = PREC == 1 ? st.lng_hi + row : nullptr;
        gl = PREC == 1 ? st.lng_lo + row : nullptr;
        H = st.H + row;
        tag = (unsigned long long *)(smem + st.Npad);
    } else {
        g = (double *)(smem + st.Npad);
        gh = (float *)(smem + st.Npad);
        gl = gh + Wpad;
        H = (uint32_t *)(smem + st.Npad + (size_t)Wpad * 8);
        tag = (unsigned long long *)(smem + st.Npad + (size_t)Wpad * 12);
    }
    const uint32_t tag_mask = (uint32_t)st.Ntag - 1u;
    // visit counts of the register cache's 64 energies during the serial
    // phase, in the first 256 bytes of the tag table (all zero outside the
    // lane-parallel phase, at least 64 entries of 8 bytes)
    uint32_t *cnt = (uint32_t *)tag;

    const uint32_t *gsp = (const uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) ((uint32_t *)sp)[i] = gsp[i];
    if (!GLOB) {
        for (int b = lane; b < W; b += 64) {
            if (PREC == 0) {
                g[b] = st.lng[row + b];
            } else {
                gh[b] = st.lng_hi[row + b];
                gl[b] = st.lng_lo[row + b];
            }
            H[b] = st.H[row + b];
        }
    }
    for (int i = lane; i < st.Ntag; i += 64) tag[i] = 0ull;
    walker_sync<WAVE>();

    const int lo = st.start[k], hi = lo + W - 1;
    const int q = st.q;
    const double lnf = st.lnf[k];
    const float lnf32 = (float)lnf;
    const bool spec = lnf <= kSpecLnf;
    int E = st.E[w];
    if (E < lo || E > hi) return;  // not walked in: leave the walker untouched

    // ln g cache: lane b holds energy ebase + b (+inf outside the window)
    int ebase = E - 32;
    double c64 = 0.0;
    float ch = 0.0f, cl = 0.0f;
    auto cache_load = [&]() {
        const int b = ebase + lane - lo;
        const bool in = b >= 0 && b < W;
        if (PREC == 0) c64 = in ? g[b] : __builtin_inf();
        else { ch = in ? gh[b] : __builtin_inff(); cl = in ? gl[b] : 0.0f; }
    };
    auto cache_store = [&]() {
        const int b = ebase + lane - lo;
        if (b >= 0 && b < W) {
            if (PREC == 0) g[b] = c64;
            else { gh[b] = ch; gl[b] = cl; }
        }
        // device-memory rows: the stores land before the lanes read the moved
        // cache range back (the ranges overlap)
        if (GLOB) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    };
    cache_load();
    int erel = 32;  // E - ebase
    // ln f as a VGPR operand: the per-attempt add then reads one SGPR pair (ln g)
    double lnf_v = lnf;
    asm volatile("" : "+v"(lnf_v));
    double gEv = 0.0, gEs = 0.0;
    float gEh = 0.0f, gEl = 0.0f;
    // proposal and ln u of lane j's attempt of the next block (they do not
    // depend on the lattice, so they are drawn while the block before runs)
    auto lnu_of = [&](uint32_t u) -> double {
        if (PREC == 0) return u == 0u ? -64.0 : log((double)u * 0x1p-32);
        return (u >> 8) == 0u ? -64.0 : log((double)(u >> 8) * 0x1p-24);
    };
    Proposal p_nx = propose(st, kDomMove, (uint64_t)(s0 + lane), (uint32_t)w);
    double lnu_nx = lnu_of(p_nx.u);
    // decision margin of lane j in a speculative segment from `start`: the
    // exact-mode slack plus, for each of the segment's earlier visits and the
    // two subtractions, ln f and the rounding of values up to |a| + |b| (the
    // two ln g read); M = M0 + (|a| + |b| + 1) Mr.  Almost every segment
    // starts its block, so those margins are computed once.
    auto margins = [&](int start, double &M0, double &Mr) {
        const double slack = (double)(lane - start + 2);
        M0 = PREC == 0 ? kMargin64 + slack * lnf * (1.0 + 0x1p-50)
                       : kMargin32 + slack * ((double)lnf32 * (1.0 + 0x1p-20) + 64.0 * lnf * 0x1p-46);
        Mr = slack * (PREC == 0 ? 0x1p-50 : 0x1p-46);
    };
    double M0b = 0.0, Mrb = 0.0;
    if (spec) margins(0, M0b, Mrb);
    PhaseClock pc;

    for (int64_t base = 0; base < n; base += 64) {
        const long long pc0 = pc.now();
        const int todo = (int)((n - base) < 64 ? (n - base) : 64);
        const bool live = lane < todo;
        if ((unsigned)(erel - 16) >= 32u) {   // keep the walker near the cache centre
            cache_store();
            ebase += erel - 32;
            erel = 32;
            cache_load();
        }
        // the current ln g rides in registers through the block
        if (PREC == 0) { gEs = readlane_d(c64, erel); gEv = gEs; }
        else { gEh = readlane_f(ch, erel); gEl = readlane_f(cl, erel); }
        // ---- lane-parallel phase: proposal, energy change, conflicts, ln u
        const Proposal p = p_nx;
        const double lnu = lnu_nx;
        // spins of the site and its neighbours at block start
        int x0 = sp[p.site], x1 = sp[p.nb0], x2 = sp[p.nb1], x3 = sp[p.nb2], x4 = sp[p.nb3];
        int nv = x0 + 1 + p.off;
        if (nv >= q) nv -= q;
        int dE = (int)(x0 == x1) + (int)(x0 == x2) + (int)(x0 == x3) + (int)(x0 == x4) - (int)(nv == x1) -
                 (int)(nv == x2) - (int)(nv == x3) - (int)(nv == x4);
        const uint32_t ti = (uint32_t)p.site & tag_mask;
        if (live) atomicOr(&tag[ti], 1ull << lane);
        const unsigned long long below = (1ull << lane) - 1ull;
        // earlier proposals of the block whose site is (or hashes like) this
        // proposal's site, resp. one of its neighbours
        unsigned long long W0 = tag[ti] & below, W1 = tag[(uint32_t)p.nb0 & tag_mask] & below,
                           W2 = tag[(uint32_t)p.nb1 & tag_mask] & below, W3 = tag[(uint32_t)p.nb2 & tag_mask] & below,
                           W4 = tag[(uint32_t)p.nb3 & tag_mask] & below;
        unsigned long long conf = W0 | W1 | W2 | W3 | W4;
        if (live) tag[ti] = 0ull;
        unsigned long long anyconf = __ballot(conf != 0ull);

        unsigned long long accepted = 0ull, flushed = 0ull;
        int hist = 0;

        // An earlier accepted flip of this block touched attempt j's site or a
        // neighbour: write the pending flips, then recompute the proposal's new
        // value and energy change from the live lattice (five reads at once).
        auto settle = [&](int j, int &nvj) -> int {
            if (((accepted & ~flushed) >> lane) & 1ull) sp[p.site] = (int8_t)nv;
            flushed = accepted;
            const int s0 = sp[__builtin_amdgcn_readlane(p.site, j)];
            const int a0 = sp[__builtin_amdgcn_readlane(p.nb0, j)];
            const int a1 = sp[__builtin_amdgcn_readlane(p.nb1, j)];
            const int a2 = sp[__builtin_amdgcn_readlane(p.nb2, j)];
            const int a3 = sp[__builtin_amdgcn_readlane(p.nb3, j)];
            const int scj = rfl(s0);
            int v = scj + 1 + __builtin_amdgcn_readlane(p.off, j);
            if (v >= q) v -= q;
            nvj = v;
            return rfl((int)(scj == a0) + (int)(scj == a1) + (int)(scj == a2) + (int)(scj == a3) -
                       (int)(v == a0) - (int)(v == a1) - (int)(v == a2) - (int)(v == a3));
        };

        // Decision of attempt j through the general path: settles its conflict
        // first (recomputing dE from the live lattice), then applies the rule
        // with the carried current ln g and the cached ln g of the new energy.
        auto slow_attempt = [&](int j) -> void {
            pc.add(kPcExact, 1);
            int dEj = __builtin_amdgcn_readlane(dE, j);
            bool now = false;
            int nvj = 0;
            if (((anyconf >> j) & 1ull) && (readlane64(conf, j) & accepted)) {
                dEj = settle(j, nvj);
                now = true;
            }
            const int Ecur = ebase + erel, En = Ecur + dEj;
            bool acc = false;
            if (En >= lo && En <= hi) {
                const uint32_t u = __builtin_amdgcn_readlane(p.u, j);
                int idx = erel + dEj;
                if ((unsigned)idx >= 64u) {
                    cache_store();
                    ebase += idx - 32;
                    cache_load();
                    erel = erel - idx + 32;
                    idx = 32;
                }
                const double luj = readlane_d(lnu, j);
                if (PREC == 0) {
                    const double gN = readlane_d(c64, idx);
                    const double d = gEv - gN;
                    const double t = d - luj;
                    if (__ballot(fabs(t) > kMargin64) != 0ull) acc = __ballot(t > 0.0) != 0ull;
                    else acc = __ballot(accept64(d, u)) != 0ull;
                    gEs = acc ? gN : gEs;
                } else {
                    const float gNh = readlane_f(ch, idx);
                    const float gNl = readlane_f(cl, idx);
                    const float d = (gEh - gNh) + (gEl - gNl);
                    const double t = (double)d - luj;
                    if (__ballot(fabs(t) > kMargin32) != 0ull) acc = __ballot(t > 0.0) != 0ull;
                    else acc = __ballot(accept32(d, u)) != 0ull;
                    gEh = acc ? gNh : gEh;
                    gEl = acc ? gNl : gEl;
                }
            }
            erel = acc ? En - ebase : erel;
            accepted |= acc ? (1ull << j) : 0ull;
            if (acc && now) {
                if (lane == 0) sp[__builtin_amdgcn_readlane(p.site, j)] = (int8_t)nvj;
                flushed |= 1ull << j;
            }
            if (PREC == 0) {
                gEv = gEs + lnf_v;
                gEs = rfl(gEv);
                c64 = (lane == erel) ? gEv : c64;
            } else {
                two_sum_add(gEh, gEl, lnf32);
                gEh = rfl(gEh);
                gEl = rfl(gEl);
                ch = (lane == erel) ? gEh : ch;
                cl = (lane == erel) ? gEl : cl;
            }
            hist = writelane_i32(ebase + erel, j, hist);
        };

        const long long pc1 = pc.now();
        pc.add(kPcLaneCycles, pc1 - pc0);
        if (spec) {
            // ---- speculative phase (small ln f): every lane evaluates its own
            // attempt from a guess of the earlier attempts of its segment (their
            // decisions and new values); the guesses are refined until they
            // reproduce themselves.  Attempt j depends only on attempts before
            // it, so the fixed point is the sequential result, reached after at
            // most one round per attempt.  Per round, lane j takes
            //  * its energy before the attempt: E0 plus dE of the accepted
            //    earlier lanes (bit counts over ballots of the dE bits),
            //  * the spins of its site and neighbours: the new value of the last
            //    accepted earlier lane that flips that site, else the spin at
            //    segment start; from them its new value and dE,
            //  * its decision from the register cache's ln g at segment start,
            //    settled only outside a margin that bounds the ln g drift of
            //    the segment's earlier visits.
            // An attempt that cannot be settled so (inside the margin, or an
            // energy outside the cache) ends the segment and runs through
            // slow_attempt; the next segment starts after it.
            const unsigned long long livem = todo == 64 ? ~0ull : ((1ull << todo) - 1ull);
            if (st.Ntag < st.N) {
                // hashed tag table: keep only proposals on exactly the same site
                unsigned long long cand = conf;
                while (__ballot(cand != 0ull)) {
                    const int i = cand ? 63 - __builtin_clzll(cand) : lane;
                    const int si = __builtin_amdgcn_ds_bpermute(i << 2, p.site);
                    const unsigned long long bit = cand ? (1ull << i) : 0ull;
                    W0 = si == p.site ? W0 : W0 & ~bit;
                    W1 = si == p.nb0 ? W1 : W1 & ~bit;
                    W2 = si == p.nb1 ? W2 : W2 & ~bit;
                    W3 = si == p.nb2 ? W3 : W3 & ~bit;
                    W4 = si == p.nb3 ? W4 : W4 & ~bit;
                    cand &= ~bit;
                }
            }
            int start = 0;
            while (start < todo) {
                pc.add(kPcSegments, 1);
                const long long pcs = pc.now();
                if ((unsigned)(erel - 16) >= 32u) {   // keep the walker near the cache centre
                    cache_store();
                    ebase += erel - 32;
                    erel = 32;
                    cache_load();
                }
                const int E0 = ebase + erel;
                const unsigned long long act = livem & (~0ull << start);
                const bool mine = (act >> lane) & 1ull;
                double M0 = M0b, Mr = Mrb;
                if (start != 0) margins(start, M0, Mr);
                unsigned long long A = 0ull, Sg = 0ull;
                int c = todo, pre = E0, nvi = nv, dEi = dE;
                bool conv = false;
                // one round; the first of a segment also draws the next block's
                // proposals (independent work that fills the round's waits)
                auto round = [&](auto first) {
                    pc.add(kPcRounds, 1);
                    if constexpr (decltype(first)::value) {
                        p_nx = propose(st, kDomMove, (uint64_t)(s0 + base + 64 + lane), (uint32_t)w);
                        lnu_nx = lnu_of(p_nx.u);
                    }
                    constexpr bool kFirst = decltype(first)::value;
                    const unsigned long long Aa = A & act;
                    // energy before the attempt, from the previous round's lanes
                    // (the first round guesses every earlier attempt rejected)
                    if constexpr (kFirst) {
                        pre = E0;
                    } else {
                        const int de4 = dEi + 4;   // in [0, 8]
                        const unsigned long long B0 = __ballot(de4 & 1), B1 = __ballot(de4 & 2);
                        const unsigned long long B2 = __ballot(de4 & 4), B3 = __ballot(de4 & 8);
                        pre = E0 - 4 * mbcnt64(Aa) + mbcnt64(B0 & Aa) + 2 * mbcnt64(B1 & Aa) +
                              4 * mbcnt64(B2 & Aa) + 8 * mbcnt64(B3 & Aa);
                    }
                    const int ip = pre - ebase;
                    // ln g before the attempt, and after it for the segment-start dE
                    // (read now; a lane whose dE changed reads again below)
                    double a = 0.0, b = 0.0;
                    float aH = 0.0f, aL = 0.0f, bH = 0.0f, bL = 0.0f;
                    const int ib0 = ip + dE;
                    if (PREC == 0) {
                        a = lane_read_d(c64, ip & 63);
                        b = lane_read_d(c64, ib0 & 63);
                    } else {
                        aH = lane_read_f(ch, ip & 63);
                        aL = lane_read_f(cl, ip & 63);
                        bH = lane_read_f(ch, ib0 & 63);
                        bL = lane_read_f(cl, ib0 & 63);
                    }
                    // new value and dE from the spins the earlier accepted lanes left
                    int nvn = nv, dEn = dE;
                    if constexpr (!kFirst) {
                        int y0 = x0, y1 = x1, y2 = x2, y3 = x3, y4 = x4;
                        const unsigned long long a0 = W0 & Aa, a1 = W1 & Aa, a2 = W2 & Aa, a3 = W3 & Aa,
                                                 a4 = W4 & Aa;
                        const int r0 = __builtin_amdgcn_ds_bpermute((a0 ? 63 - __builtin_clzll(a0) : lane) << 2, nvi);
                        const int r1 = __builtin_amdgcn_ds_bpermute((a1 ? 63 - __builtin_clzll(a1) : lane) << 2, nvi);
                        const int r2 = __builtin_amdgcn_ds_bpermute((a2 ? 63 - __builtin_clzll(a2) : lane) << 2, nvi);
                        const int r3 = __builtin_amdgcn_ds_bpermute((a3 ? 63 - __builtin_clzll(a3) : lane) << 2, nvi);
                        const int r4 = __builtin_amdgcn_ds_bpermute((a4 ? 63 - __builtin_clzll(a4) : lane) << 2, nvi);
                        y0 = a0 ? r0 : y0;
                        y1 = a1 ? r1 : y1;
                        y2 = a2 ? r2 : y2;
                        y3 = a3 ? r3 : y3;
                        y4 = a4 ? r4 : y4;
                        nvn = y0 + 1 + p.off;
                        if (nvn >= q) nvn -= q;
                        dEn = (int)(y0 == y1) + (int)(y0 == y2) + (int)(y0 == y3) + (int)(y0 == y4) -
                              (int)(nvn == y1) - (int)(nvn == y2) - (int)(nvn == y3) - (int)(nvn == y4);
                    }
                    const int En = pre + dEn;
                    const bool in_win = En >= lo && En <= hi;
                    const int inn = En - ebase;
                    if (__ballot(mine && dEn != dE)) {
                        if (PREC == 0) {
                            const double b2 = lane_read_d(c64, inn & 63);
                            b = dEn != dE ? b2 : b;
                        } else {
                            const float b2H = lane_read_f(ch, inn & 63), b2L = lane_read_f(cl, inn & 63);
                            bH = dEn != dE ? b2H : bH;
                            bL = dEn != dE ? b2L : bL;
                        }
                    }
                    const bool ok = (unsigned)ip < 64u && (!in_win || (unsigned)inn < 64u);
                    bool acc, sure;
                    if (PREC == 0) {
                        const double d0 = a - b;
                        const double t0 = d0 - lnu;
                        const double M = M0 + ((fabs(a) + fabs(b)) + 1.0) * Mr;
                        acc = dEn == 0 || d0 > M || t0 > M;
                        sure = acc || t0 < -M;
                    } else {
                        const float d0 = (aH - bH) + (aL - bL);
                        const double t0 = (double)d0 - lnu;
                        // plus the rounding of the binary32 difference itself
                        const double M = M0 + (((double)fabs(aH) + (double)fabs(bH)) + 1.0) * Mr +
                                         ((double)fabs(d0) + 1.0) * 0x1p-19;
                        acc = dEn == 0 || (double)d0 > M || t0 > M;
                        sure = acc || t0 < -M;
                    }
                    acc = in_win && acc;
                    sure = !in_win || sure;
                    const bool stop = mine && !(ok && sure);
                    const unsigned long long An = __ballot(mine && acc && !stop);
                    const unsigned long long Sn = __ballot(stop);
                    const unsigned long long Cn = __ballot(mine && (nvn != nvi || dEn != dEi));
                    c = Sn ? (int)__builtin_ctzll(Sn) : todo;
                    const unsigned long long R = act & (c >= 63 ? ~0ull : ((2ull << c) - 1ull));
                    conv = (((An ^ A) | (Sn ^ Sg) | Cn) & R) == 0ull;
                    A = An;
                    Sg = Sn;
                    nvi = nvn;
                    dEi = dEn;
                };
                const long long pcr = pc.now();
                pc.add(kPcSetupCycles, pcr - pcs);
                round(std::true_type{});
                for (int it = 1; it < 66 && !conv; ++it) round(std::false_type{});
                const long long pcc = pc.now();
                pc.add(kPcRoundCycles, pcc - pcr);
                if (!conv) c = start;   // not reached (see above); the exact path is always right
                // commit attempts [start, c): spins, visits, ln g increments per bin
                const unsigned long long seg = act & (c >= 64 ? ~0ull : ((1ull << c) - 1ull));
                const unsigned long long aseg = A & seg;
                const bool inseg = (seg >> lane) & 1ull;
                const bool mine_acc = (aseg >> lane) & 1ull;
                const int ej = pre + (mine_acc ? dEi : 0);
                if (seg) {
                    // a flip is written unless a later accepted flip of the segment
                    // hits the same site
                    unsigned long long sup = 0ull;
                    if (__ballot(mine_acc && (W0 & aseg) != 0ull)) {
                        if (mine_acc && (W0 & aseg) != 0ull) atomicOr(&tag[32], W0 & aseg);
                        wave_lds_sync();
                        sup = tag[32];
                        wave_lds_sync();
                        if (lane == 0) tag[32] = 0ull;
                    }
                    if (mine_acc && !((sup >> lane) & 1ull)) sp[p.site] = (int8_t)nvi;
                    nv = inseg ? nvi : nv;
                    dE = inseg ? dEi : dE;
                    hist = inseg ? ej : hist;
                    if (inseg) atomicAdd(&cnt[ej - ebase], 1u);
                    wave_lds_sync();
                    uint32_t nb = cnt[lane];
                    cnt[lane] = 0u;
                    // the segment's visits go to H here, one add per energy (device-
                    // memory rows: atomic, since a later block may read the bin from
                    // another lane)
                    if (nb != 0u) {
                        if (GLOB) atomicAdd(&H[ebase + lane - lo], nb);
                        else H[ebase + lane - lo] += nb;
                    }
                    if (PREC == 0 && nb != 0u) {
                        // n sequential adds of ln f in closed form: after the first
                        // add, every add moves x by the same exact step d2 while x
                        // stays in one binade (also when the adds round half-way:
                        // the parity that decides a tie is then fixed), so
                        // x_n = x_1 + (n - 1) d2 exactly; otherwise the loop below
                        const double x1 = c64 + lnf_v;
                        const double d2 = (x1 + lnf_v) - x1;
                        int ex;
                        (void)__builtin_frexp(x1, &ex);
                        const double top = __builtin_ldexp(1.0, ex);
                        const double nm1 = (double)(nb - 1u);
                        if (d2 * 64.0 <= x1 && x1 + nm1 * d2 + 4.0 * lnf_v < top * (1.0 - 0x1p-40)) {
                            c64 = x1 + nm1 * d2;
                            nb = 0u;
                        }
                    }
                    if (PREC == 1 && nb != 0u && ch + lnf32 == ch) {
                        // (hi, lo) pair whose high word ln f leaves unchanged: TwoSum
                        // then hands the whole ln f to the low word at every add, and
                        // the low word's n adds follow the closed form above in binary32
                        const float x1 = cl + lnf32;
                        const float d2 = (x1 + lnf32) - x1;
                        int ex;
                        (void)__builtin_frexpf(x1, &ex);
                        const float top = __builtin_ldexpf(1.0f, ex);
                        const float nm1 = (float)(nb - 1u);
                        if (d2 * 64.0f <= x1 &&
                            (double)x1 + (double)nm1 * (double)d2 + 4.0 * (double)lnf32 < (double)top * (1.0 - 0x1p-20)) {
                            cl = x1 + nm1 * d2;
                            nb = 0u;
                        }
                    }
                    while (__ballot(nb != 0u)) {
                        if (PREC == 0) {
                            const double x = c64 + lnf_v;
                            c64 = nb != 0u ? x : c64;
                        } else {
                            float xh = ch, xl = cl;
                            two_sum_add(xh, xl, lnf32);
                            ch = nb != 0u ? xh : ch;
                            cl = nb != 0u ? xl : cl;
                        }
                        nb = nb != 0u ? nb - 1u : 0u;
                    }
                    erel = __builtin_amdgcn_readlane(ej, c - 1) - ebase;
                }
                accepted |= aseg;
                flushed |= aseg;
                const long long pce = pc.now();
                pc.add(kPcCommitCycles, pce - pcc);
                if (c >= todo) break;
                // attempt c on the exact path, with the walker's current ln g
                // (its own new value and dE are settled there from the lattice)
                wave_lds_sync();
                if (PREC == 0) { gEs = readlane_d(c64, erel); gEv = gEs; }
                else { gEh = readlane_f(ch, erel); gEl = readlane_f(cl, erel); }
                slow_attempt(c);
                if (lane == 0) {
                    if (GLOB) atomicAdd(&H[ebase + erel - lo], 1u);
                    else H[ebase + erel - lo] += 1u;
                }
                start = c + 1;
                // every accepted flip so far goes to the lattice; proposals after
                // c that one of them touched read their spins from it again
                if (((accepted & ~flushed) >> lane) & 1ull) sp[p.site] = (int8_t)nv;
                flushed = accepted;
                wave_lds_sync();
                if (lane >= start && (conf & accepted) != 0ull) {
                    x0 = sp[p.site];
                    x1 = sp[p.nb0];
                    x2 = sp[p.nb1];
                    x3 = sp[p.nb2];
                    x4 = sp[p.nb3];
                    nv = x0 + 1 + p.off;
                    if (nv >= q) nv -= q;
                    dE = (int)(x0 == x1) + (int)(x0 == x2) + (int)(x0 == x3) + (int)(x0 == x4) -
                         (int)(nv == x1) - (int)(nv == x2) - (int)(nv == x3) - (int)(nv == x4);
                }
                const unsigned long long keep = start >= 64 ? 0ull : (~0ull << start);
                conf &= keep;
                W0 &= keep;
                W1 &= keep;
                W2 &= keep;
                W3 &= keep;
                W4 &= keep;
                anyconf = __ballot(conf != 0ull);
                pc.add(kPcExactCycles, pc.now() - pce);
            }
        } else {
            // ---- serial phase: runs of attempts with no possible conflict take the
            // inline path; the others go through slow_attempt (which settles the
            // conflict first)
            int j = 0;
            while (j < todo) {
                const unsigned long long later = anyconf & (~0ull << j);
                const int jstop = later ? min(todo, (int)__builtin_ctzll(later)) : todo;
                for (; j < jstop; ++j) {
                    const int dEj = __builtin_amdgcn_readlane(dE, j);
                    const double luj = readlane_d(lnu, j);
                    int idx = erel + dEj;
                    // rare: the proposed energy lies outside the register cache
                    // (laid out of line, the common case falls through)
                    if (__builtin_expect((unsigned)idx >= 64u, 0)) {
                        cache_store();
                        ebase += idx - 32;
                        cache_load();
                        erel = erel - idx + 32;
                        idx = 32;
                    }
                    bool acc;
                    if (PREC == 0) {
                        const double gN = readlane_d(c64, idx);
                        const double d = gEv - gN;
                        const double t = d - luj;
                        acc = __ballot(t > 0.0) != 0ull;
                        if (__builtin_expect(__ballot(!(fabs(t) > kMargin64)) != 0ull, 0))
                            acc = __ballot(ebase + idx >= lo && ebase + idx <= hi &&
                                           accept64(d, __builtin_amdgcn_readlane(p.u, j))) != 0ull;
                        gEs = acc ? gN : gEs;
                        gEv = gEs + lnf_v;
                        gEs = rfl(gEv);
                        erel = acc ? idx : erel;
                        c64 = (lane == erel) ? gEv : c64;
                    } else {
                        const float gNh = readlane_f(ch, idx);
                        const float gNl = readlane_f(cl, idx);
                        const float d = (gEh - gNh) + (gEl - gNl);
                        const double t = (double)d - luj;
                        acc = __ballot(t > 0.0) != 0ull;
                        if (__builtin_expect(__ballot(!(fabs(t) > kMargin32)) != 0ull, 0))
                            acc = __ballot(ebase + idx >= lo && ebase + idx <= hi &&
                                           accept32(d, __builtin_amdgcn_readlane(p.u, j))) != 0ull;
                        gEh = acc ? gNh : gEh;
                        gEl = acc ? gNl : gEl;
                        two_sum_add(gEh, gEl, lnf32);
                        gEh = rfl(gEh);
                        gEl = rfl(gEl);
                        erel = acc ? idx : erel;
                        ch = (lane == erel) ? gEh : ch;
                        cl = (lane == erel) ? gEl : cl;
                    }
                    accepted |= acc ? (1ull << j) : 0ull;
                    hist = writelane_i32(ebase + erel, j, hist);
                }
                if (j >= todo) break;
                slow_attempt(j);
                ++j;
            }
        }

        const long long pct = pc.now();
        if (!spec) {
            p_nx = propose(st, kDomMove, (uint64_t)(s0 + base + 64 + lane), (uint32_t)w);
            lnu_nx = lnu_of(p_nx.u);
        }
        if (((accepted & ~flushed) >> lane) & 1ull) sp[p.site] = (int8_t)nv;
        // (the speculative phase counted its visits per segment)
        if (!spec && live) atomicAdd(&H[hist - lo], 1u);
        const long long pcd = pc.now();
        pc.add(kPcTailCycles, pcd - pct);
        pc.add(kPcDecideCycles, pcd - pc1);
        pc.add(kPcBlocks, 1);
        pc.add(kPcAttempts, todo);
    }
    pc.flush(w, lane);
    cache_store();
    E = ebase + erel;
    walker_sync<WAVE>();
    uint32_t *osp = (uint32_t *)(st.spins + (size_t)w * st.Npad);
    for (int i = lane; i < st.Npad / 4; i += 64) osp[i] = ((uint32_t *)sp)[i];
    if (!GLOB) {
        for (int b = lane; b < W; b += 64) {
            if (PREC == 0) {
                st.lng[row + b] = g[b];
            } else {
                st.lng_hi[row + b] = gh[b];
                st.lng_lo[row + b] = gl[b];
            }
            st.H[row + b] = H[b];
        }
    }
    if (lane == 0) st.E[w] = E;
}

template <int PREC>
__global__ __launch_bounds__(64) void k_sweep(DevState st, int64_t s0, int64_t n) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_walker<PREC>(st, blockIdx.x, s0, n, smem);
}

// The same walk for a run whose ln g and H rows do not fit in LDS beside the
// lattice: the rows stay in device memory (see sweep_walker's GLOB form).
template <int PREC>
__global__ __launch_bounds__(64) void k_sweep_glob(DevState st, int64_t s0, int64_t n) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_walker<PREC, false, true>(st, blockIdx.x, s0, n, smem);
}

// ---------------------------------------------------------------------------
// Sync point of one window (Sec. 2), one workgroup per window:
//  1. visited bins of the window |= bins with H > 0 of any of its walkers;
//  2. (hi, lo) pairs renormalised with Fast2Sum (binary32 variant);
//  3. halving regime: every walker flat (flat_den*min H*n >= flat_num*sum H
//     over the visited bins)?  Then average ln g over the m walkers (summed in
//     walker order, divided by m), hand the mean to all, reset H, ln f /= 2,
//     and switch to ln f = 1/t once ln f <= 1/t (schedule 1);
//     1/t regime: average and reset H at every sync, ln f = 1/t;
//  4. ln f < ln f_final: the window is finished and continues with ln f = 0.
// t = attempts per walker / W (Belardinelli-Pereyra's 1/t rule, cited Sec. 2).
template <int PREC>
__device__ __forceinline__ void sync_window(const DevState &st, int k, int64_t attempts) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    if (*st.converged || st.finished[k]) return;
    const int W = st.W, m = st.m, Wpad = st.Wpad;
    const size_t base = (size_t)k * m * Wpad;
    uint8_t *vis = st.visited + (size_t)k * Wpad;
    for (int b = tid; b < W; b += 256) {
        uint8_t v = vis[b];
        for (int j = 0; j < m; ++j) v |= (st.H[base + (size_t)j * Wpad + b] != 0u) ? 1 : 0;
        vis[b] = v;
    }
    if (PREC == 1) {
        for (int idx = tid; idx < m * W; idx += 256) {
            const int j = idx / W, b = idx - j * W;
            const size_t i = base + (size_t)j * Wpad + b;
            const float h0 = st.lng_hi[i], l0 = st.lng_lo[i];
            const float s = h0 + l0;
            const float z = s - h0;
            st.lng_lo[i] = l0 - z;
            st.lng_hi[i] = s;
        }
    }
    if (st.shadow) {   // this interval's additions, (H - H_prev) * ln f, into the shadow
        const double lnf = st.lnf[k];
        for (int idx = tid; idx < m * W; idx += 256) {
            const int j = idx / W, b = idx - j * W;
            const size_t i = base + (size_t)j * Wpad + b;
            const uint32_t hv = st.H[i];
            const uint32_t n = hv - st.hprev[i];
            if (n) {
                const DD r = dd_add(DD{st.sh_hi[i], st.sh_lo[i]}, dd_mul_count(n, lnf));
                st.sh_hi[i] = r.hi;
                st.sh_lo[i] = r.lo;
            }
            st.hprev[i] = hv;
        }
    }
    if (st.fixed_lnf) return;
    __syncthreads();

    __shared__ unsigned long long s_sum[256];
    __shared__ unsigned int s_n[256], s_min[256];
    __shared__ int s_avg;
    const int regime = st.regime[k];
    if (regime == 0) {
        int all_flat = 1;
        for (int j = 0; j < m; ++j) {
            unsigned long long sum = 0;
            unsigned int cnt = 0, mn = 0xFFFFFFFFu;
            for (int b = tid; b < W; b += 256) {
                if (!vis[b]) continue;
                const unsigned int hv = st.H[base + (size_t)j * Wpad + b];
                cnt += 1;
                sum += hv;
                mn = hv < mn ? hv : mn;
            }
            s_sum[tid] = sum; s_n[tid] = cnt; s_min[tid] = mn;
            __syncthreads();
            for (int o = 128; o > 0; o >>= 1) {
                if (tid < o) {
                    s_sum[tid] += s_sum[tid + o];
                    s_n[tid] += s_n[tid + o];
                    s_min[tid] = s_min[tid + o] < s_min[tid] ? s_min[tid + o] : s_min[tid];
                }
                __syncthreads();
            }
            const unsigned long long n_act = s_n[0], tot = s_sum[0], hmin = s_min[0];
            const bool flat = n_act > 0 &&
                              (unsigned long long)st.flat_den * hmin * n_act >=
                                  (unsigned long long)st.flat_num * tot;
            all_flat = all_flat && flat;
            __syncthreads();
        }
        if (tid == 0) s_avg = all_flat;
    } else {
        if (tid == 0) s_avg = 1;
    }
    __syncthreads();
    if (!s_avg) return;
    for (int b = tid; b < W; b += 256) {
        double sum;
        if (PREC == 0) {
            sum = st.lng[base + b];
            for (int j = 1; j < m; ++j) sum = sum + st.lng[base + (size_t)j * Wpad + b];
        } else {
            sum = (double)st.lng_hi[base + b] + (double)st.lng_lo[base + b];
            for (int j = 1; j < m; ++j) {
                const size_t i = base + (size_t)j * Wpad + b;
                sum = sum + ((double)st.lng_hi[i] + (double)st.lng_lo[i]);
            }
        }
        const double mean = sum / (double)m;
        for (int j = 0; j < m; ++j) {
            const size_t i = base + (size_t)j * Wpad + b;
            if (PREC == 0) {
                st.lng[i] = mean;
            } else {
                const float h0 = (float)mean;
                st.lng_hi[i] = h0;
                st.lng_lo[i] = (float)(mean - (double)h0);
            }
            st.H[i] = 0u;
        }
        if (st.shadow) {
            DD acc{st.sh_hi[base + b], st.sh_lo[base + b]};
            for (int j = 1; j < m; ++j) {
                const size_t i = base + (size_t)j * Wpad + b;
                acc = dd_add(acc, DD{st.sh_hi[i], st.sh_lo[i]});
            }
            acc = dd_div_count(acc, m);
            for (int j = 0; j < m; ++j) {
                const size_t i = base + (size_t)j * Wpad + b;
                st.sh_hi[i] = acc.hi;
                st.sh_lo[i] = acc.lo;
                st.hprev[i] = 0u;
            }
        }
    }
    if (tid == 0) {
        const double inv_t = (double)W / (double)attempts;
        double lnf = st.lnf[k];
        if (regime == 0) {
            lnf = lnf * 0.5;
            if (st.schedule == 1 && lnf <= inv_t) {
                st.regime[k] = 1;
                lnf = inv_t;
            }
        } else {
            lnf = inv_t;
        }
        st.iterations[k] += 1;
        if (lnf < st.lnf_final) {
            st.finished[k] = 1;
            st.lnf_last[k] = lnf;
            lnf = 0.0;
        }
        st.lnf[k] = lnf;
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_sync(DevState st, int64_t attempts) {
    sync_window<PREC>(st, blockIdx.x, attempts);
}

// ---------------------------------------------------------------------------
// One replica-exchange round (Sec. 2, Eq. 1).  Workgroup b handles the window
// pair (k, k+1), k = (r mod 2) + 2b.  Walker j of window k meets walker pi(j)
// of window k+1, pi a Fisher-Yates permutation; configurations X (walker a)
// and Y (walker b) swap with probability
//   min[1, g_a(E_X)/g_a(E_Y) * g_b(E_Y)/g_b(E_X)],
// rejected outright if E_Y is outside window k or E_X outside window k+1.
// Random words: Philox blocks with counter (r, k, n, EXCH), read in order:
// m-1 words for the permutation, then one word per pair.
__device__ __forceinline__ double lng_at(const DevState &st, int w, int b, int prec) {
    const size_t i = (size_t)w * st.Wpad + b;
    if (prec == 0) return st.lng[i];
    return (double)st.lng_hi[i] + (double)st.lng_lo[i];
}

__device__ __forceinline__ void exchange_pair(const DevState &st, uint32_t r, int pair) {
#pragma clang fp contract(off)
    if (*st.converged) return;
    const int k = (int)(r & 1u) + 2 * pair;
    if (k + 1 >= st.h) return;
    const int m = st.m;
    __shared__ int s_perm[1024];
    __shared__ int s_acc[1024];
    if (threadIdx.x == 0) {
        uint32_t buf[4];
        int pos = 4;
        uint32_t n = 0;
        auto next = [&]() -> uint32_t {
            if (pos == 4) {
                const U4 v = philox10(r, (uint32_t)k, n, st.ctr3 | (kDomExch << 24), st.key0, st.key1);
                buf[0] = v.x; buf[1] = v.y; buf[2] = v.z; buf[3] = v.w;
                ++n;
                pos = 0;
            }
            return buf[pos++];
        };
        for (int j = 0; j < m; ++j) s_perm[j] = j;
        for (int i = m - 1; i >= 1; --i) {
            const int j = (int)mul_shift(next(), (uint32_t)(i + 1));
            const int t = s_perm[i]; s_perm[i] = s_perm[j]; s_perm[j] = t;
        }
        const int lo_a = st.start[k], hi_a = lo_a + st.W - 1;
        const int lo_b = st.start[k + 1], hi_b = lo_b + st.W - 1;
        unsigned long long nacc = 0;
        for (int j = 0; j < m; ++j) {
            const int a = k * m + j, b = (k + 1) * m + s_perm[j];
            const uint32_t u = next();
            const int ex = st.E[a], ey = st.E[b];
            int acc = 0;
            if (ey >= lo_a && ey <= hi_a && ex >= lo_b && ex <= hi_b) {
                const double d = ((lng_at(st, a, ex - lo_a, st.precision) -
                                   lng_at(st, a, ey - lo_a, st.precision)) +
                                  lng_at(st, b, ey - lo_b, st.precision)) -
                                 lng_at(st, b, ex - lo_b, st.precision);
                acc = accept64(d, u) ? 1 : 0;
            }
            s_acc[j] = acc;
            nacc += (unsigned long long)acc;
        }
        st.x_att[k] += (unsigned long long)m;
        st.x_acc[k] += nacc;
    }
    __syncthreads();
    // Rows are 256-byte aligned and padded: swap them in 16-byte words, four
    // per lane in flight before any is stored.
    const int n16 = st.Npad / 16;
    for (int j = 0; j < m; ++j) {
        if (!s_acc[j]) continue;
        const int a = k * m + j, b = (k + 1) * m + s_perm[j];
        uint4 *__restrict__ pa = (uint4 *)(st.spins + (size_t)a * st.Npad);
        uint4 *__restrict__ pb = (uint4 *)(st.spins + (size_t)b * st.Npad);
        for (int i0 = 0; i0 < n16; i0 += 4 * (int)blockDim.x) {
            uint4 ta[4], tb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i < n16) {
                    ta[u] = pa[i];
                    tb[u] = pb[i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i < n16) {
                    pa[i] = tb[u];
                    pb[i] = ta[u];
                }
            }
        }
        if (threadIdx.x == 0) {
            const int t = st.E[a]; st.E[a] = st.E[b]; st.E[b] = t;
            if (st.Efx) { const int64_t te = st.Efx[a]; st.Efx[a] = st.Efx[b]; st.Efx[b] = te; }
            const uint32_t rr = st.replica[a]; st.replica[a] = st.replica[b]; st.replica[b] = rr;
        }
    }
}

__global__ __launch_bounds__(64) void k_exchange(DevState st, uint32_t r) {
    exchange_pair(st, r, blockIdx.x);
}

// Replica paths (Sec. 3.2, Fig. 7).  Positions are looked up at creation, at
// every sync point (after its exchange round) and after an exchange round
// called on its own.  Each lookup adds one to visits[w][r] for the replica r
// in slot w.  A round trip takes a replica from the lowest window to the
// highest and back (the usual measure of how fast replica exchange carries
// configurations across the energy range); the return completes one and
// starts the next.  Every slot has its own row of the visit matrix and each
// replica id sits in exactly one slot, so lanes never share a counter.
__device__ __forceinline__ void track_replicas(const DevState &st, int lane, int nlanes) {
    if (st.rep_visits)
        for (int w = lane; w < st.nw; w += nlanes) st.rep_visits[(size_t)w * st.nw + st.replica[w]] += 1u;
    if (st.h < 2) return;
    const int m = st.m;
    for (int i = lane; i < 2 * m; i += nlanes) {
        const bool low = i < m;
        const int w = low ? i : (st.h - 1) * m + (i - m);
        const uint32_t r = st.replica[w];
        if (low) {
            if (st.rep_end[r] == 2) st.rep_trips[r] += 1u;
            st.rep_end[r] = 1;
        } else if (st.rep_end[r] == 1) {
            st.rep_end[r] = 2;
        }
    }
}

// Observable sampling (Sec. 3.2: distributions H(E, O) recorded while the
// walk goes on).  O = max_s n_s of walker w's current lattice, counted with
// LDS atomics over the N sites by the whole workgroup, the maximum over the
// q states taken by one wavefront; lane 0 then adds the sample to energy bin
// E - start_k of the walker's window.  Integer arithmetic throughout.
__device__ __forceinline__ void measure_walker(const DevState &st, int w) {
    __shared__ int s_cnt[128];
    __shared__ int s_max;
    const int tid = threadIdx.x;
    for (int v = tid; v < 128; v += blockDim.x) s_cnt[v] = 0;
    __syncthreads();
    const int8_t *sp = st.spins + (size_t)w * st.Npad;
    for (int i = tid; i < st.N; i += blockDim.x) atomicAdd(&s_cnt[(int)sp[i]], 1);
    __syncthreads();
    if (tid < 64) {
        int mx = 0;
        for (int v = tid; v < st.q; v += 64) mx = s_cnt[v] > mx ? s_cnt[v] : mx;
        for (int off = 32; off > 0; off >>= 1) {
            const int o = __shfl_xor(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        if (tid == 0) s_max = mx;
    }
    __syncthreads();
    if (tid == 0) {
        const int O = s_max;
        const int b = st.E[w] - st.start[w / st.m];
        if (b >= 0 && b < st.W) {
            const size_t cell = (size_t)w * st.Wpad + b;
            const int ob = (int)(((long long)O * st.obs_bins) / (st.N + 1));
            st.obs_hist[cell * st.obs_bins + ob] += 1u;
            st.obs_sum[cell] += (unsigned long long)O;
            st.obs_cnt[cell] += 1u;
        }
    }
}

__global__ __launch_bounds__(256) void k_measure(DevState st) {
    if (*st.converged) return;
    measure_walker(st, blockIdx.x);
}

// Production phase: every window keeps its walkers' current ln g as fixed
// weights (ln f = 0, marked finished; lnf_last records the ln f a window
// still had), termination off, H and the observable record cleared.
__global__ __launch_bounds__(256) void k_begin_production(DevState st) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t cells = (size_t)st.nw * st.Wpad;
    for (size_t c = i; c < cells; c += stride) {
        st.H[c] = 0u;
        if (st.obs_bins > 0) {
            st.obs_sum[c] = 0ull;
            st.obs_cnt[c] = 0u;
        }
    }
    if (st.obs_bins > 0)
        for (size_t c = i; c < cells * st.obs_bins; c += stride) st.obs_hist[c] = 0u;
    if (i == 0) {
        for (int k = 0; k < st.h; ++k) {
            if (!st.finished[k]) {
                st.finished[k] = 1;
                st.lnf_last[k] = st.lnf[k];
            }
            st.lnf[k] = 0.0;
        }
        *st.converged = 0;
        *st.production = 1;
    }
}

// Pooled microcanonical mean of O per energy bin (one thread per bin): the
// integer sums and counts of every walker whose window holds the bin.
__global__ __launch_bounds__(256) void k_obs_micro(DevState st, double *mean, unsigned long long *count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= st.B) return;
    unsigned long long s = 0, c = 0;
    for (int k = 0; k < st.h; ++k) {
        const int lb = b - (st.start[k] - st.e_lo);
        if (lb < 0 || lb >= st.W) continue;
        for (int j = 0; j < st.m; ++j) {
            const size_t cell = (size_t)(k * st.m + j) * st.Wpad + lb;
            s += st.obs_sum[cell];
            c += st.obs_cnt[cell];
        }
    }
    mean[b] = c ? (double)s / (double)c : __builtin_nan("");
    count[b] = c;
}

// Canonical average of O, one workgroup per temperature: weights
// exp(ln g(E) - E/T - max) over the bins with a finite joined ln g and
// samples of O; <O>_T = sum w mu / sum w.
__global__ __launch_bounds__(256) void k_obs_thermo(DevState st, const double *T, const double *mean,
                                                    double *out) {
    const int t = blockIdx.x, tid = threadIdx.x;
    const double temp = T[t];
    __shared__ double s[256], s2[256];
    double mx = -__builtin_inf();
    for (int b = tid; b < st.B; b += 256) {
        const double v = st.joined[b];
        if (v == -__builtin_inf() || __builtin_isnan(mean[b])) continue;
        mx = fmax(mx, v - (st.th_e0 + (double)b * st.th_de) / temp);
    }
    s[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] = fmax(s[tid], s[tid + o]);
        __syncthreads();
    }
    mx = s[0];
    __syncthreads();
    double z = 0.0, num = 0.0;
    for (int b = tid; b < st.B; b += 256) {
        const double v = st.joined[b];
        if (v == -__builtin_inf() || __builtin_isnan(mean[b])) continue;
        const double p = exp((v - (st.th_e0 + (double)b * st.th_de) / temp) - mx);
        z += p;
        num += p * mean[b];
    }
    s[tid] = z;
    s2[tid] = num;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s[tid] += s[tid + o];
            s2[tid] += s2[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) out[t] = s2[0] / s[0];
}

// Termination (Sec. 2): the run ends once every window reached ln f_final
// (never in the production phase).
__device__ __forceinline__ void check_instance(const DevState &st, int64_t step, int64_t round_after) {
    if (*st.converged || *st.production) return;
    for (int k = 0; k < st.h; ++k)
        if (!st.finished[k]) return;
    *st.converged = 1;
    st.stop[0] = step;
    st.stop[1] = round_after;
}

__global__ void k_check(DevState st, int64_t step, int64_t round_after) {
    if (!*st.converged) track_replicas(st, (int)threadIdx.x, (int)blockDim.x);
    if (threadIdx.x == 0) check_instance(st, step, round_after);
}

__global__ void k_track(DevState st) {
    if (!*st.converged) track_replicas(st, (int)threadIdx.x, (int)blockDim.x);
}

// ---------------------------------------------------------------------------
// Joining the pieces (Sec. 2, Fig. 2) in binary64.
// (a) visited flags of unfinished windows absorb the current histograms;
// (b) beta_k(E) = (ln g_k(E+) - ln g_k(E-)) / (E+ - E-) with E+-, the nearest
//     visited bins above and below E inside window k (NaN when undefined);
// (c) one workgroup walks the pairs in order: the joining energy of pair
//     (k, k+1) minimises |beta_k - beta_{k+1}| over the overlap above the
//     previous joining energy (ties: lowest E); piece k+1 is shifted to meet
//     piece k there;
// (d) every energy takes the piece whose range (cut_{k-1}, cut_k] holds it;
// (e) normalisation to sum_E g(E) = q^N by log-sum-exp.
__global__ __launch_bounds__(256) void k_fold_visited(DevState st) {
    const int k = blockIdx.x;
    if (st.finished[k]) return;
    const size_t base = (size_t)k * st.m * st.Wpad;
    uint8_t *vis = st.visited + (size_t)k * st.Wpad;
    for (int b = threadIdx.x; b < st.W; b += blockDim.x) {
        uint8_t v = vis[b];
        for (int j = 0; j < st.m; ++j) v |= (st.H[base + (size_t)j * st.Wpad + b] != 0u) ? 1 : 0;
        vis[b] = v;
    }
}

// A set of h pieces of ln g to join: piece k, bin b at p64[k * kstride + b]
// in binary64, or as the (hi, lo) pair phi/plo at the same index.
struct JoinView {
    int h, W, Wpad, B, e_lo;
    const int32_t *start;   // [h] lowest energy of each window
    const uint8_t *vis;     // [h][Wpad] visited flags
    const double *p64;
    const float *phi, *plo;
    size_t kstride;
    __device__ double piece(int k, int b) const {
        const size_t i = (size_t)k * kstride + b;
        if (p64) return p64[i];
        return (double)phi[i] + (double)plo[i];
    }
};

// The pieces of a run: walker k*m of every window (all walkers of a finished
// window hold the same averaged ln g).
__device__ __forceinline__ JoinView view_of(const DevState &st) {
    JoinView v;
    v.h = st.h; v.W = st.W; v.Wpad = st.Wpad; v.B = st.B; v.e_lo = st.e_lo;
    v.start = st.start;
    v.vis = st.visited;
    v.p64 = st.precision == 0 ? st.lng : nullptr;
    v.phi = st.lng_hi;
    v.plo = st.lng_lo;
    v.kstride = (size_t)st.m * st.Wpad;
    return v;
}

// (b) beta of piece k at bin b.
__device__ __forceinline__ void join_beta(const JoinView &v, int k, int b, double *beta) {
#pragma clang fp contract(off)
    const uint8_t *vis = v.vis + (size_t)k * v.Wpad;
    double out = __builtin_nan("");
    if (vis[b]) {
        int bp = -1, bm = -1;
        for (int t = b + 1; t < v.W; ++t) if (vis[t]) { bp = t; break; }
        for (int t = b - 1; t >= 0; --t) if (vis[t]) { bm = t; break; }
        if (bp >= 0 && bm >= 0)
            out = (v.piece(k, bp) - v.piece(k, bm)) / (double)(bp - bm);
    }
    beta[(size_t)k * v.Wpad + b] = out;
}

// (c) joining energies and shifts, one workgroup of 256 threads.
__device__ __forceinline__ void join_cuts(const JoinView &v, const double *beta, double *shift, int32_t *cuts,
                                          int32_t *status) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    __shared__ double s_d[256];
    __shared__ int s_e[256];
    __shared__ int s_prev;
    if (tid == 0) { s_prev = INT32_MIN; shift[0] = 0.0; *status = 0; }
    __syncthreads();
    const int W = v.W;
    for (int k = 0; k + 1 < v.h; ++k) {
        const int sa = v.start[k], sb = v.start[k + 1];
        int lo = sb;
        if (s_prev != INT32_MIN && s_prev + 1 > lo) lo = s_prev + 1;
        const int hi = sa + W - 1;
        double bestd = 0.0;
        int beste = INT32_MIN;
        for (int e = lo + tid; e <= hi; e += 256) {
            const double ba = beta[(size_t)k * v.Wpad + (e - sa)];
            const double bb = beta[(size_t)(k + 1) * v.Wpad + (e - sb)];
            if (ba != ba || bb != bb) continue;
            const double d = fabs(ba - bb);
            if (beste == INT32_MIN || d < bestd) { bestd = d; beste = e; }
        }
        s_d[tid] = bestd; s_e[tid] = beste;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) {
                const int e2 = s_e[tid + o];
                if (e2 != INT32_MIN) {
                    const double d2 = s_d[tid + o];
                    const int e1 = s_e[tid];
                    if (e1 == INT32_MIN || d2 < s_d[tid] || (d2 == s_d[tid] && e2 < e1)) {
                        s_d[tid] = d2; s_e[tid] = e2;
                    }
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            int best = s_e[0];
            if (best == INT32_MIN) {
                const uint8_t *va = v.vis + (size_t)k * v.Wpad;
                const uint8_t *vb = v.vis + (size_t)(k + 1) * v.Wpad;
                for (int e = lo; e <= hi; ++e)
                    if (va[e - sa] && vb[e - sb]) { best = e; break; }
            }
            if (best == INT32_MIN) {
                *status = -1;
                best = hi;
            }
            cuts[k] = best;
            shift[k + 1] = (v.piece(k, best - sa) + shift[k]) - v.piece(k + 1, best - sb);
            s_prev = best;
        }
        __syncthreads();
    }
}

// (d) the joined value of bin b: piece k holds (cut_{k-1}, cut_k].
__device__ __forceinline__ void join_assemble(const JoinView &v, const int32_t *cuts, const double *shift, int b,
                                              double *out) {
#pragma clang fp contract(off)
    const int e = v.e_lo + b;
    int k = 0;
    while (k < v.h - 1 && e > cuts[k]) ++k;
    const int bb = e - v.start[k];
    double r = -__builtin_inf();
    if (bb >= 0 && bb < v.W && v.vis[(size_t)k * v.Wpad + bb]) r = v.piece(k, bb) + shift[k];
    out[b] = r;
}

// (e) log-sum-exp over the joined curve in one workgroup, then the shift to
// sum_E g(E) = exp(log_total).
__device__ __forceinline__ void join_normalise(double *joined, int B, double log_total) {
    const int tid = threadIdx.x;
    __shared__ double s[256];
    double mx = -__builtin_inf();
    for (int b = tid; b < B; b += 256) mx = fmax(mx, joined[b]);
    s[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] = fmax(s[tid], s[tid + o]);
        __syncthreads();
    }
    mx = s[0];
    __syncthreads();
    double acc = 0.0;
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v != -__builtin_inf()) acc += exp(v - mx);
    }
    s[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    const double lse = mx + log(s[0]);
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v != -__builtin_inf()) joined[b] = (v - lse) + log_total;
    }
}

// Canonical averages (Sec. 3.1, Fig. 3b) from a joined ln g at temperature
// temp, one workgroup: ln Z = LSE_E(ln g(E) - E/T), U = sum P E,
// C_v = sum P (E - U)^2 / T^2 with P = exp(ln g(E) - E/T - ln Z); bin b at
// energy e0 + b de.  out[0..2] = ln Z, U, C_v.
__device__ __forceinline__ void thermo_one(const double *joined, int B, double e0, double de, double temp,
                                           double *out) {
    const int tid = threadIdx.x;
    __shared__ double s[256];
    double mx = -__builtin_inf();
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        mx = fmax(mx, v - (e0 + (double)b * de) / temp);
    }
    s[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] = fmax(s[tid], s[tid + o]);
        __syncthreads();
    }
    mx = s[0];
    __syncthreads();
    double z = 0.0;
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        z += exp((v - (e0 + (double)b * de) / temp) - mx);
    }
    s[tid] = z;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    const double lnz = mx + log(s[0]);
    __syncthreads();
    double u = 0.0;
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        const double e = e0 + (double)b * de;
        u += exp((v - e / temp) - lnz) * e;
    }
    s[tid] = u;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    const double U = s[0];
    __syncthreads();
    double var = 0.0;
    for (int b = tid; b < B; b += 256) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        const double e = e0 + (double)b * de;
        const double d = e - U;
        var += exp((v - e / temp) - lnz) * d * d;
    }
    s[tid] = var;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = lnz;
        out[1] = U;
        out[2] = s[0] / (temp * temp);
    }
}

__global__ __launch_bounds__(256) void k_beta(DevState st, double *beta) {
    const int k = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= st.W) return;
    join_beta(view_of(st), k, b, beta);
}

__global__ __launch_bounds__(256) void k_join_cuts(DevState st, const double *beta, double *shift) {
    join_cuts(view_of(st), beta, shift, st.cuts, st.join_status);
}

__global__ __launch_bounds__(256) void k_join_assemble(DevState st, const double *shift) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= st.B) return;
    join_assemble(view_of(st), st.cuts, shift, b, st.joined);
}

__global__ __launch_bounds__(256) void k_join_normalise(DevState st, double log_total) {
    join_normalise(st.joined, st.B, log_total);
}

__global__ __launch_bounds__(256) void k_thermo(DevState st, const double *T, double *out) {
    const int t = blockIdx.x;
    thermo_one(st.joined, st.B, st.th_e0, st.th_de, T[t], out + 3 * t);
}

// ---------------------------------------------------------------------------
// Batched form: many independent REWL runs (instances) in the same launches.
// Each instance is one DevState in device memory; its main-phase step and
// exchange round live on the device (ctl), so a captured graph of one batched
// step can be replayed.  A batched step advances every unconverged instance
// by one sync interval (its own S attempts per walker): attempts, sync point,
// exchange round, then the counters and the termination test.  Every kernel
// does per instance exactly what the single-run kernels do, so the results
// are bit-identical to running each instance on its own.

__device__ __forceinline__ int wave_broadcast(int v) { return __builtin_amdgcn_readlane(v, 0); }

__global__ __launch_bounds__(64) void k_walkin_batch(const DevState *__restrict__ descs,
                                                     const BatchTask *__restrict__ tasks, int64_t chunk,
                                                     int64_t budget) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BatchTask t = tasks[blockIdx.x];
    const DevState st = descs[t.inst];
    walkin_walker(st, t.idx, chunk, budget, smem);
}

// One thread per instance: 0 every walker placed, 1 some still walking,
// 2 some walker exhausted the budget.
__global__ void k_walkin_status(const DevState *__restrict__ descs, int n, int64_t budget,
                                BatchStatus *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevState &st = descs[i];
    int status = 0;
    for (int w = 0; w < st.nw; ++w) {
        if (st.walkin_done[w]) continue;
        status = st.walkin_att[w] >= budget ? 2 : (status == 2 ? 2 : 1);
    }
    out[i].walkin = status;
}

__global__ void k_queue_reset(int *queue) {
    if (threadIdx.x == 0) queue[0] = 0;
}

// Attempts of one sync interval for every walker of every instance.  With a
// queue the grid is persistent: each workgroup (one wavefront, one walker at
// a time) takes the next task until none is left, so the launch shape (and
// with it walkers per CU and LDS per walker) is free of the task count.
// Tasks are ordered longest first.  Every workgroup leaves once the queue
// index passes ntasks.
template <int PREC, bool PERSISTENT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_batch(const DevState *__restrict__ descs,
                                                    const BatchTask *__restrict__ tasks, int task_lo,
                                                    int ntasks, int *queue) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (!PERSISTENT) {
        const BatchTask t = tasks[task_lo + (int)blockIdx.x];
        const DevState st = descs[t.inst];
        sweep_walker<PREC, false, true>(st, t.idx, st.ctl[0], st.sync_attempts, smem);
        return;
    }
    for (;;) {
        int ti = 0;
        if (threadIdx.x == 0) ti = atomicAdd(queue, 1);
        ti = wave_broadcast(ti);
        if (ti >= ntasks) break;
        const BatchTask t = tasks[ti];
        const DevState &st = descs[t.inst];
        sweep_walker<PREC, false, true>(st, t.idx, st.ctl[0], st.sync_attempts, smem);
        __syncthreads();
    }
}

// Mixed-slot form of the attempt step: one workgroup per CU, one walker per
// wavefront, and wavefront w owns an LDS slot sized for instance class
// plan.cls[w] (classes ordered by LDS need, largest first).  A wave takes the
// tasks of its own class from that class's queue, then those of the smaller
// classes, which fit its slot as well.  Waves share nothing but the queues.
template <int PREC>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_batch_slots(
    const DevState *__restrict__ descs, const BatchTask *__restrict__ tasks, const SlotPlan *__restrict__ plan,
    int *queues) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    unsigned char *mine = smem + plan->off[wave];
    const int nclasses = plan->nclasses;
    for (int c = plan->cls[wave]; c < nclasses; ++c) {
        const int lo = plan->task_lo[c], nt = plan->task_n[c];
        for (;;) {
            int ti = 0;
            if ((threadIdx.x & 63) == 0) ti = atomicAdd(&queues[c], 1);
            ti = wave_broadcast(ti);
            if (ti >= nt) break;
            const BatchTask t = tasks[lo + ti];
            const DevState &st = descs[t.inst];
            sweep_walker<PREC, true, true>(st, t.idx, st.ctl[0], st.sync_attempts, mine);
            walker_sync<true>();
        }
    }
}

__global__ void k_queue_reset_n(int *queue, int n) {
    if ((int)threadIdx.x < n) queue[threadIdx.x] = 0;
}

// Sync point of window t.idx of instance t.inst, at the attempt count the
// instance reaches with this step.
template <int PREC>
__global__ __launch_bounds__(256) void k_sync_batch(const DevState *__restrict__ descs,
                                                    const BatchTask *__restrict__ wtasks, int lo) {
    const BatchTask t = wtasks[lo + (int)blockIdx.x];
    const DevState st = descs[t.inst];
    sync_window<PREC>(st, t.idx, st.ctl[0] + st.sync_attempts);
}

// Observable sample of walker t.idx of instance t.inst (instances that sample one).
__global__ __launch_bounds__(256) void k_measure_batch(const DevState *__restrict__ descs,
                                                       const BatchTask *__restrict__ tasks, int lo) {
    const BatchTask t = tasks[lo + (int)blockIdx.x];
    const DevState &st = descs[t.inst];
    if (st.obs_bins <= 0 || *st.converged) return;
    measure_walker(st, t.idx);
}

// Exchange round of instance t.inst (at its own round counter), pair slot t.idx.
__global__ __launch_bounds__(64) void k_exchange_batch(const DevState *__restrict__ descs,
                                                       const BatchTask *__restrict__ xtasks, int lo) {
    const BatchTask t = xtasks[lo + (int)blockIdx.x];
    const DevState st = descs[t.inst];
    if (!st.exchange) return;
    exchange_pair(st, (uint32_t)st.ctl[1], t.idx);
}

// Step and round counters of every unconverged instance, then termination.
__global__ void k_advance_batch(const DevState *__restrict__ descs, int lo, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevState &st = descs[lo + i];
    if (*st.converged) return;
    track_replicas(st, 0, 1);
    const int64_t step = st.ctl[0] + st.sync_attempts;
    const int64_t round = st.ctl[1] + (st.exchange ? 1 : 0);
    st.ctl[0] = step;
    st.ctl[1] = round;
    check_instance(st, step, round);
}

__global__ void k_status_batch(const DevState *__restrict__ descs, int n, BatchStatus *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevState &st = descs[i];
    const int conv = *st.converged;
    out[i].converged = conv;
    out[i].step = conv ? st.stop[0] : st.ctl[0];
    out[i].round = conv ? st.stop[1] : st.ctl[1];
}

// ---------------------------------------------------------------------------
// Bootstrap error analysis (Sec. 2: the simulation is repeated, the results
// resampled, and every resampled global g(E) joined anew, so its joining
// points move).  The R instances of a batch are R independent runs of one
// system.  Replicate j draws R run indices with replacement (Philox words,
// four per block (j, i/4, 0, BOOT), r = floor(w R / 2^32)), averages the
// drawn runs' pieces window by window (summed in draw order, divided by R),
// joins them over the union of the runs' visited flags, normalises, and
// evaluates U and C_v.  Replicates are independent workgroups.
struct BootView {
    int R, h, W, Wpad, B, Bpad, e_lo, m, nboot;
    const int32_t *start;   // [h]
    int32_t *draws;         // [nboot][R]
    double *pieces;         // [nboot][h][Wpad]
    uint8_t *vis;           // [h][Wpad] union of the runs' flags
    double *beta;           // [nboot][h][Wpad]
    double *shift;          // [nboot][h]
    int32_t *cuts;          // [nboot][h]
    int32_t *status;        // [nboot]
    double *joined;         // [nboot][Bpad]
    __device__ JoinView view(int j) const {
        JoinView v;
        v.h = h; v.W = W; v.Wpad = Wpad; v.B = B; v.e_lo = e_lo;
        v.start = start;
        v.vis = vis;
        v.p64 = pieces + (size_t)j * h * Wpad;
        v.phi = v.plo = nullptr;
        v.kstride = (size_t)Wpad;
        return v;
    }
};

__global__ __launch_bounds__(256) void k_boot_draws(BootView bv, uint32_t key0, uint32_t key1) {
    const int nblk = (bv.R + 3) / 4;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)bv.nboot * nblk) return;
    const int j = (int)(t / nblk), c = (int)(t % nblk);
    const U4 w = philox10((uint32_t)j, (uint32_t)c, 0u, kDomBoot << 24, key0, key1);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * c + q;
        if (i < bv.R) bv.draws[(size_t)j * bv.R + i] = (int32_t)mul_shift(ws[q], (uint32_t)bv.R);
    }
}

__global__ __launch_bounds__(256) void k_boot_visited(BootView bv, const DevState *__restrict__ descs) {
    const int k = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bv.W) return;
    uint8_t v = 0;
    for (int r = 0; r < bv.R; ++r) v |= descs[r].visited[(size_t)k * bv.Wpad + b] ? 1 : 0;
    bv.vis[(size_t)k * bv.Wpad + b] = v;
}

__global__ __launch_bounds__(256) void k_boot_pieces(BootView bv, const DevState *__restrict__ descs) {
#pragma clang fp contract(off)
    const int k = blockIdx.y, j = blockIdx.z;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bv.W) return;
    const int32_t *dr = bv.draws + (size_t)j * bv.R;
    double sum = 0.0;
    for (int i = 0; i < bv.R; ++i) {
        const DevState &st = descs[dr[i]];
        sum = sum + lng_at(st, k * bv.m, b, st.precision);
    }
    bv.pieces[((size_t)j * bv.h + k) * bv.Wpad + b] = sum / (double)bv.R;
}

__global__ __launch_bounds__(256) void k_boot_beta(BootView bv) {
    const int k = blockIdx.y, j = blockIdx.z;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bv.W) return;
    join_beta(bv.view(j), k, b, bv.beta + (size_t)j * bv.h * bv.Wpad);
}

__global__ __launch_bounds__(256) void k_boot_cuts(BootView bv) {
    const int j = blockIdx.x;
    join_cuts(bv.view(j), bv.beta + (size_t)j * bv.h * bv.Wpad, bv.shift + (size_t)j * bv.h,
              bv.cuts + (size_t)j * bv.h, bv.status + j);
}

__global__ __launch_bounds__(256) void k_boot_assemble(BootView bv) {
    const int j = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bv.B) return;
    join_assemble(bv.view(j), bv.cuts + (size_t)j * bv.h, bv.shift + (size_t)j * bv.h, b,
                  bv.joined + (size_t)j * bv.Bpad);
}

__global__ __launch_bounds__(256) void k_boot_normalise(BootView bv, double log_total) {
    join_normalise(bv.joined + (size_t)blockIdx.x * bv.Bpad, bv.B, log_total);
}

// Canonical averages of replicate j at temperature T[t], one wavefront: the
// same four passes as thermo_one, reduced across lanes with shuffles.
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(64) void k_boot_thermo(BootView bv, const double *T, int nT, double e0, double de,
                                                   double *out) {
    const int t = blockIdx.x, j = blockIdx.y, lane = threadIdx.x;
    const double *joined = bv.joined + (size_t)j * bv.Bpad;
    const double temp = T[t];
    double mx = -__builtin_inf();
    for (int b = lane; b < bv.B; b += 64) {
        const double v = joined[b];
        if (v != -__builtin_inf()) mx = fmax(mx, v - (e0 + (double)b * de) / temp);
    }
    mx = wave_max(mx);
    double z = 0.0;
    for (int b = lane; b < bv.B; b += 64) {
        const double v = joined[b];
        if (v != -__builtin_inf()) z += exp((v - (e0 + (double)b * de) / temp) - mx);
    }
    const double lnz = mx + log(wave_sum(z));
    double u = 0.0;
    for (int b = lane; b < bv.B; b += 64) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        const double e = e0 + (double)b * de;
        u += exp((v - e / temp) - lnz) * e;
    }
    const double U = wave_sum(u);
    double var = 0.0;
    for (int b = lane; b < bv.B; b += 64) {
        const double v = joined[b];
        if (v == -__builtin_inf()) continue;
        const double e = e0 + (double)b * de;
        const double d = e - U;
        var += exp((v - e / temp) - lnz) * d * d;
    }
    var = wave_sum(var);
    if (lane == 0) {
        double *o = out + ((size_t)j * nT + t) * 3;
        o[0] = lnz;
        o[1] = U;
        o[2] = var / (temp * temp);
    }
}

// Mean and sample standard deviation of one series over the replicates
// (x[j * stride], j < n) where it is finite, one workgroup of 256 threads
// (two passes, tree sums); mean -inf and std 0 if no value is finite.
__device__ __forceinline__ void finite_stats_wg(const double *x, int n, size_t stride, double *mean, double *sd) {
    const int tid = threadIdx.x;
    __shared__ double s_v[256];
    __shared__ int s_c[256];
    double acc = 0.0;
    int c = 0;
    for (int j = tid; j < n; j += 256) {
        const double v = x[(size_t)j * stride];
        if (__builtin_isfinite(v)) { acc += v; ++c; }
    }
    s_v[tid] = acc; s_c[tid] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) { s_v[tid] += s_v[tid + o]; s_c[tid] += s_c[tid + o]; }
        __syncthreads();
    }
    const int cnt = s_c[0];
    const double mu = cnt ? s_v[0] / (double)cnt : 0.0;
    __syncthreads();
    double q = 0.0;
    for (int j = tid; j < n; j += 256) {
        const double v = x[(size_t)j * stride];
        if (__builtin_isfinite(v)) { const double d = v - mu; q += d * d; }
    }
    s_v[tid] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s_v[tid] += s_v[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        *mean = cnt ? mu : -__builtin_inf();
        *sd = cnt > 1 ? sqrt(s_v[0] / (double)(cnt - 1)) : 0.0;
    }
}

// Series i < B: ln g of bin i; then U and C_v of every temperature.
__global__ __launch_bounds__(256) void k_boot_stats(BootView bv, const double *th, int nT, double *out) {
    const int i = blockIdx.x;
    if (i < bv.B) {
        finite_stats_wg(bv.joined + i, bv.nboot, (size_t)bv.Bpad, out + i, out + bv.B + i);
    } else {
        const int t = (i - bv.B) >> 1, which = (i - bv.B) & 1;   // 0: U, 1: C_v
        double *o = out + 2 * (size_t)bv.B + (size_t)which * 2 * nT;
        finite_stats_wg(th + (size_t)t * 3 + 1 + which, bv.nboot, (size_t)nT * 3, o + t, o + nT + t);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

size_t sweep_lds_bytes(const DevState &st) {
    return (size_t)st.Npad + (st.rows_glob ? (size_t)0 : (size_t)st.Wpad * 12) + (size_t)st.Ntag * 8;
}

size_t walkin_lds_bytes(const DevState &st) { return (size_t)st.Npad + (size_t)st.Bpad * 4; }

static hipError_t allow_lds(const void *fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_init_energy(const DevState &st, hipStream_t s) {
    if (st.model == kModelTrimer3D) return launch_trimer_init(st, s);
    if (st.model == kModelLipid3D) return launch_lipid_init(st, s);
    hipLaunchKernelGGL(k_init_energy, dim3(st.nw), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s) {
    if (st.model == kModelTrimer3D) return launch_trimer_walkin(st, chunk, budget, s);
    if (st.model == kModelLipid3D) return launch_lipid_walkin(st, chunk, budget, s);
    const size_t lds = walkin_lds_bytes(st);
    hipError_t e = allow_lds((const void *)k_walkin, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_walkin, dim3(st.nw), dim3(64), lds, s, st, chunk, budget);
    return hipGetLastError();
}

hipError_t launch_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s) {
    if (st.model == kModelTrimer3D) return launch_trimer_sweep(st, s0, n, s);
    if (st.model == kModelLipid3D) return launch_lipid_sweep(st, s0, n, s);
    const size_t lds = sweep_lds_bytes(st);
    auto go = [&](auto kernel) -> hipError_t {
        hipError_t e = allow_lds((const void *)kernel, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kernel, dim3(st.nw), dim3(64), lds, s, st, s0, n);
        return hipGetLastError();
    };
    if (st.rows_glob) return st.precision == 0 ? go(k_sweep_glob<0>) : go(k_sweep_glob<1>);
    return st.precision == 0 ? go(k_sweep<0>) : go(k_sweep<1>);
}

hipError_t launch_sync(const DevState &st, int64_t attempts, hipStream_t s) {
    if (st.precision == 0)
        hipLaunchKernelGGL(k_sync<0>, dim3(st.h), dim3(256), 0, s, st, attempts);
    else
        hipLaunchKernelGGL(k_sync<1>, dim3(st.h), dim3(256), 0, s, st, attempts);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState &st, uint32_t round, hipStream_t s) {
    const int pairs = (st.h - (int)(round & 1u)) / 2;
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exchange, dim3(pairs), dim3(64), 0, s, st, round);
    return hipGetLastError();
}

hipError_t launch_check(const DevState &st, int64_t step, int64_t round_after, hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, s, st, step, round_after);
    return hipGetLastError();
}

hipError_t launch_track(const DevState &st, hipStream_t s) {
    hipLaunchKernelGGL(k_track, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_measure(const DevState &st, hipStream_t s) {
    hipLaunchKernelGGL(k_measure, dim3(st.nw), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_begin_production(const DevState &st, hipStream_t s) {
    const size_t cells = (size_t)st.nw * st.Wpad * (st.obs_bins > 0 ? st.obs_bins : 1);
    const size_t blocks = std::min<size_t>((cells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_begin_production, dim3((unsigned)blocks), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_obs_micro(const DevState &st, double *mean, unsigned long long *count, hipStream_t s) {
    hipLaunchKernelGGL(k_obs_micro, dim3((st.B + 255) / 256), dim3(256), 0, s, st, mean, count);
    return hipGetLastError();
}

hipError_t launch_obs_thermo(const DevState &st, const double *T, int nT, const double *mean, double *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_obs_thermo, dim3(nT), dim3(256), 0, s, st, T, mean, out);
    return hipGetLastError();
}

hipError_t launch_join(const DevState &st, double log_total, hipStream_t s) {
    double *beta = st.scratch;                                  // [h][Wpad]
    double *shift = st.scratch + (size_t)st.h * st.Wpad;        // [h]
    hipLaunchKernelGGL(k_fold_visited, dim3(st.h), dim3(256), 0, s, st);
    hipLaunchKernelGGL(k_beta, dim3((st.W + 255) / 256, st.h), dim3(256), 0, s, st, beta);
    hipLaunchKernelGGL(k_join_cuts, dim3(1), dim3(256), 0, s, st, (const double *)beta, shift);
    hipLaunchKernelGGL(k_join_assemble, dim3((st.B + 255) / 256), dim3(256), 0, s, st,
                       (const double *)shift);
    hipLaunchKernelGGL(k_join_normalise, dim3(1), dim3(256), 0, s, st, log_total);
    return hipGetLastError();
}

hipError_t launch_bootstrap(const BootArgs &a, const DevState *descs, hipStream_t s) {
    BootView bv;
    bv.R = a.R; bv.h = a.h; bv.W = a.W; bv.Wpad = a.Wpad; bv.B = a.B; bv.Bpad = a.Bpad; bv.e_lo = a.e_lo;
    bv.m = a.m; bv.nboot = a.nboot;
    bv.start = a.start; bv.draws = a.draws; bv.pieces = a.pieces; bv.vis = a.vis; bv.beta = a.beta;
    bv.shift = a.shift; bv.cuts = a.cuts; bv.status = a.status; bv.joined = a.joined;
    const long long ndraw = (long long)a.nboot * ((a.R + 3) / 4);
    const unsigned wb = (unsigned)((a.W + 255) / 256);
    hipLaunchKernelGGL(k_boot_draws, dim3((unsigned)((ndraw + 255) / 256)), dim3(256), 0, s, bv, a.key0, a.key1);
    hipLaunchKernelGGL(k_boot_visited, dim3(wb, a.h), dim3(256), 0, s, bv, descs);
    hipLaunchKernelGGL(k_boot_pieces, dim3(wb, a.h, a.nboot), dim3(256), 0, s, bv, descs);
    hipLaunchKernelGGL(k_boot_beta, dim3(wb, a.h, a.nboot), dim3(256), 0, s, bv);
    hipLaunchKernelGGL(k_boot_cuts, dim3(a.nboot), dim3(256), 0, s, bv);
    hipLaunchKernelGGL(k_boot_assemble, dim3((unsigned)((a.B + 255) / 256), a.nboot), dim3(256), 0, s, bv);
    hipLaunchKernelGGL(k_boot_normalise, dim3(a.nboot), dim3(256), 0, s, bv, a.log_total);
    if (a.nT > 0)
        hipLaunchKernelGGL(k_boot_thermo, dim3(a.nT, a.nboot), dim3(64), 0, s, bv, a.T, a.nT, a.e0, a.de, a.th);
    hipLaunchKernelGGL(k_boot_stats, dim3((unsigned)(a.B + 2 * a.nT)), dim3(256), 0, s, bv, (const double *)a.th,
                       a.nT, a.out);
    return hipGetLastError();
}

hipError_t launch_thermo(const DevState &st, const double *T, int nT, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_thermo, dim3(nT), dim3(256), 0, s, st, T, out);
    return hipGetLastError();
}

hipError_t launch_walkin_batch(const DevState *descs, const BatchTask *tasks, int ntasks,
                               size_t lds_bytes, int64_t chunk, int64_t budget, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipError_t e = allow_lds((const void *)k_walkin_batch, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_walkin_batch, dim3(ntasks), dim3(64), lds_bytes, s, descs, tasks, chunk, budget);
    return hipGetLastError();
}

hipError_t launch_walkin_status(const DevState *descs, int n, int64_t budget, BatchStatus *out,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walkin_status, dim3((n + 255) / 256), dim3(256), 0, s, descs, n, budget, out);
    return hipGetLastError();
}

hipError_t launch_queue_reset(int *queue, hipStream_t s) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
    return hipGetLastError();
}

hipError_t launch_sweep_batch(int precision, const DevState *descs, const BatchTask *tasks, int task_lo,
                              int ntasks, int *queue, int grid, size_t lds_bytes, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    const void *fn = queue ? (precision == 0 ? (const void *)k_sweep_batch<0, true>
                                             : (const void *)k_sweep_batch<1, true>)
                           : (precision == 0 ? (const void *)k_sweep_batch<0, false>
                                             : (const void *)k_sweep_batch<1, false>);
    hipError_t e = allow_lds(fn, lds_bytes);
    if (e != hipSuccess) return e;
    if (queue && precision == 0)
        hipLaunchKernelGGL((k_sweep_batch<0, true>), dim3(grid), dim3(64), lds_bytes, s, descs, tasks, task_lo,
                           ntasks, queue);
    else if (queue)
        hipLaunchKernelGGL((k_sweep_batch<1, true>), dim3(grid), dim3(64), lds_bytes, s, descs, tasks, task_lo,
                           ntasks, queue);
    else if (precision == 0)
        hipLaunchKernelGGL((k_sweep_batch<0, false>), dim3(ntasks), dim3(64), lds_bytes, s, descs, tasks,
                           task_lo, ntasks, queue);
    else
        hipLaunchKernelGGL((k_sweep_batch<1, false>), dim3(ntasks), dim3(64), lds_bytes, s, descs, tasks,
                           task_lo, ntasks, queue);
    return hipGetLastError();
}

hipError_t launch_sweep_batch_slots(int precision, const DevState *descs, const BatchTask *tasks,
                                    const SlotPlan *plan, int nclasses, int nslots, int *queues, int grid,
                                    size_t lds_bytes, hipStream_t s) {
    const void *fn = precision == 0 ? (const void *)k_sweep_batch_slots<0> : (const void *)k_sweep_batch_slots<1>;
    hipError_t e = allow_lds(fn, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_queue_reset_n, dim3(1), dim3(64), 0, s, queues, nclasses);
    if (precision == 0)
        hipLaunchKernelGGL(k_sweep_batch_slots<0>, dim3(grid), dim3(64 * nslots), lds_bytes, s, descs, tasks,
                           plan, queues);
    else
        hipLaunchKernelGGL(k_sweep_batch_slots<1>, dim3(grid), dim3(64 * nslots), lds_bytes, s, descs, tasks,
                           plan, queues);
    return hipGetLastError();
}

hipError_t sweep_batch_slots_fits(int precision, size_t lds_bytes, int nslots, int *fits) {
    const void *fn = precision == 0 ? (const void *)k_sweep_batch_slots<0> : (const void *)k_sweep_batch_slots<1>;
    hipError_t e = allow_lds(fn, lds_bytes);
    if (e != hipSuccess) return e;
    int blocks = 0;
    if (precision == 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep_batch_slots<0>, 64 * nslots, lds_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep_batch_slots<1>, 64 * nslots, lds_bytes);
    *fits = blocks >= 1 ? 1 : 0;
    return e;
}

hipError_t launch_sync_batch(int precision, const DevState *descs, const BatchTask *wtasks, int lo, int n,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(k_sync_batch<0>, dim3(n), dim3(256), 0, s, descs, wtasks, lo);
    else
        hipLaunchKernelGGL(k_sync_batch<1>, dim3(n), dim3(256), 0, s, descs, wtasks, lo);
    return hipGetLastError();
}

hipError_t launch_measure_batch(const DevState *descs, const BatchTask *tasks, int lo, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_measure_batch, dim3(n), dim3(256), 0, s, descs, tasks, lo);
    return hipGetLastError();
}

hipError_t launch_exchange_batch(const DevState *descs, const BatchTask *xtasks, int lo, int n,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exchange_batch, dim3(n), dim3(64), 0, s, descs, xtasks, lo);
    return hipGetLastError();
}

hipError_t launch_advance_batch(const DevState *descs, int lo, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance_batch, dim3((n + 255) / 256), dim3(256), 0, s, descs, lo, n);
    return hipGetLastError();
}

hipError_t launch_status_batch(const DevState *descs, int n, BatchStatus *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_status_batch, dim3((n + 255) / 256), dim3(256), 0, s, descs, n, out);
    return hipGetLastError();
}

hipError_t sweep_batch_occupancy(int precision, size_t lds_bytes, int *blocks_per_cu) {
    const void *fn = precision == 0 ? (const void *)k_sweep_batch<0, true> : (const void *)k_sweep_batch<1, true>;
    hipError_t e = allow_lds(fn, lds_bytes);
    if (e != hipSuccess) return e;
    if (precision == 0)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_batch<0, true>, 64, lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_batch<1, true>, 64, lds_bytes);
}

}  // namespace rewl_gpu

#ifdef REWL_PHASE_CLOCKS
// Profiling build: copies rows [0, min(rows, 4096)) of the phase counters
// (12 per walker, in the order of the kPc* slots) to host memory and, if
// `reset`, zeroes all of them.  Synchronous on the null stream.
extern "C" int rewl_phase_clocks(unsigned long long *host, size_t rows, int reset) {
    const size_t n = (rows < (size_t)rewl_gpu::kPcRows ? rows : (size_t)rewl_gpu::kPcRows) * rewl_gpu::kPcSlots;
    if (host && n && hipMemcpyFromSymbol(host, HIP_SYMBOL(rewl_gpu::g_phase_ctr), n * 8) != hipSuccess) return -1;
    if (reset) {
        static unsigned long long zero[rewl_gpu::kPcRows * rewl_gpu::kPcSlots];
        if (hipMemcpyToSymbol(HIP_SYMBOL(rewl_gpu::g_phase_ctr), zero, sizeof(zero)) != hipSuccess) return -1;
    }
    return 0;
}
#endif
