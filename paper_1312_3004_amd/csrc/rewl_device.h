// rewl_device.h -- device-side building blocks of the REWL walker update and
// the state layout shared by the kernels and the host runtime of librewl.
//
// Method: Vogel, Li, Wuest, Landau, J. Phys.: Conf. Ser. (2014), Sec. 2
// (Wang-Landau walkers in overlapping windows with replica exchange).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl_gpu {

constexpr uint32_t kDomMove = 0;    // main-phase attempts
constexpr uint32_t kDomWalkin = 2;  // walk-in attempts
constexpr uint32_t kDomExch = 3;    // exchange permutation and acceptance words
constexpr uint32_t kDomMoveU = 5;   // trimer model: uniform word of a main-phase attempt
constexpr uint32_t kDomWalkinU = 6; // trimer model: uniform word of a walk-in attempt
constexpr uint32_t kDomBoot = 7;    // bootstrap: run indices drawn for the resamples

constexpr int kModelPotts2D = 0;
constexpr int kModelTrimer3D = 1;
constexpr int kModelLipid3D = 2;

// Everything a kernel needs to find one run's state in the device workspace.
// Per-walker rows are padded so every row starts on a 256-byte boundary.
// Largest walker count for which the walker-by-replica visit matrix is kept
// (4096^2 counters = 64 MiB).
constexpr int kMaxVisitWalkers = 4096;

struct DevState {
    int model;                   // kModelPotts2D or kModelTrimer3D
    // Potts: L x L lattice, q states, N = L*L sites, energies e_lo .. e_lo+B-1.
    // Trimer: N = bytes of one configuration (3 nmol beads x 3 binary32
    // coordinates), B energy bins of width bin_w from e_min, e_lo = 0 and
    // E[] holds each walker's bin, Efx[] its energy (units of 2^-32).
    int L, q, N, h, m, nw, W, B, e_lo;
    int nmol, nb;                // trimer: molecules, beads; lipid model: lipids, particles
    // lipid model: W-W Lennard-Jones depth, reptation threshold of a 32-bit
    // word, and byte offsets of the types, lipid rows and position table in
    // a walker's state row
    double lip_eps_ww;
    uint32_t lip_rep_thr;
    int lip_off_type, lip_off_lip, lip_off_where;
    float box;                   // trimer: side of the periodic cube
    double e_min, bin_w;         // trimer: energy of bin 0's lower edge, bin width
    int64_t emin_fx, binw_fx;    // the same in units of 2^-32 (rint(x 2^32))
    double binw_inv;             // 1 / binw_fx (binary64), for the bin estimate
    double th_e0, th_de;         // energy of bin b for thermodynamics: th_e0 + b th_de
    int Npad, Wpad, Bpad;        // row strides (elements)
    int Ntag;                    // entries of the LDS conflict-tag table (power of two)
    int rows_glob;               // single runs: 1 if ln g and H rows stay in device memory
                                 // (lattice plus rows exceed the LDS), 0 if staged in LDS
    uint32_t key0, key1, ctr3;   // Philox key and instance bits of counter word 3
    uint32_t flat_num, flat_den;
    double lnf_final;
    int schedule, precision, fixed_lnf, exchange, shadow;
    int64_t sync_attempts;       // S: attempts per walker between sync points
    int walkin_slack;            // walk-in lid/floor distance (0: no lid)
    int64_t *ctl;                // [2] main-phase step and exchange round, kept on the
                                 // device by the batched form (null otherwise)
    const int32_t *start;        // [h] lowest energy of each window
    int8_t *spins;               // [nw][Npad]
    int32_t *E;                  // [nw] energy (Potts) or energy bin (trimer)
    int64_t *Efx;                // [nw] continuous models: energy in units of 2^-32 (null for Potts)
    double *lng;                 // [nw][Wpad]            (precision 0)
    float *lng_hi, *lng_lo;      // [nw][Wpad] each       (precision 1)
    uint32_t *H;                 // [nw][Wpad]
    double *sh_hi, *sh_lo;       // [nw][Wpad] exact reference of ln g (double-double), if kept
    uint32_t *hprev;             // [nw][Wpad] H at the previous sync point (shadow only)
    uint32_t *replica;           // [nw] replica id held by each walker slot
    int32_t *rep_end;            // [nw] per replica id: 0 lowest window not reached yet, 1 reached
                                 // (highest not since), 2 highest reached since
    uint32_t *rep_trips;         // [nw] per replica id: completed lowest-highest-lowest round trips
    uint32_t *rep_visits;        // [nw][nw] lookups that found replica r in slot w (null above
                                 // kMaxVisitWalkers walkers)
    int obs_bins;                // O bins of H(E, O); 0: observables not sampled
    int obs_field;               // lipid model: record field binned as O (3: largest cluster)
    double obs_lo, obs_hi;       // lipid model: range of a floating-point O field
    uint32_t *obs_hist;          // [nw][Wpad][obs_bins] H(E, O) per walker
    unsigned long long *obs_sum; // [nw][Wpad] sum of O per energy bin
    uint32_t *obs_cnt;           // [nw][Wpad] samples per energy bin
    int32_t *production;         // [1] 1: weights frozen, no termination
    double *obs_rec;             // [nw][8] lipid model: structural records of the last measurement
    int64_t *walkin_att;         // [nw]
    int32_t *walkin_done;        // [nw]
    int32_t *walkin_bound;       // [nw] walk-in lid (walker above its window) or floor
    uint32_t *walkin_cnt;        // [nw][Bpad] visit counts of the walk-in ln g (ln f = 1)
    double *lnf, *lnf_last;      // [h]
    int32_t *regime, *finished;  // [h]
    int64_t *iterations;         // [h]
    uint8_t *visited;            // [h][Wpad]
    unsigned long long *x_att, *x_acc;  // [h] exchange attempts / accepts of pair (k, k+1)
    int32_t *converged;          // [1]
    int64_t *stop;               // [2] main-phase step and exchange round at convergence
    double *joined;              // [Bpad] joined ln g
    int32_t *cuts;               // [h]
    int32_t *join_status;        // [1]
    double *scratch;             // [max(h, 4096)] small reduction scratch
};

// One unit of work of the batched form: walker, window or window pair `idx`
// of instance `inst`.
struct BatchTask {
    int32_t inst, idx;
};

// Mixed-slot plan of the batched attempt step: nslots wavefronts per
// workgroup (one workgroup per CU); wavefront w owns the LDS slot at byte
// offset off[w] and serves class cls[w] first, then the smaller classes.
// Class c's tasks are tasks[task_lo[c] .. task_lo[c] + task_n[c]).
constexpr int kMaxSlots = 16;
constexpr int kMaxClasses = 8;
struct SlotPlan {
    int nslots, nclasses;
    int cls[kMaxSlots];
    int off[kMaxSlots];
    int task_lo[kMaxClasses];
    int task_n[kMaxClasses];
};

// Per-instance progress gathered after batched steps.
struct BatchStatus {
    int64_t step, round;    // device-side counters (or the stop point once converged)
    int32_t converged;      // every window reached ln f_final
    int32_t walkin;         // walk-in: 0 all placed, 1 pending, 2 some walker hit the budget
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each
// multiplying counter words 0 and 2 by fixed 32-bit constants, xor-ing the
// high halves with the other words and the round key, then bumping the key by
// the Weyl constants.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // full 64-bit products: one multiply instruction gives both halves
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return U4{c0, c1, c2, c3};
}

// floor(r * n / 2^32): Lemire's multiply-shift map of a 32-bit word to [0, n).
__device__ __forceinline__ uint32_t mul_shift(uint32_t r, uint32_t n) { return __umulhi(r, n); }

// ---------------------------------------------------------------------------
// Energies of the continuous models (trimer, lipid) in fixed point: a pair
// term V (binary64) is rounded once to a multiple of 2^-32, fx(V) =
// rint(V 2^32), and a total or a change of energy is the exact int64 sum of
// such terms, the same in whatever order the lanes add them.  A term of
// magnitude 2^18 or more (or one that is not finite) is a hard overlap: a
// move that would create one is rejected, a start holding one is refused.
// Energies stay below 2^29 in magnitude (2^61 units); a change below 2^62.
constexpr int64_t kFxBad = INT64_MIN;   // marks a hard-overlap term in buffers
constexpr int64_t kFxELimit = (int64_t)1 << 61;

__device__ __forceinline__ bool fx_term(double v, int64_t &out) {
#pragma clang fp contract(off)
    if (!(__builtin_fabs(v) < 0x1p18)) return false;
    // rint(v 2^32) without a binary64 -> int64 conversion: |v 2^32| < 2^50
    // (the scaling is exact), so adding 1.5 2^52 rounds it to the nearest
    // integer, ties to even, which then sits in the low bits of the sum's
    // significand (the sum lies in [2^52, 2^53), where the spacing is 1)
    const double y = v * 0x1p32 + 0x1.8p52;
    out = (int64_t)__double_as_longlong(y) - (int64_t)0x4338000000000000ll;
    return true;
}

// E + dE if it stays in range (|E| < 2^61, |dE| < 2^62: the sum cannot overflow).
__device__ __forceinline__ bool fx_add(int64_t e, int64_t de, int64_t &out) {
    const int64_t s = e + de;
    if (s >= kFxELimit || s <= -kFxELimit) return false;
    out = s;
    return true;
}

// Bin of a fixed-point energy: floor((E - e_min) / bin_w) on the 2^-32 grid,
// also outside [0, B) (bounded to +-2^30) so the walk-in's lid can follow it.
// The quotient comes from binary64, E - e_min times binw_inv = 1 / bin_w
// (three roundings, relative error below 2^-50, so the estimate's floor is
// within one of the exact one for quotients up to 2^31), and is then
// corrected with exact integer products, which stay below 2^63 because
// |E - e_min| < 2^62 and bin_w < 2^61 units.
__device__ __forceinline__ int fx_bin(int64_t emin_fx, int64_t binw_fx, double binw_inv, int64_t e) {
#pragma clang fp contract(off)
    const int64_t diff = e - emin_fx;
    const double qd = __builtin_floor((double)diff * binw_inv);
    if (qd <= -1073741825.0) return -1073741824;   // the exact quotient is <= -2^30
    if (qd >= 1073741825.0) return 1073741824;     // ... >= 2^30
    int64_t q = (int64_t)(int)qd;
    if (q * binw_fx > diff) q -= 1;
    else if ((q + 1) * binw_fx <= diff) q += 1;
    if (q < -1073741824) return -1073741824;
    if (q > 1073741824) return 1073741824;
    return (int)q;
}

// Lane-to-lane move of an int64 by a DPP row pattern (the two 32-bit halves
// separately); lanes of rows outside ROWS read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)v >> 32), CTRL, ROWS,
                                                              0xF, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sum of an int64 over the 64 lanes of a wavefront (all lanes active; any
// order gives the same value, integer addition being exact); every lane
// returns the total.  DPP steps: pairs and quads (quad_perm), half rows and
// rows (mirrors), then row 0 into 1 and row 2 into 3 (row_bcast:15) and the
// first half into row 3 (row_bcast:31); lane 63 holds the total.
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
    v += dpp64<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp64<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp64<0x141, 0xF>(v);   // row_half_mirror
    v += dpp64<0x140, 0xF>(v);   // row_mirror
    v += dpp64<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp64<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// exp(x) for x < 0, the acceptance ratio min[1, g_old/g_new] of Sec. 2 written
// as exp(ln g_old - ln g_new).  Cody-Waite reduction x = k ln2 + r with ln 2
// split as C1 (40 significant bits, so k*C1 is exact) + C2, then the degree-13
// Taylor polynomial of exp(r) by Horner's rule with coefficients 1/n! rounded
// to binary64, then scaling by 2^k.  Every operation is a separately rounded
// binary64 operation (no contraction), so the result is reproducible bit for
// bit on any IEEE machine that follows the same order.
__device__ __forceinline__ double exp_neg(double x) {
#pragma clang fp contract(off)
    if (x < -64.0) return 0.0;
    const double inv_ln2 = 0x1.71547652b82fep+0;
    const double c1 = 0x1.62e42fefa4000p-1;
    const double c2 = -0x1.8432a1b0e2634p-43;
    const double kd = __builtin_rint(x * inv_ln2);
    const double r = (x - kd * c1) - kd * c2;
    double p = 0x1.6124613a86d09p-33;            // 1/13!
    p = 0x1.1eed8eff8d898p-29 + r * p;           // 1/12!
    p = 0x1.ae64567f544e4p-26 + r * p;           // 1/11!
    p = 0x1.27e4fb7789f5cp-22 + r * p;           // 1/10!
    p = 0x1.71de3a556c734p-19 + r * p;           // 1/9!
    p = 0x1.a01a01a01a01ap-16 + r * p;           // 1/8!
    p = 0x1.a01a01a01a01ap-13 + r * p;           // 1/7!
    p = 0x1.6c16c16c16c17p-10 + r * p;           // 1/6!
    p = 0x1.1111111111111p-7 + r * p;            // 1/5!
    p = 0x1.5555555555555p-5 + r * p;            // 1/4!
    p = 0x1.5555555555555p-3 + r * p;            // 1/3!
    p = 0x1.0000000000000p-1 + r * p;            // 1/2!
    p = 1.0 + r * p;                             // 1/1!
    p = 1.0 + r * p;                             // 1/0!
    return __builtin_ldexp(p, (int)kd);
}

// Binary32 twin for the (hi, lo) ln g variant: C1 of 16 bits, degree 7.
__device__ __forceinline__ float exp_neg32(float x) {
#pragma clang fp contract(off)
    if (x < -64.0f) return 0.0f;
    const float inv_ln2 = 0x1.715476p+0f;
    const float c1 = 0x1.62e4p-1f;
    const float c2 = 0x1.7f7d1cp-20f;
    const float kf = __builtin_rintf(x * inv_ln2);
    const float r = (x - kf * c1) - kf * c2;
    float p = 0x1.a01a02p-13f;                   // 1/7!
    p = 0x1.6c16c2p-10f + r * p;                 // 1/6!
    p = 0x1.111112p-7f + r * p;                  // 1/5!
    p = 0x1.555556p-5f + r * p;                  // 1/4!
    p = 0x1.555556p-3f + r * p;                  // 1/3!
    p = 0x1.000000p-1f + r * p;                  // 1/2!
    p = 1.0f + r * p;
    p = 1.0f + r * p;
    return __builtin_ldexpf(p, (int)kf);
}

// Wang-Landau acceptance (Sec. 2): accept iff d >= 0 or u < exp(d), with
// d = ln g(E_old) - ln g(E_new) and u = r / 2^32.
__device__ __forceinline__ bool accept64(double d, uint32_t r) {
#pragma clang fp contract(off)
    if (d >= 0.0) return true;
    return (double)r * 0x1p-32 < exp_neg(d);
}

// Same decision in binary32 with a 24-bit uniform u = (r >> 8) / 2^24.
__device__ __forceinline__ bool accept32(float d, uint32_t r) {
#pragma clang fp contract(off)
    if (d >= 0.0f) return true;
    return (float)(r >> 8) * 0x1p-24f < exp_neg32(d);
}

// ln g(E) += ln f on a binary32 (hi, lo) pair by Knuth's TwoSum: the rounding
// error of the high part is carried into the low part.
__device__ __forceinline__ void two_sum_add(float &hi, float &lo, float x) {
#pragma clang fp contract(off)
    const float s = hi + x;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (x - bb);
    hi = s;
    lo = lo + err;
}

// ---------------------------------------------------------------------------
// Double-double arithmetic of the ln g shadow (an exact reference of the
// accumulated ln g, kept at sync points): TwoSum (Knuth), Fast2Sum (Dekker),
// product residuals by fused multiply-add, and the accurate double-double
// addition of Hida, Li and Bailey.  Every step is one rounded binary64 op.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return DD{s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD dd_quick(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return DD{s, b - (s - a)};
}

__device__ __forceinline__ DD dd_add(DD x, DD y) {
#pragma clang fp contract(off)
    DD s = dd_sum(x.hi, y.hi);
    const DD t = dd_sum(x.lo, y.lo);
    s = dd_quick(s.hi, s.lo + t.hi);
    return dd_quick(s.hi, s.lo + t.lo);
}

// exact n * x as a double-double (n < 2^32)
__device__ __forceinline__ DD dd_mul_count(uint32_t n, double x) {
#pragma clang fp contract(off)
    const double dn = (double)n;
    const double p = dn * x;
    return DD{p, __builtin_fma(dn, x, -p)};
}

__device__ __forceinline__ DD dd_div_count(DD x, int m) {
#pragma clang fp contract(off)
    const double dm = (double)m;
    const double q1 = x.hi / dm;
    const double r = __builtin_fma(-q1, dm, x.hi) + x.lo;
    return dd_quick(q1, r / dm);
}

}  // namespace rewl_gpu

// Launchers implemented in rewl_kernels.hip, used by the host runtime.
namespace rewl_gpu {
hipError_t launch_init_energy(const DevState &st, hipStream_t s);
hipError_t launch_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s);
hipError_t launch_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s);
hipError_t launch_sync(const DevState &st, int64_t attempts, hipStream_t s);
hipError_t launch_exchange(const DevState &st, uint32_t round, hipStream_t s);
hipError_t launch_check(const DevState &st, int64_t step, int64_t round_after, hipStream_t s);
hipError_t launch_track(const DevState &st, hipStream_t s);
hipError_t launch_measure(const DevState &st, hipStream_t s);
hipError_t launch_begin_production(const DevState &st, hipStream_t s);
// Lipid model: structural records of every walker, then H(E, O) with O the
// lipids in the largest cluster (rewl_structure.hip).
hipError_t launch_lipid_measure(const DevState &st, hipStream_t s);
hipError_t launch_obs_micro(const DevState &st, double *mean, unsigned long long *count, hipStream_t s);
hipError_t launch_obs_thermo(const DevState &st, const double *T, int nT, const double *mean, double *out,
                             hipStream_t s);
hipError_t launch_join(const DevState &st, double log_total, hipStream_t s);
hipError_t launch_thermo(const DevState &st, const double *T, int nT, double *out, hipStream_t s);
size_t sweep_lds_bytes(const DevState &st);
size_t walkin_lds_bytes(const DevState &st);

// Trimer model (rewl_trimer.hip).
hipError_t launch_trimer_init(const DevState &st, hipStream_t s);
hipError_t launch_lipid_init(const DevState &st, hipStream_t s);
hipError_t launch_lipid_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s);
hipError_t launch_lipid_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s);
size_t lipid_sweep_lds_bytes(const DevState &st);
hipError_t launch_trimer_walkin(const DevState &st, int64_t chunk, int64_t budget, hipStream_t s);
hipError_t launch_trimer_sweep(const DevState &st, int64_t s0, int64_t n, hipStream_t s);
size_t trimer_sweep_lds_bytes(const DevState &st);
size_t trimer_walkin_lds_bytes(const DevState &st);

// Batched form: many independent runs, each described by one DevState in
// device memory (`descs`).  Tasks are (instance, index) pairs.
hipError_t launch_walkin_batch(const DevState *descs, const BatchTask *tasks, int ntasks,
                               size_t lds_bytes, int64_t chunk, int64_t budget, hipStream_t s);
hipError_t launch_walkin_status(const DevState *descs, int n, int64_t budget, BatchStatus *out,
                                hipStream_t s);
hipError_t launch_queue_reset(int *queue, hipStream_t s);
// persistent (queue != null): `grid` workgroups pull tasks [0, ntasks) from the
// queue; otherwise one workgroup per task of [task_lo, task_lo + ntasks).
hipError_t launch_sweep_batch(int precision, const DevState *descs, const BatchTask *tasks, int task_lo,
                              int ntasks, int *queue, int grid, size_t lds_bytes, hipStream_t s);
hipError_t launch_sync_batch(int precision, const DevState *descs, const BatchTask *wtasks, int lo, int n,
                             hipStream_t s);
// Bootstrap over the R instances of a batch (device buffers carved by the host).
struct BootArgs {
    int R, h, W, Wpad, B, Bpad, e_lo, m, nboot, nT;
    uint32_t key0, key1;
    double log_total, e0, de;
    const int32_t *start;
    int32_t *draws;     // [nboot][R]
    double *pieces;     // [nboot][h][Wpad]
    uint8_t *vis;       // [h][Wpad]
    double *beta;       // [nboot][h][Wpad]
    double *shift;      // [nboot][h]
    int32_t *cuts;      // [nboot][h]
    int32_t *status;    // [nboot]
    double *joined;     // [nboot][Bpad]
    const double *T;    // [nT]
    double *th;         // [nboot][nT][3]
    double *out;        // [2B + 4 nT]: ln g mean, std; U mean, std; C mean, std
};
hipError_t launch_bootstrap(const BootArgs &a, const DevState *descs, hipStream_t s);
hipError_t launch_measure_batch(const DevState *descs, const BatchTask *tasks, int lo, int n, hipStream_t s);
hipError_t launch_exchange_batch(const DevState *descs, const BatchTask *xtasks, int lo, int n,
                                 hipStream_t s);
hipError_t launch_advance_batch(const DevState *descs, int lo, int n, hipStream_t s);
hipError_t launch_status_batch(const DevState *descs, int n, BatchStatus *out, hipStream_t s);
hipError_t sweep_batch_occupancy(int precision, size_t lds_bytes, int *blocks_per_cu);
// Mixed-slot attempt step (queue reset included); grid = workgroups (one per CU).
// plan: device copy of the slot plan.
hipError_t launch_sweep_batch_slots(int precision, const DevState *descs, const BatchTask *tasks,
                                    const SlotPlan *plan, int nclasses, int nslots, int *queues, int grid,
                                    size_t lds_bytes, hipStream_t s);
hipError_t sweep_batch_slots_fits(int precision, size_t lds_bytes, int nslots, int *fits);
}  // namespace rewl_gpu
