/*
 * rewl.h -- C ABI of the MI355X Replica-Exchange Wang-Landau library.
 *
 * Method: T. Vogel, Y. W. Li, T. Wuest, D. P. Landau, "Exploring new
 * frontiers in statistical physics with a new, parallel Wang-Landau
 * framework", J. Phys.: Conf. Ser. (2014), Sec. 2.  The global energy range
 * is split into h overlapping windows (Fig. 1); m independent Wang-Landau
 * walkers sample each window, each with its own ln g(E) and H(E); walkers in
 * neighbouring windows exchange configurations with the probability of
 * Eq. (1); when all m walkers of a window are flat their ln g are averaged
 * and ln f is reduced; the run ends when every window reached ln f_final, and
 * the pieces are joined where d ln g/dE agree best (Fig. 2).
 *
 * Model: the 2D q-state Potts model of Eq. (2) on an L x L periodic lattice,
 * single-spin-flip moves (Sec. 3.1); energies are the integers [-2N, 0].
 *
 * Conventions
 *  - Every function returns a rewl_status: 0 (REWL_OK) or 1
 *    (REWL_CONVERGED) on success, a negative code on failure; the message of
 *    the last failure in the calling thread is rewl_last_error().
 *  - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *    pointers are GPU global memory.  The library never frees caller memory.
 *  - All GPU work is enqueued on the caller's HIP stream given to
 *    rewl_create; calls that return host data synchronise that stream.
 *  - One handle must not be used from two threads at once; distinct handles
 *    are independent.
 *  - Walker w = k*m + j is walker j of window k.  Window k covers the
 *    energies [start_k, start_k + W - 1]; bin b of a window is energy
 *    start_k + b.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed
 *    and counter (step_lo, step_hi, walker, domain << 24 | instance).
 *  - Identical inputs give bitwise-identical results, and rewl_run(a)
 *    followed by rewl_run(b) equals rewl_run(a + b).
 */
#ifndef REWL_H
#define REWL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rewl rewl_t; /* opaque handle, owned by the library */

enum rewl_model { REWL_POTTS2D = 0, REWL_TRIMER3D = 1 /* rewl_create_trimer */,
                  REWL_LIPID3D = 2 /* rewl_create_lipid */ };

enum rewl_status {
    REWL_OK = 0,
    REWL_CONVERGED = 1, /* every window reached ln f_final                    */
    REWL_EINVAL = -1,   /* argument out of range                               */
    REWL_ENOMEM = -2,   /* workspace too small / host allocation failed        */
    REWL_EDEVICE = -3,  /* a HIP call failed (message in rewl_last_error)      */
    REWL_ESTATE = -4,   /* call not valid in the current state                 */
    REWL_EBUDGET = -5   /* walk-in exceeded its attempt budget                 */
};

/* Run options.  rewl_default_opts fills the values in brackets. */
typedef struct {
    uint64_t seed;          /* [1] Philox key                                       */
    uint32_t instance;      /* [0] low 24 bits enter the Philox counter             */
    uint32_t flat_num;      /* [4] flatness: H is flat when                          */
    uint32_t flat_den;      /* [5]   flat_den*min(H)*n >= flat_num*sum(H) (n = bins) */
    double lnf_init;        /* [1.0] initial ln f                                   */
    double lnf_final;       /* [1e-6] a window is finished once ln f < lnf_final    */
    int32_t schedule;       /* [0] 0: ln f halves (f -> sqrt f) at each flat sync;   */
                            /*     1: halving until ln f <= 1/t, then ln f = 1/t    */
                            /*     with t = attempts per walker / W                 */
    int32_t exchange;       /* [1] replica-exchange round at every sync point        */
    int64_t sync_attempts;  /* [1000] attempts per walker between sync points        */
    int32_t precision;      /* [0] 0: ln g in binary64; 1: binary32 (hi, lo) pair    */
    int32_t fixed_lnf;      /* [0] 1: sync points never change ln f (fixed weights) */
    int32_t shadow;         /* [0] 1: keep an exact reference of ln g (see           */
                            /*     rewl_get_shadow); costs 20 bytes per bin and walker */
    int32_t walkin_slack;   /* [16] walk-in lid width (energy units), 0 = no lid    */
    int32_t obs_bins;       /* [0] > 0 samples an observable O at every sync point  */
                            /*     into H(E, O) with this many O bins (see         */
                            /*     rewl_get_obs): Potts O = max_s n_s, at most     */
                            /*     L*L+1 bins; lipid model O = lipids in the       */
                            /*     largest cluster or another structural field     */
                            /*     (rewl_lipid_obs_field), at most 4096 bins;      */
                            /*     costs 4*obs_bins + 12 bytes per bin and walker  */
    int32_t reserved;       /* [0] must be 0                                        */
} rewl_opts;

void rewl_default_opts(rewl_opts *o);

/* Energy-range splitting of Sec. 2 / Fig. 1 for the L x L Potts model:
 * h windows of equal width W at overlap fraction o over the 2N+1 energies;
 * W = ceil((2N+1) / (1 + (h-1)(1-o))), start_k = -2N + round(k(2N+1-W)/(h-1)).
 * starts: host int32[windows].  REWL_EINVAL for L < 3, windows < 1,
 * o outside [0, 1) or W < 8.                                                 */
int rewl_window_layout(int L, int windows, double overlap, int32_t *W, int32_t *starts);

/* Device workspace needed by rewl_create for these parameters (bytes), or 0
 * if the parameters are invalid.                                             */
size_t rewl_workspace_bytes(int model, int L, int q, int windows, double overlap, int walkers,
                            const rewl_opts *opts);

/* Create a run: `windows` windows at `overlap`, `walkers` walkers per window.
 * init_spins: host int8[windows*walkers][L*L], values in [0, q): the starting
 *   lattice of every walker (copied; the caller keeps ownership).
 * dev_workspace: device memory of at least rewl_workspace_bytes(...) bytes,
 *   owned by the caller and required to outlive the handle.
 * hip_stream: the hipStream_t all work is enqueued on (NULL = default stream).
 * Limits: 3 <= L <= 724, 2 <= q <= 127, 1 <= windows, 1 <= walkers,
 *   windows*walkers <= 65535, 0 <= overlap < 1, W >= 8, 1 <= flat_den <= 1000,
 *   flat_num <= flat_den, sync_attempts >= 1.  The handle is written to *out. */
int rewl_create(rewl_t **out, int model, int L, int q, int windows, double overlap, int walkers,
                const rewl_opts *opts, const int8_t *init_spins, void *dev_workspace,
                size_t ws_bytes, void *hip_stream);

void rewl_destroy(rewl_t *r);

/* ---- Lipid model with explicit solvent (Sec. 3.2, Eqs. (3)-(5), Fig. 5) ---
 * nlip lipids of a polar head P and two hydrophobic tails H (P-H-H) and nsol
 * solvent particles W in a periodic cube of side `box`; particles 3i, 3i+1,
 * 3i+2 start as lipid i (head first), the others as solvent.  Non-bonded
 * pairs: H-W and H-P repel by 4 (1.05/r)^9 (Eq. 3), all other pairs are
 * Lennard-Jones 4 eps (r^-12 - r^-6) (Eq. 4) with eps = 1, or eps_ww for
 * W-W; both cut at r = 2.5 unshifted.  Bonded neighbours of a lipid: FENE,
 * -0.5 K R^2 ln(1 - (r/R)^2) with K = 30, R = 1.3, plus the WCA repulsion
 * (LJ + 1 below 2^(1/6)) (Eq. 5); r >= R is forbidden.  Moves: with
 * probability rep_prob (a negative value selects the paper's 3 nlip /
 * (10 np), np = 3 nlip + nsol) a reptation: a uniformly drawn lipid and end;
 * one of the n_c solvent particles within R of that end (drawn uniformly, in
 * index order) becomes the new end bead, the beads shift along the chain and
 * the far end is released as solvent; positions are unchanged; acceptance
 * min[1, g(E)/g(E') n_c / n_r] with n_r the solvent particles within R of the
 * new end next to the released particle.  Otherwise a displacement of one
 * uniformly drawn particle by a uniform vector in [-0.1, 0.1)^3.  Energy
 * changes are summed over partners in the fixed order of the trimer model;
 * the FENE logarithm is computed from basic IEEE operations, so runs are
 * reproducible bit for bit.  Energy bins and windows as for the trimer model.
 * init_coords: host float[windows*walkers][np][3] in [0, box).  opts:
 * precision 0 and shadow 0 only; obs_bins > 0 (at most 4096, with nlip <=
 * 512) samples H(E, O) with O the lipids in the largest cluster or another
 * structural field (see rewl_structure, rewl_lipid_obs_field and
 * rewl_get_obs).  rewl_get_particles returns a
 * walker's coordinates, types (0 P, 1 H, 2 W) and lipid rows (particle
 * indices, head first).  Limits: nlip >= 1, np <= 4096, the state row plus
 * 12 bytes per window bin within the 160 KiB LDS of a CU.
 * Errors: REWL_EINVAL on invalid arguments, REWL_ENOMEM if the workspace is
 * too small, REWL_EDEVICE on a HIP failure.                                   */
size_t rewl_lipid_workspace_bytes(int nlip, int nsol, float box, double eps_ww, double rep_prob, double e_min,
                                  double bin_w, int bins, int windows, double overlap, int walkers,
                                  const rewl_opts *opts);
int rewl_create_lipid(rewl_t **out, int nlip, int nsol, float box, double eps_ww, double rep_prob, double e_min,
                      double bin_w, int bins, int windows, double overlap, int walkers, const rewl_opts *opts,
                      const float *init_coords, void *dev_workspace, size_t ws_bytes, void *hip_stream);
int rewl_get_particles(rewl_t *r, int walker, float *coords, int8_t *types, int32_t *lipids);

/* ---- Structural observables of lipid configurations (Sec. 3.2, Eqs. 6-8) --
 * For each configuration, an 8-double record:
 *   [0] S_mol^head (Eq. 6): (3 <cos^2 theta> - 1) / 2 over the bonds from each
 *       lipid's head to its first tail bead, theta measured against the box
 *       axis that maximises it;  [1] that axis (0 x, 1 y, 2 z; the first on
 *       ties);
 *   [2] number of lipid clusters: lipids are neighbours when a tail bead of
 *       one lies within 1.4 of a tail bead of the other (squared minimum-image
 *       distance < 1.96), clusters are the connected components;
 *   [3] lipids in the largest cluster (the one holding the lowest lipid index
 *       on ties);
 *   [4..6] Q_xx, Q_yy, Q_zz (Eq. 7 with the square): the diagonal of the
 *       gyration tensor of the 3 x [3] beads of the largest cluster in unfolded
 *       coordinates, all beads of equal mass;
 *   [7] prolateness P = 9 sum_i (Q_ii - lambda)^3 / (sum_i Q_ii)^3 with lambda
 *       = (sum_i Q_ii) / 3 (Eq. 8): 2 for a rod, -1/4 for a flat disc.
 * Unfolding grows the cluster breadth first from its lowest-index lipid; a
 * lipid found at level k+1 hangs from the lowest-index lipid of level k it
 * touches and is placed through their first touching tail pair (parent
 * centre, then end bead; child centre, then end bead), its other beads through
 * its bonds; the root keeps its stored head position.  Minimum images are
 * taken per axis in binary32 (one wrap by +-box), everything else in binary64.
 * Integer fields are exact; floating fields agree with a plain evaluation to
 * rounding (lane sums are taken in butterfly order).
 *
 * rewl_lipid_structure: device pointers.  Configuration c has coordinates
 *   float[np][3] at (char *)coords + c * coord_stride and lipid rows int32
 *   [nlip][3] (particle indices, head first) at (char *)lipids + c *
 *   lipid_stride; out double[nconf][8].  The work is queued on hip_stream
 *   (NULL: the default stream) and the call returns without waiting.  A
 *   configuration holding a particle index outside [0, np) gets a NaN record.
 *   Limits: 1 <= nlip <= 512, np >= 3 nlip; pointers and strides 4-byte
 *   aligned, out 8-byte aligned.  REWL_EINVAL on invalid arguments,
 *   REWL_EDEVICE if the launch fails.
 * rewl_structure: the records of every walker of a lipid-model run (walker
 *   order), into host out double[windows * walkers][8]; waits for the result.
 *   REWL_EINVAL for a null argument, a run of another model or one of more
 *   than 512 lipids, REWL_EDEVICE on a HIP failure.                           */
int rewl_lipid_structure(const float *coords, size_t coord_stride, const int32_t *lipids, size_t lipid_stride,
                         int nconf, int np, int nlip, float box, double *out, void *hip_stream);
int rewl_structure(rewl_t *r, double *out);

/* rewl_structure for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same records, staged in a static device buffer of 4,096 records (256
 * KiB on every GPU the library runs on, held until the process ends) instead
 * of an allocation per call.  Calls no hipMalloc or hipFree.  Every call on
 * one GPU shares that GPU's buffer: calls that overlap on one GPU (from
 * several host threads or streams) race and must be serialised by the caller.
 * Errors as rewl_structure, and REWL_EINVAL for a run of more than 4,096
 * walkers.                                                                   */
int rewl_structure_noalloc(rewl_t *r, double *out);

/* Which structural observable a lipid run with obs_bins > 0 histograms in
 * H(E, O) (Sec. 3.2 records H(E, O) for S_mol, Q_ii and P).  field 3 (the
 * default at creation): O = lipids in the largest cluster, O bin O obs_bins /
 * (nlip + 1).  field 0, 4, 5, 6 or 7 (S_mol, Q_xx, Q_yy, Q_zz, P of the
 * rewl_structure record): O = floor((v - lo) / (hi - lo) * obs_bins), held to
 * [0, obs_bins - 1], is both the O bin and the value summed by rewl_get_obs
 * (rewl_obs_micro then gives the mean bin index).  Applies from the next sync
 * point; rewl_begin_production clears what was sampled before.  Not part of a
 * checkpoint: after rewl_load the default applies.  Errors: REWL_EINVAL for a
 * null handle, a run of another model or without obs_bins, another field, or
 * lo, hi not finite with lo < hi.                                            */
int rewl_lipid_obs_field(rewl_t *r, int field, double lo, double hi);

/* ---- Continuous-move model: amphiphilic trimers ---------------------------
 * nmol head-tail-tail molecules (bead 3i the head, 3i+1 and 3i+2 its tails)
 * in a periodic cube of side `box` (the paper's bead-spring amphiphile with
 * local displacement moves, Sec. 3.2, with a simpler force field): bonds
 * head-tail1 and tail1-tail2 harmonic, 100 (r - 1)^2; every other pair
 * 4 (r^-12 - r^-6), tail-tail cut at r = 2.5 unshifted, pairs with a head cut
 * at r = 2^(1/6) and shifted by +1.  A move displaces one uniformly chosen
 * bead by a uniform vector in [-0.1, 0.1)^3 (periodic wrap).  Energies are
 * binned: bin b = floor((E - e_min) / bin_w), b in [0, bins); the windows of
 * Sec. 2 are laid over the bins exactly as over the Potts energies.
 * Energies are fixed point in units of 2^-32: every pair term V (binary64)
 * is rounded once, rint(V 2^32), and totals and the change of a move are
 * exact integer sums of such terms (independent of the order of summation,
 * so runs are reproducible bit for bit); bins are floor((E - e_min) / bin_w)
 * on that grid, with e_min and bin_w rounded to it.  A pair term of magnitude
 * 2^18 or more (or not finite) is a hard overlap: a move creating one is
 * rejected, and a start holding one (or an energy of magnitude 2^29 or more)
 * is refused with REWL_EINVAL.  Limits: bin_w in [2^-32, 2^28], |e_min| <
 * 2^28.
 * init_coords: host float[windows*walkers][3 nmol][3], values in [0, box).
 * For these runs rewl_get_walker returns the configuration's bytes in
 * `spins` (float[3 nmol][3]) and the energy bin in `E`; rewl_get_energy
 * gives the energy.  rewl_join normalises to sum over bins of g = 1, and
 * rewl_thermo takes bin centres as energies.  Limits: 1 <= nmol <= 1024,
 * bins >= 8.                                                                */
size_t rewl_trimer_workspace_bytes(int nmol, float box, double e_min, double bin_w, int bins, int windows,
                                   double overlap, int walkers, const rewl_opts *opts);
int rewl_create_trimer(rewl_t **out, int nmol, float box, double e_min, double bin_w, int bins, int windows,
                       double overlap, int walkers, const rewl_opts *opts, const float *init_coords,
                       void *dev_workspace, size_t ws_bytes, void *hip_stream);

/* Windows over `bins` energy bins (bin indices, first window at 0).        */
int rewl_window_layout_bins(int bins, int windows, double overlap, int32_t *W, int32_t *starts);

/* Current energy of walker w (the Potts energy as a double, or the
 * continuous models' energy, the nearest binary64 of the fixed-point value).
 * rewl_get_energy_fx: the continuous models' energy in units of 2^-32
 * exactly (the Potts energy as an integer for Potts runs).                  */
int rewl_get_energy(rewl_t *r, int walker, double *E);
int rewl_get_energy_fx(rewl_t *r, int walker, int64_t *E);

/* Walk-in: move every walker whose energy lies outside its window into it
 * (each walker starts inside its own window, Sec. 3.2 on Fig. 7) by a
 * Wang-Landau walk with ln f = 1 over all energies, under a lid: a walker
 * above its window rejects moves to energies more than walkin_slack above the
 * lowest energy it has reached (a walker below, symmetrically, stays above a
 * floor), so it floods a band of that width instead of the whole range.  REWL_EBUDGET if some
 * walker needs more than max_attempts attempts (its state is left where the
 * walk stopped).  Called implicitly with a budget of 2^40 by the first run. */
int rewl_walkin(rewl_t *r, int64_t max_attempts);

/* Main phase: attempts per walker (rewl_run: sweeps * L*L attempts).  Sync
 * points (flatness, averaging and ln f update per window, then an exchange
 * round) fall at every multiple of sync_attempts counted from the start of
 * the main phase.  Returns REWL_CONVERGED, and stops at that sync point, once
 * every window is finished; later calls return REWL_CONVERGED at once.       */
int rewl_run(rewl_t *r, int64_t sweeps);
int rewl_run_attempts(rewl_t *r, int64_t attempts);

/* One replica-exchange round now (Eq. (1)); round r pairs windows (k, k+1)
 * with k = r mod 2, r mod 2 + 2, ...                                          */
int rewl_exchange(rewl_t *r);

/* Replica paths under exchange (Sec. 2; Sec. 3.2, Fig. 7): replica r starts
 * in walker slot r (window r / m) and moves with every accepted exchange.
 * Positions are looked up at creation, at every sync point (after its
 * exchange round) and after every rewl_exchange call.  window_of[r] receives
 * the window replica r is in now and trips[r] the round trips it completed:
 * paths window 0 -> window h-1 -> window 0, counted on the return, which also
 * starts the next (a run with one window has none).  Host buffers of h*m
 * entries, indexed by replica id; either may be NULL.
 * Errors: REWL_EINVAL on a null handle.                                       */
int rewl_get_replicas(rewl_t *r, uint32_t *window_of, uint32_t *trips);

/* Replicas seen by walker slot w (Fig. 7c): counts[r] = lookups (as above)
 * that found replica r in slot w; a host buffer of h*m entries.  Kept for
 * runs of at most 4096 walkers (h*m*h*m counters in the workspace).
 * Errors: REWL_EINVAL on a null handle or buffer, w out of range, or a run
 * with more than 4096 walkers.                                                */
int rewl_get_replica_visits(rewl_t *r, int walker, uint32_t *counts);

/* Production phase (Sec. 3.2: after g(E) is estimated, sampling goes on
 * with fixed weights 1/g(E) while observables are recorded).  From this call
 * on every walker keeps its current ln g as fixed weights: each window gets
 * ln f = 0 and is marked finished (a window not finished before records its
 * current ln f as lnf_last), the run no longer terminates, and H and the
 * observable record restart from zero; step and round counters continue.
 * Usually called once rewl_run has returned REWL_CONVERGED; rewl_run then
 * keeps sampling.  Errors: REWL_EINVAL on a null handle, REWL_ESTATE before
 * the walk-in or on an instance of a batch.                                   */
int rewl_begin_production(rewl_t *r);

/* Observable record of walker w (runs with opts.obs_bins > 0).  At every
 * sync point, after its exchange round, each walker adds the configuration it
 * holds: with O = max_s n_s for the Potts model (the population of the most
 * occupied state; the order parameter is (q O / N - 1) / (q - 1)), or O = the
 * lipids in the largest cluster for the lipid model (record field [3] of
 * rewl_structure, with N read as nlip; rewl_lipid_obs_field selects another
 * field), and b its energy bin in the window, hist[b][floor(O * obs_bins /
 * (N + 1))] += 1, sum[b] += O, count[b] += 1.  Host buffers hist
 * uint32[W][obs_bins], sum uint64[W], count uint32[W]; any may be NULL.  Errors: REWL_EINVAL on a null handle,
 * w out of range, or a run without observable sampling.                      */
int rewl_get_obs(rewl_t *r, int walker, uint32_t *hist, uint64_t *sum, uint32_t *count);

/* Microcanonical mean of O per energy bin of the whole range (B bins, bin b
 * at energy e_lo + b): the samples of all walkers whose window holds the bin,
 * pooled (weights that depend only on E leave the distribution of O at fixed
 * E unchanged).  mean double[B] (NaN where no sample fell), count uint64[B]
 * (may be NULL).  Errors: REWL_EINVAL on a null handle or mean, or a run
 * without observable sampling.                                               */
int rewl_obs_micro(rewl_t *r, double *mean, uint64_t *count);

/* Canonical average of O at nT temperatures (Sec. 3.2 with the canonical
 * weights of Sec. 3.1): <O>_T = sum_E g(E) e^{-E/T} mu(E) / sum_E g(E)
 * e^{-E/T} over the bins with a finite joined ln g and samples of O, mu the
 * pooled mean of rewl_obs_micro.  Needs a current rewl_join.  out double[nT].
 * Errors: REWL_EINVAL (null argument, nT outside [1, 4096], T <= 0, no
 * observable sampling), REWL_ESTATE without a current join.                  */
int rewl_obs_thermo(rewl_t *r, const double *T, int nT, double *out);

/* Progress counters: main-phase attempts per walker, exchange rounds done,
 * and whether the run converged.  Any pointer may be NULL.                   */
int rewl_get_progress(rewl_t *r, int64_t *step, int64_t *round, int32_t *converged);

/* State of walker w into host buffers (any pointer may be NULL):
 * spins int8[L*L], E, H uint32[W], lng double[W] (the (hi, lo) pair summed in
 * binary64 when precision = 1), replica id, walk-in attempts.                */
int rewl_get_walker(rewl_t *r, int walker, int8_t *spins, int32_t *E, uint32_t *H, double *lng,
                    uint32_t *replica, int64_t *walkin_attempts);

/* The walker's state in one call (any pointer may be NULL): spins, E, H and
 * ln g as rewl_get_walker, and lnf, the current ln f of the walker's window
 * as rewl_get_window.  Errors: REWL_EINVAL on a null handle or w out of
 * range, REWL_EDEVICE on a HIP failure.                                       */
int rewl_get_state(rewl_t *r, int walker, int8_t *spins, int32_t *E, uint32_t *H, double *lng, double *lnf);

/* State of window k (any pointer may be NULL): current ln f (0 once
 * finished), the ln f that finished it, regime (0 halving, 1 1/t), finished
 * flag, number of ln f reductions, visited flags uint8[W] (union over the
 * window's walkers), and the exchange attempts/accepts of pair (k, k+1).     */
int rewl_get_window(rewl_t *r, int window, double *lnf, double *lnf_last, int32_t *regime,
                    int32_t *finished, int64_t *iterations, uint8_t *visited, uint64_t *x_att,
                    uint64_t *x_acc);

/* Shadow of walker w's ln g (runs created with opts.shadow = 1): an exact
 * reference of the values ln g should hold along the walker's own trajectory.
 * At every sync point each bin receives (visits since the previous sync
 * point) x ln f in double-double arithmetic (Knuth TwoSum, Dekker Fast2Sum,
 * exact products by fused multiply-add), and window averages are taken the
 * same way; (hi + lo) - ln g is the rounding error the ln g format has
 * accumulated (binary64, or the binary32 pair).  Valid at sync points.
 * hi, lo: host double[W].  REWL_ESTATE if the run keeps no shadow.          */
int rewl_get_shadow(rewl_t *r, int walker, double *hi, double *lo);

/* Checkpoint / resume.  rewl_save writes the whole state of the run (its
 * device workspace and the host-side counters, behind a header that records
 * the run's parameters) into host memory: with buf = NULL it only stores the
 * required size in *n; with cap smaller than that it fails with REWL_ENOMEM.
 * rewl_load restores such a checkpoint into a handle created with the same
 * model, sizes and options (REWL_EINVAL otherwise); the run then continues
 * bit for bit as the saved one would have.  Both synchronise the stream.     */
int rewl_save(rewl_t *r, void *buf, size_t cap, size_t *n);
int rewl_load(rewl_t *r, const void *buf, size_t n);

/* Overwrite ln g of walker w from host double[W] (sampling with the fixed
 * weights 1/g(E) of a converged run, Sec. 3.2).                             */
int rewl_set_lng(rewl_t *r, int walker, const double *lng);

/* ln g of window k (walker 0 of the window) into host double[W], or with
 * window = -1 the joined and normalised ln g over all 2N+1 energies (see
 * rewl_join).  Unvisited bins are -INFINITY.  *n_out = number of values,
 * *e_first_out = energy of the first value.  REWL_EINVAL if cap is too small. */
int rewl_get_lng(rewl_t *r, int window, double *host_out, int64_t cap, int64_t *n_out,
                 int64_t *e_first_out);

/* Join the h pieces on the GPU in binary64 (Sec. 2, Fig. 2): for each pair of
 * neighbouring windows the joining energy E* is where the finite-difference
 * slopes d ln g/dE of the two pieces agree best (ties: lowest E, and E* above
 * the previous joining energy); piece k+1 is shifted to meet piece k at E*;
 * the result is normalised to sum_E g(E) = q^N.  host_out: double[2N+1]
 * (may be NULL), cuts: int32[windows-1] (may be NULL).  REWL_ESTATE if two
 * neighbouring pieces share no visited energy.  The joined ln g stays on the
 * device for rewl_thermo.                                                    */
int rewl_join(rewl_t *r, double *host_out, int32_t *cuts);

/* Canonical thermodynamics from the joined ln g (Sec. 3.1, Fig. 3b), binary64
 * on the GPU: ln Z(T) = log-sum-exp_E (ln g(E) - E/T), U = <E>,
 * C_v = (<E^2> - <E>^2)/T^2.  T, lnZ, U, C: host double[nT].  Requires a
 * previous rewl_join (REWL_ESTATE otherwise).                                */
int rewl_thermo(rewl_t *r, const double *T, int nT, double *lnZ, double *U, double *C);

/* Kernel timing.  While enabled, HIP events on the run's stream bracket every
 * launch of the attempt kernel and every sync point (flatness, averaging,
 * exchange, termination test); rewl_get_timing returns the summed elapsed
 * milliseconds and launch counts since timing was last enabled.            */
int rewl_set_timing(rewl_t *r, int enable);
int rewl_get_timing(rewl_t *r, double *sweep_ms, int64_t *sweep_launches, double *sync_ms,
                    int64_t *sync_points);

/* Message of the last failing call in this thread ("" if none). */
const char *rewl_last_error(void);

/* ---- Batched form ---------------------------------------------------------
 * A batch holds n independent runs ("instances") of the method above, each
 * with its own L, q, windows, walkers and options, in one device workspace.
 * One batched step advances every unconverged instance by one sync interval:
 * sync_attempts attempts for each of its walkers, then its sync point and
 * exchange round, exactly as rewl_run_attempts does at a sync point.  The
 * attempts of all walkers of all instances run in one persistent launch: a
 * grid of walkers_per_cu x (compute units) one-wavefront workgroups takes
 * walker tasks, longest first, from a device-side queue.  The step (queue
 * reset, attempts, sync points, exchange rounds, counters) is captured once
 * in a HIP graph and replayed.  Whatever the plan, every instance ends in the
 * bit-identical state rewl_run_attempts gives it alone (the plan changes only
 * where and when a walker's attempts run).
 * Instances must share `precision`; each keeps its own seed and `instance`
 * counter bits (give instances distinct `instance` values or seeds, else
 * equal inputs give equal streams).                                          */
typedef struct rewl_batch rewl_batch_t; /* opaque, owned by the library */

typedef struct {
    int32_t model;          /* REWL_POTTS2D */
    int32_t L, q, windows, walkers;
    int32_t reserved;
    double overlap;
    rewl_opts opts;
} rewl_instance;

typedef struct {
    int32_t walkers_per_cu; /* persistent grid = walkers_per_cu x CUs workgroups    */
    int32_t tag_policy;     /* 0: each instance's conflict-tag table as large as the */
                            /*    LDS share 160 KiB / walkers_per_cu allows;         */
                            /*    1: 64-entry tables (least LDS, more recomputation) */
    int32_t use_graph;      /* 1: replay a captured HIP graph per step; 0: launch    */
    int32_t lds_bytes;      /* out: LDS per workgroup of the attempt kernel          */
    int32_t grid;           /* out: workgroups of the attempt kernel                 */
    int32_t resident;       /* out: workgroups per CU the occupancy calculator allows */
    double ms_per_step;     /* out (rewl_batch_tune): measured ms per batched step   */
    /* Mixed-slot form (mixed = 1): one workgroup per CU whose wavefronts own LDS
     * slots sized per instance class (classes = instances of equal LDS need,
     * largest first, at most 8); a wave serves its class, then the smaller ones.
     * walkers_per_cu and tag_policy are then ignored.                          */
    int32_t mixed;
    int32_t tag_bytes;      /* mixed: conflict-tag table of a walker at most this    */
                            /*    many bytes (power-of-two entries, >= 64)           */
    int32_t slot_count[8];  /* mixed: slots per CU of each class (sum <= 16)         */
    int32_t nclasses;       /* out: instance classes of the batch                    */
    int32_t class_lds[8];   /* out: LDS bytes of a walker of each class              */
} rewl_batch_plan;

/* Device workspace for these instances (bytes), 0 if any is invalid.        */
size_t rewl_batch_workspace_bytes(int n, const rewl_instance *inst);

/* Create a batch of n instances.  init_spins: host int8, the starting lattices
 * of instance 0's walkers, then instance 1's, ... (windows*walkers*L*L values
 * per instance).  dev_workspace / ws_bytes / hip_stream as for rewl_create.
 * The initial plan is the one rewl_batch_set_plan picks for walkers_per_cu =
 * 0 (the most resident walkers per CU with tag_policy 0).                   */
int rewl_batch_create(rewl_batch_t **out, int n, const rewl_instance *inst, const int8_t *init_spins,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream);
void rewl_batch_destroy(rewl_batch_t *b);

/* Handle of instance i, for every single-run query (rewl_get_walker,
 * rewl_get_window, rewl_get_lng, rewl_join, rewl_thermo, ...).  The batch
 * owns it: rewl_destroy ignores it, and it dies with the batch.             */
int rewl_batch_instance(rewl_batch_t *b, int i, rewl_t **out);

/* Walk-in of every walker of every instance in one launch per chunk (see
 * rewl_walkin).  Called with a budget of 2^40 by the first batched step.    */
int rewl_batch_walkin(rewl_batch_t *b, int64_t max_attempts);

/* Set the launch plan (walkers_per_cu = 0: the largest count the occupancy
 * calculator allows).  Fills the out fields.  REWL_EINVAL if the LDS of an
 * instance does not fit the share or the CU cannot hold that many walkers.  */
int rewl_batch_set_plan(rewl_batch_t *b, rewl_batch_plan *plan);
int rewl_batch_get_plan(rewl_batch_t *b, rewl_batch_plan *plan);

/* Autotuner: time `steps_per_plan` batched steps under every feasible plan
 * (uniform: walkers per CU from 1 to the occupancy limit x both tag policies;
 * mixed-slot: slot mixes proportional to each class's work for several slot
 * totals and tag-table sizes), keep the fastest (with use_graph = 1).  The trial steps are ordinary steps of the
 * runs (results do not depend on the plan).  tried: host array of `cap`
 * plans (may be NULL) receiving every trial with its ms_per_step; *n_tried
 * the number of trials.                                                      */
int rewl_batch_tune(rewl_batch_t *b, int steps_per_plan, rewl_batch_plan *tried, int cap, int *n_tried);

/* `steps` batched steps under the current plan.  Every instance's step must
 * be a multiple of its sync_attempts (true unless the instance handles were
 * run on their own).  REWL_CONVERGED once every instance has converged.     */
int rewl_batch_run(rewl_batch_t *b, int64_t steps);

/* Same steps with one launch per instance for each kernel (attempts, sync
 * point, exchange, counters): the one-run-at-a-time baseline of the batched
 * form.  Results are identical to rewl_batch_run.                           */
int rewl_batch_run_per_instance(rewl_batch_t *b, int64_t steps);

/* Bootstrap error analysis over the instances of a batch (Sec. 2: repeat the
 * simulation, resample, and join every resampled g(E) anew, so the joining
 * points move).  The R instances must be independent converged runs of one
 * Potts system (same L, q, windows, overlap and walkers; different seeds or
 * instance ids).  Replicate j draws R instances with replacement (Philox4x32-10
 * keyed by `seed`, block (j, i/4, 0, 7 << 24), index floor(w R / 2^32) for
 * its four words w), averages their final ln g window by window (summed in
 * draw order, divided by R), joins the pieces over the union of the runs'
 * visited flags, normalises to q^N and evaluates U and C_v at the nT
 * temperatures T.  Outputs, host double buffers: lng_mean/lng_std[B] (mean
 * and sample standard deviation over the replicates where ln g is finite;
 * -inf and 0 where it never is), U_mean/U_std/C_mean/C_std[nT] (may be NULL
 * when nT = 0).  dev_scratch: device memory of rewl_batch_bootstrap_bytes
 * bytes, owned by the caller.  Errors: REWL_EINVAL (null argument, nboot
 * outside [1, 65535], nT outside [0, 4096], T <= 0, instances of different
 * systems, scratch too small), REWL_ESTATE (an instance not converged, or a
 * resample without a common visited bin for a pair of windows).              */
size_t rewl_batch_bootstrap_bytes(rewl_batch_t *b, int nboot, int nT);
int rewl_batch_bootstrap(rewl_batch_t *b, int nboot, uint64_t seed, const double *T, int nT, void *dev_scratch,
                         size_t scratch_bytes, double *lng_mean, double *lng_std, double *U_mean, double *U_std,
                         double *C_mean, double *C_std);

/* Batched steps done by the batch, and how many instances have converged.   */
int rewl_batch_progress(rewl_batch_t *b, int64_t *steps, int32_t *converged);

/* While enabled, HIP events on the batch's stream bracket every batched step
 * (graph replay or launches); rewl_batch_get_timing returns the summed
 * milliseconds and step count since timing was last enabled.                */
int rewl_batch_set_timing(rewl_batch_t *b, int enable);
int rewl_batch_get_timing(rewl_batch_t *b, double *ms, int64_t *steps);

#ifdef __cplusplus
}
#endif

#endif /* REWL_H */
