/*
 * rewl_oracle.c -- plain, sequential CPU reference of Replica-Exchange
 * Wang-Landau (REWL) sampling, written for checking the GPU library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the HIP
 * library: every routine below is written out from the paper and from the
 * published definitions it names.
 *
 * Paper: T. Vogel, Y. W. Li, T. Wuest, D. P. Landau, "Exploring new
 * frontiers in statistical physics with a new, parallel Wang-Landau
 * framework", J. Phys.: Conf. Ser. (2014).  Citations below give the section,
 * equation or figure of that paper.
 *
 * Arithmetic is IEEE binary64 unless a routine says otherwise.  Build with
 * -ffp-contract=off (no fused multiply-add) and without -ffast-math: the
 * acceptance decisions must follow the exact operation order written here.
 *
 * Parity status: every routine has a pin in tests/ (rocRAND for Philox,
 * mpmath for exp_poly, brute-force enumeration for the converged density of
 * states, closed forms for the exchange rule and the thermodynamics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Status codes returned by the oracle entry points.                         */
enum { ORC_OK = 0, ORC_CONVERGED = 1, ORC_EINVAL = -1, ORC_ENOMEM = -2,
       ORC_ESTATE = -4, ORC_EBUDGET = -5 };

/* Philox counter domains: the fourth counter word carries domain << 24 | instance. */
enum { DOM_MOVE = 0, DOM_WALKIN = 2, DOM_EXCH = 3, DOM_MOVE_U = 5, DOM_WALKIN_U = 6, DOM_BOOT = 7 };

/* Models. */
enum { MODEL_POTTS2D = 0, MODEL_TRIMER3D = 1, MODEL_LIPID3D = 2 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
 * Shaw (SC'11): ten rounds of two 32x32->64 multiplications with a Weyl key
 * schedule.  The paper names no generator; this one is keyed by
 * (seed, walker, step) so every draw is reproducible independently of the
 * order in which walkers are simulated.                                      */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {               /* key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* exp(x) for x < 0 by Cody-Waite range reduction and the Taylor series of
 * degree 13 evaluated by Horner's rule, every step rounded separately.
 * Needed for the Wang-Landau acceptance min[1, g(E_old)/g(E_new)] (Sec. 2)
 * evaluated as exp(ln g(E_old) - ln g(E_new)).
 *   k = rint(x / ln 2),  r = (x - k*C1) - k*C2,  exp(x) = 2^k * exp(r).
 * C1 is ln 2 rounded to 40 significant bits (so k*C1 is exact for |k| < 2^13)
 * and C2 = ln 2 - C1 rounded to double.  Coefficients are 1/n! rounded to
 * double; n! is exact in binary64 for n <= 18 so 1.0/n! is correctly rounded. */
static const double ORC_INV_LN2 = 0x1.71547652b82fep+0;   /* RN(1/ln 2)          */
static const double ORC_LN2_C1  = 0x1.62e42fefa4000p-1;   /* ln 2, 40 bits       */
static const double ORC_LN2_C2  = -0x1.8432a1b0e2634p-43; /* RN(ln 2 - C1)       */

static double exp_poly(double x)
{
    if (x < -64.0) return 0.0;
    double kd = rint(x * ORC_INV_LN2);
    double r = (x - kd * ORC_LN2_C1) - kd * ORC_LN2_C2;
    double coef[14];
    double fact = 1.0;
    coef[0] = 1.0;
    for (int n = 1; n <= 13; ++n) { fact = fact * (double)n; coef[n] = 1.0 / fact; }
    double p = coef[13];
    for (int n = 12; n >= 0; --n) {
        double t = r * p;
        p = coef[n] + t;
    }
    return ldexp(p, (int)kd);
}

/* Single-precision twin used by the FP32 (hi, lo) ln g variant: the same
 * reduction with C1 of 16 significant bits and a degree-7 Taylor series.     */
static const float ORC_INV_LN2_F = 0x1.715476p+0f;
static const float ORC_LN2_C1_F  = 0x1.62e4p-1f;
static const float ORC_LN2_C2_F  = 0x1.7f7d1cp-20f;

static float exp_poly32(float x)
{
    if (x < -64.0f) return 0.0f;
    float kf = rintf(x * ORC_INV_LN2_F);
    float r = (x - kf * ORC_LN2_C1_F) - kf * ORC_LN2_C2_F;
    float coef[8];
    float fact = 1.0f;
    coef[0] = 1.0f;
    for (int n = 1; n <= 7; ++n) { fact = fact * (float)n; coef[n] = 1.0f / fact; }
    float p = coef[7];
    for (int n = 6; n >= 0; --n) {
        float t = r * p;
        p = coef[n] + t;
    }
    return ldexpf(p, (int)kf);
}

/* ------------------------------------------------------------------------ */
/* Energy-range splitting (Sec. 2, Fig. 1): h windows of equal size W with a
 * constant overlap o over the B = 2N+1 integer energies of the Potts model.
 * W = ceil(B / (1 + (h-1)(1-o))); window k starts at
 * E_lo + round(k (B - W) / (h - 1)) so the last window ends at E = 0.        */
static int window_layout(int B, int h, double o, int e_lo, int *W_out, int *start)
{
    if (h < 1 || !(o >= 0.0 && o < 1.0) || B < 1) return ORC_EINVAL;
    int W;
    if (h == 1) {
        W = B;
    } else {
        double denom = 1.0 + (double)(h - 1) * (1.0 - o);
        W = (int)ceil((double)B / denom);
        if (W > B) W = B;
    }
    for (int k = 0; k < h; ++k) {
        if (h == 1) { start[k] = e_lo; continue; }
        /* floor(k(B-W)/(h-1) + 1/2) in integers */
        int64_t num = 2 * (int64_t)k * (int64_t)(B - W) + (int64_t)(h - 1);
        int64_t den = 2 * (int64_t)(h - 1);
        start[k] = e_lo + (int)(num / den);
    }
    *W_out = W;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 2D q-state Potts model, Eq. (2): H = -sum over nearest-neighbour pairs of
 * delta(s_i, s_j), on an L x L periodic lattice (each bond counted once via
 * the right and lower neighbour), so E lies in [-2N, 0].                    */
static int potts_energy(const int8_t *s, int L)
{
    int e = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int i = y * L + x;
            int right = y * L + (x + 1) % L;
            int down = ((y + 1) % L) * L + x;
            if (s[i] == s[right]) e -= 1;
            if (s[i] == s[down]) e -= 1;
        }
    return e;
}

/* Energy change of setting site i to value nv (single spin flip, Sec. 3.1). */
static int potts_delta_e(const int8_t *s, int L, int i, int nv)
{
    int x = i % L, y = i / L;
    int nb[4];
    nb[0] = y * L + (x + 1) % L;
    nb[1] = y * L + (x + L - 1) % L;
    nb[2] = ((y + 1) % L) * L + x;
    nb[3] = ((y + L - 1) % L) * L + x;
    int de = 0;
    for (int t = 0; t < 4; ++t) {
        int sn = s[nb[t]];
        de += (s[i] == sn) ? 1 : 0;
        de -= (nv == sn) ? 1 : 0;
    }
    return de;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int model;             /* MODEL_POTTS2D or MODEL_TRIMER3D                 */
    /* trimer model: nmol head-tail-tail molecules (nb = 3 nmol beads, bead
     * 3i is a head, 3i+1 and 3i+2 its tails), FP32 coordinates in a periodic
     * cube of side `box`, energy bins of width bin_w from e_min             */
    int nmol, nb;
    float box;
    double e_min, bin_w;
    int64_t *Efx;          /* [nw] energy of each walker in units of 2^-32 (trimer, lipid) */
    int64_t emin_fx, binw_fx; /* e_min and bin_w in units of 2^-32          */
    /* lipid model (explicit solvent): np particles, nlip P-H-H lipids, the
     * rest solvent W; per-walker bytes: coordinates float[np][3], types
     * int8[np] (padded to 4), lipid table int32[nlip][3] (head first),
     * position table int32[np] (3 lipid + bead, -1 for solvent)            */
    int np, nlip;
    double eps_ww;         /* W-W Lennard-Jones depth                         */
    uint32_t rep_thr;      /* reptation when a 32-bit word is below this      */
    size_t off_type, off_lip, off_where;
    int L, q, N;
    int h, m, nw;          /* windows, walkers per window, walkers            */
    int W, B, e_lo;        /* bins per window, global bins, lowest energy     */
    int *start;            /* [h] lowest energy of window k                   */
    uint32_t key[2];
    uint32_t instance;
    uint32_t flat_num, flat_den;
    double lnf_init, lnf_final;
    int schedule;          /* 0: halve ln f; 1: halve, then the 1/t rule     */
    int64_t S;             /* attempts per walker between sync points        */
    int exchange;          /* exchange round at every sync point             */
    int precision;         /* 0: binary64 ln g; 1: binary32 (hi, lo) pair    */
    int fixed_lnf;         /* 1: sync points never change ln f or average    */
    int shadow;            /* 1: keep the exact reference of ln g (below)    */
    int walkin_slack;      /* walk-in lid/floor distance (0: no lid)          */
    int threads;
    /* walker state, walker w = k*m + j */
    int8_t *spin;          /* [nw][N] */
    int32_t *E;            /* [nw]    */
    double *lng;           /* [nw][W] (precision 0) */
    float *lng_hi, *lng_lo;/* [nw][W] (precision 1) */
    uint32_t *H;           /* [nw][W] */
    double *sh_hi, *sh_lo; /* [nw][W] shadow: ln g in double-double          */
    uint32_t *hprev;       /* [nw][W] H at the previous sync point           */
    uint8_t *vis;          /* [nw][W] bins this walker reached since creation */
    uint32_t *replica;     /* [nw] replica id held by walker slot w */
    int32_t *rep_end;      /* [nw] by replica id: 0 lowest window not reached yet,
                              1 lowest reached (highest not since), 2 highest since */
    uint32_t *rep_trips;   /* [nw] by replica id: completed round trips lowest-highest-lowest */
    uint32_t *rep_visits;  /* [nw][nw] lookups that found replica r in slot w (nw <= 4096) */
    /* observable O = max_s n_s (Potts), sampled at sync points              */
    int obs_bins;          /* 0: not sampled; else O bins of H(E, O)         */
    uint32_t *obs_hist;    /* [nw][W][obs_bins] H(E, O) per walker           */
    uint64_t *obs_sum;     /* [nw][W] sum of O per energy bin                */
    uint32_t *obs_cnt;     /* [nw][W] samples per energy bin                 */
    int production;        /* 1: weights frozen, no termination              */
    int64_t *walkin_att;   /* [nw] */
    /* window state */
    double *lnf;           /* [h] current ln f (0 once finished)             */
    double *lnf_last;      /* [h] ln f value at which the window finished     */
    int32_t *regime;       /* [h] 0 halving, 1 1/t                           */
    int32_t *finished;     /* [h] */
    int64_t *iterations;   /* [h] ln f reductions so far                      */
    uint8_t *visited;      /* [h][W] union of the walkers' visited bins       */
    uint64_t *x_att, *x_acc;/* [h] exchange attempts/accepts of pair (k,k+1)  */
    int64_t step;          /* main-phase attempts per walker                  */
    int64_t round;         /* exchange rounds performed                       */
    int walked_in;
    int converged;
} orc_t;

static void orc_free(orc_t *o)
{
    if (!o) return;
    free(o->start); free(o->spin); free(o->E); free(o->lng); free(o->lng_hi);
    free(o->lng_lo); free(o->H); free(o->sh_hi); free(o->sh_lo); free(o->hprev); free(o->vis); free(o->replica); free(o->walkin_att);
    free(o->lnf); free(o->lnf_last); free(o->regime); free(o->finished);
    free(o->iterations); free(o->visited); free(o->x_att); free(o->x_acc);
    free(o->Efx); free(o->rep_end); free(o->rep_trips); free(o->rep_visits);
    free(o->obs_hist); free(o->obs_sum); free(o->obs_cnt);
    free(o);
}

void orc_destroy(orc_t *o) { orc_free(o); }

/* Replica-path diagnostics (Sec. 3.2, Fig. 7): the position of every replica
 * is looked up at creation, at every sync point (after its exchange round)
 * and after every exchange round called on its own.  Each lookup adds one to
 * visits[w][r] for the replica r held by walker slot w.  A round trip is a
 * path from the lowest window to the highest and back to the lowest; the
 * return to the lowest window completes one and starts the next.           */
static void replica_track(orc_t *o)
{
    if (o->rep_visits)
        for (int w = 0; w < o->nw; ++w) o->rep_visits[(size_t)w * o->nw + o->replica[w]] += 1;
    if (o->h < 2) return;
    for (int w = 0; w < o->nw; ++w) {
        int k = w / o->m;
        uint32_t r = o->replica[w];
        if (k == 0) {
            if (o->rep_end[r] == 2) o->rep_trips[r] += 1;
            o->rep_end[r] = 1;
        } else if (k == o->h - 1 && o->rep_end[r] == 1) {
            o->rep_end[r] = 2;
        }
    }
}

void orc_get_replicas(const orc_t *o, uint32_t *window_of, uint32_t *trips)
{
    for (int w = 0; w < o->nw; ++w) {
        if (window_of) window_of[o->replica[w]] = (uint32_t)(w / o->m);
    }
    if (trips) for (int r = 0; r < o->nw; ++r) trips[r] = o->rep_trips[r];
}

/* counts[r] = lookups that found replica r in walker slot w; -1 if the
 * matrix is not kept (more than 4096 walkers).                              */
int orc_get_replica_visits(const orc_t *o, int w, uint32_t *counts)
{
    if (!o->rep_visits || w < 0 || w >= o->nw) return ORC_EINVAL;
    memcpy(counts, o->rep_visits + (size_t)w * o->nw, (size_t)o->nw * sizeof(uint32_t));
    return ORC_OK;
}

/* Exposed for the tests. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox4x32_10(ctr, key, out); }
double orc_exp_poly(double x) { return exp_poly(x); }
float orc_exp_poly32(float x) { return exp_poly32(x); }
int orc_window_layout(int B, int h, double o, int e_lo, int *W, int *start)
{
    return window_layout(B, h, o, e_lo, W, start);
}
int orc_potts_energy(const int8_t *s, int L) { return potts_energy(s, L); }
void orc_constants(double *c) { c[0] = ORC_INV_LN2; c[1] = ORC_LN2_C1; c[2] = ORC_LN2_C2; }
void orc_constants32(float *c) { c[0] = ORC_INV_LN2_F; c[1] = ORC_LN2_C1_F; c[2] = ORC_LN2_C2_F; }

/* Options and state arrays shared by both models: B energy bins from e_lo,
 * N bytes of configuration per walker.  Returns NULL on invalid options.    */
static orc_t *orc_new(int B, int e_lo, int N, int h, double overlap, int m, uint64_t seed,
                      uint32_t instance, uint32_t flat_num, uint32_t flat_den, double lnf_init,
                      double lnf_final, int schedule, int64_t sync_attempts, int exchange,
                      int precision, int fixed_lnf, int shadow, int walkin_slack)
{
    if (h < 1 || m < 1) return NULL;
    if (!(overlap >= 0.0 && overlap < 1.0)) return NULL;
    if (flat_den == 0 || flat_den > 1000 || flat_num > flat_den) return NULL;
    if (sync_attempts < 1 || precision < 0 || precision > 1 || schedule < 0 || schedule > 1) return NULL;
    if (walkin_slack < 0) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    if (!o) return NULL;
    o->N = N; o->h = h; o->m = m; o->nw = h * m;
    o->B = B; o->e_lo = e_lo;
    o->start = (int *)calloc((size_t)h, sizeof(int));
    if (!o->start || window_layout(o->B, h, overlap, o->e_lo, &o->W, o->start) != ORC_OK || o->W < 8) {
        orc_free(o);
        return NULL;
    }
    o->key[0] = (uint32_t)seed; o->key[1] = (uint32_t)(seed >> 32);
    o->instance = instance & 0xFFFFFFu;
    o->flat_num = flat_num; o->flat_den = flat_den;
    o->lnf_init = lnf_init; o->lnf_final = lnf_final;
    o->schedule = schedule; o->S = sync_attempts; o->exchange = exchange;
    o->precision = precision; o->fixed_lnf = fixed_lnf; o->shadow = shadow != 0; o->threads = 1;
    o->walkin_slack = walkin_slack;
    size_t nw = (size_t)o->nw, W = (size_t)o->W;
    o->spin = (int8_t *)malloc(nw * (size_t)N);
    o->E = (int32_t *)calloc(nw, sizeof(int32_t));
    if (precision == 0) o->lng = (double *)calloc(nw * W, sizeof(double));
    else { o->lng_hi = (float *)calloc(nw * W, sizeof(float)); o->lng_lo = (float *)calloc(nw * W, sizeof(float)); }
    o->H = (uint32_t *)calloc(nw * W, sizeof(uint32_t));
    if (o->shadow) {
        o->sh_hi = (double *)calloc(nw * W, sizeof(double));
        o->sh_lo = (double *)calloc(nw * W, sizeof(double));
        o->hprev = (uint32_t *)calloc(nw * W, sizeof(uint32_t));
        if (!o->sh_hi || !o->sh_lo || !o->hprev) { orc_free(o); return NULL; }
    }
    o->vis = (uint8_t *)calloc(nw * W, 1);
    o->replica = (uint32_t *)calloc(nw, sizeof(uint32_t));
    o->rep_end = (int32_t *)calloc(nw, sizeof(int32_t));
    o->rep_trips = (uint32_t *)calloc(nw, sizeof(uint32_t));
    if (nw <= 4096) {
        o->rep_visits = (uint32_t *)calloc((size_t)nw * nw, sizeof(uint32_t));
        if (!o->rep_visits) { orc_free(o); return NULL; }
    }
    o->walkin_att = (int64_t *)calloc(nw, sizeof(int64_t));
    o->lnf = (double *)calloc((size_t)h, sizeof(double));
    o->lnf_last = (double *)calloc((size_t)h, sizeof(double));
    o->regime = (int32_t *)calloc((size_t)h, sizeof(int32_t));
    o->finished = (int32_t *)calloc((size_t)h, sizeof(int32_t));
    o->iterations = (int64_t *)calloc((size_t)h, sizeof(int64_t));
    o->visited = (uint8_t *)calloc((size_t)h * W, 1);
    o->x_att = (uint64_t *)calloc((size_t)h, sizeof(uint64_t));
    o->x_acc = (uint64_t *)calloc((size_t)h, sizeof(uint64_t));
    if (!o->spin || !o->E || !(o->lng || (o->lng_hi && o->lng_lo)) || !o->H || !o->vis ||
        !o->replica || !o->rep_end || !o->rep_trips || !o->walkin_att || !o->lnf || !o->lnf_last || !o->regime ||
        !o->finished || !o->iterations || !o->visited || !o->x_att || !o->x_acc) {
        orc_free(o);
        return NULL;
    }
    for (int w = 0; w < o->nw; ++w) o->replica[w] = (uint32_t)w;
    replica_track(o);
    for (int k = 0; k < h; ++k) o->lnf[k] = lnf_init;
    return o;
}

/* Create a REWL run of the 2D Potts model: h windows with overlap o and m
 * walkers each (Sec. 2).  init_spins holds one starting lattice per walker
 * ([h*m][L*L], values in [0, q)).  Returns NULL on invalid arguments.       */
orc_t *orc_create(int L, int q, int h, double overlap, int m, uint64_t seed, uint32_t instance,
                  uint32_t flat_num, uint32_t flat_den, double lnf_init, double lnf_final,
                  int schedule, int64_t sync_attempts, int exchange, int precision, int fixed_lnf,
                  int shadow, int walkin_slack, int obs_bins, const int8_t *init_spins)
{
    if (L < 3 || L > 724 || q < 2 || q > 127) return NULL;
    if (!init_spins) return NULL;
    int N = L * L;
    if (obs_bins < 0 || obs_bins > N + 1) return NULL;
    orc_t *o = orc_new(2 * N + 1, -2 * N, N, h, overlap, m, seed, instance, flat_num, flat_den,
                       lnf_init, lnf_final, schedule, sync_attempts, exchange, precision, fixed_lnf,
                       shadow, walkin_slack);
    if (!o) return NULL;
    o->model = MODEL_POTTS2D;
    o->L = L; o->q = q;
    size_t nw = (size_t)o->nw;
    for (size_t i = 0; i < nw * (size_t)N; ++i) {
        if (init_spins[i] < 0 || init_spins[i] >= q) { orc_free(o); return NULL; }
        o->spin[i] = init_spins[i];
    }
    for (int w = 0; w < o->nw; ++w) o->E[w] = potts_energy(o->spin + (size_t)w * N, L);
    o->obs_bins = obs_bins;
    if (obs_bins > 0) {
        size_t cells = nw * (size_t)o->W;
        o->obs_hist = (uint32_t *)calloc(cells * (size_t)obs_bins, sizeof(uint32_t));
        o->obs_sum = (uint64_t *)calloc(cells, sizeof(uint64_t));
        o->obs_cnt = (uint32_t *)calloc(cells, sizeof(uint32_t));
        if (!o->obs_hist || !o->obs_sum || !o->obs_cnt) { orc_free(o); return NULL; }
    }
    return o;
}

void orc_set_threads(orc_t *o, int n) { o->threads = n < 1 ? 1 : n; }

/* ------------------------------------------------------------------------ */
/* ln g of walker w at bin b, as a binary64 value (the (hi, lo) pair is summed
 * in binary64 for the exchange, averaging and joining steps).               */
static double lng_get(const orc_t *o, int w, int b)
{
    size_t i = (size_t)w * o->W + b;
    if (o->precision == 0) return o->lng[i];
    return (double)o->lng_hi[i] + (double)o->lng_lo[i];
}

/* The accept test of one Wang-Landau move (Sec. 2): accept with probability
 * min[1, g(E_old)/g(E_new)], decided as  d >= 0  or  u < exp(d)  with
 * d = ln g(E_old) - ln g(E_new) and u = r/2^32 from one 32-bit random word. */
static int accept64(double d, uint32_t r)
{
    if (d >= 0.0) return 1;
    double u = (double)r * 0x1p-32;
    return u < exp_poly(d);
}

/* The same test on the binary32 (hi, lo) representation: d is formed in
 * binary32 as (hi_old - hi_new) + (lo_old - lo_new) and compared with a
 * 24-bit uniform u = (r >> 8) / 2^24, exact in binary32.                    */
static int accept32(float d, uint32_t r)
{
    if (d >= 0.0f) return 1;
    float u = (float)(r >> 8) * 0x1p-24f;
    return u < exp_poly32(d);
}

/* Knuth's TwoSum: ln g(E) += ln f on the (hi, lo) pair; the rounding error
 * of the high part is carried into the low part.                            */
static void twosum_add(float *hi, float *lo, float x)
{
    float s = *hi + x;
    float bb = s - *hi;
    float err = (*hi - (s - bb)) + (x - bb);
    *hi = s;
    *lo = *lo + err;
}

/* Exposed for the tests: n additions of x to the pair (hi, lo).            */
void orc_twosum_accumulate(float *hi, float *lo, float x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) twosum_add(hi, lo, x);
}

/* One Wang-Landau attempt of walker w in window k (Sec. 2, Sec. 3.1):
 * propose a single spin flip, accept with min[1, g(E_old)/g(E_new)] (moves
 * leaving the window are rejected), then g(E) -> f g(E) and H(E) += 1 at the
 * energy after the decision.  ctr selects the Philox draw.                  */
static void potts_attempt(orc_t *o, int w, int k, double lnf, uint32_t domain, uint64_t cnt)
{
    int N = o->N, L = o->L, q = o->q, W = o->W;
    int8_t *s = o->spin + (size_t)w * N;
    uint32_t ctr[4] = { (uint32_t)cnt, (uint32_t)(cnt >> 32), (uint32_t)w, (domain << 24) | o->instance };
    uint32_t r[4];
    philox4x32_10(ctr, o->key, r);
    int i = (int)(((uint64_t)r[0] * (uint64_t)N) >> 32);
    int off = (int)(((uint64_t)r[1] * (uint64_t)(q - 1)) >> 32);
    int nv = s[i] + 1 + off;
    if (nv >= q) nv -= q;
    int e_old = o->E[w];
    int e_new = e_old + potts_delta_e(s, L, i, nv);
    int lo = o->start[k], hi = o->start[k] + W - 1;
    int acc = 0;
    if (e_new >= lo && e_new <= hi) {
        int bo = e_old - lo, bn = e_new - lo;
        if (o->precision == 0) {
            double d = o->lng[(size_t)w * W + bo] - o->lng[(size_t)w * W + bn];
            acc = accept64(d, r[2]);
        } else {
            size_t io = (size_t)w * W + bo, in = (size_t)w * W + bn;
            float d = (o->lng_hi[io] - o->lng_hi[in]) + (o->lng_lo[io] - o->lng_lo[in]);
            acc = accept32(d, r[2]);
        }
    }
    if (acc) {
        s[i] = (int8_t)nv;
        o->E[w] = e_new;
    }
    int b = o->E[w] - lo;
    size_t ib = (size_t)w * W + b;
    if (o->precision == 0) o->lng[ib] += lnf;
    else twosum_add(&o->lng_hi[ib], &o->lng_lo[ib], (float)lnf);
    o->H[ib] += 1u;
    if (!o->finished[k]) o->vis[ib] = 1;
}

/* ------------------------------------------------------------------------ */
/* Coarse-grained amphiphile of three beads, head-tail-tail (the paper's lipid
 * model, Sec. 3.2, is a bead-spring amphiphile sampled with local bead
 * displacements; this workload keeps that structure with a simpler force
 * field): bonds H-T1 and T1-T2 are harmonic, k (r - r0)^2 with k = 100,
 * r0 = 1 (no factor 1/2); every other pair interacts by Lennard-Jones,
 * 4 (r^-12 - r^-6) (sigma = epsilon = 1): tail-tail pairs cut at r = 2.5
 * without shift, every pair involving a head cut at r = 2^(1/6) and shifted
 * by +1 (WCA).  Periodic cube, minimum image per axis in binary32; pair
 * energies in binary64 from the binary32 coordinate differences; the bond
 * length by the correctly rounded binary64 square root.                    */
static const double TRI_K = 100.0;
static const double TRI_R0 = 1.0;
static const double TRI_LJ_RC2 = 6.25;                    /* 2.5^2                 */
static const double TRI_WCA_RC2 = 0x1.428a2f98d728bp+0;   /* RN(2^(1/3)) = RN((2^(1/6))^2) */

static void tri_min_image(float box, const float *a, const float *b, double d[3])
{
    float half = 0.5f * box;
    for (int c = 0; c < 3; ++c) {
        float x = b[c] - a[c];
        if (x > half) x = x - box;
        else if (x < -half) x = x + box;
        d[c] = (double)x;
    }
}

static double tri_pair(const orc_t *o, int i, int j, const float *xi, const float *xj)
{
    double d[3];
    tri_min_image(o->box, xi, xj, d);
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    int ti = i % 3, tj = j % 3;
    if (i / 3 == j / 3 && (ti - tj == 1 || tj - ti == 1)) {
        double x = sqrt(r2) - TRI_R0;
        return TRI_K * (x * x);
    }
    int tails = ti > 0 && tj > 0;
    if (r2 >= (tails ? TRI_LJ_RC2 : TRI_WCA_RC2)) return 0.0;
    double s2 = 1.0 / r2;
    double s6 = (s2 * s2) * s2;
    double v = 4.0 * ((s6 * s6) - s6);
    return tails ? v : v + 1.0;
}

/* ------------------------------------------------------------------------ */
/* Energies of the continuous models (trimer, lipid) in fixed point.  Each
 * pair term V of the force field (binary64) is rounded once to a multiple of
 * 2^-32, fx(V) = rint(V 2^32); a total or a change of energy is the exact
 * integer sum of such terms, so it is the same in whatever order the terms
 * are added, and a change always equals the difference of the two totals.
 * A term of magnitude 2^18 or more, or one that is not finite, is a hard
 * overlap: a configuration never holds one (a move that would create one is
 * rejected, a start that holds one is refused).  Energies must stay below
 * 2^29 in magnitude (2^61 units).  The bin of an energy E is
 * floor((E - e_min) / bin_w) on the same grid.                              */
static const double FX_ONE = 0x1p32;
static const double FX_TERM_LIMIT = 0x1p18;
#define FX_E_LIMIT (((__int128)1) << 61)

static int fx_term(double v, int64_t *out)
{
    if (!(fabs(v) < FX_TERM_LIMIT)) return 0;
    *out = (int64_t)rint(v * FX_ONE);
    return 1;
}

static int fx_in_range(__int128 e) { return e < FX_E_LIMIT && e > -FX_E_LIMIT; }

static double fx_to_double(int64_t e) { return (double)e / FX_ONE; }

/* Total energy, every pair i < j (only at creation and in the tests). */
static int tri_energy(const orc_t *o, const float *x, int64_t *e)
{
    __int128 acc = 0;
    for (int i = 0; i < o->nb; ++i)
        for (int j = i + 1; j < o->nb; ++j) {
            int64_t t;
            if (!fx_term(tri_pair(o, i, j, x + 3 * i, x + 3 * j), &t)) return 0;
            acc += t;
        }
    if (!fx_in_range(acc)) return 0;
    *e = (int64_t)acc;
    return 1;
}

/* Energy change of moving bead b to xn: the sum over its partners j of
 * fx(V(b at xn, j)) - fx(V(b, j)).  0 if a term is a hard overlap.         */
static int tri_delta_e(const orc_t *o, const float *x, int b, const float *xn, int64_t *de)
{
    __int128 acc = 0;
    for (int j = 0; j < o->nb; ++j) {
        if (j == b) continue;
        int64_t tn, to;
        if (!fx_term(tri_pair(o, b, j, xn, x + 3 * j), &tn)) return 0;
        if (!fx_term(tri_pair(o, b, j, x + 3 * b, x + 3 * j), &to)) return 0;
        acc += (__int128)tn - (__int128)to;
    }
    *de = (int64_t)acc;
    return 1;
}

/* Energy bin: floor((E - e_min) / bin_w) in units of 2^-32, also outside
 * [0, B) (bounded to +-2^30), so that the walk-in's lid can follow energies
 * above the range.                                                          */
static int tri_bin(const orc_t *o, int64_t e)
{
    int64_t diff = e - o->emin_fx;
    int64_t q = diff / o->binw_fx;
    if (diff % o->binw_fx != 0 && diff < 0) q -= 1;
    if (q < -1073741824) return -1073741824;
    if (q > 1073741824) return 1073741824;
    return (int)q;
}

/* New energy of a valid move, or 0 if it leaves the energy range.          */
static int fx_add(int64_t e, int64_t de, int64_t *out)
{
    __int128 s = (__int128)e + (__int128)de;
    if (!fx_in_range(s)) return 0;
    *out = (int64_t)s;
    return 1;
}

/* Displacement of one axis, uniform in [-0.1, 0.1) (0.1 (2u - 1) with u a
 * 23-bit uniform), and the periodic wrap into [0, box).                    */
static float tri_disp(uint32_t r) { return 0.1f * ((float)(r >> 9) * 0x1p-22f - 1.0f); }
static float tri_wrap(float v, float box)
{
    if (v < 0.0f) v = v + box;
    if (v >= box) v = v - box;
    return v;
}

/* One bead-displacement attempt of walker w (Wang-Landau acceptance as in
 * potts_attempt, on energy bins).  Philox block (step, walker, MOVE): bead,
 * dx, dy, dz; block (step, walker, MOVE_U): the uniform word.               */
static void trimer_attempt(orc_t *o, int w, int k, double lnf, uint64_t cnt)
{
    int W = o->W;
    float *x = (float *)(o->spin + (size_t)w * o->N);
    uint32_t ctr[4] = { (uint32_t)cnt, (uint32_t)(cnt >> 32), (uint32_t)w,
                        ((uint32_t)DOM_MOVE << 24) | o->instance };
    uint32_t r[4], ru[4];
    philox4x32_10(ctr, o->key, r);
    ctr[3] = ((uint32_t)DOM_MOVE_U << 24) | o->instance;
    philox4x32_10(ctr, o->key, ru);
    int b = (int)(((uint64_t)r[0] * (uint64_t)o->nb) >> 32);
    float xn[3];
    for (int c = 0; c < 3; ++c) xn[c] = tri_wrap(x[3 * b + c] + tri_disp(r[1 + c]), o->box);
    int64_t de = 0, e_new = 0;
    int ok = tri_delta_e(o, x, b, xn, &de) && fx_add(o->Efx[w], de, &e_new);
    int bn = ok ? tri_bin(o, e_new) : 0;
    int lo = o->start[k], hi = o->start[k] + W - 1;
    int acc = 0;
    if (ok && bn >= lo && bn <= hi) {
        size_t io = (size_t)w * W + (o->E[w] - lo), in = (size_t)w * W + (bn - lo);
        if (o->precision == 0) {
            acc = accept64(o->lng[io] - o->lng[in], ru[0]);
        } else {
            float d = (o->lng_hi[io] - o->lng_hi[in]) + (o->lng_lo[io] - o->lng_lo[in]);
            acc = accept32(d, ru[0]);
        }
    }
    if (acc) {
        for (int c = 0; c < 3; ++c) x[3 * b + c] = xn[c];
        o->Efx[w] = e_new;
        o->E[w] = bn;
    }
    size_t ib = (size_t)w * W + (o->E[w] - lo);
    if (o->precision == 0) o->lng[ib] += lnf;
    else twosum_add(&o->lng_hi[ib], &o->lng_lo[ib], (float)lnf);
    o->H[ib] += 1u;
    if (!o->finished[k]) o->vis[ib] = 1;
}

/* Walk-in of a trimer walker: the Potts walk-in rule on energy bins (counts
 * over the B bins, an energy outside the range counted at the nearest end
 * bin), same lid.                                                           */
static int trimer_walkin(orc_t *o, int w, int64_t max_attempts)
{
    int k = w / o->m;
    int lo = o->start[k], hi = o->start[k] + o->W - 1;
    float *x = (float *)(o->spin + (size_t)w * o->N);
    double *g = (double *)calloc((size_t)o->B, sizeof(double));
    if (!g) return ORC_ENOMEM;
    int64_t t = 0;
    int slack = o->walkin_slack;
    int down = o->E[w] > hi;
    int bound = down ? o->E[w] + slack : o->E[w] - slack;
    int status = ORC_OK;
    while (!(o->E[w] >= lo && o->E[w] <= hi)) {
        if (t >= max_attempts) { status = ORC_EBUDGET; break; }
        uint32_t ctr[4] = { (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)w,
                            ((uint32_t)DOM_WALKIN << 24) | o->instance };
        uint32_t r[4], ru[4];
        philox4x32_10(ctr, o->key, r);
        ctr[3] = ((uint32_t)DOM_WALKIN_U << 24) | o->instance;
        philox4x32_10(ctr, o->key, ru);
        int b = (int)(((uint64_t)r[0] * (uint64_t)o->nb) >> 32);
        float xn[3];
        for (int c = 0; c < 3; ++c) xn[c] = tri_wrap(x[3 * b + c] + tri_disp(r[1 + c]), o->box);
        int64_t de = 0, e_new = 0;
        int ok = tri_delta_e(o, x, b, xn, &de) && fx_add(o->Efx[w], de, &e_new);
        int bn = ok ? tri_bin(o, e_new) : 0;
        int co = o->E[w] < 0 ? 0 : (o->E[w] >= o->B ? o->B - 1 : o->E[w]);
        int cn = bn < 0 ? 0 : (bn >= o->B ? o->B - 1 : bn);
        double d = g[co] - g[cn];
        int inside = slack == 0 || (down ? bn <= bound : bn >= bound);
        if (ok && inside && accept64(d, ru[0])) {
            for (int c = 0; c < 3; ++c) x[3 * b + c] = xn[c];
            o->Efx[w] = e_new;
            o->E[w] = bn;
            if (slack && down && o->E[w] + slack < bound) bound = o->E[w] + slack;
            if (slack && !down && o->E[w] - slack > bound) bound = o->E[w] - slack;
        }
        int ci = o->E[w] < 0 ? 0 : (o->E[w] >= o->B ? o->B - 1 : o->E[w]);
        g[ci] += 1.0;
        ++t;
    }
    o->walkin_att[w] = t;
    free(g);
    return status;
}

/* Create a REWL run of the trimer model: nmol molecules in a periodic cube
 * of side box; `bins` energy bins of width bin_w from e_min; windows as for
 * the Potts model, over the bins.  init_coords: [h*m][3 nmol][3] binary32
 * positions in [0, box).  Returns NULL on invalid arguments.               */
orc_t *orc_create_trimer(int nmol, float box, double e_min, double bin_w, int bins, int h,
                         double overlap, int m, uint64_t seed, uint32_t instance, uint32_t flat_num,
                         uint32_t flat_den, double lnf_init, double lnf_final, int schedule,
                         int64_t sync_attempts, int exchange, int precision, int fixed_lnf, int shadow,
                         int walkin_slack, const float *init_coords)
{
    if (nmol < 1 || nmol > 1024 || !(box > 0.0f) || !(bin_w * FX_ONE >= 1.0 && bin_w * FX_ONE <= 0x1p60) ||
        !(fabs(e_min) < 0x1p28) || bins < 8 || !init_coords)
        return NULL;
    int nb = 3 * nmol;
    orc_t *o = orc_new(bins, 0, nb * 3 * (int)sizeof(float), h, overlap, m, seed, instance, flat_num,
                       flat_den, lnf_init, lnf_final, schedule, sync_attempts, exchange, precision,
                       fixed_lnf, shadow, walkin_slack);
    if (!o) return NULL;
    o->model = MODEL_TRIMER3D;
    o->nmol = nmol; o->nb = nb; o->box = box; o->e_min = e_min; o->bin_w = bin_w;
    o->emin_fx = (int64_t)rint(e_min * FX_ONE);
    o->binw_fx = (int64_t)rint(bin_w * FX_ONE);
    o->Efx = (int64_t *)calloc((size_t)o->nw, sizeof(int64_t));
    if (!o->Efx) { orc_free(o); return NULL; }
    for (int w = 0; w < o->nw; ++w) {
        float *x = (float *)(o->spin + (size_t)w * o->N);
        for (int i = 0; i < 3 * nb; ++i) {
            float v = init_coords[(size_t)w * 3 * nb + i];
            if (!(v >= 0.0f && v < box)) { orc_free(o); return NULL; }
            x[i] = v;
        }
        if (!tri_energy(o, x, &o->Efx[w])) { orc_free(o); return NULL; }
        o->E[w] = tri_bin(o, o->Efx[w]);
    }
    return o;
}

/* Test exports of the trimer model. */
/* Energies in units of 2^-32 (fixed point); the return value is 0 for a
 * hard overlap.                                                             */
int orc_trimer_energy_fx(const orc_t *o, int w, int64_t *e)
{
    return tri_energy(o, (const float *)(o->spin + (size_t)w * o->N), e);
}
int64_t orc_get_energy_fx(const orc_t *o, int w) { return o->model != MODEL_POTTS2D ? o->Efx[w] : (int64_t)o->E[w]; }
double orc_get_energy(const orc_t *o, int w) { return o->model != MODEL_POTTS2D ? fx_to_double(o->Efx[w]) : (double)o->E[w]; }
int orc_trimer_delta_fx(const orc_t *o, int w, int b, const float *xn, int64_t *de)
{
    return tri_delta_e(o, (const float *)(o->spin + (size_t)w * o->N), b, xn, de);
}

/* ------------------------------------------------------------------------ */
/* Lipid model with explicit solvent (Sec. 3.2, Eqs. (3)-(5), Fig. 5).
 * Particles: nlip amphiphiles of a polar head P and two hydrophobic tails H
 * (P-H-H), the rest solvent W, in a periodic cube.  Non-bonded pairs: H-W
 * and H-P repel by 4 (1.05/r)^9 (Eq. 3); all other pairs (H-H, P-P, P-W,
 * W-W) are Lennard-Jones 4 eps (r^-12 - r^-6) (Eq. 4) with eps = 1, or
 * eps_ww for W-W; both cut at r = 2.5 without shift.  Bonded neighbours of a
 * lipid: FENE with K = 30, R = 1.3 plus the WCA repulsion (LJ + 1 below
 * 2^(1/6), 0 above) (Eq. 5); r >= R is forbidden.  Moves: with probability
 * rep_thr / 2^32 a reptation (Fig. 5), else a displacement of one particle
 * by 0.1 (2u - 1) per axis.  Reptation: a lipid and one of its ends are
 * drawn; one of the n_c solvent particles within R of that end is captured
 * and becomes the new end bead, the lipid's beads shift along the chain and
 * the bead at the other end is released as solvent; positions do not
 * change.  The reverse move would capture the released particle among the
 * n_r solvent particles within R of the new end next to it, so the
 * acceptance carries the ratio of selection probabilities n_c / n_r.      */
static const double LIP_RC2 = 6.25;                      /* 2.5^2                 */
static const double LIP_WCA_RC2 = 0x1.428a2f98d728bp+0;  /* RN(2^(1/3))           */
static const double LIP_R2 = 1.69;                       /* FENE R^2, R = 1.3     */
static const double LIP_SQRT2 = 0x1.6a09e667f3bcdp+0;    /* RN(sqrt 2)            */
enum { LIP_P = 0, LIP_H = 1, LIP_W = 2 };

/* Natural logarithm of a positive normal x from basic IEEE operations: x =
 * 2^k m with m in [sqrt(1/2), sqrt(2)), f = (m - 1)/(m + 1), ln m = 2 atanh f
 * = 2 f (1 + s/3 + s^2/5 + ... + s^12/25) with s = f^2 by Horner (no fused
 * operations; coefficients 1/(2n + 1) rounded once), and ln x = k C1 +
 * (k C2 + ln m) with the Cody-Waite split of ln 2 used by exp_poly.         */
static double log_poly(double x)
{
    int k;
    double m = frexp(x, &k);
    m = m * 2.0;
    k -= 1;
    if (m > LIP_SQRT2) { m = m * 0.5; k += 1; }
    double f = (m - 1.0) / (m + 1.0);
    double s2 = f * f;
    double p = 1.0 / 25.0;
    for (int n = 11; n >= 0; --n) {
        double t = s2 * p;
        p = 1.0 / (double)(2 * n + 1) + t;
    }
    double lm = (2.0 * f) * p;
    return (double)k * ORC_LN2_C1 + ((double)k * ORC_LN2_C2 + lm);
}

static float *lip_x(const orc_t *o, int w) { return (float *)(o->spin + (size_t)w * o->N); }
static int8_t *lip_type(const orc_t *o, int w) { return (int8_t *)(o->spin + (size_t)w * o->N + o->off_type); }
static int32_t *lip_lip(const orc_t *o, int w) { return (int32_t *)(o->spin + (size_t)w * o->N + o->off_lip); }
static int32_t *lip_where(const orc_t *o, int w) { return (int32_t *)(o->spin + (size_t)w * o->N + o->off_where); }

/* Squared minimum-image distance (per-axis difference in binary32). */
static double lip_r2(float box, const float *a, const float *b)
{
    double d[3];
    tri_min_image(box, a, b, d);
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* Pair energy of particles of types ti, tj at squared distance r2; bonded
 * marks consecutive beads of one lipid.                                     */
static double lip_pair(const orc_t *o, int ti, int tj, int bonded, double r2)
{
    if (bonded) {
        if (r2 >= LIP_R2) return INFINITY;
        double fene = -(0.5 * 30.0 * 1.69) * log_poly(1.0 - r2 / LIP_R2);
        double wca = 0.0;
        if (r2 < LIP_WCA_RC2) {
            double s2 = 1.0 / r2;
            double s6 = (s2 * s2) * s2;
            wca = 4.0 * ((s6 * s6) - s6) + 1.0;
        }
        return fene + wca;
    }
    if (r2 >= LIP_RC2) return 0.0;
    int rep = (ti == LIP_H && tj != LIP_H) || (tj == LIP_H && ti != LIP_H);
    if (rep) {
        double q = 1.05 / sqrt(r2);
        double q3 = (q * q) * q;
        return 4.0 * ((q3 * q3) * q3);
    }
    double s2 = 1.0 / r2;
    double s6 = (s2 * s2) * s2;
    double v = 4.0 * ((s6 * s6) - s6);
    return (ti == LIP_W && tj == LIP_W) ? o->eps_ww * v : v;
}

static int lip_bonded(const int32_t *where, int i, int j)
{
    int a = where[i], b = where[j];
    if (a < 0 || b < 0 || a / 3 != b / 3) return 0;
    return (a - b == 1) || (b - a == 1);
}

/* Energy of the pair (i, j) with particle i at xi. */
static double lip_pair_ij(const orc_t *o, const float *x, const int8_t *type, const int32_t *where, int i,
                          const float *xi, int j)
{
    return lip_pair(o, type[i], type[j], lip_bonded(where, i, j), lip_r2(o->box, xi, x + 3 * j));
}

/* Total energy in fixed point, every pair i < j (creation and tests only);
 * 0 for a hard overlap (a bond stretched to R or beyond included).          */
static int lip_energy(const orc_t *o, int w, int64_t *e)
{
    const float *x = lip_x(o, w);
    const int8_t *type = lip_type(o, w);
    const int32_t *where = lip_where(o, w);
    __int128 acc = 0;
    for (int i = 0; i < o->np; ++i)
        for (int j = i + 1; j < o->np; ++j) {
            int64_t t;
            if (!fx_term(lip_pair_ij(o, x, type, where, i, x + 3 * i, j), &t)) return 0;
            acc += t;
        }
    if (!fx_in_range(acc)) return 0;
    *e = (int64_t)acc;
    return 1;
}

/* Energy change of displacing particle b to xn: the sum over partners j of
 * fx(V(b at xn, j)) - fx(V(b, j)); 0 if a term is a hard overlap.          */
static int lip_delta_move(const orc_t *o, int w, int b, const float *xn, int64_t *de)
{
    const float *x = lip_x(o, w);
    const int8_t *type = lip_type(o, w);
    const int32_t *where = lip_where(o, w);
    __int128 acc = 0;
    for (int j = 0; j < o->np; ++j) {
        if (j == b) continue;
        int64_t tn, to;
        if (!fx_term(lip_pair_ij(o, x, type, where, b, xn, j), &tn)) return 0;
        if (!fx_term(lip_pair_ij(o, x, type, where, b, x + 3 * b, j), &to)) return 0;
        acc += (__int128)tn - (__int128)to;
    }
    *de = (int64_t)acc;
    return 1;
}

/* A reptation proposal: the four particles whose role changes (captured,
 * and the lipid's three beads), sorted ascending, with their new types and
 * positions in the chain; the new lipid row; n_c and n_r.                   */
typedef struct {
    int c[4];
    int8_t nt[4];
    int32_t nwh[4];
    int32_t nlip[3];
    int lipid, nc, nr;
} lip_rep_t;

/* Solvent particles within R of particle e under the given types (counted
 * in index order); if pick >= 0, the pick-th of them is returned in *found. */
static int lip_near_solvent(const orc_t *o, const float *x, const int8_t *type, int e, int pick, int *found)
{
    int n = 0;
    for (int j = 0; j < o->np; ++j) {
        if (j == e || type[j] != LIP_W) continue;
        if (lip_r2(o->box, x + 3 * e, x + 3 * j) < LIP_R2) {
            if (n == pick) *found = j;
            ++n;
        }
    }
    return n;
}

/* Build the reptation of `lipid` at its head (end 0) or tail (end 1), the
 * captured particle being the pick_word-selected solvent particle near that
 * end.  Returns 0 (no proposal) when no solvent particle is within R.       */
static int lip_reptation(const orc_t *o, int w, int lipid, int end, uint32_t pick_word, lip_rep_t *rp)
{
    const float *x = lip_x(o, w);
    const int8_t *type = lip_type(o, w);
    const int32_t *lp = lip_lip(o, w) + 3 * lipid;
    int e = end == 0 ? lp[0] : lp[2];
    int nc = lip_near_solvent(o, x, type, e, -1, NULL);
    if (nc == 0) return 0;
    int cap = -1;
    lip_near_solvent(o, x, type, e, (int)(((uint64_t)pick_word * (uint64_t)nc) >> 32), &cap);
    int nl[3], rel;
    if (end == 0) { nl[0] = cap; nl[1] = lp[0]; nl[2] = lp[1]; rel = lp[2]; }
    else          { nl[0] = lp[1]; nl[1] = lp[2]; nl[2] = cap; rel = lp[0]; }
    int all[4] = { cap, lp[0], lp[1], lp[2] };
    for (int a = 1; a < 4; ++a)                 /* sort ascending */
        for (int b = a; b > 0 && all[b - 1] > all[b]; --b) { int t = all[b]; all[b] = all[b - 1]; all[b - 1] = t; }
    for (int a = 0; a < 4; ++a) {
        int p = all[a];
        rp->c[a] = p;
        if (p == rel) { rp->nt[a] = LIP_W; rp->nwh[a] = -1; }
        else {
            int pos = p == nl[0] ? 0 : (p == nl[1] ? 1 : 2);
            rp->nt[a] = pos == 0 ? LIP_P : LIP_H;
            rp->nwh[a] = 3 * lipid + pos;
        }
    }
    for (int a = 0; a < 3; ++a) rp->nlip[a] = nl[a];
    rp->lipid = lipid;
    rp->nc = nc;
    /* n_r: solvent near the new end next to the released particle (lp[1]) */
    int8_t *t2 = (int8_t *)malloc((size_t)o->np);
    memcpy(t2, type, (size_t)o->np);
    for (int a = 0; a < 4; ++a) t2[rp->c[a]] = rp->nt[a];
    rp->nr = lip_near_solvent(o, x, t2, lp[1], -1, NULL);
    free(t2);
    return 1;
}

/* Energy change of a reptation: the sum of fx(V_new(i, j)) - fx(V_old(i, j))
 * over the pairs that hold a changed particle i (each such pair once);
 * positions stay, types and bonds change.  0 if a term is a hard overlap.  */
static int lip_delta_rep(const orc_t *o, int w, const lip_rep_t *rp, int64_t *de)
{
    const float *x = lip_x(o, w);
    const int8_t *type = lip_type(o, w);
    const int32_t *where = lip_where(o, w);
    int8_t *nt = (int8_t *)malloc((size_t)o->np);
    int32_t *nw = (int32_t *)malloc((size_t)o->np * sizeof(int32_t));
    memcpy(nt, type, (size_t)o->np);
    memcpy(nw, where, (size_t)o->np * sizeof(int32_t));
    for (int a = 0; a < 4; ++a) { nt[rp->c[a]] = rp->nt[a]; nw[rp->c[a]] = rp->nwh[a]; }
    __int128 acc = 0;
    int ok = 1;
    for (int j = 0; j < o->np && ok; ++j) {
        int jin = j == rp->c[0] || j == rp->c[1] || j == rp->c[2] || j == rp->c[3];
        for (int a = 0; a < 4; ++a) {
            int i = rp->c[a];
            if (i == j || (jin && i > j)) continue;
            double r2 = lip_r2(o->box, x + 3 * i, x + 3 * j);
            int64_t tn, to;
            if (!fx_term(lip_pair(o, nt[i], nt[j], lip_bonded(nw, i, j), r2), &tn) ||
                !fx_term(lip_pair(o, type[i], type[j], lip_bonded(where, i, j), r2), &to)) {
                ok = 0;
                break;
            }
            acc += (__int128)tn - (__int128)to;
        }
    }
    free(nt); free(nw);
    if (!ok) return 0;
    *de = (int64_t)acc;
    return 1;
}

static void lip_apply_rep(orc_t *o, int w, const lip_rep_t *rp)
{
    int8_t *type = lip_type(o, w);
    int32_t *where = lip_where(o, w);
    for (int a = 0; a < 4; ++a) { type[rp->c[a]] = rp->nt[a]; where[rp->c[a]] = rp->nwh[a]; }
    for (int a = 0; a < 3; ++a) lip_lip(o, w)[3 * rp->lipid + a] = rp->nlip[a];
}

/* Acceptance of a reptation with Wang-Landau weights and the selection
 * ratio: accept with probability min[1, e^d n_c / n_r], d = ln g(old) -
 * ln g(new), decided with u = r / 2^32 as
 *   d >= 0:  (u n_r) exp_poly(-d) < n_c,     d < 0:  u n_r < exp_poly(d) n_c. */
static int lip_accept_rep(double d, uint32_t r, int nc, int nr)
{
    double u = (double)r * 0x1p-32;
    if (d >= 0.0) return (u * (double)nr) * exp_poly(-d) < (double)nc;
    return u * (double)nr < exp_poly(d) * (double)nc;
}

/* One lipid-model attempt of walker w from Philox blocks (cnt, w, dom) and
 * (cnt, w, domu): block words a0 particle (or lipid), a1..a3 displacement;
 * u0 acceptance, u1 move type, u2 end (top bit), u3 captured particle.
 * lng_of(b) gives the walker's ln g at bin b; returns 1 if accepted.        */
typedef struct { int64_t e_new; int bn; int ok; int is_rep; lip_rep_t rp; int b; float xn[3]; int nc, nr; } lip_prop_t;

static void lip_propose(const orc_t *o, int w, uint64_t cnt, uint32_t dom, uint32_t domu, uint32_t u_out[4],
                        lip_prop_t *pr)
{
    uint32_t ctr[4] = { (uint32_t)cnt, (uint32_t)(cnt >> 32), (uint32_t)w, (dom << 24) | o->instance };
    uint32_t a[4];
    philox4x32_10(ctr, o->key, a);
    ctr[3] = (domu << 24) | o->instance;
    philox4x32_10(ctr, o->key, u_out);
    pr->ok = 0;
    pr->is_rep = u_out[1] < o->rep_thr;
    int64_t de = 0;
    int valid;
    if (pr->is_rep) {
        int lipid = (int)(((uint64_t)a[0] * (uint64_t)o->nlip) >> 32);
        if (!lip_reptation(o, w, lipid, (int)(u_out[2] >> 31), u_out[3], &pr->rp)) return;
        valid = lip_delta_rep(o, w, &pr->rp, &de);
    } else {
        const float *x = lip_x(o, w);
        pr->b = (int)(((uint64_t)a[0] * (uint64_t)o->np) >> 32);
        for (int c = 0; c < 3; ++c) pr->xn[c] = tri_wrap(x[3 * pr->b + c] + tri_disp(a[1 + c]), o->box);
        valid = lip_delta_move(o, w, pr->b, pr->xn, &de);
    }
    /* a hard overlap (a bond stretched to R or beyond included) or an energy
     * out of range: no move                                                  */
    if (!valid || !fx_add(o->Efx[w], de, &pr->e_new)) return;
    pr->bn = tri_bin(o, pr->e_new);
    pr->ok = 1;
}

static void lip_apply(orc_t *o, int w, const lip_prop_t *pr)
{
    if (pr->is_rep) lip_apply_rep(o, w, &pr->rp);
    else {
        float *x = lip_x(o, w);
        for (int c = 0; c < 3; ++c) x[3 * pr->b + c] = pr->xn[c];
    }
    o->Efx[w] = pr->e_new;
    o->E[w] = pr->bn;
}

static int lip_decide(const lip_prop_t *pr, double d, uint32_t u0)
{
    return pr->is_rep ? lip_accept_rep(d, u0, pr->rp.nc, pr->rp.nr) : accept64(d, u0);
}

static void lipid_attempt(orc_t *o, int w, int k, double lnf, uint64_t cnt)
{
    int W = o->W;
    uint32_t u[4];
    lip_prop_t pr;
    lip_propose(o, w, cnt, DOM_MOVE, DOM_MOVE_U, u, &pr);
    int lo = o->start[k], hi = o->start[k] + W - 1;
    if (pr.ok && pr.bn >= lo && pr.bn <= hi) {
        size_t io = (size_t)w * W + (o->E[w] - lo), in = (size_t)w * W + (pr.bn - lo);
        if (lip_decide(&pr, o->lng[io] - o->lng[in], u[0])) lip_apply(o, w, &pr);
    }
    size_t ib = (size_t)w * W + (o->E[w] - lo);
    o->lng[ib] += lnf;
    o->H[ib] += 1u;
    if (!o->finished[k]) o->vis[ib] = 1;
}

/* Walk-in of a lipid walker: the trimer walk-in rule with the lipid moves. */
static int lipid_walkin(orc_t *o, int w, int64_t max_attempts)
{
    int k = w / o->m;
    int lo = o->start[k], hi = o->start[k] + o->W - 1;
    double *g = (double *)calloc((size_t)o->B, sizeof(double));
    if (!g) return ORC_ENOMEM;
    int64_t n = 0;
    int slack = o->walkin_slack;
    int down = o->E[w] > hi;
    int bound = down ? o->E[w] + slack : o->E[w] - slack;
    int status = ORC_OK;
    while (!(o->E[w] >= lo && o->E[w] <= hi)) {
        if (n >= max_attempts) { status = ORC_EBUDGET; break; }
        uint32_t u[4];
        lip_prop_t pr;
        lip_propose(o, w, (uint64_t)n, DOM_WALKIN, DOM_WALKIN_U, u, &pr);
        if (pr.ok) {
            int co = o->E[w] < 0 ? 0 : (o->E[w] >= o->B ? o->B - 1 : o->E[w]);
            int cn = pr.bn < 0 ? 0 : (pr.bn >= o->B ? o->B - 1 : pr.bn);
            int inside = slack == 0 || (down ? pr.bn <= bound : pr.bn >= bound);
            if (inside && lip_decide(&pr, g[co] - g[cn], u[0])) {
                lip_apply(o, w, &pr);
                if (slack && down && o->E[w] + slack < bound) bound = o->E[w] + slack;
                if (slack && !down && o->E[w] - slack > bound) bound = o->E[w] - slack;
            }
        }
        int ci = o->E[w] < 0 ? 0 : (o->E[w] >= o->B ? o->B - 1 : o->E[w]);
        g[ci] += 1.0;
        ++n;
    }
    o->walkin_att[w] = n;
    free(g);
    return status;
}

/* Create a REWL run of the lipid model: nlip lipids and nsol solvent
 * particles in a periodic cube of side box; particles 3i, 3i+1, 3i+2 start as
 * lipid i (head, tail, tail), the rest as solvent.  rep_thr: reptation when
 * a word is below it (2^32 * 3 nlip / (10 np) in the paper's protocol).
 * Energy bins and windows as for the trimer model; binary64 ln g only.
 * init_coords: [h*m][np][3] in [0, box).  NULL on invalid arguments.        */
orc_t *orc_create_lipid(int nlip, int nsol, float box, double eps_ww, uint32_t rep_thr, double e_min,
                        double bin_w, int bins, int h, double overlap, int m, uint64_t seed, uint32_t instance,
                        uint32_t flat_num, uint32_t flat_den, double lnf_init, double lnf_final, int schedule,
                        int64_t sync_attempts, int exchange, int fixed_lnf, int walkin_slack,
                        const float *init_coords)
{
    if (nlip < 1 || nsol < 0 || nlip * 3 + nsol > 4096 || !(box > 0.0f) ||
        !(bin_w * FX_ONE >= 1.0 && bin_w * FX_ONE <= 0x1p60) || !(fabs(e_min) < 0x1p28) || bins < 8 ||
        !init_coords || !(eps_ww >= 0.0))
        return NULL;
    int np = 3 * nlip + nsol;
    size_t off_type = (size_t)np * 12;
    size_t off_lip = off_type + ((size_t)np + 3) / 4 * 4;
    size_t off_where = off_lip + (size_t)nlip * 12;
    size_t bytes = off_where + (size_t)np * 4;
    orc_t *o = orc_new(bins, 0, (int)bytes, h, overlap, m, seed, instance, flat_num, flat_den, lnf_init,
                       lnf_final, schedule, sync_attempts, exchange, 0, fixed_lnf, 0, walkin_slack);
    if (!o) return NULL;
    o->model = MODEL_LIPID3D;
    o->np = np; o->nlip = nlip; o->box = box; o->eps_ww = eps_ww; o->rep_thr = rep_thr;
    o->e_min = e_min; o->bin_w = bin_w;
    o->emin_fx = (int64_t)rint(e_min * FX_ONE);
    o->binw_fx = (int64_t)rint(bin_w * FX_ONE);
    o->off_type = off_type; o->off_lip = off_lip; o->off_where = off_where;
    o->Efx = (int64_t *)calloc((size_t)o->nw, sizeof(int64_t));
    if (!o->Efx) { orc_free(o); return NULL; }
    for (int w = 0; w < o->nw; ++w) {
        float *x = lip_x(o, w);
        for (int i = 0; i < 3 * np; ++i) {
            float v = init_coords[(size_t)w * 3 * np + i];
            if (!(v >= 0.0f && v < box)) { orc_free(o); return NULL; }
            x[i] = v;
        }
        int8_t *type = lip_type(o, w);
        int32_t *where = lip_where(o, w), *lp = lip_lip(o, w);
        for (int i = 0; i < np; ++i) {
            int lipid = i < 3 * nlip;
            type[i] = lipid ? (i % 3 == 0 ? LIP_P : LIP_H) : LIP_W;
            where[i] = lipid ? i : -1;
        }
        for (int i = 0; i < 3 * nlip; ++i) lp[i] = i;
        if (!lip_energy(o, w, &o->Efx[w])) { orc_free(o); return NULL; }
        o->E[w] = tri_bin(o, o->Efx[w]);
    }
    return o;
}

/* Test exports of the lipid model. */
int orc_lipid_energy_fx(const orc_t *o, int w, int64_t *e) { return lip_energy(o, w, e); }
double orc_log_poly(double x) { return log_poly(x); }
double orc_lipid_pair(const orc_t *o, int ti, int tj, int bonded, double r2) { return lip_pair(o, ti, tj, bonded, r2); }

/* Particles of walker w: coordinates [np][3], types [np], lipid rows [nlip][3]. */
void orc_lipid_state(const orc_t *o, int w, float *x, int8_t *type, int32_t *lip)
{
    if (x) memcpy(x, lip_x(o, w), (size_t)o->np * 12);
    if (type) memcpy(type, lip_type(o, w), (size_t)o->np);
    if (lip) memcpy(lip, lip_lip(o, w), (size_t)o->nlip * 12);
}

/* Energy change (units of 2^-32) of displacing particle b of walker w to xn
 * (no state change); 0 for a hard overlap.                                  */
int orc_lipid_delta_move_fx(const orc_t *o, int w, int b, const float *xn, int64_t *de)
{
    return lip_delta_move(o, w, b, xn, de);
}

/* Apply the reptation of `lipid` at `end` capturing the pick-th nearby
 * solvent particle (the word pick * 2^32 / n_c selects it); out: n_c, n_r,
 * energy change.  Returns 0 if no solvent particle is near that end.       */
int orc_lipid_reptate(orc_t *o, int w, int lipid, int end, int pick, int *nc, int *nr, int64_t *de)
{
    const float *x = lip_x(o, w);
    int e = end == 0 ? lip_lip(o, w)[3 * lipid] : lip_lip(o, w)[3 * lipid + 2];
    int n = lip_near_solvent(o, x, lip_type(o, w), e, -1, NULL);
    if (n == 0 || pick < 0 || pick >= n) return 0;
    uint32_t word = (uint32_t)((((uint64_t)pick << 32) + (uint64_t)n - 1) / (uint64_t)n);
    lip_rep_t rp;
    if (!lip_reptation(o, w, lipid, end, word, &rp)) return 0;
    int64_t d = 0, e_new = 0;
    if (!lip_delta_rep(o, w, &rp, &d) || !fx_add(o->Efx[w], d, &e_new)) return 0;
    lip_apply_rep(o, w, &rp);
    o->Efx[w] = e_new;
    o->E[w] = tri_bin(o, o->Efx[w]);
    *nc = rp.nc; *nr = rp.nr; *de = d;
    return 1;
}

/* Placement before the run: each walker must carry a configuration whose
 * energy lies inside its own window (Sec. 3.2, discussion of Fig. 7).  The
 * paper does not say how; here a Wang-Landau walk with its own ln g over all
 * B energies and ln f = 1 moves the configuration until its energy first
 * lies in the window.  A walker above its window walks under a lid: moves to
 * energies more than `walkin_slack` above the lowest energy it has reached
 * are rejected (a walker below its window, symmetrically, walks above a
 * floor).  Without the lid the walk floods the whole range between the start
 * and the window, at a cost that grows with the square of that range; with
 * it the flooded band stays `walkin_slack` wide.  walkin_slack = 0 means no
 * lid.  Returns ORC_EBUDGET if a walker needs more than max_attempts
 * attempts.                                                                 */
int orc_walkin(orc_t *o, int64_t max_attempts)
{
    if (o->walked_in) return ORC_OK;
    int status = ORC_OK;
    int nt = o->threads;
    (void)nt;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int w = 0; w < o->nw; ++w) {
        if (o->model == MODEL_TRIMER3D || o->model == MODEL_LIPID3D) {
            int st = o->model == MODEL_TRIMER3D ? trimer_walkin(o, w, max_attempts)
                                                : lipid_walkin(o, w, max_attempts);
            if (st != ORC_OK) {
#pragma omp atomic write
                status = st;
            }
            continue;
        }
        int k = w / o->m;
        int lo = o->start[k], hi = o->start[k] + o->W - 1;
        int N = o->N, L = o->L, q = o->q;
        int8_t *s = o->spin + (size_t)w * N;
        double *g = (double *)calloc((size_t)o->B, sizeof(double));
        int64_t t = 0;
        int slack = o->walkin_slack;
        int down = o->E[w] > hi;
        int bound = down ? o->E[w] + slack : o->E[w] - slack;   /* lid, or floor */
        while (!(o->E[w] >= lo && o->E[w] <= hi)) {
            if (t >= max_attempts || !g) {
#pragma omp atomic write
                status = ORC_EBUDGET;
                break;
            }
            uint32_t ctr[4] = { (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)w,
                                ((uint32_t)DOM_WALKIN << 24) | o->instance };
            uint32_t r[4];
            philox4x32_10(ctr, o->key, r);
            int i = (int)(((uint64_t)r[0] * (uint64_t)N) >> 32);
            int off = (int)(((uint64_t)r[1] * (uint64_t)(q - 1)) >> 32);
            int nv = s[i] + 1 + off;
            if (nv >= q) nv -= q;
            int e_new = o->E[w] + potts_delta_e(s, L, i, nv);
            double d = g[o->E[w] - o->e_lo] - g[e_new - o->e_lo];
            int inside = slack == 0 || (down ? e_new <= bound : e_new >= bound);
            if (inside && accept64(d, r[2])) {
                s[i] = (int8_t)nv;
                o->E[w] = e_new;
                if (slack && down && o->E[w] + slack < bound) bound = o->E[w] + slack;
                if (slack && !down && o->E[w] - slack > bound) bound = o->E[w] - slack;
            }
            g[o->E[w] - o->e_lo] += 1.0;
            ++t;
        }
        o->walkin_att[w] = t;
        free(g);
    }
    if (status == ORC_OK) o->walked_in = 1;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Shadow: an exact reference of every walker's ln g along its own trajectory.
 * Between two sync points ln f of a window is constant, so bin b of walker w
 * received (H - H_prev) additions of ln f; the shadow adds that product in
 * double-double arithmetic (about 106 significant bits) and follows the
 * window averages the same way.  The difference between ln g and its shadow
 * is then the rounding error the ln g format accumulated (binary64, or the
 * binary32 (hi, lo) pair).  It plays no part in the sampling.
 * Double-double routines: Knuth's TwoSum, Dekker's Fast2Sum, and the exact
 * product residual by fused multiply-add, combined as in the accurate
 * double-double addition of Hida, Li and Bailey (QD library, 2001).          */
static void dd_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bb = x - a;
    *e = (a - (x - bb)) + (b - bb);
    *s = x;
}

static void dd_fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

static void dd_add(double *hi, double *lo, double bh, double bl)
{
    double s, e, t, f;
    dd_two_sum(*hi, bh, &s, &e);
    dd_two_sum(*lo, bl, &t, &f);
    e = e + t;
    dd_fast_two_sum(s, e, &s, &e);
    e = e + f;
    dd_fast_two_sum(s, e, hi, lo);
}

/* (hi, lo) / m for a small positive integer m */
static void dd_div_int(double *hi, double *lo, int m)
{
    double dm = (double)m;
    double q1 = *hi / dm;
    double r = fma(-q1, dm, *hi);
    r = r + *lo;
    double q2 = r / dm;
    dd_fast_two_sum(q1, q2, hi, lo);
}

/* test exports of the double-double steps */
void orc_dd_add(double *hi, double *lo, double bh, double bl) { dd_add(hi, lo, bh, bl); }
void orc_dd_div_int(double *hi, double *lo, int m) { dd_div_int(hi, lo, m); }
void orc_dd_mul_count(uint32_t n, double x, double *hi, double *lo)
{
    double dn = (double)n;
    *hi = dn * x;
    *lo = fma(dn, x, -*hi);
}

/* sync point of window k: the interval's additions, n * ln f, into the shadow */
static void shadow_accumulate(orc_t *o, int k, double lnf)
{
    int W = o->W, m = o->m;
    for (int j = 0; j < m; ++j)
        for (int b = 0; b < W; ++b) {
            size_t i = (size_t)(k * m + j) * W + b;
            uint32_t n = o->H[i] - o->hprev[i];
            if (n) {
                double dn = (double)n;
                double ph = dn * lnf;
                double pl = fma(dn, lnf, -ph);
                dd_add(&o->sh_hi[i], &o->sh_lo[i], ph, pl);
            }
            o->hprev[i] = o->H[i];
        }
}

/* window average of the shadows (walker order, then / m), H_prev reset */
static void shadow_average(orc_t *o, int k)
{
    int W = o->W, m = o->m;
    for (int b = 0; b < W; ++b) {
        size_t i0 = (size_t)(k * m) * W + b;
        double hi = o->sh_hi[i0], lo = o->sh_lo[i0];
        for (int j = 1; j < m; ++j) {
            size_t i = (size_t)(k * m + j) * W + b;
            dd_add(&hi, &lo, o->sh_hi[i], o->sh_lo[i]);
        }
        dd_div_int(&hi, &lo, m);
        for (int j = 0; j < m; ++j) {
            size_t i = (size_t)(k * m + j) * W + b;
            o->sh_hi[i] = hi;
            o->sh_lo[i] = lo;
            o->hprev[i] = 0;
        }
    }
}

/* Average the m estimators of window k and hand the mean back to every
 * walker (Sec. 2: the window's estimators are averaged and every walker
 * continues from the mean).  The mean is taken of ln g,
 * summed in walker order and divided by m.                                   */
static void window_average(orc_t *o, int k)
{
    int W = o->W, m = o->m;
    for (int b = 0; b < W; ++b) {
        double sum = lng_get(o, k * m, b);
        for (int j = 1; j < m; ++j) sum = sum + lng_get(o, k * m + j, b);
        double mean = sum / (double)m;
        for (int j = 0; j < m; ++j) {
            size_t i = (size_t)(k * m + j) * W + b;
            if (o->precision == 0) o->lng[i] = mean;
            else {
                float hi = (float)mean;
                o->lng_hi[i] = hi;
                o->lng_lo[i] = (float)(mean - (double)hi);
            }
        }
    }
}

/* Sync point of window k after every S attempts per walker (Sec. 2):
 * each walker must be flat on its own; when all m are flat their ln g are
 * averaged, H is reset and ln f is halved (f -> sqrt f); optionally the
 * 1/t rule of Belardinelli and Pereyra takes over once ln f <= 1/t with
 * t = attempts per walker / W.  The window is finished once ln f < ln f_final. */
static void window_sync(orc_t *o, int k)
{
    int W = o->W, m = o->m;
    if (o->finished[k]) return;
    for (int j = 0; j < m; ++j)
        for (int b = 0; b < W; ++b)
            if (o->vis[(size_t)(k * m + j) * W + b]) o->visited[(size_t)k * W + b] = 1;
    if (o->precision == 1) {
        /* renormalise the (hi, lo) pairs with Dekker's Fast2Sum */
        for (int j = 0; j < m; ++j)
            for (int b = 0; b < W; ++b) {
                size_t i = (size_t)(k * m + j) * W + b;
                float s = o->lng_hi[i] + o->lng_lo[i];
                float z = s - o->lng_hi[i];
                o->lng_lo[i] = o->lng_lo[i] - z;
                o->lng_hi[i] = s;
            }
    }
    if (o->shadow) shadow_accumulate(o, k, o->lnf[k]);
    if (o->fixed_lnf) return;
    double inv_t = (double)W / (double)o->step;
    if (o->regime[k] == 0) {
        int all_flat = 1;
        for (int j = 0; j < m; ++j) {
            uint64_t n_act = 0, sum = 0, mn = UINT64_MAX;
            for (int b = 0; b < W; ++b) {
                if (!o->visited[(size_t)k * W + b]) continue;
                uint64_t hv = o->H[(size_t)(k * m + j) * W + b];
                n_act += 1;
                sum += hv;
                if (hv < mn) mn = hv;
            }
            int flat = n_act > 0 && (uint64_t)o->flat_den * mn * n_act >= (uint64_t)o->flat_num * sum;
            if (!flat) all_flat = 0;
        }
        if (!all_flat) return;
        window_average(o, k);
        if (o->shadow) shadow_average(o, k);
        memset(o->H + (size_t)k * m * W, 0, (size_t)m * W * sizeof(uint32_t));
        o->lnf[k] = o->lnf[k] * 0.5;
        o->iterations[k] += 1;
        if (o->schedule == 1 && o->lnf[k] <= inv_t) {
            o->regime[k] = 1;
            o->lnf[k] = inv_t;
        }
    } else {
        window_average(o, k);
        if (o->shadow) shadow_average(o, k);
        memset(o->H + (size_t)k * m * W, 0, (size_t)m * W * sizeof(uint32_t));
        o->lnf[k] = inv_t;
        o->iterations[k] += 1;
    }
    if (o->lnf[k] < o->lnf_final) {
        o->finished[k] = 1;
        o->lnf_last[k] = o->lnf[k];
        o->lnf[k] = 0.0;
    }
}

/* One round of replica exchange (Sec. 2, Eq. (1)).  Round r pairs windows
 * (k, k+1) with k = r mod 2, r mod 2 + 2, ...  Within a pair, walker j of
 * window k is matched with walker pi(j) of window k+1 for a uniformly random
 * permutation pi (Fisher-Yates).  Configurations X (walker a) and Y (walker b)
 * swap with probability min[1, g_a(E_X)/g_a(E_Y) * g_b(E_Y)/g_b(E_X)]; the
 * exchange is rejected if either energy lies outside the other window.
 * ln g and H stay with their walkers.                                        */
typedef struct { uint32_t ctr[4]; uint32_t buf[4]; int pos; const uint32_t *key; } word_stream;

static uint32_t next_word(word_stream *ws)
{
    if (ws->pos == 4) {
        philox4x32_10(ws->ctr, ws->key, ws->buf);
        ws->ctr[2] += 1u;      /* block index n */
        ws->pos = 0;
    }
    return ws->buf[ws->pos++];
}

static int exchange_round(orc_t *o)
{
    int h = o->h, m = o->m, W = o->W, N = o->N;
    uint32_t r = (uint32_t)o->round;
    int *perm = (int *)malloc((size_t)m * sizeof(int));
    int8_t *tmp = (int8_t *)malloc((size_t)N);
    if (!perm || !tmp) { free(perm); free(tmp); return ORC_ENOMEM; }
    for (int k = (int)(r & 1u); k + 1 < h; k += 2) {
        word_stream ws;
        ws.ctr[0] = r; ws.ctr[1] = (uint32_t)k; ws.ctr[2] = 0u;
        ws.ctr[3] = ((uint32_t)DOM_EXCH << 24) | o->instance;
        ws.pos = 4; ws.key = o->key;
        for (int j = 0; j < m; ++j) perm[j] = j;
        for (int i = m - 1; i >= 1; --i) {
            int j = (int)(((uint64_t)next_word(&ws) * (uint64_t)(i + 1)) >> 32);
            int t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        int lo_a = o->start[k], hi_a = o->start[k] + W - 1;
        int lo_b = o->start[k + 1], hi_b = o->start[k + 1] + W - 1;
        for (int j = 0; j < m; ++j) {
            int a = k * m + j, b = (k + 1) * m + perm[j];
            uint32_t u = next_word(&ws);
            int ex = o->E[a], ey = o->E[b];
            int acc = 0;
            o->x_att[k] += 1;
            if (ey >= lo_a && ey <= hi_a && ex >= lo_b && ex <= hi_b) {
                double d = ((lng_get(o, a, ex - lo_a) - lng_get(o, a, ey - lo_a))
                            + lng_get(o, b, ey - lo_b)) - lng_get(o, b, ex - lo_b);
                acc = accept64(d, u);
            }
            if (acc) {
                o->x_acc[k] += 1;
                memcpy(tmp, o->spin + (size_t)a * N, (size_t)N);
                memcpy(o->spin + (size_t)a * N, o->spin + (size_t)b * N, (size_t)N);
                memcpy(o->spin + (size_t)b * N, tmp, (size_t)N);
                o->E[a] = ey; o->E[b] = ex;
                if (o->Efx) { int64_t te = o->Efx[a]; o->Efx[a] = o->Efx[b]; o->Efx[b] = te; }
                uint32_t t = o->replica[a]; o->replica[a] = o->replica[b]; o->replica[b] = t;
            }
        }
    }
    o->round += 1;
    free(perm); free(tmp);
    return ORC_OK;
}

/* One exchange round on its own (no sync point); nothing once converged.   */
int orc_exchange(orc_t *o)
{
    if (o->converged) return ORC_CONVERGED;
    int st = exchange_round(o);
    if (st == ORC_OK) replica_track(o);
    return st;
}

/* Observable sampling (Sec. 3.2: after the density of states is known, the
 * paper keeps sampling with fixed weights 1/g(E) and records distributions
 * H(E, O) of observables O).  For the Potts model O is the population of the
 * most occupied state, O = max_s n_s, from which the usual order parameter
 * (q O / N - 1) / (q - 1) follows.  At every sync point (after its exchange
 * round) each walker adds its current configuration: H(E, O) gains one count
 * in O bin floor(O * obs_bins / (N + 1)), and the exact sum of O and the
 * sample count of bin E grow.                                               */
static void obs_measure(orc_t *o)
{
    if (o->obs_bins <= 0) return;
    int N = o->N, W = o->W, nb = o->obs_bins;
    int *cnt = (int *)calloc((size_t)o->q, sizeof(int));
    if (!cnt) return;
    for (int w = 0; w < o->nw; ++w) {
        const int8_t *s = o->spin + (size_t)w * N;
        for (int v = 0; v < o->q; ++v) cnt[v] = 0;
        for (int i = 0; i < N; ++i) cnt[s[i]] += 1;
        int O = 0;
        for (int v = 0; v < o->q; ++v) if (cnt[v] > O) O = cnt[v];
        int b = o->E[w] - o->start[w / o->m];
        if (b < 0 || b >= W) continue;
        size_t cell = (size_t)w * W + (size_t)b;
        int ob = (int)(((int64_t)O * nb) / (N + 1));
        o->obs_hist[cell * nb + ob] += 1;
        o->obs_sum[cell] += (uint64_t)O;
        o->obs_cnt[cell] += 1;
    }
    free(cnt);
}

/* Production phase: from now on every window keeps its current ln g as
 * fixed weights (ln f = 0, window marked finished; a window that had not
 * finished records its current ln f as the last one), the run no longer
 * terminates, and H and the observable histograms restart from zero.
 * Needs a walked-in run.                                                    */
int orc_begin_production(orc_t *o)
{
    if (!o->walked_in) return ORC_EINVAL;
    for (int k = 0; k < o->h; ++k) {
        if (!o->finished[k]) {
            o->finished[k] = 1;
            o->lnf_last[k] = o->lnf[k];
        }
        o->lnf[k] = 0.0;
    }
    memset(o->H, 0, (size_t)o->nw * o->W * sizeof(uint32_t));
    if (o->obs_bins > 0) {
        size_t cells = (size_t)o->nw * o->W;
        memset(o->obs_hist, 0, cells * (size_t)o->obs_bins * sizeof(uint32_t));
        memset(o->obs_sum, 0, cells * sizeof(uint64_t));
        memset(o->obs_cnt, 0, cells * sizeof(uint32_t));
    }
    o->converged = 0;
    o->production = 1;
    return ORC_OK;
}

/* Run `attempts` more Wang-Landau attempts per walker.  Sync points (flatness,
 * averaging, ln f update, then an exchange round) fall at every multiple of S
 * attempts counted from the start of the main phase, so splitting a run into
 * several calls gives the same result.  Stops at the first sync point at
 * which every window is finished (Sec. 2: the simulation terminates when all
 * h windows reached f_final).                                               */
int orc_run(orc_t *o, int64_t attempts, int64_t walkin_budget)
{
    if (!o->walked_in) {
        int st = orc_walkin(o, walkin_budget);
        if (st != ORC_OK) return st;
    }
    if (o->converged) return ORC_CONVERGED;
    int nt = o->threads;
    (void)nt;
    while (attempts > 0) {
        int64_t seg = o->S - (o->step % o->S);
        if (seg > attempts) seg = attempts;
        int64_t s0 = o->step;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
        for (int w = 0; w < o->nw; ++w) {
            int k = w / o->m;
            double lnf = o->lnf[k];
            if (o->model == MODEL_LIPID3D) {
                for (int64_t t = 0; t < seg; ++t) lipid_attempt(o, w, k, lnf, (uint64_t)(s0 + t));
            } else if (o->model == MODEL_TRIMER3D)
                for (int64_t t = 0; t < seg; ++t) trimer_attempt(o, w, k, lnf, (uint64_t)(s0 + t));
            else
                for (int64_t t = 0; t < seg; ++t) potts_attempt(o, w, k, lnf, DOM_MOVE, (uint64_t)(s0 + t));
        }
        o->step += seg;
        attempts -= seg;
        if (o->step % o->S == 0) {
            for (int k = 0; k < o->h; ++k) window_sync(o, k);
            if (o->exchange) {
                int st = exchange_round(o);
                if (st != ORC_OK) return st;
            }
            replica_track(o);
            obs_measure(o);
            int all = !o->production;
            for (int k = 0; k < o->h; ++k) all = all && o->finished[k];
            if (all) { o->converged = 1; return ORC_CONVERGED; }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Accessors for the tests.                                                  */
void orc_info(const orc_t *o, int64_t *out)
{
    out[0] = o->N; out[1] = o->W; out[2] = o->B; out[3] = o->e_lo; out[4] = o->nw;
    out[5] = o->step; out[6] = o->round; out[7] = o->converged; out[8] = o->walked_in;
}

void orc_starts(const orc_t *o, int32_t *out)
{
    for (int k = 0; k < o->h; ++k) out[k] = o->start[k];
}

void orc_get_walker(const orc_t *o, int w, int8_t *spins, int32_t *E, uint32_t *H, double *lng,
                    float *lng_hi, float *lng_lo, uint32_t *replica, int64_t *walkin_attempts)
{
    size_t N = (size_t)o->N, W = (size_t)o->W;
    if (spins) memcpy(spins, o->spin + (size_t)w * N, N);
    if (E) *E = o->E[w];
    if (H) memcpy(H, o->H + (size_t)w * W, W * sizeof(uint32_t));
    if (lng) for (size_t b = 0; b < W; ++b) lng[b] = lng_get(o, w, (int)b);
    if (lng_hi && o->precision == 1) memcpy(lng_hi, o->lng_hi + (size_t)w * W, W * sizeof(float));
    if (lng_lo && o->precision == 1) memcpy(lng_lo, o->lng_lo + (size_t)w * W, W * sizeof(float));
    if (replica) *replica = o->replica[w];
    if (walkin_attempts) *walkin_attempts = o->walkin_att[w];
}

/* Window state; visited is the union of the walkers' visited bins so far.   */
void orc_get_window(const orc_t *o, int k, double *lnf, double *lnf_last, int32_t *regime,
                    int32_t *finished, int64_t *iterations, uint8_t *visited, uint64_t *xatt,
                    uint64_t *xacc)
{
    int W = o->W, m = o->m;
    if (lnf) *lnf = o->lnf[k];
    if (lnf_last) *lnf_last = o->lnf_last[k];
    if (regime) *regime = o->regime[k];
    if (finished) *finished = o->finished[k];
    if (iterations) *iterations = o->iterations[k];
    if (visited) {
        for (int b = 0; b < W; ++b) {
            uint8_t v = o->visited[(size_t)k * W + b];
            if (!o->finished[k])
                for (int j = 0; j < m; ++j) v |= o->vis[(size_t)(k * m + j) * W + b];
            visited[b] = v;
        }
    }
    if (xatt) *xatt = o->x_att[k];
    if (xacc) *xacc = o->x_acc[k];
}

/* Shadow of walker w (zeros if the run keeps none).                        */
void orc_get_shadow(const orc_t *o, int w, double *hi, double *lo)
{
    size_t W = (size_t)o->W;
    for (size_t b = 0; b < W; ++b) {
        hi[b] = o->shadow ? o->sh_hi[(size_t)w * W + b] : 0.0;
        lo[b] = o->shadow ? o->sh_lo[(size_t)w * W + b] : 0.0;
    }
}

/* Test hooks for the sync step on its own: plant walker w's histogram and
 * the bins it has visited, the main-phase attempt count (which fixes the 1/t
 * value W/t), and window k's ln f and regime; then run window k's sync step
 * (flatness, averaging, ln f reduction, termination) without any attempts.  */
void orc_plant_walker(orc_t *o, int w, const uint32_t *H, const uint8_t *vis)
{
    size_t W = (size_t)o->W;
    memcpy(o->H + (size_t)w * W, H, W * sizeof(uint32_t));
    memcpy(o->vis + (size_t)w * W, vis, W);
}

void orc_set_step(orc_t *o, int64_t step) { o->step = step; }

void orc_set_window(orc_t *o, int k, double lnf, int regime)
{
    o->lnf[k] = lnf;
    o->regime[k] = regime;
}

void orc_sync_window(orc_t *o, int k) { window_sync(o, k); }

/* Test hook: overwrite the ln g of walker w (precision 0 or 1); the shadow
 * restarts from the given values.                                           */
void orc_set_lng(orc_t *o, int w, const double *lng)
{
    size_t W = (size_t)o->W;
    for (size_t b = 0; b < W; ++b) {
        if (o->shadow) {
            o->sh_hi[(size_t)w * W + b] = lng[b];
            o->sh_lo[(size_t)w * W + b] = 0.0;
            o->hprev[(size_t)w * W + b] = o->H[(size_t)w * W + b];
        }
        if (o->precision == 0) o->lng[(size_t)w * W + b] = lng[b];
        else {
            float hi = (float)lng[b];
            o->lng_hi[(size_t)w * W + b] = hi;
            o->lng_lo[(size_t)w * W + b] = (float)(lng[b] - (double)hi);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Joining the h pieces (Sec. 2, Fig. 2): for neighbouring windows k, k+1
 * the joining energy E* is the energy of their overlap at which the
 * microcanonical inverse temperatures beta(E) = d ln g / dE of the two pieces
 * agree best; beta is the finite difference between the nearest visited bins
 * above and below E inside the piece.  Ties go to the lowest E*, and E* must
 * lie above the previous joining point.  Piece k+1 is shifted to equal piece
 * k at E*; the joined curve takes piece k up to E* and piece k+1 above it.
 * Finally ln g is normalised so that sum_E g(E) = q^N.
 * pieces: [h][W] ln g, vis: [h][W] visited flags.  out: [B] (unvisited bins
 * are -inf).  cuts: [h-1] joining energies.  Returns ORC_ESTATE if two
 * neighbouring pieces share no visited energy.                              */
static int beta_at(const double *g, const uint8_t *v, int W, int b, double *beta)
{
    if (!v[b]) return 0;
    int bp = -1, bm = -1;
    for (int t = b + 1; t < W; ++t) if (v[t]) { bp = t; break; }
    for (int t = b - 1; t >= 0; --t) if (v[t]) { bm = t; break; }
    if (bp < 0 || bm < 0) return 0;
    *beta = (g[bp] - g[bm]) / (double)(bp - bm);
    return 1;
}

int orc_join_pieces(int h, int W, const int32_t *start, int e_lo, int B, const double *pieces,
                    const uint8_t *vis, double log_total, double *out, int32_t *cuts)
{
    double *shift = (double *)calloc((size_t)h, sizeof(double));
    if (!shift) return ORC_ENOMEM;
    int prev_cut = INT32_MIN;
    for (int k = 0; k + 1 < h; ++k) {
        const double *ga = pieces + (size_t)k * W, *gb = pieces + (size_t)(k + 1) * W;
        const uint8_t *va = vis + (size_t)k * W, *vb = vis + (size_t)(k + 1) * W;
        int lo = start[k + 1], hi = start[k] + W - 1;
        if (prev_cut != INT32_MIN && prev_cut + 1 > lo) lo = prev_cut + 1;
        int best = INT32_MIN;
        double bestd = 0.0;
        for (int e = lo; e <= hi; ++e) {
            double ba, bb;
            if (!beta_at(ga, va, W, e - start[k], &ba)) continue;
            if (!beta_at(gb, vb, W, e - start[k + 1], &bb)) continue;
            double d = fabs(ba - bb);
            if (best == INT32_MIN || d < bestd) { best = e; bestd = d; }
        }
        if (best == INT32_MIN)
            for (int e = lo; e <= hi; ++e)
                if (va[e - start[k]] && vb[e - start[k + 1]]) { best = e; break; }
        if (best == INT32_MIN) { free(shift); return ORC_ESTATE; }
        cuts[k] = best;
        shift[k + 1] = (ga[best - start[k]] + shift[k]) - gb[best - start[k + 1]];
        prev_cut = best;
    }
    for (int b = 0; b < B; ++b) out[b] = -INFINITY;
    for (int k = 0; k < h; ++k) {
        int from = (k == 0) ? start[0] : cuts[k - 1] + 1;
        int to = (k == h - 1) ? start[h - 1] + W - 1 : cuts[k];
        for (int e = from; e <= to; ++e) {
            int b = e - start[k];
            if (b < 0 || b >= W || !vis[(size_t)k * W + b]) continue;
            out[e - e_lo] = pieces[(size_t)k * W + b] + shift[k];
        }
    }
    free(shift);
    /* normalisation: ln g <- ln g - ln(sum_E g(E)) + ln(total) */
    double mx = -INFINITY;
    for (int b = 0; b < B; ++b) if (out[b] > mx) mx = out[b];
    if (mx == -INFINITY) return ORC_ESTATE;
    double s = 0.0;
    for (int b = 0; b < B; ++b) if (out[b] != -INFINITY) s += exp(out[b] - mx);
    double lse = mx + log(s);
    for (int b = 0; b < B; ++b) if (out[b] != -INFINITY) out[b] = (out[b] - lse) + log_total;
    return ORC_OK;
}

/* Joined ln g of a run, from walker 0 of every window. */
int orc_join(const orc_t *o, double *out, int32_t *cuts)
{
    int h = o->h, W = o->W;
    double *pieces = (double *)malloc((size_t)h * W * sizeof(double));
    uint8_t *vis = (uint8_t *)malloc((size_t)h * W);
    int32_t *st = (int32_t *)malloc((size_t)h * sizeof(int32_t));
    if (!pieces || !vis || !st) { free(pieces); free(vis); free(st); return ORC_ENOMEM; }
    for (int k = 0; k < h; ++k) {
        st[k] = o->start[k];
        orc_get_window(o, k, NULL, NULL, NULL, NULL, NULL, vis + (size_t)k * W, NULL, NULL);
        for (int b = 0; b < W; ++b) pieces[(size_t)k * W + b] = lng_get(o, k * o->m, b);
    }
    /* Potts: sum_E g(E) = q^N; trimer: no total count, sum over bins of g = 1 */
    double log_total = o->model == MODEL_POTTS2D ? (double)o->N * log((double)o->q) : 0.0;
    int st_code = orc_join_pieces(h, W, st, o->e_lo, o->B, pieces, vis, log_total, out, cuts);
    free(pieces); free(vis); free(st);
    return st_code;
}

/* Canonical averages from g(E) (Sec. 3.1, Fig. 3b): P(E,T) = g(E) e^{-E/T}/Z.
 * ln Z = LSE_E(ln g(E) - E/T), U = <E>, C_v = (<E^2> - <E>^2)/T^2, with the
 * variance summed as sum P (E - U)^2.  Bin b stands for the energy
 * e_first + b de (Potts: integer energies, de = 1; trimer: bin centres).
 * Bins with ln g = -inf are skipped.                                         */
void orc_thermo(const double *lng, int B, double e_first, double de, const double *T, int nT,
                double *lnZ, double *U, double *C)
{
    for (int t = 0; t < nT; ++t) {
        double mx = -INFINITY;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY) continue;
            double x = lng[b] - (e_first + (double)b * de) / T[t];
            if (x > mx) mx = x;
        }
        double s = 0.0;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY) continue;
            s += exp((lng[b] - (e_first + (double)b * de) / T[t]) - mx);
        }
        double lz = mx + log(s);
        double u = 0.0;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY) continue;
            double p = exp((lng[b] - (e_first + (double)b * de) / T[t]) - lz);
            u += p * (e_first + (double)b * de);
        }
        double var = 0.0;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY) continue;
            double p = exp((lng[b] - (e_first + (double)b * de) / T[t]) - lz);
            double d = (e_first + (double)b * de) - u;
            var += p * d * d;
        }
        lnZ[t] = lz;
        U[t] = u;
        C[t] = var / (T[t] * T[t]);
    }
}

/* Mean and sample standard deviation of x[0], x[stride], ... (n values, in
 * order) over the finite ones; mean -inf and std 0 when none is finite.     */
static void finite_stats(const double *x, int n, size_t stride, double *mean, double *sd)
{
    double s = 0.0;
    int c = 0;
    for (int j = 0; j < n; ++j) {
        double v = x[(size_t)j * stride];
        if (isfinite(v)) { s += v; ++c; }
    }
    if (c == 0) { *mean = -INFINITY; *sd = 0.0; return; }
    double m = s / (double)c, q = 0.0;
    for (int j = 0; j < n; ++j) {
        double v = x[(size_t)j * stride];
        if (isfinite(v)) { double d = v - m; q += d * d; }
    }
    *mean = m;
    *sd = c > 1 ? sqrt(q / (double)(c - 1)) : 0.0;
}

/* Bootstrap error analysis (Sec. 2: the simulation is repeated and the
 * results resampled; every resampled global g(E) is joined anew, so its
 * joining points move).  Inputs: R independent runs of one system, each
 * window's final ln g as pieces[R][h][W] and its visited flags vis[R][h][W].
 * Replicate j draws R run indices with replacement: r_i = floor(w_i R / 2^32)
 * for the Philox words w_i, four per block (j, i / 4, 0, BOOT << 24), keyed
 * by seed.  Its piece k is the mean over i, summed in order, of the drawn
 * runs' piece k; the pieces are joined (orc_join_pieces) over the union of
 * all runs' visited flags and normalised to log_total, and U and C_v follow
 * at the nT temperatures (orc_thermo, bin b at energy e_first + b de).
 * Outputs: over the nboot replicates, mean and sample standard deviation of
 * the joined ln g per bin (over the replicates where it is finite) and of U
 * and C_v per temperature.  Returns ORC_ESTATE if a replicate cannot be
 * joined.                                                                   */
int orc_bootstrap(int R, int h, int W, const int32_t *start, int e_lo, int B, const double *pieces,
                  const uint8_t *vis, double log_total, int nboot, uint64_t seed, const double *T,
                  int nT, double e_first, double de, double *lng_mean, double *lng_std,
                  double *U_mean, double *U_std, double *C_mean, double *C_std)
{
    if (R < 1 || h < 1 || W < 1 || nboot < 1 || nT < 0) return ORC_EINVAL;
    size_t HW = (size_t)h * W;
    int *draw = (int *)malloc((size_t)R * sizeof(int));
    uint8_t *vu = (uint8_t *)calloc(HW, 1);
    double *mp = (double *)malloc(HW * sizeof(double));
    double *reps = (double *)malloc((size_t)nboot * B * sizeof(double));
    double *ru = (double *)malloc(((size_t)nboot * nT + 1) * sizeof(double));
    double *rc = (double *)malloc(((size_t)nboot * nT + 1) * sizeof(double));
    double *lz = (double *)malloc(((size_t)nT + 1) * sizeof(double));
    int32_t *cuts = (int32_t *)malloc((size_t)(h > 1 ? h - 1 : 1) * sizeof(int32_t));
    int st = ORC_OK;
    if (!draw || !vu || !mp || !reps || !ru || !rc || !lz || !cuts) { st = ORC_ENOMEM; goto done; }
    for (int r = 0; r < R; ++r)
        for (size_t i = 0; i < HW; ++i) vu[i] |= vis[(size_t)r * HW + i] ? 1 : 0;
    {
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        for (int j = 0; j < nboot && st == ORC_OK; ++j) {
            for (int i = 0; i < R; i += 4) {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(i / 4), 0u, (uint32_t)DOM_BOOT << 24};
                uint32_t w[4];
                philox4x32_10(ctr, key, w);
                for (int t = 0; t < 4 && i + t < R; ++t)
                    draw[i + t] = (int)(((uint64_t)w[t] * (uint64_t)R) >> 32);
            }
            for (size_t c = 0; c < HW; ++c) {
                double sum = 0.0;
                for (int i = 0; i < R; ++i) sum = sum + pieces[(size_t)draw[i] * HW + c];
                mp[c] = sum / (double)R;
            }
            st = orc_join_pieces(h, W, start, e_lo, B, mp, vu, log_total, reps + (size_t)j * B, cuts);
            if (st == ORC_OK && nT > 0)
                orc_thermo(reps + (size_t)j * B, B, e_first, de, T, nT, lz, ru + (size_t)j * nT,
                           rc + (size_t)j * nT);
        }
    }
    if (st != ORC_OK) goto done;
    for (int b = 0; b < B; ++b) finite_stats(reps + b, nboot, (size_t)B, lng_mean + b, lng_std + b);
    for (int t = 0; t < nT; ++t) {
        finite_stats(ru + t, nboot, (size_t)nT, U_mean + t, U_std + t);
        finite_stats(rc + t, nboot, (size_t)nT, C_mean + t, C_std + t);
    }
done:
    free(draw); free(vu); free(mp); free(reps); free(ru); free(rc); free(lz); free(cuts);
    return st;
}

/* Walker w's observable record: H(E, O) [W][obs_bins], sum of O [W] and
 * samples [W] per energy bin of its window; -1 if O is not sampled.         */
int orc_get_obs(const orc_t *o, int w, uint32_t *hist, uint64_t *sum, uint32_t *count)
{
    if (o->obs_bins <= 0 || w < 0 || w >= o->nw) return ORC_EINVAL;
    size_t W = (size_t)o->W, nb = (size_t)o->obs_bins;
    if (hist) memcpy(hist, o->obs_hist + (size_t)w * W * nb, W * nb * sizeof(uint32_t));
    if (sum) memcpy(sum, o->obs_sum + (size_t)w * W, W * sizeof(uint64_t));
    if (count) memcpy(count, o->obs_cnt + (size_t)w * W, W * sizeof(uint32_t));
    return ORC_OK;
}

/* Microcanonical mean of O per energy bin of the whole range: the samples of
 * every walker whose window holds the bin, pooled (with weights that depend
 * on E only, the distribution of O at fixed E does not depend on them).
 * mean[b] = NaN where no sample fell.                                       */
int orc_obs_micro(const orc_t *o, double *mean, uint64_t *count)
{
    if (o->obs_bins <= 0) return ORC_EINVAL;
    for (int b = 0; b < o->B; ++b) {
        uint64_t s = 0, c = 0;
        for (int k = 0; k < o->h; ++k) {
            int lb = b - (o->start[k] - o->e_lo);
            if (lb < 0 || lb >= o->W) continue;
            for (int j = 0; j < o->m; ++j) {
                size_t cell = (size_t)(k * o->m + j) * o->W + (size_t)lb;
                s += o->obs_sum[cell];
                c += o->obs_cnt[cell];
            }
        }
        mean[b] = c ? (double)s / (double)c : NAN;
        if (count) count[b] = c;
    }
    return ORC_OK;
}

/* Canonical average of O at temperature T (Sec. 3.2 with Sec. 3.1's
 * canonical weights): <O>_T = sum_E g(E) e^{-E/T} mu(E) / sum_E g(E) e^{-E/T}
 * over the bins where ln g is finite and mu(E) was sampled, with the
 * largest exponent factored out.                                            */
void orc_obs_thermo(const double *lng, const double *mu, int B, double e_first, double de,
                    const double *T, int nT, double *out)
{
    for (int t = 0; t < nT; ++t) {
        double mx = -INFINITY;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY || isnan(mu[b])) continue;
            double x = lng[b] - (e_first + (double)b * de) / T[t];
            if (x > mx) mx = x;
        }
        double z = 0.0, num = 0.0;
        for (int b = 0; b < B; ++b) {
            if (lng[b] == -INFINITY || isnan(mu[b])) continue;
            double p = exp((lng[b] - (e_first + (double)b * de) / T[t]) - mx);
            z += p;
            num += p * mu[b];
        }
        out[t] = num / z;
    }
}
