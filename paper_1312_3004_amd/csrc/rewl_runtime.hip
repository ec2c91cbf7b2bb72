// rewl_runtime.hip -- host side of librewl: the C ABI declared in
// include/rewl.h.  Validates arguments, carves the caller's device workspace
// into the run's state arrays, and enqueues the kernels of rewl_kernels.hip
// on the caller's stream in the order of the method (Sec. 2 of Vogel, Li,
// Wuest, Landau): attempts, then at every sync point flatness/averaging/ln f
// per window, a replica-exchange round, and the termination test.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rewl_host.h"

using rewl_gpu::DevState;
using namespace rewl_host;

namespace rewl_host {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Conflict-tag table of the attempt kernel: one 64-bit lane mask per site
// (exact) up to 4096 sites, hashed by site mod the table size beyond or when
// the LDS left after lattice and window state is smaller (a hash collision
// only sends an attempt down the exact recomputation path).
int tag_entries(int N, size_t lds_free) {
    int t = 64;
    while (t < N && t < 4096 && (size_t)t * 16 <= lds_free) t *= 2;
    return t;
}

size_t sweep_state_lds(int Npad, int Wpad, bool lng_in_lds) {
    return (size_t)Npad + (lng_in_lds ? (size_t)Wpad * 12 : 0);
}

}  // namespace rewl_host

namespace {

constexpr int kMaxThermo = 4096;
constexpr int64_t kWalkinChunk = int64_t(1) << 20;

struct Params {
    int L, q, N, h, m, nw, W, B, e_lo, Npad, Wpad, Bpad, Ntag;
    bool rows_glob = false;   // ln g and H rows in device memory (too large for LDS)
};

Layout make_layout(const Params &p, int precision, int shadow, bool trimer, int obs_bins) {
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = round_up(off + bytes, kAlign);
        return at;
    };
    l.start = take(sizeof(int32_t) * p.h);
    l.spins = take((size_t)p.nw * p.Npad);
    l.E = take(sizeof(int32_t) * p.nw);
    l.Ed = trimer ? take(sizeof(int64_t) * p.nw) : 0;
    l.lng = precision == 0 ? take(sizeof(double) * p.nw * p.Wpad) : 0;
    l.lng_hi = precision == 1 ? take(sizeof(float) * p.nw * p.Wpad) : 0;
    l.lng_lo = precision == 1 ? take(sizeof(float) * p.nw * p.Wpad) : 0;
    l.H = take(sizeof(uint32_t) * p.nw * p.Wpad);
    l.sh_hi = shadow ? take(sizeof(double) * p.nw * p.Wpad) : 0;
    l.sh_lo = shadow ? take(sizeof(double) * p.nw * p.Wpad) : 0;
    l.hprev = shadow ? take(sizeof(uint32_t) * p.nw * p.Wpad) : 0;
    l.replica = take(sizeof(uint32_t) * p.nw);
    l.rep_end = take(sizeof(int32_t) * p.nw);
    l.rep_trips = take(sizeof(uint32_t) * p.nw);
    l.rep_visits = p.nw <= rewl_gpu::kMaxVisitWalkers ? take(sizeof(uint32_t) * (size_t)p.nw * p.nw) : 0;
    l.walkin_att = take(sizeof(int64_t) * p.nw);
    l.walkin_done = take(sizeof(int32_t) * p.nw);
    l.walkin_bound = take(sizeof(int32_t) * p.nw);
    l.walkin_cnt = take(sizeof(uint32_t) * (size_t)p.nw * p.Bpad);
    l.lnf = take(sizeof(double) * p.h);
    l.lnf_last = take(sizeof(double) * p.h);
    l.regime = take(sizeof(int32_t) * p.h);
    l.finished = take(sizeof(int32_t) * p.h);
    l.iterations = take(sizeof(int64_t) * p.h);
    l.visited = take((size_t)p.h * p.Wpad);
    l.x_att = take(sizeof(uint64_t) * p.h);
    l.x_acc = take(sizeof(uint64_t) * p.h);
    l.converged = take(sizeof(int32_t));
    l.stop = take(sizeof(int64_t) * 2);
    l.joined = take(sizeof(double) * p.Bpad);
    l.cuts = take(sizeof(int32_t) * p.h);
    l.join_status = take(sizeof(int32_t));
    l.scratch = take(sizeof(double) * ((size_t)p.h * p.Wpad + p.h + 16));
    l.T = take(sizeof(double) * kMaxThermo);
    l.thermo_out = take(sizeof(double) * 3 * kMaxThermo);
    l.production = take(sizeof(int32_t));
    if (obs_bins > 0) {
        l.obs_hist = take(sizeof(uint32_t) * (size_t)p.nw * p.Wpad * obs_bins);
        l.obs_sum = take(sizeof(unsigned long long) * (size_t)p.nw * p.Wpad);
        l.obs_cnt = take(sizeof(uint32_t) * (size_t)p.nw * p.Wpad);
        l.obs_mean = take(sizeof(double) * p.Bpad);
        l.obs_count = take(sizeof(unsigned long long) * p.Bpad);
        if (trimer) l.obs_rec = take(sizeof(double) * 8 * (size_t)p.nw);
    }
    l.total = off;
    return l;
}

// Windows over B bins from e_lo (Sec. 2, Fig. 1): h windows of equal width W
// at overlap o, the first starting at e_lo and the last ending at e_lo+B-1.
int layout_bins(int B, int e_lo, int h, double o, int *W_out, int32_t *starts) {
    if (h < 1) return fail(REWL_EINVAL, "windows must be >= 1");
    if (!(o >= 0.0 && o < 1.0)) return fail(REWL_EINVAL, "overlap must be in [0, 1)");
    int W = B;
    if (h > 1) {
        const double denom = 1.0 + (double)(h - 1) * (1.0 - o);
        W = (int)std::ceil((double)B / denom);
        if (W > B) W = B;
    }
    if (W < 8) return fail(REWL_EINVAL, "windows narrower than 8 energies");
    for (int k = 0; k < h; ++k) {
        if (h == 1) { starts[k] = e_lo; continue; }
        const int64_t num = 2 * (int64_t)k * (B - W) + (h - 1);
        starts[k] = e_lo + (int32_t)(num / (2 * (int64_t)(h - 1)));
    }
    *W_out = W;
    return REWL_OK;
}

int layout_windows(int L, int h, double o, int *W_out, int32_t *starts) {
    if (L < 3 || L > 724) return fail(REWL_EINVAL, "L must be in [3, 724]");
    const int N = L * L;
    return layout_bins(2 * N + 1, -2 * N, h, o, W_out, starts);
}

int check_opts(int h, int m, const rewl_opts &op) {
    if (m < 1 || m > 1024) return fail(REWL_EINVAL, "walkers per window must be in [1, 1024]");
    if ((int64_t)h * m > 65535) return fail(REWL_EINVAL, "at most 65535 walkers");
    if (op.flat_den == 0 || op.flat_den > 1000 || op.flat_num > op.flat_den)
        return fail(REWL_EINVAL, "flatness must satisfy flat_num <= flat_den <= 1000");
    if (op.sync_attempts < 1) return fail(REWL_EINVAL, "sync_attempts must be >= 1");
    if (op.precision < 0 || op.precision > 1) return fail(REWL_EINVAL, "precision must be 0 or 1");
    if (op.schedule < 0 || op.schedule > 1) return fail(REWL_EINVAL, "schedule must be 0 or 1");
    if (op.shadow < 0 || op.shadow > 1) return fail(REWL_EINVAL, "shadow must be 0 or 1");
    if (op.walkin_slack < 0) return fail(REWL_EINVAL, "walkin_slack must be >= 0");
    if (op.obs_bins < 0) return fail(REWL_EINVAL, "obs_bins must be >= 0");
    if (op.reserved != 0) return fail(REWL_EINVAL, "opts.reserved must be 0");
    if (!(op.lnf_init >= 0.0) || !(op.lnf_final >= 0.0)) return fail(REWL_EINVAL, "ln f must be >= 0");
    return REWL_OK;
}

// Geometry of the continuous models (rewl_create_trimer, rewl_create_lipid).
struct TrimerGeom {
    int nmol;
    float box;
    double e_min, bin_w;
    int bins;
    int model = rewl_gpu::kModelTrimer3D;
    int nsol = 0;                 // lipid model: solvent particles
    double eps_ww = 1.0;          // lipid model: W-W depth
    uint32_t rep_thr = 0;         // lipid model: reptation threshold
    int off_type = 0, off_lip = 0, off_where = 0;
};

// Lipid model: check the geometry and lay out a walker's state row.
int check_lipid(TrimerGeom &g, int h, double o, int m, const rewl_opts &op, Params *p,
                std::vector<int32_t> *starts) {
    if (g.nmol < 1 || g.nsol < 0 || 3 * g.nmol + g.nsol > 4096)
        return fail(REWL_EINVAL, "lipids >= 1, solvent >= 0, at most 4096 particles");
    if (!(g.box > 0.0f) || !(g.box < 1e6f)) return fail(REWL_EINVAL, "box must be positive");
    if (!(g.bin_w * 0x1p32 >= 1.0 && g.bin_w * 0x1p32 <= 0x1p60) || !(std::fabs(g.e_min) < 0x1p28))
        return fail(REWL_EINVAL, "bin_w must lie in [2^-32, 2^28], |e_min| below 2^28");
    if (!(g.eps_ww >= 0.0) || !std::isfinite(g.eps_ww)) return fail(REWL_EINVAL, "eps_ww must be >= 0");
    if (g.bins < 8) return fail(REWL_EINVAL, "at least 8 energy bins");
    int st = check_opts(h, m, op);
    if (st != REWL_OK) return st;
    if (op.precision != 0 || op.shadow != 0)
        return fail(REWL_EINVAL, "the lipid model runs in binary64 without shadow");
    if (op.obs_bins > 0 && (op.obs_bins > 4096 || g.nmol > 512))
        return fail(REWL_EINVAL, "lipid observable sampling: obs_bins at most 4096, nlip at most 512");
    starts->assign((size_t)std::max(h, 1), 0);
    int W = 0;
    st = layout_bins(g.bins, 0, h, o, &W, starts->data());
    if (st != REWL_OK) return st;
    const int np = 3 * g.nmol + g.nsol;
    g.off_type = 12 * np;
    g.off_lip = g.off_type + (np + 3) / 4 * 4;
    g.off_where = g.off_lip + 12 * g.nmol;
    p->L = 0; p->q = 0; p->N = g.off_where + 4 * np; p->h = h; p->m = m; p->nw = h * m;
    p->W = W; p->B = g.bins; p->e_lo = 0;
    p->Npad = (int)round_up((size_t)p->N, kAlign);
    p->Wpad = (int)round_up((size_t)W, 64);
    p->Bpad = (int)round_up((size_t)p->B, 64);
    p->Ntag = 64;
    const size_t nch = (size_t)(np + 63) / 64;   // partner chunks of the attempt kernel's term buffer
    if ((size_t)p->Npad + (size_t)p->Wpad * 12 + nch * 64 * 8 + nch * 16 > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "particle state plus window state exceed the 160 KiB LDS of a CU");
    if ((size_t)p->Npad + (size_t)p->Bpad * 4 > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "walk-in counts over all bins exceed the 160 KiB LDS (too many bins)");
    return REWL_OK;
}

int check_trimer(const TrimerGeom &g, int h, double o, int m, const rewl_opts &op, Params *p,
                 std::vector<int32_t> *starts) {
    if (g.nmol < 1 || g.nmol > 1024) return fail(REWL_EINVAL, "nmol must be in [1, 1024]");
    if (!(g.box > 0.0f) || !(g.box < 1e6f)) return fail(REWL_EINVAL, "box must be positive");
    if (!(g.bin_w * 0x1p32 >= 1.0 && g.bin_w * 0x1p32 <= 0x1p60) || !(std::fabs(g.e_min) < 0x1p28))
        return fail(REWL_EINVAL, "bin_w must lie in [2^-32, 2^28], |e_min| below 2^28");
    if (g.bins < 8) return fail(REWL_EINVAL, "at least 8 energy bins");
    int st = check_opts(h, m, op);
    if (st != REWL_OK) return st;
    if (op.obs_bins != 0) return fail(REWL_EINVAL, "observable sampling (obs_bins) is defined for the Potts model only");
    starts->assign((size_t)std::max(h, 1), 0);
    int W = 0;
    st = layout_bins(g.bins, 0, h, o, &W, starts->data());
    if (st != REWL_OK) return st;
    p->L = 0; p->q = 0; p->N = 3 * g.nmol * 3 * (int)sizeof(float); p->h = h; p->m = m; p->nw = h * m;
    p->W = W; p->B = g.bins; p->e_lo = 0;
    p->Npad = (int)round_up((size_t)p->N, kAlign);
    p->Wpad = (int)round_up((size_t)W, 64);
    p->Bpad = (int)round_up((size_t)p->B, 64);
    p->Ntag = 64;
    // attempt kernel: coordinates, ln g and H, and up to two partner-term buffers
    const size_t tbuf = (size_t)2 * ((3 * g.nmol + 63) / 64) * 64 * 8;
    if ((size_t)p->Npad + (size_t)p->Wpad * 12 + tbuf > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "coordinates plus window state exceed the 160 KiB LDS of a CU");
    if ((size_t)p->Npad + (size_t)p->Bpad * 4 > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "walk-in counts over all bins exceed the 160 KiB LDS");
    return REWL_OK;
}

int check_params(int model, int L, int q, int h, double o, int m, const rewl_opts &op, Params *p,
                 std::vector<int32_t> *starts) {
    if (model != REWL_POTTS2D) return fail(REWL_EINVAL, "unknown model (the trimer model has rewl_create_trimer)");
    if (q < 2 || q > 127) return fail(REWL_EINVAL, "q must be in [2, 127]");
    int st = check_opts(h, m, op);
    if (st != REWL_OK) return st;
    if (L >= 3 && L <= 724 && op.obs_bins > L * L + 1) return fail(REWL_EINVAL, "obs_bins must be at most L*L+1");
    starts->assign((size_t)std::max(h, 1), 0);
    int W = 0;
    st = layout_windows(L, h, o, &W, starts->data());
    if (st != REWL_OK) return st;
    p->L = L; p->q = q; p->N = L * L; p->h = h; p->m = m; p->nw = h * m; p->W = W;
    p->B = 2 * p->N + 1; p->e_lo = -2 * p->N;
    p->Npad = (int)round_up((size_t)p->N, kAlign);
    p->Wpad = (int)round_up((size_t)W, 64);
    p->Bpad = (int)round_up((size_t)p->B, 64);
    // the attempt kernel stages the walker's ln g and H rows in LDS when they
    // fit beside the lattice and a minimal tag table, else reads them from
    // device memory (the same code, rows touched when the register cache moves)
    p->rows_glob = sweep_state_lds(p->Npad, p->Wpad) + 64 * 8 > (size_t)kMaxLds;
    const size_t lds_state = sweep_state_lds(p->Npad, p->Wpad, !p->rows_glob);
    p->Ntag = tag_entries(p->N, lds_state < (size_t)kMaxLds ? (size_t)kMaxLds - lds_state : 0);
    if (lds_state + (size_t)p->Ntag * 8 > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "the lattice exceeds the 160 KiB LDS of a CU");
    // one workgroup per walker: halve the tag table (down to 256 entries) while
    // that lets more of the walkers a CU must hold share its LDS, so that a
    // launch runs in one pass over the CUs where it can (a smaller table only
    // adds hashed candidates, which the kernel checks site by site)
    const int per_cu = (p->nw + kCUs - 1) / kCUs;
    auto fits = [&](int t) { return (int)((size_t)kMaxLds / (lds_state + (size_t)t * 8)); };
    while (p->Ntag > 256 && fits(p->Ntag) < per_cu && fits(p->Ntag / 2) > fits(p->Ntag)) p->Ntag /= 2;
    if ((size_t)p->Npad + (size_t)p->Bpad * 4 > (size_t)kMaxLds)
        return fail(REWL_EINVAL, "walk-in ln g over all energies exceeds the 160 KiB LDS (L too large)");
    return REWL_OK;
}

}  // namespace

namespace {

hipError_t timer_event(Timer &t, hipEvent_t *ev) {
    if (!t.pool.empty()) {
        *ev = t.pool.back();
        t.pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

hipError_t timer_fold(Timer &t) {
    for (int kind = 0; kind < 2; ++kind) {
        for (auto &pr : t.pending[kind]) {
            hipError_t e = hipEventSynchronize(pr.second);
            if (e != hipSuccess) return e;
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, pr.first, pr.second);
            if (e != hipSuccess) return e;
            t.ms[kind] += ms;
            t.count[kind] += 1;
            t.pool.push_back(pr.first);
            t.pool.push_back(pr.second);
        }
        t.pending[kind].clear();
    }
    return hipSuccess;
}

// Record the start event of a timed region of the given kind (0 attempts,
// 1 sync point) on the run's stream.
hipError_t timer_begin(rewl *r, hipEvent_t *ev) {
    if (!r->timer.on) return hipSuccess;
    if (r->timer.pending[0].size() + r->timer.pending[1].size() >= 4096) {
        hipError_t e = timer_fold(r->timer);
        if (e != hipSuccess) return e;
    }
    hipError_t e = timer_event(r->timer, ev);
    if (e != hipSuccess) return e;
    return hipEventRecord(*ev, r->stream);
}

hipError_t timer_end(rewl *r, int kind, hipEvent_t start) {
    if (!r->timer.on) return hipSuccess;
    hipEvent_t stop;
    hipError_t e = timer_event(r->timer, &stop);
    if (e != hipSuccess) return e;
    e = hipEventRecord(stop, r->stream);
    if (e != hipSuccess) return e;
    r->timer.pending[kind].push_back({start, stop});
    return hipSuccess;
}

void timer_destroy(Timer &t) {
    (void)timer_fold(t);
    for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
    t.pool.clear();
}

}  // namespace

extern "C" {

void rewl_default_opts(rewl_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->seed = 1;
    o->instance = 0;
    o->flat_num = 4;
    o->flat_den = 5;
    o->lnf_init = 1.0;
    o->lnf_final = 1e-6;
    o->schedule = 0;
    o->exchange = 1;
    o->sync_attempts = 1000;
    o->precision = 0;
    o->fixed_lnf = 0;
    o->shadow = 0;
    o->walkin_slack = 16;
}

const char *rewl_last_error(void) { return g_err.c_str(); }

int rewl_window_layout(int L, int windows, double overlap, int32_t *W, int32_t *starts) {
    if (!W || !starts) return fail(REWL_EINVAL, "null output pointer");
    int w = 0;
    const int st = layout_windows(L, windows, overlap, &w, starts);
    if (st == REWL_OK) *W = w;
    return st;
}

size_t rewl_workspace_bytes(int model, int L, int q, int windows, double overlap, int walkers,
                            const rewl_opts *opts) {
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    if (check_params(model, L, q, windows, overlap, walkers, op, &p, &starts) != REWL_OK) return 0;
    return make_layout(p, op.precision, op.shadow, false, op.obs_bins).total;
}

namespace {

// Shared part of rewl_create / rewl_create_trimer: carve the workspace, fill
// the device state, upload the starting configurations (p.N bytes per walker)
// and compute the starting energies.
int create_run(rewl_t **out, const Params &p, const std::vector<int32_t> &starts, const rewl_opts &op,
               const TrimerGeom *geom, const unsigned char *init, void *dev_workspace, size_t ws_bytes,
               void *hip_stream) {
    const Layout lay = make_layout(p, op.precision, op.shadow, geom != nullptr, op.obs_bins);
    if (!dev_workspace) return fail(REWL_EINVAL, "null device workspace");
    if (ws_bytes < lay.total) return fail(REWL_ENOMEM, "device workspace smaller than rewl_workspace_bytes");
    if (((uintptr_t)dev_workspace) % kAlign != 0) return fail(REWL_EINVAL, "workspace must be 256-byte aligned");

    rewl *r = new (std::nothrow) rewl();
    if (!r) return fail(REWL_ENOMEM, "host allocation failed");
    r->ws = (unsigned char *)dev_workspace;
    r->lay = lay;
    r->stream = (hipStream_t)hip_stream;
    r->opts = op;
    r->starts = starts;
    unsigned char *b = r->ws;
    DevState &d = r->st;
    std::memset(&d, 0, sizeof(d));
    d.model = geom ? geom->model : rewl_gpu::kModelPotts2D;
    if (geom) {
        d.nmol = geom->nmol; d.nb = 3 * geom->nmol + geom->nsol; d.box = geom->box;
        d.lip_eps_ww = geom->eps_ww; d.lip_rep_thr = geom->rep_thr;
        d.lip_off_type = geom->off_type; d.lip_off_lip = geom->off_lip; d.lip_off_where = geom->off_where;
        d.e_min = geom->e_min; d.bin_w = geom->bin_w;
        d.emin_fx = (int64_t)std::rint(geom->e_min * 0x1p32);
        d.binw_fx = (int64_t)std::rint(geom->bin_w * 0x1p32);
        d.binw_inv = 1.0 / (double)d.binw_fx;
        d.th_e0 = geom->e_min + 0.5 * geom->bin_w;   // bin centres
        d.th_de = geom->bin_w;
        d.Efx = (int64_t *)(b + lay.Ed);
    } else {
        d.th_e0 = (double)p.e_lo;
        d.th_de = 1.0;
    }
    d.L = p.L; d.q = p.q; d.N = p.N; d.h = p.h; d.m = p.m; d.nw = p.nw; d.W = p.W; d.B = p.B;
    d.e_lo = p.e_lo; d.Npad = p.Npad; d.Wpad = p.Wpad; d.Bpad = p.Bpad; d.Ntag = p.Ntag;
    d.rows_glob = p.rows_glob ? 1 : 0;
    d.key0 = (uint32_t)op.seed; d.key1 = (uint32_t)(op.seed >> 32);
    d.ctr3 = op.instance & 0xFFFFFFu;
    d.flat_num = op.flat_num; d.flat_den = op.flat_den;
    d.lnf_final = op.lnf_final;
    d.schedule = op.schedule; d.precision = op.precision; d.fixed_lnf = op.fixed_lnf;
    d.exchange = op.exchange; d.sync_attempts = op.sync_attempts; d.ctl = nullptr;
    d.shadow = op.shadow;
    d.walkin_slack = op.walkin_slack;
    d.start = (const int32_t *)(b + lay.start);
    d.spins = (int8_t *)(b + lay.spins);
    d.E = (int32_t *)(b + lay.E);
    d.lng = op.precision == 0 ? (double *)(b + lay.lng) : nullptr;
    d.lng_hi = op.precision == 1 ? (float *)(b + lay.lng_hi) : nullptr;
    d.lng_lo = op.precision == 1 ? (float *)(b + lay.lng_lo) : nullptr;
    d.H = (uint32_t *)(b + lay.H);
    d.sh_hi = op.shadow ? (double *)(b + lay.sh_hi) : nullptr;
    d.sh_lo = op.shadow ? (double *)(b + lay.sh_lo) : nullptr;
    d.hprev = op.shadow ? (uint32_t *)(b + lay.hprev) : nullptr;
    d.replica = (uint32_t *)(b + lay.replica);
    d.rep_end = (int32_t *)(b + lay.rep_end);
    d.rep_trips = (uint32_t *)(b + lay.rep_trips);
    d.rep_visits = p.nw <= rewl_gpu::kMaxVisitWalkers ? (uint32_t *)(b + lay.rep_visits) : nullptr;
    d.obs_bins = op.obs_bins;
    d.obs_hist = op.obs_bins > 0 ? (uint32_t *)(b + lay.obs_hist) : nullptr;
    d.obs_sum = op.obs_bins > 0 ? (unsigned long long *)(b + lay.obs_sum) : nullptr;
    d.obs_cnt = op.obs_bins > 0 ? (uint32_t *)(b + lay.obs_cnt) : nullptr;
    d.obs_rec = op.obs_bins > 0 && geom != nullptr ? (double *)(b + lay.obs_rec) : nullptr;
    d.obs_field = 3;
    d.obs_lo = d.obs_hi = 0.0;
    d.production = (int32_t *)(b + lay.production);
    d.walkin_att = (int64_t *)(b + lay.walkin_att);
    d.walkin_done = (int32_t *)(b + lay.walkin_done);
    d.walkin_bound = (int32_t *)(b + lay.walkin_bound);
    d.walkin_cnt = (uint32_t *)(b + lay.walkin_cnt);
    d.lnf = (double *)(b + lay.lnf);
    d.lnf_last = (double *)(b + lay.lnf_last);
    d.regime = (int32_t *)(b + lay.regime);
    d.finished = (int32_t *)(b + lay.finished);
    d.iterations = (int64_t *)(b + lay.iterations);
    d.visited = (uint8_t *)(b + lay.visited);
    d.x_att = (unsigned long long *)(b + lay.x_att);
    d.x_acc = (unsigned long long *)(b + lay.x_acc);
    d.converged = (int32_t *)(b + lay.converged);
    d.stop = (int64_t *)(b + lay.stop);
    d.joined = (double *)(b + lay.joined);
    d.cuts = (int32_t *)(b + lay.cuts);
    d.join_status = (int32_t *)(b + lay.join_status);
    d.scratch = (double *)(b + lay.scratch);

    auto bail = [&](int code) { delete r; return code; };
    // Conflict-tag table: as large as fits when every walker of the run is to
    // be resident at once (walkers per CU = walkers / CUs, at most 16, the
    // register limit of the attempt kernel), so no workgroup waits for a slot.
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("device query: ") + hipGetErrorString(e)));
    if (ncu > 0 && !geom) {
        const int per_cu = std::min((p.nw + ncu - 1) / ncu, 16);
        const size_t share = (size_t)kMaxLds / (size_t)per_cu;
        const size_t state = sweep_state_lds(p.Npad, p.Wpad, !p.rows_glob);
        if (share > state + 64 * 8) d.Ntag = std::min(d.Ntag, tag_entries(p.N, share - state));
        else d.Ntag = 64;
    }
    e = hipMemsetAsync(r->ws, 0, lay.total, r->stream);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e)));
    std::vector<int8_t> sp((size_t)p.nw * p.Npad, 0);
    for (int w = 0; w < p.nw; ++w) std::memcpy(&sp[(size_t)w * p.Npad], init + (size_t)w * p.N, p.N);
    std::vector<uint32_t> rep(p.nw);
    for (int w = 0; w < p.nw; ++w) rep[w] = (uint32_t)w;
    std::vector<double> lnf(p.h, op.lnf_init);
    e = hipMemcpyAsync((void *)d.start, starts.data(), sizeof(int32_t) * p.h, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.spins, sp.data(), sp.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.replica, rep.data(), sizeof(uint32_t) * p.nw, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.lnf, lnf.data(), sizeof(double) * p.h, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = rewl_gpu::launch_init_energy(d, r->stream);
    // replica paths start from the initial placement (replica w in slot w)
    if (e == hipSuccess) e = rewl_gpu::launch_track(d, r->stream);
    std::vector<int32_t> e0(geom ? p.nw : 0);
    if (e == hipSuccess && geom)
        e = hipMemcpyAsync(e0.data(), d.E, sizeof(int32_t) * p.nw, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("rewl_create: ") + hipGetErrorString(e)));
    // continuous models: the set-up kernel marks a start that holds a hard
    // overlap (a pair term of 2^18 or more) or lies out of the energy range
    for (int w = 0; w < (int)e0.size(); ++w)
        if (e0[w] == INT32_MIN)
            return bail(fail(REWL_EINVAL, "starting configuration " + std::to_string(w) +
                                              " holds a hard overlap (a pair energy of 2^18 or more) or an energy "
                                              "beyond 2^29"));
    *out = r;
    return REWL_OK;
}

}  // namespace


int rewl_create(rewl_t **out, int model, int L, int q, int windows, double overlap, int walkers,
                const rewl_opts *opts, const int8_t *init_spins, void *dev_workspace, size_t ws_bytes,
                void *hip_stream) {
    if (!out) return fail(REWL_EINVAL, "null handle pointer");
    *out = nullptr;
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    int st = check_params(model, L, q, windows, overlap, walkers, op, &p, &starts);
    if (st != REWL_OK) return st;
    if (!init_spins) return fail(REWL_EINVAL, "init_spins is required");
    for (size_t i = 0; i < (size_t)p.nw * p.N; ++i)
        if (init_spins[i] < 0 || init_spins[i] >= q) return fail(REWL_EINVAL, "spin value outside [0, q)");
    return create_run(out, p, starts, op, nullptr, (const unsigned char *)init_spins, dev_workspace, ws_bytes,
                      hip_stream);
}

size_t rewl_trimer_workspace_bytes(int nmol, float box, double e_min, double bin_w, int bins, int windows,
                                   double overlap, int walkers, const rewl_opts *opts) {
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    const TrimerGeom g{nmol, box, e_min, bin_w, bins};
    if (check_trimer(g, windows, overlap, walkers, op, &p, &starts) != REWL_OK) return 0;
    return make_layout(p, op.precision, op.shadow, true, op.obs_bins).total;
}

size_t rewl_lipid_workspace_bytes(int nlip, int nsol, float box, double eps_ww, double rep_prob, double e_min,
                                  double bin_w, int bins, int windows, double overlap, int walkers,
                                  const rewl_opts *opts) {
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    TrimerGeom g{nlip, box, e_min, bin_w, bins};
    g.model = rewl_gpu::kModelLipid3D; g.nsol = nsol; g.eps_ww = eps_ww;
    (void)rep_prob;
    if (check_lipid(g, windows, overlap, walkers, op, &p, &starts) != REWL_OK) return 0;
    return make_layout(p, op.precision, op.shadow, true, op.obs_bins).total;
}

int rewl_create_lipid(rewl_t **out, int nlip, int nsol, float box, double eps_ww, double rep_prob, double e_min,
                      double bin_w, int bins, int windows, double overlap, int walkers, const rewl_opts *opts,
                      const float *init_coords, void *dev_workspace, size_t ws_bytes, void *hip_stream) {
    if (!out) return fail(REWL_EINVAL, "null handle pointer");
    *out = nullptr;
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    TrimerGeom g{nlip, box, e_min, bin_w, bins};
    g.model = rewl_gpu::kModelLipid3D; g.nsol = nsol; g.eps_ww = eps_ww;
    const int np = 3 * nlip + nsol;
    if (rep_prob < 0.0) rep_prob = 3.0 * nlip / (10.0 * np);
    if (!(rep_prob <= 1.0)) return fail(REWL_EINVAL, "rep_prob must be <= 1");
    const double thr = std::nearbyint(rep_prob * 4294967296.0);
    g.rep_thr = thr >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)thr;
    int st = check_lipid(g, windows, overlap, walkers, op, &p, &starts);
    if (st != REWL_OK) return st;
    if (!init_coords) return fail(REWL_EINVAL, "init_coords is required");
    for (size_t i = 0; i < (size_t)p.nw * 3 * np; ++i)
        if (!(init_coords[i] >= 0.0f && init_coords[i] < box))
            return fail(REWL_EINVAL, "coordinate outside [0, box)");
    // state rows: particles 3i, 3i+1, 3i+2 start as lipid i (head, tail, tail)
    std::vector<unsigned char> rows((size_t)p.nw * p.N, 0);
    for (int w = 0; w < p.nw; ++w) {
        unsigned char *row = rows.data() + (size_t)w * p.N;
        std::memcpy(row, init_coords + (size_t)w * 3 * np, (size_t)12 * np);
        int8_t *type = (int8_t *)(row + g.off_type);
        int32_t *lip = (int32_t *)(row + g.off_lip);
        int32_t *where = (int32_t *)(row + g.off_where);
        for (int i = 0; i < np; ++i) {
            const bool in_lipid = i < 3 * nlip;
            type[i] = (int8_t)(in_lipid ? (i % 3 == 0 ? 0 : 1) : 2);
            where[i] = in_lipid ? i : -1;
        }
        for (int i = 0; i < 3 * nlip; ++i) lip[i] = i;
    }
    return create_run(out, p, starts, op, &g, rows.data(), dev_workspace, ws_bytes, hip_stream);
}

int rewl_get_particles(rewl_t *r, int w, float *coords, int8_t *types, int32_t *lipids) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    if (d.model != rewl_gpu::kModelLipid3D) return fail(REWL_EINVAL, "not a run of the lipid model");
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    const unsigned char *row = (const unsigned char *)(d.spins + (size_t)w * d.Npad);
    if (coords) HIP_TRY(hipMemcpyAsync(coords, row, (size_t)12 * d.nb, hipMemcpyDeviceToHost, r->stream));
    if (types) HIP_TRY(hipMemcpyAsync(types, row + d.lip_off_type, (size_t)d.nb, hipMemcpyDeviceToHost, r->stream));
    if (lipids)
        HIP_TRY(hipMemcpyAsync(lipids, row + d.lip_off_lip, (size_t)12 * d.nmol, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_create_trimer(rewl_t **out, int nmol, float box, double e_min, double bin_w, int bins, int windows,
                       double overlap, int walkers, const rewl_opts *opts, const float *init_coords,
                       void *dev_workspace, size_t ws_bytes, void *hip_stream) {
    if (!out) return fail(REWL_EINVAL, "null handle pointer");
    *out = nullptr;
    rewl_opts op;
    if (opts) op = *opts; else rewl_default_opts(&op);
    Params p;
    std::vector<int32_t> starts;
    const TrimerGeom g{nmol, box, e_min, bin_w, bins};
    int st = check_trimer(g, windows, overlap, walkers, op, &p, &starts);
    if (st != REWL_OK) return st;
    if (!init_coords) return fail(REWL_EINVAL, "init_coords is required");
    for (size_t i = 0; i < (size_t)p.nw * 9 * nmol; ++i)
        if (!(init_coords[i] >= 0.0f && init_coords[i] < box))
            return fail(REWL_EINVAL, "coordinate outside [0, box)");
    return create_run(out, p, starts, op, &g, (const unsigned char *)init_coords, dev_workspace, ws_bytes,
                      hip_stream);
}

int rewl_window_layout_bins(int bins, int windows, double overlap, int32_t *W, int32_t *starts) {
    if (!W || !starts) return fail(REWL_EINVAL, "null output pointer");
    if (bins < 8) return fail(REWL_EINVAL, "at least 8 bins");
    int w = 0;
    const int st = layout_bins(bins, 0, windows, overlap, &w, starts);
    if (st == REWL_OK) *W = w;
    return st;
}

int rewl_get_energy(rewl_t *r, int w, double *E) {
    if (!r || !E) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    if (d.Efx) {
        int64_t e = 0;
        HIP_TRY(hipMemcpyAsync(&e, d.Efx + w, sizeof(int64_t), hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
        *E = (double)e / 0x1p32;
    } else {
        int32_t e = 0;
        HIP_TRY(hipMemcpyAsync(&e, d.E + w, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
        *E = (double)e;
    }
    return REWL_OK;
}

int rewl_get_energy_fx(rewl_t *r, int w, int64_t *E) {
    if (!r || !E) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    if (d.Efx) {
        HIP_TRY(hipMemcpyAsync(E, d.Efx + w, sizeof(int64_t), hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
    } else {
        int32_t e = 0;
        HIP_TRY(hipMemcpyAsync(&e, d.E + w, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
        *E = e;
    }
    return REWL_OK;
}

void rewl_destroy(rewl_t *r) {
    if (!r || r->in_batch) return;
    timer_destroy(r->timer);
    delete r;
}

int rewl_set_timing(rewl_t *r, int enable) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    HIP_TRY(timer_fold(r->timer));
    r->timer.on = enable != 0;
    r->timer.ms[0] = r->timer.ms[1] = 0.0;
    r->timer.count[0] = r->timer.count[1] = 0;
    return REWL_OK;
}

int rewl_get_timing(rewl_t *r, double *sweep_ms, int64_t *sweep_launches, double *sync_ms,
                    int64_t *sync_points) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    HIP_TRY(timer_fold(r->timer));
    if (sweep_ms) *sweep_ms = r->timer.ms[0];
    if (sweep_launches) *sweep_launches = r->timer.count[0];
    if (sync_ms) *sync_ms = r->timer.ms[1];
    if (sync_points) *sync_points = r->timer.count[1];
    return REWL_OK;
}

int rewl_walkin(rewl_t *r, int64_t max_attempts) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (r->walked_in) return REWL_OK;
    if (max_attempts < 0) return fail(REWL_EINVAL, "negative walk-in budget");
    const int nw = r->st.nw;
    std::vector<int32_t> done(nw);
    std::vector<int64_t> att(nw);
    for (;;) {
        // the lipid model's attempts cost thousands of pair terms: shorter launches
        const int64_t chunk = r->st.model == rewl_gpu::kModelLipid3D ? int64_t(1) << 12 : kWalkinChunk;
        HIP_TRY(rewl_gpu::launch_walkin(r->st, chunk, max_attempts, r->stream));
        HIP_TRY(hipMemcpyAsync(done.data(), r->st.walkin_done, sizeof(int32_t) * nw, hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipMemcpyAsync(att.data(), r->st.walkin_att, sizeof(int64_t) * nw, hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
        bool all = true, stuck = false;
        for (int w = 0; w < nw; ++w) {
            if (!done[w]) {
                all = false;
                if (att[w] >= max_attempts) stuck = true;
            }
        }
        if (all) break;
        if (stuck) return fail(REWL_EBUDGET, "walk-in exceeded its attempt budget");
    }
    r->walked_in = true;
    return REWL_OK;
}

static int read_converged(rewl_t *r) {
    int32_t conv = 0;
    int64_t stop[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&conv, r->st.converged, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipMemcpyAsync(stop, r->st.stop, sizeof(stop), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (conv) {
        r->converged = true;
        r->step = stop[0];
        r->round = stop[1];
    }
    return REWL_OK;
}

int rewl_run_attempts(rewl_t *r, int64_t attempts) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (attempts < 0) return fail(REWL_EINVAL, "negative attempt count");
    if (!r->walked_in) {
        const int st = rewl_walkin(r, int64_t(1) << 40);
        if (st != REWL_OK) return st;
    }
    if (r->converged) return REWL_CONVERGED;
    r->joined = false;
    const int64_t S = r->opts.sync_attempts;
    int syncs_since_read = 0;
    while (attempts > 0) {
        int64_t seg = S - (r->step % S);
        if (seg > attempts) seg = attempts;
        hipEvent_t ev = nullptr;
        HIP_TRY(timer_begin(r, &ev));
        HIP_TRY(rewl_gpu::launch_sweep(r->st, r->step, seg, r->stream));
        HIP_TRY(timer_end(r, 0, ev));
        r->step += seg;
        attempts -= seg;
        if (r->step % S == 0) {
            HIP_TRY(timer_begin(r, &ev));
            HIP_TRY(rewl_gpu::launch_sync(r->st, r->step, r->stream));
            if (r->opts.exchange) {
                HIP_TRY(rewl_gpu::launch_exchange(r->st, (uint32_t)r->round, r->stream));
                r->round += 1;
            }
            if (r->st.obs_bins > 0) {
                if (r->st.model == rewl_gpu::kModelLipid3D)
                    HIP_TRY(rewl_gpu::launch_lipid_measure(r->st, r->stream));
                else
                    HIP_TRY(rewl_gpu::launch_measure(r->st, r->stream));
            }
            HIP_TRY(rewl_gpu::launch_check(r->st, r->step, r->round, r->stream));
            HIP_TRY(timer_end(r, 1, ev));
            if (!r->opts.fixed_lnf && ++syncs_since_read >= 64) {
                syncs_since_read = 0;
                const int st = read_converged(r);
                if (st != REWL_OK) return st;
                if (r->converged) return REWL_CONVERGED;
            }
        }
    }
    const int st = read_converged(r);
    if (st != REWL_OK) return st;
    return r->converged ? REWL_CONVERGED : REWL_OK;
}

int rewl_run(rewl_t *r, int64_t sweeps) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (sweeps < 0) return fail(REWL_EINVAL, "negative sweep count");
    return rewl_run_attempts(r, sweeps * (int64_t)r->st.N);
}

int rewl_exchange(rewl_t *r) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (r->converged) return REWL_CONVERGED;
    HIP_TRY(rewl_gpu::launch_exchange(r->st, (uint32_t)r->round, r->stream));
    HIP_TRY(rewl_gpu::launch_track(r->st, r->stream));
    r->round += 1;
    r->joined = false;
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_get_progress(rewl_t *r, int64_t *step, int64_t *round, int32_t *converged) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (step) *step = r->step;
    if (round) *round = r->round;
    if (converged) *converged = r->converged ? 1 : 0;
    return REWL_OK;
}

int rewl_begin_production(rewl_t *r) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (r->in_batch) return fail(REWL_ESTATE, "production runs are standalone, not instances of a batch");
    if (!r->walked_in) return fail(REWL_ESTATE, "rewl_begin_production needs a walked-in run");
    HIP_TRY(rewl_gpu::launch_begin_production(r->st, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    r->converged = false;
    r->joined = false;
    return REWL_OK;
}

int rewl_get_obs(rewl_t *r, int w, uint32_t *hist, uint64_t *sum, uint32_t *count) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    if (d.obs_bins <= 0) return fail(REWL_EINVAL, "the run samples no observable (opts.obs_bins = 0)");
    const size_t row = (size_t)w * d.Wpad;
    if (hist)
        HIP_TRY(hipMemcpyAsync(hist, d.obs_hist + row * d.obs_bins, sizeof(uint32_t) * d.W * d.obs_bins,
                               hipMemcpyDeviceToHost, r->stream));
    if (sum) HIP_TRY(hipMemcpyAsync(sum, d.obs_sum + row, sizeof(uint64_t) * d.W, hipMemcpyDeviceToHost, r->stream));
    if (count) HIP_TRY(hipMemcpyAsync(count, d.obs_cnt + row, sizeof(uint32_t) * d.W, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_obs_micro(rewl_t *r, double *mean, uint64_t *count) {
    if (!r || !mean) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (d.obs_bins <= 0) return fail(REWL_EINVAL, "the run samples no observable (opts.obs_bins = 0)");
    double *dmean = (double *)(r->ws + r->lay.obs_mean);
    unsigned long long *dcount = (unsigned long long *)(r->ws + r->lay.obs_count);
    HIP_TRY(rewl_gpu::launch_obs_micro(d, dmean, dcount, r->stream));
    HIP_TRY(hipMemcpyAsync(mean, dmean, sizeof(double) * d.B, hipMemcpyDeviceToHost, r->stream));
    if (count) HIP_TRY(hipMemcpyAsync(count, dcount, sizeof(uint64_t) * d.B, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_obs_thermo(rewl_t *r, const double *T, int nT, double *out) {
    if (!r || !T || !out) return fail(REWL_EINVAL, "null argument");
    if (nT < 1 || nT > kMaxThermo) return fail(REWL_EINVAL, "nT must be in [1, 4096]");
    const DevState &d = r->st;
    if (d.obs_bins <= 0) return fail(REWL_EINVAL, "the run samples no observable (opts.obs_bins = 0)");
    if (!r->joined) return fail(REWL_ESTATE, "rewl_obs_thermo needs a current rewl_join");
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0)) return fail(REWL_EINVAL, "temperatures must be positive");
    double *dT = (double *)(r->ws + r->lay.T);
    double *dout = (double *)(r->ws + r->lay.thermo_out);
    double *dmean = (double *)(r->ws + r->lay.obs_mean);
    unsigned long long *dcount = (unsigned long long *)(r->ws + r->lay.obs_count);
    HIP_TRY(hipMemcpyAsync(dT, T, sizeof(double) * nT, hipMemcpyHostToDevice, r->stream));
    HIP_TRY(rewl_gpu::launch_obs_micro(d, dmean, dcount, r->stream));
    HIP_TRY(rewl_gpu::launch_obs_thermo(d, dT, nT, dmean, dout, r->stream));
    HIP_TRY(hipMemcpyAsync(out, dout, sizeof(double) * nT, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_get_replicas(rewl_t *r, uint32_t *window_of, uint32_t *trips) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    std::vector<uint32_t> rep(d.nw);
    if (window_of)
        HIP_TRY(hipMemcpyAsync(rep.data(), d.replica, sizeof(uint32_t) * d.nw, hipMemcpyDeviceToHost, r->stream));
    if (trips) HIP_TRY(hipMemcpyAsync(trips, d.rep_trips, sizeof(uint32_t) * d.nw, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (window_of)
        for (int w = 0; w < d.nw; ++w) window_of[rep[w]] = (uint32_t)(w / d.m);
    return REWL_OK;
}

int rewl_get_replica_visits(rewl_t *r, int w, uint32_t *counts) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    if (!d.rep_visits) return fail(REWL_EINVAL, "visit matrix not kept for more than 4096 walkers");
    if (!counts) return fail(REWL_EINVAL, "null buffer");
    HIP_TRY(hipMemcpyAsync(counts, d.rep_visits + (size_t)w * d.nw, sizeof(uint32_t) * d.nw,
                           hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_get_walker(rewl_t *r, int w, int8_t *spins, int32_t *E, uint32_t *H, double *lng,
                    uint32_t *replica, int64_t *walkin_attempts) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    const size_t row = (size_t)w * d.Wpad;
    std::vector<float> hi, lo;
    if (spins) HIP_TRY(hipMemcpyAsync(spins, d.spins + (size_t)w * d.Npad, d.N, hipMemcpyDeviceToHost, r->stream));
    if (E) HIP_TRY(hipMemcpyAsync(E, d.E + w, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
    if (H) HIP_TRY(hipMemcpyAsync(H, d.H + row, sizeof(uint32_t) * d.W, hipMemcpyDeviceToHost, r->stream));
    if (lng && d.precision == 0)
        HIP_TRY(hipMemcpyAsync(lng, d.lng + row, sizeof(double) * d.W, hipMemcpyDeviceToHost, r->stream));
    if (lng && d.precision == 1) {
        hi.resize(d.W); lo.resize(d.W);
        HIP_TRY(hipMemcpyAsync(hi.data(), d.lng_hi + row, sizeof(float) * d.W, hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipMemcpyAsync(lo.data(), d.lng_lo + row, sizeof(float) * d.W, hipMemcpyDeviceToHost, r->stream));
    }
    if (replica) HIP_TRY(hipMemcpyAsync(replica, d.replica + w, sizeof(uint32_t), hipMemcpyDeviceToHost, r->stream));
    if (walkin_attempts)
        HIP_TRY(hipMemcpyAsync(walkin_attempts, d.walkin_att + w, sizeof(int64_t), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (lng && d.precision == 1)
        for (int b = 0; b < d.W; ++b) lng[b] = (double)hi[b] + (double)lo[b];
    return REWL_OK;
}

int rewl_get_state(rewl_t *r, int w, int8_t *spins, int32_t *E, uint32_t *H, double *lng, double *lnf) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    if (w < 0 || w >= r->st.nw) return fail(REWL_EINVAL, "walker index out of range");
    const int st = rewl_get_walker(r, w, spins, E, H, lng, nullptr, nullptr);
    if (st != REWL_OK || !lnf) return st;
    return rewl_get_window(r, w / r->st.m, lnf, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int rewl_get_window(rewl_t *r, int k, double *lnf, double *lnf_last, int32_t *regime, int32_t *finished,
                    int64_t *iterations, uint8_t *visited, uint64_t *x_att, uint64_t *x_acc) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    if (k < 0 || k >= d.h) return fail(REWL_EINVAL, "window index out of range");
    int32_t fin = 0;
    HIP_TRY(hipMemcpyAsync(&fin, d.finished + k, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
    if (lnf) HIP_TRY(hipMemcpyAsync(lnf, d.lnf + k, sizeof(double), hipMemcpyDeviceToHost, r->stream));
    if (lnf_last) HIP_TRY(hipMemcpyAsync(lnf_last, d.lnf_last + k, sizeof(double), hipMemcpyDeviceToHost, r->stream));
    if (regime) HIP_TRY(hipMemcpyAsync(regime, d.regime + k, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
    if (iterations) HIP_TRY(hipMemcpyAsync(iterations, d.iterations + k, sizeof(int64_t), hipMemcpyDeviceToHost, r->stream));
    if (x_att) HIP_TRY(hipMemcpyAsync(x_att, d.x_att + k, sizeof(uint64_t), hipMemcpyDeviceToHost, r->stream));
    if (x_acc) HIP_TRY(hipMemcpyAsync(x_acc, d.x_acc + k, sizeof(uint64_t), hipMemcpyDeviceToHost, r->stream));
    std::vector<uint32_t> Hs;
    if (visited) {
        HIP_TRY(hipMemcpyAsync(visited, d.visited + (size_t)k * d.Wpad, d.W, hipMemcpyDeviceToHost, r->stream));
        Hs.resize((size_t)d.m * d.Wpad);
        HIP_TRY(hipMemcpyAsync(Hs.data(), d.H + (size_t)k * d.m * d.Wpad, sizeof(uint32_t) * Hs.size(),
                               hipMemcpyDeviceToHost, r->stream));
    }
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (finished) *finished = fin;
    if (visited && !fin)
        for (int j = 0; j < d.m; ++j)
            for (int b = 0; b < d.W; ++b)
                if (Hs[(size_t)j * d.Wpad + b]) visited[b] = 1;
    return REWL_OK;
}

namespace {

// Checkpoint header: the run's identity (sizes and options that fix the
// workspace layout and the trajectory) and its host-side counters.
struct SaveHeader {
    char magic[8];          // "REWLCKP1" (Potts), "REWLCKP2" (continuous models)
    uint64_t ws_bytes;
    int32_t model, L, q, N, h, m, W, B, nmol, precision, shadow, fixed_lnf, schedule, exchange;
    float box;
    int32_t walkin_slack;
    double e_min, bin_w, lnf_init, lnf_final;
    uint64_t seed;
    uint32_t instance, flat_num, flat_den, reserved;
    int64_t sync_attempts, step, round;
    int32_t walked_in, converged;
};

SaveHeader make_header(const rewl *r) {
    SaveHeader h;
    std::memset(&h, 0, sizeof(h));
    // "REWLCKP2": continuous-model energies in fixed point (Potts rows unchanged)
    std::memcpy(h.magic, r->st.model == rewl_gpu::kModelPotts2D ? "REWLCKP1" : "REWLCKP2", 8);
    const DevState &d = r->st;
    h.ws_bytes = r->lay.total;
    h.model = d.model; h.L = d.L; h.q = d.q; h.N = d.N; h.h = d.h; h.m = d.m; h.W = d.W; h.B = d.B;
    h.nmol = d.nmol; h.precision = d.precision; h.shadow = d.shadow; h.fixed_lnf = d.fixed_lnf;
    h.schedule = d.schedule; h.exchange = d.exchange; h.box = d.box; h.walkin_slack = d.walkin_slack;
    h.e_min = d.e_min; h.bin_w = d.bin_w;
    h.lnf_init = r->opts.lnf_init; h.lnf_final = r->opts.lnf_final;
    h.seed = r->opts.seed; h.instance = r->opts.instance;
    h.flat_num = r->opts.flat_num; h.flat_den = r->opts.flat_den;
    h.reserved = (uint32_t)r->opts.obs_bins;
    h.sync_attempts = r->opts.sync_attempts;
    h.step = r->step; h.round = r->round;
    h.walked_in = r->walked_in ? 1 : 0;
    h.converged = r->converged ? 1 : 0;
    return h;
}

}  // namespace

int rewl_save(rewl_t *r, void *buf, size_t cap, size_t *n) {
    if (!r || !n) return fail(REWL_EINVAL, "null argument");
    const size_t need = sizeof(SaveHeader) + r->lay.total;
    *n = need;
    if (!buf) return REWL_OK;
    if (cap < need) return fail(REWL_ENOMEM, "checkpoint buffer smaller than the required size");
    const SaveHeader h = make_header(r);
    std::memcpy(buf, &h, sizeof(h));
    HIP_TRY(hipMemcpyAsync((unsigned char *)buf + sizeof(h), r->ws, r->lay.total, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_load(rewl_t *r, const void *buf, size_t n) {
    if (!r || !buf) return fail(REWL_EINVAL, "null argument");
    if (n < sizeof(SaveHeader)) return fail(REWL_EINVAL, "checkpoint too short");
    SaveHeader h;
    std::memcpy(&h, buf, sizeof(h));
    SaveHeader mine = make_header(r);
    if (std::memcmp(h.magic, "REWLCKP", 7) != 0) return fail(REWL_EINVAL, "not a checkpoint");
    // everything but the counters must match the handle
    SaveHeader a = h, b = mine;
    a.step = b.step = 0; a.round = b.round = 0;
    a.walked_in = b.walked_in = 0; a.converged = b.converged = 0;
    if (std::memcmp(&a, &b, sizeof(a)) != 0)
        return fail(REWL_EINVAL, "checkpoint of a run with other sizes or options");
    if (n < sizeof(SaveHeader) + h.ws_bytes) return fail(REWL_EINVAL, "checkpoint truncated");
    HIP_TRY(hipMemcpyAsync(r->ws, (const unsigned char *)buf + sizeof(h), r->lay.total, hipMemcpyHostToDevice,
                           r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    r->step = h.step;
    r->round = h.round;
    r->walked_in = h.walked_in != 0;
    r->converged = h.converged != 0;
    r->joined = false;
    return REWL_OK;
}

int rewl_get_shadow(rewl_t *r, int w, double *hi, double *lo) {
    if (!r || !hi || !lo) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    if (!d.shadow) return fail(REWL_ESTATE, "the run keeps no shadow (opts.shadow = 0)");
    const size_t row = (size_t)w * d.Wpad;
    HIP_TRY(hipMemcpyAsync(hi, d.sh_hi + row, sizeof(double) * d.W, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipMemcpyAsync(lo, d.sh_lo + row, sizeof(double) * d.W, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

int rewl_set_lng(rewl_t *r, int w, const double *lng) {
    if (!r || !lng) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (w < 0 || w >= d.nw) return fail(REWL_EINVAL, "walker index out of range");
    const size_t row = (size_t)w * d.Wpad;
    if (d.shadow) {   // the shadow restarts from the given values
        HIP_TRY(hipMemcpyAsync(d.sh_hi + row, lng, sizeof(double) * d.W, hipMemcpyHostToDevice, r->stream));
        HIP_TRY(hipMemsetAsync(d.sh_lo + row, 0, sizeof(double) * d.W, r->stream));
        HIP_TRY(hipMemcpyAsync(d.hprev + row, d.H + row, sizeof(uint32_t) * d.W, hipMemcpyDeviceToDevice,
                               r->stream));
    }
    if (d.precision == 0) {
        HIP_TRY(hipMemcpyAsync(d.lng + row, lng, sizeof(double) * d.W, hipMemcpyHostToDevice, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
    } else {
        std::vector<float> hi(d.W), lo(d.W);
        for (int b = 0; b < d.W; ++b) {
            hi[b] = (float)lng[b];
            lo[b] = (float)(lng[b] - (double)hi[b]);
        }
        HIP_TRY(hipMemcpyAsync(d.lng_hi + row, hi.data(), sizeof(float) * d.W, hipMemcpyHostToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(d.lng_lo + row, lo.data(), sizeof(float) * d.W, hipMemcpyHostToDevice, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
    }
    r->joined = false;
    return REWL_OK;
}

int rewl_join(rewl_t *r, double *host_out, int32_t *cuts) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    const DevState &d = r->st;
    // Potts: sum_E g(E) = q^N; trimer (no total count): sum over bins of g = 1
    const double log_total = d.model == rewl_gpu::kModelPotts2D ? (double)d.N * std::log((double)d.q) : 0.0;
    HIP_TRY(rewl_gpu::launch_join(d, log_total, r->stream));
    int32_t status = 0;
    HIP_TRY(hipMemcpyAsync(&status, d.join_status, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream));
    if (host_out) HIP_TRY(hipMemcpyAsync(host_out, d.joined, sizeof(double) * d.B, hipMemcpyDeviceToHost, r->stream));
    if (cuts && d.h > 1)
        HIP_TRY(hipMemcpyAsync(cuts, d.cuts, sizeof(int32_t) * (d.h - 1), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (status != 0) return fail(REWL_ESTATE, "two neighbouring windows share no visited energy");
    r->joined = true;
    return REWL_OK;
}

int rewl_get_lng(rewl_t *r, int k, double *host_out, int64_t cap, int64_t *n_out, int64_t *e_first_out) {
    if (!r || !host_out) return fail(REWL_EINVAL, "null argument");
    const DevState &d = r->st;
    if (k == -1) {
        if (cap < d.B) return fail(REWL_EINVAL, "output buffer too small");
        const int st = rewl_join(r, host_out, nullptr);
        if (n_out) *n_out = d.B;
        if (e_first_out) *e_first_out = d.e_lo;
        return st;
    }
    if (k < 0 || k >= d.h) return fail(REWL_EINVAL, "window index out of range");
    if (cap < d.W) return fail(REWL_EINVAL, "output buffer too small");
    std::vector<uint8_t> vis(d.W);
    int st = rewl_get_window(r, k, nullptr, nullptr, nullptr, nullptr, nullptr, vis.data(), nullptr, nullptr);
    if (st != REWL_OK) return st;
    st = rewl_get_walker(r, k * d.m, nullptr, nullptr, nullptr, host_out, nullptr, nullptr);
    if (st != REWL_OK) return st;
    for (int b = 0; b < d.W; ++b)
        if (!vis[b]) host_out[b] = -INFINITY;
    if (n_out) *n_out = d.W;
    if (e_first_out) *e_first_out = r->starts[k];
    return REWL_OK;
}

int rewl_thermo(rewl_t *r, const double *T, int nT, double *lnZ, double *U, double *C) {
    if (!r || !T) return fail(REWL_EINVAL, "null argument");
    if (nT < 1 || nT > kMaxThermo) return fail(REWL_EINVAL, "nT must be in [1, 4096]");
    if (!r->joined) return fail(REWL_ESTATE, "rewl_thermo needs a current rewl_join");
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0)) return fail(REWL_EINVAL, "temperatures must be positive");
    const DevState &d = r->st;
    double *dT = (double *)(r->ws + r->lay.T);
    double *dout = (double *)(r->ws + r->lay.thermo_out);
    std::vector<double> out(3 * (size_t)nT);
    HIP_TRY(hipMemcpyAsync(dT, T, sizeof(double) * nT, hipMemcpyHostToDevice, r->stream));
    HIP_TRY(rewl_gpu::launch_thermo(d, dT, nT, dout, r->stream));
    HIP_TRY(hipMemcpyAsync(out.data(), dout, sizeof(double) * 3 * nT, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    for (int i = 0; i < nT; ++i) {
        if (lnZ) lnZ[i] = out[3 * i + 0];
        if (U) U[i] = out[3 * i + 1];
        if (C) C[i] = out[3 * i + 2];
    }
    return REWL_OK;
}

}  // extern "C"
