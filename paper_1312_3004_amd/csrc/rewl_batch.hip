// rewl_batch.hip -- host side of the batched form (include/rewl.h, "Batched
// form"): many independent REWL runs advanced together by one persistent
// attempt kernel, batched sync/exchange kernels and a replayed HIP graph,
// plus the launch-plan autotuner.
//
// Workspace: [descriptor table | task lists | counters | status | queue]
// followed by one single-run workspace per instance (rewl_create layout).
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "rewl_host.h"

using rewl_gpu::BatchStatus;
using rewl_gpu::BatchTask;
using rewl_gpu::DevState;
using namespace rewl_host;

namespace {

constexpr int64_t kWalkinChunk = int64_t(1) << 20;
constexpr int kStatusEvery = 16;   // batched steps between convergence reads

struct BatchLayout {
    size_t descs, tasks, tasks_inst, tasks_cls, wtasks, xtasks, ctl, status, queue, slots, inst0, total;
    std::vector<size_t> inst;      // offset of each instance's workspace
    std::vector<size_t> inst_bytes;
};

bool valid_instances(int n, const rewl_instance *inst) {
    if (n < 1 || n > 65535 || !inst) return false;
    for (int i = 0; i < n; ++i)
        if (rewl_workspace_bytes(inst[i].model, inst[i].L, inst[i].q, inst[i].windows, inst[i].overlap,
                                 inst[i].walkers, &inst[i].opts) == 0)
            return false;
    return true;
}

BatchLayout batch_layout(int n, const rewl_instance *inst) {
    BatchLayout l{};
    int64_t walkers = 0, windows = 0, pairs = 0;
    for (int i = 0; i < n; ++i) {
        walkers += (int64_t)inst[i].windows * inst[i].walkers;
        windows += inst[i].windows;
        pairs += std::max(inst[i].windows / 2, 0);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = round_up(off + std::max(bytes, (size_t)1), kAlign);
        return at;
    };
    l.descs = take(sizeof(DevState) * n);
    l.tasks = take(sizeof(BatchTask) * walkers);
    l.tasks_inst = take(sizeof(BatchTask) * walkers);
    l.tasks_cls = take(sizeof(BatchTask) * walkers);
    l.wtasks = take(sizeof(BatchTask) * windows);
    l.xtasks = take(sizeof(BatchTask) * pairs);
    l.ctl = take(sizeof(int64_t) * 2 * n);
    l.status = take(sizeof(BatchStatus) * n);
    l.queue = take(sizeof(int) * 64);
    l.slots = take(sizeof(rewl_gpu::SlotPlan));
    l.inst0 = off;
    for (int i = 0; i < n; ++i) {
        const size_t bytes = rewl_workspace_bytes(inst[i].model, inst[i].L, inst[i].q, inst[i].windows,
                                                  inst[i].overlap, inst[i].walkers, &inst[i].opts);
        l.inst.push_back(take(bytes));
        l.inst_bytes.push_back(bytes);
    }
    l.total = off;
    return l;
}

}  // namespace

struct rewl_batch {
    int n = 0, precision = 0, cus = 0;
    std::vector<rewl *> inst;
    BatchLayout lay;
    unsigned char *ws = nullptr;
    hipStream_t stream = nullptr;     // caller's stream
    hipStream_t capture = nullptr;    // library stream used only to capture the step graph
    DevState *d_descs = nullptr;
    BatchTask *d_tasks = nullptr, *d_tasks_inst = nullptr, *d_tasks_cls = nullptr, *d_wtasks = nullptr,
              *d_xtasks = nullptr;
    int64_t *d_ctl = nullptr;
    BatchStatus *d_status = nullptr;
    int *d_queue = nullptr;
    std::vector<int> task_lo, win_lo, pair_lo;   // per-instance offsets in the instance-major lists
    int ntasks = 0, nwin = 0, npairs = 0;
    std::vector<int> ntag;                        // per-instance tag entries under the plan
    std::vector<size_t> lds_inst;                 // per-instance attempt-kernel LDS under the plan
    // instance classes of the mixed-slot form: instances of equal LDS state and
    // lattice size, largest LDS need first (at most kMaxClasses)
    int nclasses = 0;
    std::vector<int> cls_of;                      // class of each instance
    std::vector<int> cls_task_lo, cls_task_n;     // class ranges of d_tasks_cls
    rewl_gpu::SlotPlan slots{};
    rewl_gpu::SlotPlan *d_slots = nullptr;
    rewl_batch_plan plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t steps = 0;
    int32_t n_converged = 0;
    bool any_obs = false;                         // some instance samples an observable
    Timer timer;
};

namespace {

void drop_graph(rewl_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Upload the descriptor table with the plan's tag-table sizes and the batch's
// device counters.
int upload_descs(rewl_batch *b) {
    std::vector<DevState> d(b->n);
    for (int i = 0; i < b->n; ++i) {
        d[i] = b->inst[i]->st;
        d[i].Ntag = b->ntag[i];
        d[i].ctl = b->d_ctl + 2 * i;
    }
    HIP_TRY(hipMemcpyAsync(b->d_descs, d.data(), sizeof(DevState) * b->n, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return REWL_OK;
}

// Counters from the instance handles (which the single-run API may have
// moved) to the device; every instance must sit on a sync point.
int upload_ctl(rewl_batch *b) {
    std::vector<int64_t> ctl(2 * (size_t)b->n);
    for (int i = 0; i < b->n; ++i) {
        const rewl *r = b->inst[i];
        if (!r->converged && r->step % r->opts.sync_attempts != 0)
            return fail(REWL_ESTATE, "instance " + std::to_string(i) + " is between sync points");
        ctl[2 * i] = r->step;
        ctl[2 * i + 1] = r->round;
    }
    HIP_TRY(hipMemcpyAsync(b->d_ctl, ctl.data(), sizeof(int64_t) * ctl.size(), hipMemcpyHostToDevice, b->stream));
    return REWL_OK;
}

// Device counters and convergence back into the instance handles.
int download_status(rewl_batch *b) {
    std::vector<BatchStatus> s(b->n);
    HIP_TRY(rewl_gpu::launch_status_batch(b->d_descs, b->n, b->d_status, b->stream));
    HIP_TRY(hipMemcpyAsync(s.data(), b->d_status, sizeof(BatchStatus) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    int conv = 0;
    for (int i = 0; i < b->n; ++i) {
        rewl *r = b->inst[i];
        r->step = s[i].step;
        r->round = s[i].round;
        r->converged = s[i].converged != 0;
        r->joined = false;
        conv += r->converged ? 1 : 0;
    }
    b->n_converged = conv;
    return REWL_OK;
}

int walkin_all(rewl_batch *b, int64_t budget) {
    bool all = true;
    for (rewl *r : b->inst) all = all && r->walked_in;
    if (all) return REWL_OK;
    size_t lds = 0;
    for (rewl *r : b->inst) lds = std::max(lds, rewl_gpu::walkin_lds_bytes(r->st));
    std::vector<BatchStatus> s(b->n);
    for (;;) {
        HIP_TRY(rewl_gpu::launch_walkin_batch(b->d_descs, b->d_tasks_inst, b->ntasks, lds, kWalkinChunk, budget,
                                              b->stream));
        HIP_TRY(rewl_gpu::launch_walkin_status(b->d_descs, b->n, budget, b->d_status, b->stream));
        HIP_TRY(hipMemcpyAsync(s.data(), b->d_status, sizeof(BatchStatus) * b->n, hipMemcpyDeviceToHost,
                               b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        bool pending = false, stuck = false;
        for (int i = 0; i < b->n; ++i) {
            pending = pending || s[i].walkin != 0;
            stuck = stuck || s[i].walkin == 2;
        }
        if (stuck) return fail(REWL_EBUDGET, "walk-in exceeded its attempt budget");
        if (!pending) break;
    }
    for (rewl *r : b->inst) r->walked_in = true;
    return REWL_OK;
}

// Enqueue one persistent batched step on `s`.
hipError_t enqueue_step(rewl_batch *b, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (b->plan.mixed) {
        e = rewl_gpu::launch_sweep_batch_slots(b->precision, b->d_descs, b->d_tasks_cls, b->d_slots,
                                               b->slots.nclasses, b->slots.nslots, b->d_queue, b->plan.grid,
                                               (size_t)b->plan.lds_bytes, s);
    } else {
        e = rewl_gpu::launch_queue_reset(b->d_queue, s);
        if (e == hipSuccess)
            e = rewl_gpu::launch_sweep_batch(b->precision, b->d_descs, b->d_tasks, 0, b->ntasks, b->d_queue,
                                             b->plan.grid, (size_t)b->plan.lds_bytes, s);
    }
    if (e == hipSuccess) e = rewl_gpu::launch_sync_batch(b->precision, b->d_descs, b->d_wtasks, 0, b->nwin, s);
    if (e == hipSuccess) e = rewl_gpu::launch_exchange_batch(b->d_descs, b->d_xtasks, 0, b->npairs, s);
    if (e == hipSuccess && b->any_obs) e = rewl_gpu::launch_measure_batch(b->d_descs, b->d_tasks_inst, 0, b->ntasks, s);
    if (e == hipSuccess) e = rewl_gpu::launch_advance_batch(b->d_descs, 0, b->n, s);
    return e;
}

int capture_graph(rewl_batch *b) {
    drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
    const hipError_t e = enqueue_step(b, b->capture);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(REWL_EDEVICE, std::string("batched step capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(REWL_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return REWL_OK;
}

hipError_t batch_timer_begin(rewl_batch *b, hipEvent_t *ev) {
    if (!b->timer.on) return hipSuccess;
    hipError_t e = hipEventCreate(ev);
    if (e != hipSuccess) return e;
    return hipEventRecord(*ev, b->stream);
}

hipError_t batch_timer_end(rewl_batch *b, hipEvent_t start) {
    if (!b->timer.on) return hipSuccess;
    hipEvent_t stop;
    hipError_t e = hipEventCreate(&stop);
    if (e != hipSuccess) return e;
    e = hipEventRecord(stop, b->stream);
    if (e != hipSuccess) return e;
    b->timer.pending[0].push_back({start, stop});
    return hipSuccess;
}

hipError_t batch_timer_fold(rewl_batch *b) {
    for (auto &pr : b->timer.pending[0]) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return e;
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return e;
        b->timer.ms[0] += ms;
        b->timer.count[0] += 1;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    b->timer.pending[0].clear();
    return hipSuccess;
}

int run_steps(rewl_batch *b, int64_t steps, bool per_instance) {
    if (steps < 0) return fail(REWL_EINVAL, "negative step count");
    int st = walkin_all(b, int64_t(1) << 40);
    if (st != REWL_OK) return st;
    st = upload_ctl(b);
    if (st != REWL_OK) return st;
    if (!per_instance && b->plan.use_graph && !b->exec) {
        st = capture_graph(b);
        if (st != REWL_OK) return st;
    }
    for (int64_t s = 0; s < steps; ++s) {
        hipEvent_t ev = nullptr;
        HIP_TRY(batch_timer_begin(b, &ev));
        if (per_instance) {
            for (int i = 0; i < b->n; ++i) {
                const rewl *r = b->inst[i];
                const int nw = r->st.nw, h = r->st.h;
                HIP_TRY(rewl_gpu::launch_sweep_batch(b->precision, b->d_descs, b->d_tasks_inst, b->task_lo[i], nw,
                                                     nullptr, 0, b->lds_inst[i], b->stream));
                HIP_TRY(rewl_gpu::launch_sync_batch(b->precision, b->d_descs, b->d_wtasks, b->win_lo[i], h,
                                                    b->stream));
                HIP_TRY(rewl_gpu::launch_exchange_batch(b->d_descs, b->d_xtasks, b->pair_lo[i], h / 2, b->stream));
                if (r->st.obs_bins > 0)
                    HIP_TRY(rewl_gpu::launch_measure_batch(b->d_descs, b->d_tasks_inst, b->task_lo[i], nw, b->stream));
                HIP_TRY(rewl_gpu::launch_advance_batch(b->d_descs, i, 1, b->stream));
            }
        } else if (b->plan.use_graph) {
            HIP_TRY(hipGraphLaunch(b->exec, b->stream));
        } else {
            HIP_TRY(enqueue_step(b, b->stream));
        }
        HIP_TRY(batch_timer_end(b, ev));
        b->steps += 1;
        if ((s + 1) % kStatusEvery == 0 && s + 1 < steps) {
            st = download_status(b);
            if (st != REWL_OK) return st;
            if (b->n_converged == b->n) break;
        }
    }
    st = download_status(b);
    if (st != REWL_OK) return st;
    return b->n_converged == b->n ? REWL_CONVERGED : REWL_OK;
}

// Tag-table entries and LDS of every instance for a plan; false if some
// instance does not fit the LDS share.
bool plan_layout(const rewl_batch *b, int wpc, int policy, std::vector<int> *ntag, std::vector<size_t> *lds,
                 size_t *lds_max) {
    const size_t share = wpc > 0 ? ((size_t)kMaxLds / (size_t)wpc) / 512 * 512 : (size_t)kMaxLds;
    ntag->assign(b->n, 64);
    lds->assign(b->n, 0);
    *lds_max = 0;
    for (int i = 0; i < b->n; ++i) {
        const DevState &d = b->inst[i]->st;
        const size_t state = sweep_state_lds(d.Npad, d.Wpad, false);
        if (state + 64 * 8 > share) return false;
        (*ntag)[i] = policy == 0 ? tag_entries(d.N, share - state) : 64;
        (*lds)[i] = state + (size_t)(*ntag)[i] * 8;
        *lds_max = std::max(*lds_max, (*lds)[i]);
    }
    return true;
}

// Tag entries of a walker with N sites when its table may take `tag_bytes`.
int capped_tags(int N, int tag_bytes) {
    int t = 64;
    while (t < N && t < 4096 && 2 * t * 8 <= tag_bytes) t *= 2;
    return t;
}

int apply_mixed(rewl_batch *b, rewl_batch_plan *p) {
    if (p->tag_bytes < 512) return fail(REWL_EINVAL, "tag_bytes must be >= 512");
    std::vector<int> ntag(b->n);
    std::vector<size_t> lds(b->n);
    std::vector<size_t> cls_lds(b->nclasses, 0);
    for (int i = 0; i < b->n; ++i) {
        const DevState &d = b->inst[i]->st;
        ntag[i] = capped_tags(d.N, p->tag_bytes);
        lds[i] = sweep_state_lds(d.Npad, d.Wpad, false) + (size_t)ntag[i] * 8;
        size_t &cl = cls_lds[b->cls_of[i]];
        cl = std::max(cl, round_up(lds[i], 256));
    }
    rewl_gpu::SlotPlan sp{};
    sp.nclasses = b->nclasses;
    int nslots = 0;
    size_t total = 0;
    for (int c = 0; c < b->nclasses; ++c) {
        const int k = p->slot_count[c];
        if (k < 0) return fail(REWL_EINVAL, "slot counts must be >= 0");
        for (int j = 0; j < k; ++j) {
            if (nslots >= rewl_gpu::kMaxSlots) return fail(REWL_EINVAL, "at most 16 slots per CU");
            sp.cls[nslots] = c;
            sp.off[nslots] = (int)total;
            total += cls_lds[c];
            ++nslots;
        }
        sp.task_lo[c] = b->cls_task_lo[c];
        sp.task_n[c] = b->cls_task_n[c];
    }
    if (nslots < 1 || p->slot_count[0] < 1)
        return fail(REWL_EINVAL, "the largest class needs at least one slot (it serves every class)");
    if (total > (size_t)kMaxLds) return fail(REWL_EINVAL, "slots exceed the 160 KiB LDS of a CU");
    sp.nslots = nslots;
    int fits = 0;
    HIP_TRY(rewl_gpu::sweep_batch_slots_fits(b->precision, total, nslots, &fits));
    if (!fits) return fail(REWL_EINVAL, "a CU cannot hold this slot mix");
    drop_graph(b);
    b->ntag = ntag;
    b->lds_inst = lds;
    b->slots = sp;
    HIP_TRY(hipMemcpyAsync(b->d_slots, &sp, sizeof(sp), hipMemcpyHostToDevice, b->stream));
    rewl_batch_plan q = *p;
    q.mixed = 1;
    q.use_graph = p->use_graph ? 1 : 0;
    q.lds_bytes = (int32_t)total;
    q.grid = b->cus;
    q.resident = nslots;
    q.nclasses = b->nclasses;
    for (int c = 0; c < 8; ++c) {
        q.class_lds[c] = c < b->nclasses ? (int32_t)cls_lds[c] : 0;
        if (c >= b->nclasses) q.slot_count[c] = 0;
    }
    b->plan = q;
    *p = q;
    return upload_descs(b);
}

int apply_plan(rewl_batch *b, rewl_batch_plan *p) {
    if (p->mixed) return apply_mixed(b, p);
    if (p->tag_policy < 0 || p->tag_policy > 1) return fail(REWL_EINVAL, "tag_policy must be 0 or 1");
    if (p->walkers_per_cu < 0) return fail(REWL_EINVAL, "walkers_per_cu must be >= 0");
    std::vector<int> ntag;
    std::vector<size_t> lds;
    size_t lds_max = 0;
    int wpc = p->walkers_per_cu;
    int resident = 0;
    if (wpc == 0) {
        // largest count whose LDS share fits every instance and the CU's registers
        for (int c = 64; c >= 1; --c) {
            if (!plan_layout(b, c, p->tag_policy, &ntag, &lds, &lds_max)) continue;
            HIP_TRY(rewl_gpu::sweep_batch_occupancy(b->precision, lds_max, &resident));
            if (resident >= c) { wpc = c; break; }
        }
        if (wpc == 0) return fail(REWL_EINVAL, "an instance does not fit the LDS of a CU");
    }
    if (!plan_layout(b, wpc, p->tag_policy, &ntag, &lds, &lds_max))
        return fail(REWL_EINVAL, "an instance does not fit an LDS share of 160 KiB / walkers_per_cu");
    HIP_TRY(rewl_gpu::sweep_batch_occupancy(b->precision, lds_max, &resident));
    if (resident < wpc) return fail(REWL_EINVAL, "the CU cannot hold walkers_per_cu attempt workgroups");
    drop_graph(b);
    b->ntag = ntag;
    b->lds_inst = lds;
    b->plan = rewl_batch_plan{};
    b->plan.nclasses = b->nclasses;
    b->plan.walkers_per_cu = wpc;
    b->plan.tag_policy = p->tag_policy;
    b->plan.use_graph = p->use_graph ? 1 : 0;
    b->plan.lds_bytes = (int32_t)lds_max;
    b->plan.grid = wpc * b->cus;
    b->plan.resident = resident;
    b->plan.ms_per_step = p->ms_per_step;
    *p = b->plan;
    return upload_descs(b);
}

}  // namespace

extern "C" {

size_t rewl_batch_workspace_bytes(int n, const rewl_instance *inst) {
    if (!valid_instances(n, inst)) return 0;
    return batch_layout(n, inst).total;
}

void rewl_batch_destroy(rewl_batch_t *b) {
    if (!b) return;
    drop_graph(b);
    (void)batch_timer_fold(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (rewl *r : b->inst) {
        r->in_batch = false;
        rewl_destroy(r);
    }
    delete b;
}

int rewl_batch_create(rewl_batch_t **out, int n, const rewl_instance *inst, const int8_t *init_spins,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream) {
    if (!out) return fail(REWL_EINVAL, "null handle pointer");
    *out = nullptr;
    if (!inst || n < 1 || n > 65535) return fail(REWL_EINVAL, "n must be in [1, 65535] with instances");
    for (int i = 0; i < n; ++i)
        if (inst[i].opts.precision != inst[0].opts.precision)
            return fail(REWL_EINVAL, "instances of a batch must share precision");
    if (!valid_instances(n, inst)) {
        // report the first invalid instance's own message
        for (int i = 0; i < n; ++i)
            if (rewl_workspace_bytes(inst[i].model, inst[i].L, inst[i].q, inst[i].windows, inst[i].overlap,
                                     inst[i].walkers, &inst[i].opts) == 0)
                return fail(REWL_EINVAL, "instance " + std::to_string(i) + ": " + rewl_last_error());
    }
    if (!init_spins) return fail(REWL_EINVAL, "init_spins is required");
    const BatchLayout lay = batch_layout(n, inst);
    if (!dev_workspace) return fail(REWL_EINVAL, "null device workspace");
    if (ws_bytes < lay.total) return fail(REWL_ENOMEM, "device workspace smaller than rewl_batch_workspace_bytes");
    if (((uintptr_t)dev_workspace) % kAlign != 0) return fail(REWL_EINVAL, "workspace must be 256-byte aligned");

    rewl_batch *b = new (std::nothrow) rewl_batch();
    if (!b) return fail(REWL_ENOMEM, "host allocation failed");
    auto bail = [&](int code) { rewl_batch_destroy(b); return code; };
    b->n = n;
    b->precision = inst[0].opts.precision;
    b->lay = lay;
    b->ws = (unsigned char *)dev_workspace;
    b->stream = (hipStream_t)hip_stream;
    b->d_descs = (DevState *)(b->ws + lay.descs);
    b->d_tasks = (BatchTask *)(b->ws + lay.tasks);
    b->d_tasks_inst = (BatchTask *)(b->ws + lay.tasks_inst);
    b->d_wtasks = (BatchTask *)(b->ws + lay.wtasks);
    b->d_xtasks = (BatchTask *)(b->ws + lay.xtasks);
    b->d_ctl = (int64_t *)(b->ws + lay.ctl);
    b->d_status = (BatchStatus *)(b->ws + lay.status);
    b->d_queue = (int *)(b->ws + lay.queue);
    b->d_slots = (rewl_gpu::SlotPlan *)(b->ws + lay.slots);

    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("rewl_batch_create: ") + hipGetErrorString(e)));
    b->cus = prop.multiProcessorCount;
    e = hipMemsetAsync(b->ws, 0, lay.inst0, b->stream);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e)));

    // instances, in their own slices of the workspace
    size_t spin_off = 0;
    for (int i = 0; i < n; ++i) {
        rewl_t *r = nullptr;
        const int st = rewl_create(&r, inst[i].model, inst[i].L, inst[i].q, inst[i].windows, inst[i].overlap,
                                   inst[i].walkers, &inst[i].opts, init_spins + spin_off, b->ws + lay.inst[i],
                                   lay.inst_bytes[i], hip_stream);
        if (st != REWL_OK) {
            const std::string msg = rewl_last_error();
            return bail(fail(st, "instance " + std::to_string(i) + ": " + msg));
        }
        r->in_batch = true;
        b->any_obs = b->any_obs || r->st.obs_bins > 0;
        b->inst.push_back(r);
        spin_off += (size_t)inst[i].windows * inst[i].walkers * inst[i].L * inst[i].L;
    }

    // task lists: instance-major, and the persistent order (longest first:
    // attempts per walker per step, ties in instance-major order)
    std::vector<BatchTask> tasks_inst, wtasks, xtasks;
    for (int i = 0; i < n; ++i) {
        const DevState &d = b->inst[i]->st;
        b->task_lo.push_back((int)tasks_inst.size());
        for (int w = 0; w < d.nw; ++w) tasks_inst.push_back({i, w});
        b->win_lo.push_back((int)wtasks.size());
        for (int k = 0; k < d.h; ++k) wtasks.push_back({i, k});
        b->pair_lo.push_back((int)xtasks.size());
        for (int p = 0; p < d.h / 2; ++p) xtasks.push_back({i, p});
    }
    std::vector<BatchTask> tasks = tasks_inst;
    std::stable_sort(tasks.begin(), tasks.end(), [&](const BatchTask &x, const BatchTask &y) {
        return b->inst[x.inst]->opts.sync_attempts > b->inst[y.inst]->opts.sync_attempts;
    });
    // classes: distinct (LDS state, sites), ordered by LDS need with exact tags
    {
        std::vector<std::pair<size_t, int>> keys;   // (need, sites) per instance
        for (int i = 0; i < n; ++i) {
            const DevState &d = b->inst[i]->st;
            keys.push_back({sweep_state_lds(d.Npad, d.Wpad, false) + (size_t)std::min(d.N, 4096) * 8, d.N});
        }
        std::vector<std::pair<size_t, int>> uniq = keys;
        std::sort(uniq.begin(), uniq.end(), [](const auto &x, const auto &y) { return x > y; });
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        b->cls_of.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            const int pos = (int)(std::find(uniq.begin(), uniq.end(), keys[i]) - uniq.begin());
            b->cls_of[i] = std::min(pos, rewl_gpu::kMaxClasses - 1);
        }
        b->nclasses = std::min((int)uniq.size(), rewl_gpu::kMaxClasses);
        std::vector<BatchTask> tcls;
        for (int c = 0; c < b->nclasses; ++c) {
            b->cls_task_lo.push_back((int)tcls.size());
            for (const BatchTask &t : tasks_inst)
                if (b->cls_of[t.inst] == c) tcls.push_back(t);
            b->cls_task_n.push_back((int)tcls.size() - b->cls_task_lo.back());
        }
        b->d_tasks_cls = (BatchTask *)(b->ws + lay.tasks_cls);
        e = hipMemcpyAsync(b->d_tasks_cls, tcls.data(), sizeof(BatchTask) * tcls.size(), hipMemcpyHostToDevice,
                           b->stream);
        if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("rewl_batch_create: ") + hipGetErrorString(e)));
    }
    b->ntasks = (int)tasks.size();
    b->nwin = (int)wtasks.size();
    b->npairs = (int)xtasks.size();
    e = hipMemcpyAsync(b->d_tasks, tasks.data(), sizeof(BatchTask) * tasks.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_tasks_inst, tasks_inst.data(), sizeof(BatchTask) * tasks_inst.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_wtasks, wtasks.data(), sizeof(BatchTask) * wtasks.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && !xtasks.empty())
        e = hipMemcpyAsync(b->d_xtasks, xtasks.data(), sizeof(BatchTask) * xtasks.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bail(fail(REWL_EDEVICE, std::string("rewl_batch_create: ") + hipGetErrorString(e)));

    rewl_batch_plan p{};
    p.use_graph = 1;
    const int st = apply_plan(b, &p);
    if (st != REWL_OK) return bail(st);
    *out = b;
    return REWL_OK;
}

int rewl_batch_instance(rewl_batch_t *b, int i, rewl_t **out) {
    if (!b || !out) return fail(REWL_EINVAL, "null argument");
    if (i < 0 || i >= b->n) return fail(REWL_EINVAL, "instance index out of range");
    *out = b->inst[i];
    return REWL_OK;
}

int rewl_batch_walkin(rewl_batch_t *b, int64_t max_attempts) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    if (max_attempts < 0) return fail(REWL_EINVAL, "negative walk-in budget");
    return walkin_all(b, max_attempts);
}

int rewl_batch_set_plan(rewl_batch_t *b, rewl_batch_plan *plan) {
    if (!b || !plan) return fail(REWL_EINVAL, "null argument");
    return apply_plan(b, plan);
}

int rewl_batch_get_plan(rewl_batch_t *b, rewl_batch_plan *plan) {
    if (!b || !plan) return fail(REWL_EINVAL, "null argument");
    *plan = b->plan;
    return REWL_OK;
}

int rewl_batch_run(rewl_batch_t *b, int64_t steps) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    return run_steps(b, steps, false);
}

int rewl_batch_run_per_instance(rewl_batch_t *b, int64_t steps) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    return run_steps(b, steps, true);
}

int rewl_batch_tune(rewl_batch_t *b, int steps_per_plan, rewl_batch_plan *tried, int cap, int *n_tried) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    if (steps_per_plan < 1) return fail(REWL_EINVAL, "steps_per_plan must be >= 1");
    int st = walkin_all(b, int64_t(1) << 40);
    if (st != REWL_OK) return st;
    // candidates: walkers-per-CU counts (1..6, then every second or fourth up
    // to what the LDS and registers allow), for both tag policies; a plan
    // whose layout equals an earlier one is skipped
    std::vector<rewl_batch_plan> cands;
    std::vector<std::vector<int>> seen;
    for (int policy = 0; policy <= (b->nclasses > 1 ? 0 : 1); ++policy) {
        for (int c = 1; c <= 64; c += (c < 6 ? 1 : c < 16 ? 2 : 4)) {
            std::vector<int> ntag;
            std::vector<size_t> lds;
            size_t lds_max = 0;
            if (!plan_layout(b, c, policy, &ntag, &lds, &lds_max)) break;
            int resident = 0;
            HIP_TRY(rewl_gpu::sweep_batch_occupancy(b->precision, lds_max, &resident));
            if (resident < c) break;
            std::vector<int> key = ntag;
            key.push_back(c);
            if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
            seen.push_back(key);
            rewl_batch_plan p{};
            p.walkers_per_cu = c;
            p.tag_policy = policy;
            p.use_graph = 0;
            cands.push_back(p);
        }
    }
    // mixed-slot plans.  Tasks of class c run on slots of classes 0..c, so with
    // k_c slots of class c the step takes at least
    //   max_c (work of classes 0..c) / (slots of classes 0..c);
    // every slot mix within the LDS and the 16 waves of a CU is ranked by that
    // bound and the best few (per tag-table cap) are timed.
    if (b->nclasses > 1 && b->nclasses <= 6) {
        std::vector<double> work(b->nclasses, 0.0);
        for (int i = 0; i < b->n; ++i)
            work[b->cls_of[i]] += (double)b->inst[i]->st.nw * (double)b->inst[i]->opts.sync_attempts;
        for (int tag_bytes : {4096, 8192, 16384}) {
            std::vector<size_t> cl(b->nclasses, 0);
            for (int i = 0; i < b->n; ++i) {
                const DevState &d = b->inst[i]->st;
                const size_t need = sweep_state_lds(d.Npad, d.Wpad, false) + (size_t)capped_tags(d.N, tag_bytes) * 8;
                cl[b->cls_of[i]] = std::max(cl[b->cls_of[i]], round_up(need, 256));
            }
            std::vector<std::pair<double, std::vector<int>>> ranked;
            std::vector<int> k(b->nclasses, 0);
            // depth-first over slot counts, class 0 first
            std::vector<int> stack_pos;
            std::function<void(int, int, size_t)> rec = [&](int c, int used, size_t lds) {
                if (c == b->nclasses) {
                    if (k[0] < 1) return;
                    double bound = 0.0, wsum = 0.0;
                    int ksum = 0;
                    for (int x = 0; x < b->nclasses; ++x) {
                        wsum += work[x];
                        ksum += k[x];
                        bound = std::max(bound, ksum > 0 ? wsum / ksum : 1e300);
                    }
                    ranked.push_back({bound, k});
                    return;
                }
                for (int v = 0; used + v <= rewl_gpu::kMaxSlots && lds + (size_t)v * cl[c] <= (size_t)kMaxLds; ++v) {
                    k[c] = v;
                    rec(c + 1, used + v, lds + (size_t)v * cl[c]);
                }
                k[c] = 0;
            };
            rec(0, 0, 0);
            std::sort(ranked.begin(), ranked.end(),
                      [](const auto &x, const auto &y) { return x.first < y.first; });
            int taken = 0;
            for (const auto &rk : ranked) {
                if (taken >= 4) break;
                size_t lds = 0;
                int ns = 0;
                for (int c = 0; c < b->nclasses; ++c) { lds += (size_t)rk.second[c] * cl[c]; ns += rk.second[c]; }
                int fits = 0;
                HIP_TRY(rewl_gpu::sweep_batch_slots_fits(b->precision, lds, ns, &fits));
                if (!fits) continue;
                rewl_batch_plan p{};
                p.mixed = 1;
                p.tag_bytes = tag_bytes;
                for (int c = 0; c < b->nclasses; ++c) p.slot_count[c] = rk.second[c];
                cands.push_back(p);
                ++taken;
            }
        }
    }
    if (cands.empty()) return fail(REWL_EINVAL, "no feasible plan");
    const bool timing_was_on = b->timer.on;
    HIP_TRY(batch_timer_fold(b));
    const double saved_ms = b->timer.ms[0];
    const int64_t saved_n = b->timer.count[0];
    int best = -1;
    int done = 0;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        rewl_batch_plan p = cands[ci];
        st = apply_plan(b, &p);
        if (st != REWL_OK) return st;
        b->timer.on = true;
        b->timer.ms[0] = 0.0;
        b->timer.count[0] = 0;
        st = run_steps(b, steps_per_plan, false);
        HIP_TRY(batch_timer_fold(b));
        if (st < 0) return st;
        p.ms_per_step = b->timer.count[0] > 0 ? b->timer.ms[0] / (double)b->timer.count[0] : 0.0;
        cands[ci] = p;
        if (tried && done < cap) tried[done] = p;
        ++done;
        if (best < 0 || p.ms_per_step < cands[best].ms_per_step) best = (int)ci;
        if (st == REWL_CONVERGED) break;
    }
    b->timer.on = timing_was_on;
    b->timer.ms[0] = saved_ms;
    b->timer.count[0] = saved_n;
    if (n_tried) *n_tried = done;
    rewl_batch_plan p = cands[best];
    p.use_graph = 1;
    st = apply_plan(b, &p);
    if (st != REWL_OK) return st;
    return b->n_converged == b->n ? REWL_CONVERGED : REWL_OK;
}

namespace {

// Device scratch of a bootstrap: offsets of its buffers (256-byte aligned).
struct BootLayout {
    size_t draws, pieces, vis, beta, shift, cuts, status, joined, T, th, out, total;
};

BootLayout boot_layout(const DevState &d, int R, int nboot, int nT) {
    BootLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = round_up(off + bytes, 256);
        return at;
    };
    const size_t hw = (size_t)d.h * d.Wpad;
    l.draws = take(sizeof(int32_t) * (size_t)nboot * R);
    l.pieces = take(sizeof(double) * (size_t)nboot * hw);
    l.vis = take(hw);
    l.beta = take(sizeof(double) * (size_t)nboot * hw);
    l.shift = take(sizeof(double) * (size_t)nboot * d.h);
    l.cuts = take(sizeof(int32_t) * (size_t)nboot * d.h);
    l.status = take(sizeof(int32_t) * (size_t)nboot);
    l.joined = take(sizeof(double) * (size_t)nboot * d.Bpad);
    l.T = take(sizeof(double) * (size_t)(nT > 0 ? nT : 1));
    l.th = take(sizeof(double) * 3 * (size_t)nboot * (nT > 0 ? nT : 1));
    l.out = take(sizeof(double) * (2 * (size_t)d.B + 4 * (size_t)nT));
    l.total = off;
    return l;
}

// Every instance a run of the same Potts system (lattice, q, windows, walkers).
int check_same_system(const rewl_batch *b) {
    const rewl *a = b->inst[0];
    if (a->st.model != rewl_gpu::kModelPotts2D) return fail(REWL_EINVAL, "bootstrap needs Potts instances");
    for (const rewl *r : b->inst) {
        const DevState &d = r->st;
        if (d.model != a->st.model || d.L != a->st.L || d.q != a->st.q || d.h != a->st.h || d.m != a->st.m ||
            d.W != a->st.W || r->starts != a->starts)
            return fail(REWL_EINVAL, "bootstrap needs instances of one system (same L, q, windows, walkers, overlap)");
    }
    return REWL_OK;
}

}  // namespace

size_t rewl_batch_bootstrap_bytes(rewl_batch_t *b, int nboot, int nT) {
    if (!b || b->n < 1 || nboot < 1 || nT < 0) return 0;
    return boot_layout(b->inst[0]->st, b->n, nboot, nT).total;
}

int rewl_batch_bootstrap(rewl_batch_t *b, int nboot, uint64_t seed, const double *T, int nT, void *dev_scratch,
                         size_t scratch_bytes, double *lng_mean, double *lng_std, double *U_mean, double *U_std,
                         double *C_mean, double *C_std) {
    if (!b || !dev_scratch || !lng_mean || !lng_std) return fail(REWL_EINVAL, "null argument");
    if (nboot < 1 || nboot > 65535) return fail(REWL_EINVAL, "nboot must be in [1, 65535]");
    if (nT < 0 || nT > 4096) return fail(REWL_EINVAL, "nT must be in [0, 4096]");
    if (nT > 0 && (!T || !U_mean || !U_std || !C_mean || !C_std)) return fail(REWL_EINVAL, "null argument");
    for (int i = 0; i < nT; ++i)
        if (!(T[i] > 0.0)) return fail(REWL_EINVAL, "temperatures must be positive");
    int st = check_same_system(b);
    if (st != REWL_OK) return st;
    st = download_status(b);
    if (st != REWL_OK) return st;
    if (b->n_converged != b->n) return fail(REWL_ESTATE, "bootstrap needs every instance converged");
    const DevState &d = b->inst[0]->st;
    const BootLayout l = boot_layout(d, b->n, nboot, nT);
    if (scratch_bytes < l.total) return fail(REWL_EINVAL, "scratch smaller than rewl_batch_bootstrap_bytes");
    unsigned char *w = (unsigned char *)dev_scratch;
    rewl_gpu::BootArgs a{};
    a.R = b->n; a.h = d.h; a.W = d.W; a.Wpad = d.Wpad; a.B = d.B; a.Bpad = d.Bpad; a.e_lo = d.e_lo; a.m = d.m;
    a.nboot = nboot; a.nT = nT;
    a.key0 = (uint32_t)seed; a.key1 = (uint32_t)(seed >> 32);
    a.log_total = (double)d.N * std::log((double)d.q);
    a.e0 = (double)d.e_lo; a.de = 1.0;
    a.start = d.start;
    a.draws = (int32_t *)(w + l.draws);
    a.pieces = (double *)(w + l.pieces);
    a.vis = (uint8_t *)(w + l.vis);
    a.beta = (double *)(w + l.beta);
    a.shift = (double *)(w + l.shift);
    a.cuts = (int32_t *)(w + l.cuts);
    a.status = (int32_t *)(w + l.status);
    a.joined = (double *)(w + l.joined);
    a.T = (const double *)(w + l.T);
    a.th = (double *)(w + l.th);
    a.out = (double *)(w + l.out);
    if (nT > 0) HIP_TRY(hipMemcpyAsync((void *)a.T, T, sizeof(double) * nT, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(rewl_gpu::launch_bootstrap(a, b->d_descs, b->stream));
    std::vector<double> out(2 * (size_t)d.B + 4 * (size_t)nT);
    std::vector<int32_t> status(nboot);
    HIP_TRY(hipMemcpyAsync(out.data(), a.out, sizeof(double) * out.size(), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(status.data(), a.status, sizeof(int32_t) * nboot, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int j = 0; j < nboot; ++j)
        if (status[j] != 0) return fail(REWL_ESTATE, "a resample could not be joined (no common visited bin)");
    std::memcpy(lng_mean, out.data(), sizeof(double) * d.B);
    std::memcpy(lng_std, out.data() + d.B, sizeof(double) * d.B);
    const double *o = out.data() + 2 * (size_t)d.B;
    if (nT > 0) {
        std::memcpy(U_mean, o, sizeof(double) * nT);
        std::memcpy(U_std, o + nT, sizeof(double) * nT);
        std::memcpy(C_mean, o + 2 * nT, sizeof(double) * nT);
        std::memcpy(C_std, o + 3 * nT, sizeof(double) * nT);
    }
    return REWL_OK;
}

int rewl_batch_progress(rewl_batch_t *b, int64_t *steps, int32_t *converged) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    if (steps) *steps = b->steps;
    if (converged) *converged = b->n_converged;
    return REWL_OK;
}

int rewl_batch_set_timing(rewl_batch_t *b, int enable) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    HIP_TRY(batch_timer_fold(b));
    b->timer.on = enable != 0;
    b->timer.ms[0] = 0.0;
    b->timer.count[0] = 0;
    return REWL_OK;
}

int rewl_batch_get_timing(rewl_batch_t *b, double *ms, int64_t *steps) {
    if (!b) return fail(REWL_EINVAL, "null handle");
    HIP_TRY(batch_timer_fold(b));
    if (ms) *ms = b->timer.ms[0];
    if (steps) *steps = b->timer.count[0];
    return REWL_OK;
}

}  // extern "C"
