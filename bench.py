"""Benchmark: spin-flip attempts/s of REWL on one MI355X, q=10 Potts L=32.

Workload potts_q10_L32: 2D q=10 Potts, 32x32 periodic, 16 windows at 75%
overlap, 4 walkers per window (64 walkers), flatness 0.8, ln f 1 -> 1e-8
(halving, then 1/t), exchange every 10^4 attempts per walker, binary64 ln g.
One step = one sync interval: 10^4 attempts for every walker, then the sync
point (flatness, averaging, ln f update) and a replica-exchange round.
Inputs are synthetic (uniform random starting lattices from a seed) and
resident on the GPU before the timed region; walk-in is timed separately.
The timed steps run where the workload spends its attempts: once every window
is in the 1/t regime (98% of the 4.3e10 attempts per walker to ln f < 1e-8);
the first steps after walk-in (ln f = 1) and the halving phase that leads to
the timed steps are measured and reported beside them.

Prints one JSON line; the roofline constants below carry their derivations.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic ALU work of one Potts attempt, in VALU issue slots per lane (a
# full-rate 32-bit or binary64 vector operation is one slot: unpacked fp32 and
# fp64 both issue at one operation per lane per clock on this part; a 32x32->64
# integer multiply is quarter rate, four slots):
#   Philox4x32-10 block: 10 rounds x (2 multiplies x 4 + 4 xor) + 9 key bumps x 2 adds = 138
#   proposal: site and new value by multiply-high (2 x 4) + add, compare, subtract      =  11
#   neighbour indices with periodic wrap: 4 x 3                                          =  12
#   energy change: 8 compares + 8 adds                                                   =  16
#   window test and E': 2 compares + 1 add                                               =   3
#   acceptance: d (1) + sign test (1) + uniform (3) + exp_poly (32) in the half of the
#     attempts with d < 0 (16)                                                           =  21
#   WL update: ln g add, H add, E select (2)                                             =   4
ALU_SLOTS_ITEMS = dict(philox=10 * (2 * 4 + 4) + 9 * 2, proposal=2 * 4 + 3, neighbours=4 * 3, delta_e=16,
                       window=3, acceptance=1 + 1 + 3 + 32 // 2, update=4)
ALU_SLOTS_PER_ATTEMPT = sum(ALU_SLOTS_ITEMS.values())
# MI355X vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13
# lane-slots/s (the 157.3 TFLOP/s fp32 figure counts packed FMAs as four flops;
# these kernels issue no packed fp32 and no FMA).
CU, SIMD_LANES, CLOCK_HZ = 256, 4 * 16, 2.4e9
VALU_LANE_SLOTS_PEAK = CU * SIMD_LANES * CLOCK_HZ
ALU_PEAK_TOPS = VALU_LANE_SLOTS_PEAK / 1e12
# Binary64 vector peak without FMA: one operation per lane per clock, 39.3
# TFLOP/s (the published 78.6 TFLOP/s counts an FMA as two flops).
FP64_UNFUSED_PEAK_TFLOPS = VALU_LANE_SLOTS_PEAK / 1e12
# Algorithmic LDS bytes per attempt (site and neighbours 5, ln g(E') 8, ln g(E)
# read-modify-write 16, H 8, spin 1); spec LDS peak 256 CUs x 128 B/clock x 2.4 GHz.
LDS_BYTES_PER_ATTEMPT = 38
LDS_PEAK_GBS = CU * 128 * CLOCK_HZ / 1e9
# HBM bytes per k_sweep launch of the potts_q10_L32 workload in its timed (1/t)
# phase, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a torch.neg
# copy of known size (profiles/k_sweep_potts_q10_L32_pmc.md): 268.18 KiB x 2.000
# + 390.0 KiB x 1.000.  Valid for the kernel as profiled.
K_SWEEP_L32_HBM_BYTES = 948_600
# VALU instructions (wave64) per attempt of the same kernel, rocprofv3 SQ_INSTS_VALU
# over the same workload (same profile).
K_SWEEP_L32_VALU_PER_ATTEMPT = 9.76
# 1/t phase ends once W/t < 1e-8, i.e. after W/1e-8 attempts per walker.


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """Host cores this process may use, and what the machine reports.

    usable = the CPUs in this process's affinity mask, capped by a cgroup CPU
    quota when one is set (a container's share of a larger host)."""
    info = {"nproc": os.cpu_count()}
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    info["affinity"] = aff
    usable = aff
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            quota, period = f.read().split()[:2]
        if quota != "max":
            info["cgroup_quota_cpus"] = int(quota) / int(period)
            usable = max(1, min(usable, int(int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    info["usable"] = usable
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    info["model"] = model
    return info


def oracle_threads(n_walkers):
    """One oracle thread per usable host core, at most one per walker."""
    hc = host_cpu()
    return max(1, min(hc["usable"], n_walkers)), hc


def cpu_baseline(cfg, spins, attempts_per_walker):
    import oracle

    nw = cfg["windows"] * cfg["walkers"]
    threads, hc = oracle_threads(nw)
    o = oracle.Rewl(cfg["L"], cfg["q"], cfg["windows"], cfg["overlap"], cfg["walkers"], spins,
                    seed=cfg["seed"], flat=cfg["flat"], lnf_init=cfg["lnf_init"],
                    lnf_final=cfg["lnf_final"], schedule=cfg["schedule"],
                    sync_attempts=cfg["sync_attempts"], exchange=cfg["exchange"],
                    precision=cfg["precision"], threads=threads)
    t0 = time.perf_counter()
    o.walkin()
    t1 = time.perf_counter()
    o.run(attempts_per_walker)
    t2 = time.perf_counter()
    return dict(value=nw * attempts_per_walker / (t2 - t1), unit="attempts/s", cores=threads,
                kind="oracle", host=hc,
                sample=(f"oracle walk-in ({t1 - t0:.1f} s, excluded) then {attempts_per_walker:,} "
                        f"main-phase attempts per walker of the same workload ({nw} walkers), "
                        f"{threads} OpenMP threads on {hc['model']}"))


def batched_roofline(attempts_per_step, step_s):
    """ALU and LDS roofline of the batched persistent step (k_sweep_batch*),
    priced per attempt like the single-run kernel, over the step wall time."""
    achieved = ALU_SLOTS_PER_ATTEMPT * attempts_per_step / step_s / 1e12
    lds = LDS_BYTES_PER_ATTEMPT * attempts_per_step / step_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / ALU_PEAK_TOPS, "traffic": None, "kernel": "k_sweep_batch_slots",
            "time_basis": "wall time of one batched step (graph replay)",
            "lds": {"achieved_gb_per_s": lds, "peak_gb_per_s": LDS_PEAK_GBS, "frac": lds / LDS_PEAK_GBS}}


def batched(args):
    """The 256-instance batched workload: autotuned persistent launch (graph
    replay) against one launch per instance, alternating step by step."""
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = workloads.BATCHED
    pairs = workloads.batched_instances(cfg)
    insts, spins = [], []
    for i, (L, q) in enumerate(pairs):
        insts.append(dict(L=L, q=q, windows=cfg["windows"], overlap=cfg["overlap"], walkers=cfg["walkers"],
                          seed=cfg["seed"], instance=i, flat=cfg["flat"], lnf_init=cfg["lnf_init"],
                          lnf_final=cfg["lnf_final"], schedule=cfg["schedule"],
                          sync_attempts=cfg["sweeps_per_sync"] * L * L, exchange=cfg["exchange"],
                          precision=cfg["precision"]))
        spins.append(workloads.init_spins(L, q, cfg["windows"] * cfg["walkers"], cfg["seed"] + i))
    attempts_per_step = sum(d["windows"] * d["walkers"] * d["sync_attempts"] for d in insts)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = pk.Batch(insts, spins, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.walkin()
    torch.cuda.synchronize()
    walkin_s = time.perf_counter() - t0
    log(f"[bench] batched walk-in done in {walkin_s:.2f} s")
    t0 = time.perf_counter()
    plan, trials = b.tune(steps_per_plan=1)
    tune_s = time.perf_counter() - t0
    log(f"[bench] tuned in {tune_s:.1f} s over {len(trials)} plans: {plan}")
    if args.warmup:
        b.run(args.warmup)
    torch.cuda.synchronize()
    # persistent steps, with one step of one-launch-per-instance in the middle
    t_batch = t_single = 0.0
    for i in range(args.steps):
        if i == args.steps // 2 and not args.no_per_instance:
            t0 = time.perf_counter()
            b.run_per_instance(1)
            torch.cuda.synchronize()
            t_single = time.perf_counter() - t0
            log(f"[bench] one launch per instance: {1e3 * t_single:.1f} ms per step")
        t0 = time.perf_counter()
        b.run(1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_batch += dt
        log(f"[bench] persistent step {i}: {1e3 * dt:.1f} ms")
    steps, conv = b.progress()
    value = attempts_per_step * args.steps / t_batch
    out = {
        "metric": "spin-flip attempts/s (1 GPU), 256 batched REWL instances",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_batch / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256 instances of 2D Potts, L in {16,24,32,48} and q in {2,4,8,10} drawn "
                               "from a seed, 8 windows at 75% overlap, 4 walkers each, sync every 1000 sweeps",
                   "instances": len(insts), "walkers": sum(d["windows"] * d["walkers"] for d in insts),
                   "attempts_per_step": attempts_per_step},
        "plan": plan,
        "tuner_trials": trials,
        "per_instance_launches": ({"value": attempts_per_step / t_single, "ms_per_step": 1e3 * t_single,
                                   "steps": 1} if t_single else None),
        "speedup_vs_per_instance": t_single / (t_batch / args.steps) if t_single else None,
        # the same per-attempt work as the single-run kernel (205 VALU issue
        # slots, 38 LDS bytes) against the step's wall time: one graph replay
        # is the attempt launch plus the small sync-point kernels
        "roofline": batched_roofline(attempts_per_step, t_batch / args.steps),
        "walkin_s": walkin_s,
        "tune_s": tune_s,
        "converged_instances": conv,
    }
    print(json.dumps(out), flush=True)


def walkin_with_progress(g, tag, budget=1 << 22):
    """Walk-in in growing attempt budgets, logging progress (placed walkers)."""
    import paper_1312_3004_amd as pk

    t0 = time.perf_counter()
    while True:
        try:
            g.walkin(budget=budget)
            break
        except pk.RewlError:
            placed = sum(1 for w in range(g.nw)
                         if g.starts[w // g.m] <= g.walker(w)["E"] <= g.starts[w // g.m] + g.W - 1)
            log(f"[bench] {tag} walk-in: {placed}/{g.nw} placed after {budget:,} attempts budget, "
                f"{time.perf_counter() - t0:.1f} s")
            budget *= 2
    return time.perf_counter() - t0


def precision_study(args):
    """The L=80 workload (64 windows x 16 walkers, ln f halved to 1e-9) to
    convergence three times: binary64 (seed 1), the binary32 (hi, lo) pair
    (seed 1, the same trajectory until the formats' roundings part it) and
    binary64 with seed 2.  Each run keeps the exact double-double shadow of
    its ln g.  Reports per run the wall time and its own accumulation error
    max |ln g - shadow|, and for the joined, normalised curves the largest
    difference between the two formats beside the spread between the two
    binary64 seeds.  --to-convergence sets this process's budget of seconds
    (default 600); with --checkpoint DIR the three runs can span several
    processes (the run in progress saved in DIR when the budget is spent and
    continued on the next call)."""
    import zlib

    import numpy as np
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS["potts_q10_L80"])
    L, q, h, m = cfg["L"], cfg["q"], cfg["windows"], cfg["walkers"]
    nw, S = h * m, cfg["sync_attempts"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spins = workloads.init_spins(L, q, nw, cfg["seed"])
    d = args.checkpoint or ""
    if d:
        os.makedirs(d, exist_ok=True)
    state_path = os.path.join(d, "precision.json") if d else None
    lnf_final = args.lnf_final if args.lnf_final > 0 else cfg["lnf_final"]
    state = {"runs": {}, "lnf_final": lnf_final}
    if state_path and os.path.exists(state_path):
        with open(state_path) as f:
            state = json.load(f)
        if state.get("lnf_final") != lnf_final:
            raise SystemExit(f"{state_path} holds runs to ln f < {state.get('lnf_final')}, not {lnf_final}")
    budget = args.to_convergence if args.to_convergence > 0 else 600.0
    t_start = time.perf_counter()
    runs = (("f64", 0, cfg["seed"]), ("f32x2", 1, cfg["seed"]), ("f64_seed2", 0, cfg["seed"] + 1))
    curves = {}
    started = 0
    for name, prec, seed in runs:
        rs = state["runs"].setdefault(name, {"seconds": 0.0, "segments": 0})
        npy = os.path.join(d, name + "_lng.npy") if d else None
        if rs.get("converged"):
            curves[name] = np.load(npy)
            continue
        if time.perf_counter() - t_start >= budget or (args.max_runs and started >= args.max_runs):
            break
        started += 1
        g = pk.Rewl(L, q, h, cfg["overlap"], m, spins, device=dev, seed=seed, flat=cfg["flat"],
                    lnf_init=cfg["lnf_init"], lnf_final=lnf_final, schedule=cfg["schedule"],
                    sync_attempts=S, exchange=cfg["exchange"], precision=prec, shadow=1)
        # saved states are zlib-compressed (the walk-in counts are mostly zeros)
        ck = os.path.join(d, name + ".bin.z") if d else None
        if ck and os.path.exists(ck):
            with open(ck, "rb") as f:
                g.load(zlib.decompress(f.read()))
        elif rs["segments"]:
            # its saved state is gone: the run starts again
            rs.update(seconds=0.0, segments=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, last = pk.OK, t0
        while time.perf_counter() - t_start < budget:
            st = g.run(200 * S)
            if st == pk.CONVERGED:
                break
            if time.perf_counter() - last > 30:
                torch.cuda.synchronize()
                ws = [g.window(k) for k in range(h)]
                lnf = [w["lnf"] for w in ws if not w["finished"]]
                log(f"[bench] precision {name}: step {g.step}, {rs['seconds'] + time.perf_counter() - t0:.0f} s, "
                    f"{h - len(lnf)}/{h} windows finished, ln f max {max(lnf) if lnf else 0.0:.3g}")
                last = time.perf_counter()
        torch.cuda.synchronize()
        rs["seconds"] += time.perf_counter() - t0
        rs["segments"] += 1
        rs["attempts_per_walker"] = g.step
        if st == pk.CONVERGED:
            err = 0.0
            for w in range(nw):
                hi, lo = g.shadow(w)
                err = max(err, float(np.max(np.abs((g.walker(w)["lng"] - hi) - lo))))
            sj, lng, _ = g.join()
            rs.update(converged=True, max_abs_lng_minus_shadow=err, join_status=sj,
                      attempts_per_s=nw * g.step / rs["seconds"])
            curves[name] = lng
            if npy:
                np.save(npy, lng)
            log(f"[bench] precision {name}: converged after {rs['seconds']:.0f} s, {g.step} attempts per walker, "
                f"max |ln g - shadow| {err:.3g}")
        elif ck:
            with open(ck, "wb") as f:
                f.write(zlib.compress(g.save(), 1))
        if state_path:
            with open(state_path, "w") as f:
                json.dump(state, f)
        del g
    done = all(state["runs"].get(n, {}).get("converged") for n, _, _ in runs)
    res = {
        "metric": "max |delta ln g| of converged q=10 Potts L=80 REWL, binary32 (hi, lo) against binary64",
        "unit": "ln g", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32x2",
        "config": {"workload": "potts_q10_L80: 2D q=10 Potts 80x80 periodic, 64 windows at 75% overlap, "
                               f"16 walkers/window, ln f halving to {lnf_final:g}", "walkers": nw,
                   "lnf_final": lnf_final},
        "runs": state["runs"], "complete": done,
    }
    if done:
        def diff(a, b):
            both = np.isfinite(a) & np.isfinite(b)
            return float(np.max(np.abs(a[both] - b[both]))), int(both.sum())

        res["f32x2_vs_f64"], res["bins_compared"] = diff(curves["f32x2"], curves["f64"])
        res["f64_seed_spread"], _ = diff(curves["f64_seed2"], curves["f64"])
        res["value"] = res["f32x2_vs_f64"]
    print(json.dumps(res), flush=True)


# Floating-point work of one trimer attempt counted as the binary64 squared
# distance (3 multiplies, 2 adds) for the old and the new position of the
# moved bead against each of its 191 partners; cut-off tests, potentials and
# the sum come on top.
TRIMER_FLOPS_PER_ATTEMPT = 2 * 191 * 5
# Lipid model, binary64 flops of one displacement attempt: the squared
# minimum-image distance (3 mul + 2 add) to each of the 999 partners at the
# old and the new position, and the Lennard-Jones / r^-9 term (1 div + 5
# mul/add) of the ~52 partners inside the 2.5 cut-off at density 0.8, twice.
# HBM bytes of one k_trimer_sweep launch of the trimer workload (64 walkers x
# 20,000 attempts): FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a
# 256 MiB torch.neg copy in the same program), 227.75 KiB and 308.0 KiB.
TRIMER_SWEEP_HBM_BYTES = 781_800
LIPID_FLOPS_PER_ATTEMPT = 2 * 999 * 5 + 2 * 52 * 6
# HBM bytes of one k_lipid_sweep launch of the lipid workload (64 walkers x 2,000
# attempts): FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a 256 MiB
# torch.neg copy in the same program), 792.7 KiB and 1,302.0 KiB per launch.
LIPID_SWEEP_HBM_BYTES = 2_956_600


def trimer(args):
    """The continuous-move workload: 64 head-tail-tail trimers, bead displacements."""
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = workloads.TRIMER
    h, m = cfg["windows"], cfg["walkers"]
    nw, S = h * m, cfg["sync_attempts"]
    x = workloads.init_trimers(cfg["nmol"], cfg["box"], nw, cfg["seed"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = pk.Rewl.trimer(cfg["nmol"], cfg["box"], cfg["e_min"], cfg["bin_w"], cfg["bins"], h, cfg["overlap"], m, x,
                       device=dev, seed=cfg["seed"], flat=cfg["flat"], lnf_init=cfg["lnf_init"],
                       lnf_final=cfg["lnf_final"], schedule=cfg["schedule"], sync_attempts=S,
                       exchange=cfg["exchange"], precision=cfg["precision"])
    walkin_s = walkin_with_progress(g, "trimer")
    log(f"[bench] trimer walk-in done in {walkin_s:.1f} s")
    if args.warmup:
        g.run(args.warmup * S)
    torch.cuda.synchronize()
    g.set_timing(True)
    t0 = time.perf_counter()
    g.run(args.steps * S)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sweep_ms, launches, sync_ms, syncs = g.timing()
    g.set_timing(False)
    value = nw * S * args.steps / el
    avg_ms = sweep_ms / max(launches, 1)
    achieved = TRIMER_FLOPS_PER_ATTEMPT * nw * S / (avg_ms * 1e-3) / 1e12
    out = {
        "metric": "bead-displacement attempts/s (1 GPU), 64-trimer amphiphile REWL",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "trimer: 64 head-tail-tail trimers in a periodic cube of side 10, bins of 0.5 "
                               "over [-460, 40), 16 windows at 75% overlap, 4 walkers each",
                   "walkers": nw, "attempts_per_step_per_walker": S},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_UNFUSED_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_UNFUSED_PEAK_TFLOPS, "traffic": TRIMER_SWEEP_HBM_BYTES, "kernel": "k_trimer_sweep",
                     "kernel_avg_ms": avg_ms, "kernel_launches": launches,
                     "flops_per_attempt": TRIMER_FLOPS_PER_ATTEMPT},
        "per_walker_attempts_per_s": S * args.steps / el,
        "walkin_s": walkin_s,
    }
    print(json.dumps(out), flush=True)


def lipid(args):
    """The paper's lipid system (Sec. 3.2): 125 P-H-H lipids in 625 solvent
    particles at density 0.8, displacement and reptation moves; the CPU
    oracle is timed on a bounded sample of the same run."""
    import numpy as np
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.LIPID)
    if args.lipid_emin is not None:
        # the same 800 bins placed lower: the walkers walk in from the lattice start
        cfg["e_min"] = args.lipid_emin
    h, m = cfg["windows"], cfg["walkers"]
    nw, S = h * m, cfg["sync_attempts"]
    np_ = 3 * cfg["nlip"] + cfg["nsol"]
    x = workloads.init_lipids(cfg["nlip"], cfg["nsol"], cfg["box"], nw, cfg["seed"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    kw = dict(seed=cfg["seed"], flat=cfg["flat"], lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"],
              schedule=cfg["schedule"], sync_attempts=S, exchange=cfg["exchange"])
    g = pk.Rewl.lipid(cfg["nlip"], cfg["nsol"], cfg["box"], cfg["e_min"], cfg["bin_w"], cfg["bins"], h,
                      cfg["overlap"], m, x, eps_ww=cfg["eps_ww"], device=dev, **kw)
    walkin_s = walkin_with_progress(g, "lipid", budget=1 << 13)
    log(f"[bench] lipid walk-in done in {walkin_s:.1f} s")
    if args.warmup:
        g.run(args.warmup * S)
    torch.cuda.synchronize()
    g.set_timing(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        g.run(S)
        if i % 20 == 19:
            torch.cuda.synchronize()
            log(f"[bench] lipid step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sweep_ms, launches, sync_ms, syncs = g.timing()
    g.set_timing(False)
    value = nw * S * args.steps / el
    avg_ms = sweep_ms / max(launches, 1)
    flops = LIPID_FLOPS_PER_ATTEMPT
    achieved = flops * nw * S / (avg_ms * 1e-3) / 1e12
    reps = sum(int(not np.array_equal(g.lipid_state(w)[2], np.arange(3 * cfg["nlip"]).reshape(-1, 3)))
               for w in range(nw))
    out = {
        "metric": "particle-move attempts/s (1 GPU), lipid model with explicit solvent (N=1000) REWL",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "lipid: 125 P-H-H lipids + 625 solvent particles, density 0.8, reptation "
                               f"probability 0.0375, bins of 1 over [{cfg['e_min']:g}, "
                               f"{cfg['e_min'] + cfg['bins'] * cfg['bin_w']:g}), 16 windows at 75% overlap, "
                               "4 walkers each", "walkers": nw, "attempts_per_step_per_walker": S,
                   "e_min": cfg["e_min"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_UNFUSED_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_UNFUSED_PEAK_TFLOPS,
                     "traffic": LIPID_SWEEP_HBM_BYTES if cfg["e_min"] == workloads.LIPID["e_min"] else None,
                     "kernel": "k_lipid_sweep",
                     "kernel_avg_ms": avg_ms, "kernel_launches": launches, "flops_per_attempt": flops},
        "per_walker_attempts_per_s": S * args.steps / el,
        "walkin_s": walkin_s,
        "walkers_with_reptated_lipids": reps,
    }
    if not args.no_cpu_baseline:
        import oracle

        threads, hc = oracle_threads(nw)
        o = oracle.Rewl.lipid(cfg["nlip"], cfg["nsol"], cfg["box"], cfg["e_min"], cfg["bin_w"], cfg["bins"], h,
                              cfg["overlap"], m, x, eps_ww=cfg["eps_ww"], threads=threads, **kw)
        o.walkin()
        n = 1000
        t0 = time.perf_counter()
        o.run(n)
        cs = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": nw * n / cs, "unit": "attempts/s", "cores": threads, "kind": "oracle",
                               "host": hc,
                               "sample": f"oracle walk-in (excluded) then {n:,} attempts per walker of the same "
                                         f"workload ({nw} walkers), {threads} OpenMP threads"}
    print(json.dumps(out), flush=True)


def trajectory(g, S, seconds, converge_attempts, walkin_s, early_rate):
    """Continue the protocol of the run for `seconds` of wall time (from where
    the measurement left it, 2,000 sync intervals per call), logging the
    windows' ln f; returns when every window entered the 1/t regime, the rate
    there, and the time to ln f_final from those measured parts (the 1/t phase
    is deterministic: ln f = W / t)."""
    import torch

    import paper_1312_3004_amd as pk

    t0 = time.perf_counter()
    first_all_1t = None
    rates = []
    start_step = g.step
    last_t, last_s = t0, g.step
    while time.perf_counter() - t0 < seconds:
        st = g.run(2000 * S)
        torch.cuda.synchronize()
        now = time.perf_counter()
        ws = [g.window(k) for k in range(g.h)]
        lnf = [w["lnf"] if not w["finished"] else w["lnf_last"] for w in ws]
        n1t = sum(1 for w in ws if w["regime"] == 1 or w["finished"])
        rate = (g.step - last_s) / (now - last_t)
        if n1t == g.h:
            rates.append(rate)
            if first_all_1t is None:
                first_all_1t = {"attempts_per_walker": g.step, "wall_s": now - t0}
        log(f"[bench] trajectory t={now - t0:.0f} s step={g.step} rate/walker={rate:.4g} "
            f"ln f max={max(lnf):.3g} min={min(lnf):.3g} windows in 1/t: {n1t}")
        last_t, last_s = now, g.step
        if st == pk.CONVERGED:
            break
    out = {"seconds": time.perf_counter() - t0, "start_attempts_per_walker": start_step,
           "end_attempts_per_walker": g.step, "all_windows_in_1_over_t": first_all_1t}
    if first_all_1t and rates and converge_attempts:
        r1t = sum(rates) / len(rates)
        # the part before (walk-in, warm-up and timed steps) at the measured rate
        before = walkin_s + start_step / early_rate
        out["rate_1_over_t_per_walker"] = r1t
        out["time_to_lnf_final_s"] = (before + first_all_1t["wall_s"] +
                                      (converge_attempts - first_all_1t["attempts_per_walker"]) / r1t)
    return out


def to_convergence(args):
    """Wall time from creation to every window finished (the full protocol of
    the named workload).  With --checkpoint PATH the run can span several
    processes: an existing PATH (and its PATH.json sidecar of measured times)
    is loaded and continued; at convergence or when this process's budget of
    --to-convergence seconds is spent, the run is saved back to PATH.  The
    reported time is the sum of the segments' GPU wall times (creation and
    walk-in included, saving and loading not).  Unless --no-cpu-baseline (and
    the run fits one process), the CPU oracle runs the same protocol too."""
    import math

    import numpy as np
    import torch

    import oracle
    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS[args.config])
    L, q, h, m = cfg["L"], cfg["q"], cfg["windows"], cfg["walkers"]
    spins = workloads.init_spins(L, q, h * m, cfg["seed"])
    kw = dict(seed=cfg["seed"], flat=cfg["flat"], lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"],
              schedule=cfg["schedule"], sync_attempts=cfg["sync_attempts"], exchange=cfg["exchange"],
              precision=cfg["precision"])
    S = cfg["sync_attempts"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ck = args.checkpoint
    side = {"segments": [], "seconds": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = pk.Rewl(L, q, h, cfg["overlap"], m, spins, device=dev, **kw)
    if ck and os.path.exists(ck):
        with open(ck + ".json") as f:
            side = json.load(f)
        torch.cuda.synchronize()
        tl = time.perf_counter()
        with open(ck, "rb") as f:
            g.load(f.read())
        torch.cuda.synchronize()
        t0 += time.perf_counter() - tl     # loading is not part of the run
        log(f"[bench] resumed at step {g.step} after {side['seconds']:.1f} s in {len(side['segments'])} segments")
    else:
        tw = time.perf_counter()
        g.walkin()
        torch.cuda.synchronize()
        side["walkin_s"] = time.perf_counter() - tw
        log(f"[bench] walk-in {side['walkin_s']:.2f} s")
    st = pk.OK
    last = time.perf_counter()
    while st != pk.CONVERGED and time.perf_counter() - t0 < args.to_convergence:
        st = g.run(1000 * S)
        if time.perf_counter() - last > 30 or st == pk.CONVERGED:
            torch.cuda.synchronize()
            ws = [g.window(k) for k in range(h)]
            lnf = [w["lnf"] if not w["finished"] else w["lnf_last"] for w in ws]
            log(f"[bench] GPU step {g.step} after {side['seconds'] + time.perf_counter() - t0:.1f} s: "
                f"ln f max {max(lnf):.3g}, {sum(w['finished'] for w in ws)}/{h} windows finished")
            last = time.perf_counter()
    torch.cuda.synchronize()
    seg_s = time.perf_counter() - t0
    side["segments"].append({"seconds": seg_s, "end_step": g.step})
    side["seconds"] += seg_s
    gpu_s = side["seconds"]
    if ck:
        with open(ck, "wb") as f:
            f.write(g.save())
        with open(ck + ".json", "w") as f:
            json.dump(side, f)
    out = {"metric": f"time to ln f < {cfg['lnf_final']:g}, {args.config}", "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": args.config, "L": L, "q": q, "windows": h, "walkers_per_window": m},
           "gpu": {"converged": st == pk.CONVERGED, "seconds": gpu_s, "attempts_per_walker": g.step,
                   "segments": side["segments"], "walkin_s": side.get("walkin_s")}}
    if st == pk.CONVERGED:
        # the joined, normalised ln g and its canonical specific heat: the peak
        # lies near the infinite-lattice transition 1/ln(1 + sqrt(q)), shifted
        # by the finite size (Sec. 3.1)
        sj, lng, cuts = g.join()
        T = np.linspace(0.60, 0.80, 2001)
        _, U, C = g.thermo(T)
        i = int(np.argmax(C))
        out["joined"] = {"status": sj, "cuts": [int(c) for c in cuts],
                         "sum_g_check": float(np.logaddexp.reduce(lng[np.isfinite(lng)]) - L * L * math.log(q)),
                         "cv_peak_T": float(T[i]), "cv_peak": float(C[i]),
                         "Tc_infinite": 1.0 / math.log(1.0 + math.sqrt(q))}
        if args.save_lng:
            np.save(args.save_lng, lng)
    if not args.no_cpu_baseline and not ck:
        threads, hc = oracle_threads(h * m)
        t0 = time.perf_counter()
        o = oracle.Rewl(L, q, h, cfg["overlap"], m, spins, threads=threads, **kw)
        ost = o.run(10**13)
        out["cpu_oracle"] = {"converged": ost == oracle.CONVERGED, "seconds": time.perf_counter() - t0,
                             "attempts_per_walker": o.step, "cores": threads, "host": hc,
                             "same_state": o.step == g.step and o.round == g.round}
    out["value"] = gpu_s
    print(json.dumps(out), flush=True)


def production(args):
    """The potts_q10_L32 workload in the production phase (frozen weights, Sec. 3.2):
    after a WL segment, begin_production, then sample H(E, O) of O = max_s n_s at
    every sync point with full O resolution (L*L + 1 bins).  Reported beside the
    same run's WL-phase rate: the attempt kernel is the same, the sync point
    gains the observable pass."""
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS[args.config])
    L, q, h, m = cfg["L"], cfg["q"], cfg["windows"], cfg["walkers"]
    nw, S = h * m, cfg["sync_attempts"]
    spins = workloads.init_spins(L, q, nw, cfg["seed"])
    torch.cuda.set_device(0)
    g = pk.Rewl(L, q, h, cfg["overlap"], m, spins, seed=cfg["seed"], flat=cfg["flat"],
                lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"], schedule=cfg["schedule"],
                sync_attempts=S, exchange=cfg["exchange"], precision=cfg["precision"], obs_bins=L * L + 1)
    g.walkin()
    g.run(args.warmup * S)
    torch.cuda.synchronize()
    rates = {}
    for phase in ("wl", "production"):
        if phase == "production":
            g.begin_production()
            g.run(args.warmup * S)
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.run(args.steps * S)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        sweep_ms, launches, sync_ms, syncs = g.timing()
        g.set_timing(False)
        if st == pk.CONVERGED:
            raise RuntimeError("run converged inside the timed region")
        rates[phase] = dict(attempts_per_s=nw * S * args.steps / elapsed, ms_per_step=elapsed * 1e3 / args.steps,
                            k_sweep_avg_ms=sweep_ms / max(launches, 1), sync_point_avg_ms=sync_ms / max(syncs, 1))
        log(f"[bench] {phase}: {rates[phase]}")
    mean, cnt = g.obs_micro()
    p = rates["production"]
    out = {
        "metric": "spin-flip attempts/s (1 GPU), production phase with H(E, O) sampling, q=10 Potts L=32",
        "value": p["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": p["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} after {args.warmup} WL steps, weights frozen, "
                               f"O = max_s n_s in {L * L + 1} bins sampled every {S} attempts per walker",
                   "walkers": nw, "obs_bins": L * L + 1},
        "phases": rates,
        "production_over_wl": p["attempts_per_s"] / rates["wl"]["attempts_per_s"],
        "samples": int(cnt.sum()),
    }
    print(json.dumps(out), flush=True)


# Structural observables of one lipid configuration (Sec. 3.2, Eqs. 6-8),
# algorithmic ALU work in VALU issue slots (binary32 and binary64 operations
# one slot each): the tail-contact test over the M (M - 1) / 2 lipid pairs, 4
# tail pairs each, at 3 binary32 differences + 3 wrap tests + 3 widenings + 3
# binary64 products + 2 binary64 sums + 1 compare = 15 ops; S_mol, the cluster
# search and the unfolding add O(M) and are left out.
def structure_ops_per_config(M):
    return M * (M - 1) // 2 * 4 * 15


# HBM bytes of one k_lipid_structure launch over the 4,096 configurations of the
# structure workload: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a
# 256 MiB torch.neg copy in the same program), 12,588.7 KiB and 256.0 KiB.  The
# algorithmic bytes are 4,096 x (lipid rows 1,500 + bead coordinates 4,500 +
# record 64) = 24.84 MB.
STRUCT_4096_HBM_BYTES = 26_043_000


def structure_bench(args):
    """Structural observables of the N = 1000 lipid system (125 lipids in 625
    solvent particles, density 0.8) for a batch of 4,096 configurations in one
    launch (one wavefront each), timed with HIP events on the launching stream;
    the oracle's structure() of a sample of the same configurations is timed
    beside it."""
    import numpy as np
    import torch

    import paper_1312_3004_amd as pk
    import workloads

    c = workloads.LIPID
    nconf, M = 4096, c["nlip"]
    xs = workloads.init_lipids(c["nlip"], c["nsol"], c["box"], nconf, c["seed"])
    lips = np.broadcast_to(np.arange(3 * M, dtype=np.int32).reshape(1, M, 3), (nconf, M, 3)).copy()
    torch.cuda.set_device(0)
    x = torch.from_numpy(xs).cuda()
    lp = torch.from_numpy(lips).cuda()
    out = torch.empty((nconf, 8), dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        pk.lipid_structure(x, lp, c["box"], out=out)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 200))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        pk.lipid_structure(x, lp, c["box"], out=out)
        b.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    rec = out.cpu().numpy()
    ops = structure_ops_per_config(M) * nconf
    achieved = ops / (kern_ms * 1e-3) / 1e12
    log(f"[bench] structure: {nconf} configurations per launch, kernel {kern_ms:.3f} ms; largest cluster "
        f"{rec[:, 3].mean():.1f} lipids on average, {rec[:, 2].mean():.1f} clusters")
    res = {"metric": "configurations analysed/s (1 GPU), lipid structure observables (S_mol, clusters, "
                     "gyration tensor, prolateness), N = 1000",
           "value": nconf / (kern_ms * 1e-3), "unit": "configurations/s", "n_gpus": 1, "steps": steps,
           "warmup": max(args.warmup, 1), "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{nconf} configurations of the lipid system (125 lipids, 625 solvent, "
                                  f"box {c['box']:.3f}), one launch", "configurations": nconf, "lipids": M},
           "kernel_avg_ms": kern_ms,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                        "frac": achieved / ALU_PEAK_TOPS,
                        "traffic": STRUCT_4096_HBM_BYTES if (nconf, M) == (4096, 125) else None,
                        "hbm_gb_per_s": STRUCT_4096_HBM_BYTES / (kern_ms * 1e-3) / 1e9},
           "mean_largest_cluster": float(rec[:, 3].mean()), "mean_clusters": float(rec[:, 2].mean())}
    # The production phase of the lipid workload with H(E, O), O = lipids in the
    # largest cluster, sampled at every sync point (64 walkers, 2,000 attempts each).
    h, m, S_att = c["windows"], c["walkers"], c["sync_attempts"]
    x0 = workloads.init_lipids(c["nlip"], c["nsol"], c["box"], h * m, c["seed"])
    g = pk.Rewl.lipid(c["nlip"], c["nsol"], c["box"], c["e_min"], c["bin_w"], c["bins"], h, c["overlap"], m, x0,
                      eps_ww=c["eps_ww"], seed=c["seed"], flat=c["flat"], lnf_init=c["lnf_init"],
                      lnf_final=c["lnf_final"], schedule=c["schedule"], sync_attempts=S_att, exchange=c["exchange"],
                      obs_bins=M + 1)
    g.walkin()
    g.run(2 * S_att)
    g.begin_production()
    g.run(2 * S_att)
    torch.cuda.synchronize()
    g.set_timing(True)
    nsteps = 50
    t0 = time.perf_counter()
    g.run(nsteps * S_att)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sweep_ms, launches, sync_ms, syncs = g.timing()
    g.set_timing(False)
    _, cnt = g.obs_micro()
    res["production"] = {"attempts_per_s": h * m * S_att * nsteps / el, "steps": nsteps,
                         "k_lipid_sweep_avg_ms": sweep_ms / max(launches, 1),
                         "sync_point_avg_ms": sync_ms / max(syncs, 1), "samples": int(cnt.sum())}
    log(f"[bench] lipid production with H(E, O): {res['production']}")
    if not args.no_cpu_baseline:
        from oracle import structure as S

        n, t0 = 0, time.perf_counter()
        while n < nconf and (n < 8 or time.perf_counter() - t0 < 10.0):
            ref = S.structure(xs[n], lips[n], c["box"])
            if not (ref[2] == rec[n, 2] and ref[3] == rec[n, 3]):
                raise RuntimeError(f"configuration {n}: clusters differ from the oracle")
            n += 1
        cpu_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / cpu_s, "unit": "configurations/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's structure() of the first {n} of the same configurations, "
                                         f"one thread"}
    print(json.dumps(res), flush=True)


def bootstrap_bench(args):
    """Error analysis of Sec. 2 on the GPU: R = 64 independent runs of the
    potts_q10_L8 workload (instances of one batch, different Philox streams
    and starting lattices) to convergence, then 1,000 bootstrap resamples, each
    joined anew, with U and C_v on 201 temperatures; the oracle's bootstrap of
    the same runs is timed beside it."""
    import math

    import numpy as np
    import torch

    import oracle
    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS["potts_q10_L8"])
    L, q, h, m = cfg["L"], cfg["q"], cfg["windows"], cfg["walkers"]
    R, nboot = 64, 1000
    T = np.linspace(0.5, 1.0, 201)
    insts, spins = [], []
    for i in range(R):
        insts.append(dict(L=L, q=q, windows=h, overlap=cfg["overlap"], walkers=m, seed=cfg["seed"], instance=i,
                          flat=cfg["flat"], lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"],
                          schedule=cfg["schedule"], sync_attempts=cfg["sync_attempts"], exchange=cfg["exchange"],
                          precision=cfg["precision"]))
        spins.append(workloads.init_spins(L, q, h * m, cfg["seed"] + i))
    torch.cuda.set_device(0)
    b = pk.Batch(insts, spins)
    t0 = time.perf_counter()
    b.walkin()
    while b.run(200) != pk.CONVERGED:
        log(f"[bench] bootstrap workload: {b.progress()[1]}/{R} runs converged")
    torch.cuda.synchronize()
    converge_s = time.perf_counter() - t0
    log(f"[bench] {R} runs converged in {converge_s:.1f} s")
    b.bootstrap(10, 1, T)                       # first call: module load and allocation
    reps = []
    for k in range(3):
        t0 = time.perf_counter()
        out = b.bootstrap(nboot, 11, T)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
    gpu_s = min(reps)
    peak = int(np.argmax(out["C_mean"]))
    log(f"[bench] GPU bootstrap: {nboot} resamples in {gpu_s * 1e3:.1f} ms; C_v peak {out['C_mean'][peak]:.4g} "
        f"+- {out['C_std'][peak]:.2g} at T = {T[peak]:.4f}")
    res = {"metric": "bootstrap resamples/s (1 GPU), 64 converged q=10 Potts L=8 runs, 201 temperatures",
           "value": nboot / gpu_s, "unit": "resamples/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": gpu_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{R} independent runs of potts_q10_L8 ({h} windows x {m} walker, ln f 1 -> "
                                  f"1e-6), {nboot} bootstrap resamples, U and C_v at {len(T)} temperatures",
                      "runs": R, "resamples": nboot, "temperatures": len(T)},
           "runs_to_convergence_s": converge_s,
           "cv_peak": {"T": float(T[peak]), "C_mean": float(out["C_mean"][peak]),
                       "C_std": float(out["C_std"][peak])},
           "lng_std_max": float(np.max(out["lng_std"]))}
    if not args.no_cpu_baseline:
        pv = []
        for i in range(R):
            inst = b.instance(i)
            pv.append((np.stack([inst.walker(k * m)["lng"] for k in range(h)]),
                       np.stack([inst.window(k)["visited"] for k in range(h)])))
        t0 = time.perf_counter()
        st, ref = oracle.bootstrap(np.stack([p for p, _ in pv]), np.stack([v for _, v in pv]), b.instance(0).starts,
                                   -2 * L * L, 2 * L * L + 1, L * L * math.log(q), nboot, 11, T)
        cpu_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": nboot / cpu_s, "unit": "resamples/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's bootstrap of the same {R} runs, {nboot} resamples, "
                                         f"{len(T)} temperatures, one thread"}
        fin = np.isfinite(ref["lng_mean"])
        res["max_abs_diff_vs_oracle"] = {
            "lng_mean": float(np.max(np.abs(out["lng_mean"][fin] - ref["lng_mean"][fin]))),
            "lng_std": float(np.max(np.abs(out["lng_std"] - ref["lng_std"]))),
            "C_mean_rel": float(np.max(np.abs(out["C_mean"] - ref["C_mean"]) / np.abs(ref["C_mean"])))}
    print(json.dumps(res), flush=True)


def lds_peak_measured():
    """Measured LDS bandwidth of the part (GB/s): ds_read_b128 and ds_write_b64
    streams over every CU (paper_1312_3004_amd/csrc/lds_peak.hip); None if the
    library is missing."""
    import ctypes

    from paper_1312_3004_amd import build as pkbuild

    if not os.path.exists(pkbuild.LDS_PEAK_LIB):
        return None
    lib = ctypes.CDLL(pkbuild.LDS_PEAK_LIB)
    lib.lds_peak.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]
    out = {}
    for mode, name in ((0, "read_b128"), (1, "write_b64")):
        bps, ms = ctypes.c_double(0), ctypes.c_double(0)
        if lib.lds_peak(mode, 2000, ctypes.byref(bps), ctypes.byref(ms)) != 0:
            return None
        out[name + "_gb_per_s"] = bps.value / 1e9
    return out


def potts_roofline(attempts_per_launch, avg_ms, launches, traffic):
    """Roofline entry of the Potts attempt kernel: ALU issue slots (the binding
    roof) with the LDS bandwidth roof beside it, per launch of avg_ms."""
    sec = avg_ms * 1e-3
    achieved = ALU_SLOTS_PER_ATTEMPT * attempts_per_launch / sec / 1e12
    lds = LDS_BYTES_PER_ATTEMPT * attempts_per_launch / sec / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic, "kernel": "k_sweep",
            "kernel_avg_ms": avg_ms, "kernel_launches": launches,
            "slots_per_attempt": ALU_SLOTS_PER_ATTEMPT, "attempts_per_launch": attempts_per_launch,
            "lds": {"achieved_gb_per_s": lds, "peak_gb_per_s": LDS_PEAK_GBS, "frac": lds / LDS_PEAK_GBS,
                    "bytes_per_attempt": LDS_BYTES_PER_ATTEMPT}}


def trace_window(trace_dir, bench_out):
    """Kernel durations of a `rocprofv3 --kernel-trace --output-format csv`
    run of this benchmark over its timed window: the k_sweep dispatches whose
    0-based index lies in the line's `timed_k_sweep_launches` range (the
    timed sync intervals), their mean, min and max, and the other kernels
    launched inside the window's time span."""
    import csv
    import glob

    line = json.loads([x for x in open(bench_out).read().splitlines() if x.startswith("{")][-1])
    a, b = line["config"]["timed_k_sweep_launches"]
    tr = sorted(glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True))
    if not tr:
        raise SystemExit(f"no *kernel_trace.csv under {trace_dir}")
    rows = []
    with open(tr[0]) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort()
    ks = [(t0, t1) for _, name, t0, t1 in rows if "k_sweep<" in name]
    win = ks[a:b]
    if not win:
        raise SystemExit(f"the trace holds {len(ks)} k_sweep dispatches, none in [{a}, {b})")
    durs = [(t1 - t0) * 1e-6 for t0, t1 in win]
    span0, span1 = win[0][0], win[-1][1]
    other = {}
    for _, name, t0, t1 in rows:
        if t0 >= span0 and t1 <= span1 and "k_sweep<" not in name:
            c = other.setdefault(name.replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1], [0, 0.0])
            c[0] += 1
            c[1] += (t1 - t0) * 1e-6
    return {"trace": os.path.basename(tr[0]), "k_sweep_dispatches": len(ks), "window": [a, b], "window_n": len(win),
            "window_avg_ms": sum(durs) / len(durs), "window_min_ms": min(durs), "window_max_ms": max(durs),
            "window_span_ms": (span1 - span0) * 1e-6,
            "bench_kernel_avg_ms": line["roofline"]["kernel_avg_ms"], "bench_value": line["value"],
            "other_kernels_in_window": {k: {"n": v[0], "avg_ms": v[1] / v[0]} for k, v in other.items()}}


def phase_clock_summary(ctr, fields):
    """Cycle split of the attempt loop from the profiling build's per-walker
    counters (summed over the timed launches): cycles per attempt of the
    lane-parallel and decision phases, speculative segments, rounds and
    exact-path attempts per block, mean and max over the walkers."""
    import numpy as np

    c = {f: ctr[:, i].astype(np.float64) for i, f in enumerate(fields)}
    att, blocks = np.maximum(c["attempts"], 1), np.maximum(c["blocks"], 1)
    per = {
        "lane_parallel_cycles_per_attempt": c["lane_cycles"] / att,
        "decision_cycles_per_attempt": c["decide_cycles"] / att,
        "round_cycles_per_attempt": c["round_cycles"] / att,
        "segment_setup_cycles_per_attempt": c["setup_cycles"] / att,
        "commit_cycles_per_attempt": c["commit_cycles"] / att,
        "exact_path_cycles_per_attempt": c["exact_cycles"] / att,
        "block_tail_cycles_per_attempt": c["tail_cycles"] / att,
        "segments_per_block": c["segments"] / blocks,
        "rounds_per_block": c["rounds"] / blocks,
        "exact_attempts_per_block": c["exact_attempts"] / blocks,
    }
    out = {k: {"mean": float(v.mean()), "max": float(v.max())} for k, v in per.items()}
    out["rounds_per_segment"] = float(c["rounds"].sum() / max(c["segments"].sum(), 1))
    out["attempts"] = int(c["attempts"].sum())
    out["library"] = "librewl_clocks.so (profiling build: s_memtime clocks in the attempt loop)"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="potts_q10_L32")
    ap.add_argument("--cpu-attempts", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-approach", action="store_true",
                    help="time the steps right after walk-in instead of after the halving phase")
    ap.add_argument("--to-convergence", type=float, default=0.0,
                    help="run the named workload from creation to convergence (at most this many seconds) "
                         "on the GPU and, unless --no-cpu-baseline, on the CPU oracle")
    ap.add_argument("--checkpoint", default="",
                    help="with --to-convergence: continue the run saved at this path (if present) and save it "
                         "back there when this process's budget is spent or the run converged")
    ap.add_argument("--lnf-final", type=float, default=0.0,
                    help="precision study: stop each run when every window's ln f is below this instead of "
                         "the workload's own ln f_final")
    ap.add_argument("--precision", type=int, choices=(0, 1), default=None,
                    help="Potts workload: ln g in binary64 (0, the workload's own) or as the binary32 "
                         "(hi, lo) pair (1)")
    ap.add_argument("--no-per-instance", action="store_true",
                    help="batched workload: skip the step with one launch per instance (for profiler runs)")
    ap.add_argument("--lipid-emin", type=float, default=None,
                    help="lipid workload: lower end of its 800 unit-wide energy bins (default 7000, the band "
                         "just below the lattice starts)")
    ap.add_argument("--max-runs", type=int, default=0,
                    help="precision study: start at most this many of its runs in this process")
    ap.add_argument("--save-lng", default="", help="with --to-convergence: write the joined ln g (.npy) here")
    ap.add_argument("--trajectory", type=float, default=0.0,
                    help="after the measurement, continue the run for this many seconds and report "
                         "when every window reached the 1/t regime and the time to ln f_final")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy kernel (torch.neg, fp32) of this many MiB three "
                         "times first: the reference for the HBM byte counters of a profiler run")
    ap.add_argument("--trace-window", nargs=2, metavar=("TRACE_DIR", "BENCH_OUT"),
                    help="no GPU work: summarise the k_sweep durations of a rocprofv3 csv kernel trace of "
                         "this benchmark (TRACE_DIR) over the timed launches named in its output line")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="run on the profiling build librewl_clocks.so and report the attempt loop's cycle "
                         "split (lane-parallel phase, decision phase, speculative rounds) over the timed "
                         "steps; its rates are those of the profiling build")
    ap.add_argument("--workload", choices=("potts", "batched", "precision", "trimer", "production", "bootstrap",
                                           "lipid", "structure"),
                    default="potts",
                    help="potts: the single-run workload (--config); batched: 256 instances; "
                         "precision: the L=80 workload in binary64 and in the binary32 pair form; "
                         "trimer: the continuous-move workload; production: the single-run workload "
                         "with frozen weights and H(E, O) sampling; bootstrap: error analysis over 64 "
                         "independent L=8 runs; lipid: the explicit-solvent lipid system (N = 1000); "
                         "structure: its structural observables over 4,096 configurations")
    args = ap.parse_args()
    if args.trace_window:
        print(json.dumps(trace_window(*args.trace_window), indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the REWL hot path runs on a single MI355X "
              "(multi-GPU window sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.phase_clocks:
        import paper_1312_3004_amd as pk

        pk.use_phase_clocks()
    if args.copy_calibration_mib:
        import torch

        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x torch.neg over {args.copy_calibration_mib} MiB "
            f"(reads and writes {4 * n} bytes per launch)")
        del src, dst
    if args.workload == "precision":
        # --to-convergence is this study's time budget
        return precision_study(args)
    if args.to_convergence > 0:
        return to_convergence(args)
    if args.workload == "batched":
        return batched(args)
    if args.workload == "trimer":
        return trimer(args)
    if args.workload == "production":
        return production(args)
    if args.workload == "bootstrap":
        return bootstrap_bench(args)
    if args.workload == "lipid":
        return lipid(args)
    if args.workload == "structure":
        return structure_bench(args)

    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS[args.config])
    if args.precision is not None:
        cfg["precision"] = args.precision
    L, q, h, m = cfg["L"], cfg["q"], cfg["windows"], cfg["walkers"]
    nw = h * m
    S = cfg["sync_attempts"]
    spins = workloads.init_spins(L, q, nw, cfg["seed"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = pk.Rewl(L, q, h, cfg["overlap"], m, spins, device=dev, seed=cfg["seed"], flat=cfg["flat"],
                lnf_init=cfg["lnf_init"], lnf_final=cfg["lnf_final"], schedule=cfg["schedule"],
                sync_attempts=S, exchange=cfg["exchange"], precision=cfg["precision"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.walkin()
    torch.cuda.synchronize()
    walkin_s = time.perf_counter() - t0
    log(f"[bench] walk-in done in {walkin_s:.2f} s")
    W = g.W
    lnf_final = cfg["lnf_final"]
    converge_attempts = (int(W / lnf_final) // S + 1) * S if cfg["schedule"] == 1 else None

    def timed(steps):
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.run(steps * S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sweep_ms, launches, sync_ms, syncs = g.timing()
        g.set_timing(False)
        if st == pk.CONVERGED:
            raise RuntimeError("run converged inside a timed segment; the step count is not the work done")
        return el, sweep_ms / max(launches, 1), launches, sync_ms / max(syncs, 1)

    # The first steps after walk-in (ln f = 1, every attempt on the exact serial path).
    n_early = min(args.steps, 200)
    el, k_ms, _, _ = timed(n_early)
    early = {"steps": n_early, "attempts_per_s": nw * S * n_early / el, "k_sweep_avg_ms": k_ms,
             "lnf": cfg["lnf_init"]}
    log(f"[bench] early phase (ln f = {cfg['lnf_init']:g}): {early['attempts_per_s']:.4g} attempts/s")
    # The protocol up to the phase that holds almost all of the run's attempts:
    # every window in the 1/t regime (untimed for the value, reported).
    approach = None
    if cfg["schedule"] == 1 and not args.no_approach:
        t0 = time.perf_counter()
        s_start = g.step
        while True:
            g.run(2000 * S)
            torch.cuda.synchronize()
            ws = [g.window(k) for k in range(h)]
            n1t = sum(1 for w in ws if w["regime"] == 1 or w["finished"])
            log(f"[bench] halving phase: step {g.step}, {time.perf_counter() - t0:.0f} s, "
                f"{n1t}/{h} windows in the 1/t regime")
            if n1t == h:
                break
        el = time.perf_counter() - t0
        approach = {"seconds": el, "attempts_per_walker": g.step, "attempts_per_s": nw * (g.step - s_start) / el,
                    "lnf_max": max(w["lnf"] for w in ws)}
    if args.warmup:
        g.run(args.warmup * S)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")
    step_timed = g.step
    if args.phase_clocks:
        pk.phase_clocks(nw, reset=True)
    elapsed, avg_ms, launches, sync_avg = timed(args.steps)
    attempts = nw * S * args.steps
    value = attempts / elapsed
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s: {value:.4g} attempts/s")

    attempts_per_launch = nw * S
    per_walker = S * args.steps / elapsed
    phase = ("1/t regime in every window (ln f = W/t, " +
             f"from {step_timed:,} attempts per walker)" if approach else "the start of the run (ln f = 1)")
    out = {
        "metric": "spin-flip attempts/s (1 GPU) + time to ln f<1e-8, q=10 Potts L=32 REWL",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if cfg["precision"] == 0 else "f32x2",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 2D q={q} Potts {L}x{L} periodic, {h} windows at "
                               f"{int(cfg['overlap'] * 100)}% overlap, {m} walkers/window",
                   "L": L, "q": q, "windows": h, "walkers_per_window": m, "walkers": nw,
                   "attempts_per_step_per_walker": S, "attempts_per_step": nw * S,
                   "timed_phase": phase,
                   # one k_sweep launch per sync interval: the timed steps are these
                   # launches of the run (0-based, for matching a profiler's trace)
                   "timed_k_sweep_launches": [step_timed // S, step_timed // S + args.steps]},
        "roofline": potts_roofline(attempts_per_launch, avg_ms, launches,
                                   K_SWEEP_L32_HBM_BYTES if args.config == "potts_q10_L32" and approach
                                   and cfg["precision"] == 0 else None),
        "per_walker_attempts_per_s": per_walker,
        "sync_point_avg_ms": sync_avg,
        "walkin_s": walkin_s,
        "early_phase": early,
        "halving_phase": approach,
    }
    meas = lds_peak_measured()
    if meas:
        lds = out["roofline"]["lds"]
        lds["measured_peak"] = meas
        lds["frac_of_measured_read_peak"] = lds["achieved_gb_per_s"] / meas["read_b128_gb_per_s"]
    if args.config == "potts_q10_L32" and approach and cfg["precision"] == 0 and K_SWEEP_L32_VALU_PER_ATTEMPT:
        v = K_SWEEP_L32_VALU_PER_ATTEMPT * 64 * attempts_per_launch / (avg_ms * 1e-3)
        out["valu"] = {"instructions_per_attempt": K_SWEEP_L32_VALU_PER_ATTEMPT, "achieved_lane_slots_per_s": v,
                       "peak_lane_slots_per_s": VALU_LANE_SLOTS_PEAK, "frac": v / VALU_LANE_SLOTS_PEAK}
    if converge_attempts and approach:
        # walk-in, early segment, halving phase and warm-up as measured; the rest
        # of the 1/t phase (ln f = W/t is fixed by the attempt count) at the
        # timed rate
        before = walkin_s + early["steps"] * S / (early["attempts_per_s"] / nw) + approach["seconds"] + \
            args.warmup * S / per_walker
        out["time_to_lnf_final_s_projected"] = before + (converge_attempts - step_timed) / per_walker
        out["attempts_per_walker_to_lnf_final"] = converge_attempts
    if args.phase_clocks:
        out["phase_clocks"] = phase_clock_summary(pk.phase_clocks(nw), pk.PHASE_CLOCK_FIELDS)
    if args.trajectory > 0:
        out["trajectory"] = trajectory(g, S, args.trajectory, converge_attempts, walkin_s, per_walker)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg, spins, args.cpu_attempts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
