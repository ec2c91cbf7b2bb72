"""Benchmark: spin-flip attempts/s of REWL on one MI355X, q=10 Potts L=32.

Workload potts_q10_L32: 2D q=10 Potts, 32x32 periodic, 16 windows at 75%
overlap, 4 walkers per window (64 walkers), flatness 0.8, ln f 1 -> 1e-8
(halving, then 1/t), exchange every 10^4 attempts per walker, binary64 ln g.
One step = one sync interval: 10^4 attempts for every walker, then the sync
point (flatness, averaging, ln f update) and a replica-exchange round.
Inputs are synthetic (uniform random starting lattices from a seed) and
resident on the GPU before the timed region; walk-in is timed separately.

Prints one JSON line (see the design doc for the roofline accounting).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic LDS traffic of one Potts attempt: the flipped site and its four
# neighbours (5 B), ln g(E') (8 B), read-modify-write of ln g(E) (16 B) and of
# H(E) (8 B), and the accepted spin (1 B).
LDS_BYTES_PER_ATTEMPT = 38
# MI355X LDS bandwidth: 256 CUs x 128 B/clk x 2.4 GHz.
LDS_PEAK_GBS = 256 * 128 * 2.4
# 1/t phase ends once W/t < 1e-8, i.e. after W/1e-8 attempts per walker.


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, spins, attempts_per_walker):
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1, cfg["windows"] * cfg["walkers"]))
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
    nw = cfg["windows"] * cfg["walkers"]
    return dict(value=nw * attempts_per_walker / (t2 - t1), unit="attempts/s", cores=threads,
                kind="oracle",
                sample=(f"oracle walk-in ({t1 - t0:.1f} s, excluded) then {attempts_per_walker:,} "
                        f"main-phase attempts per walker of the same workload ({nw} walkers), "
                        f"{threads} OpenMP threads"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="potts_q10_L32")
    ap.add_argument("--cpu-attempts", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the whole REWL hot path on a single "
              "MI355X (multi-GPU window sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1312_3004_amd as pk
    import workloads

    cfg = dict(workloads.CONFIGS[args.config])
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
    if args.warmup:
        g.run(args.warmup * S)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.run(args.steps * S)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms, launches, sync_ms, syncs = g.timing()
    g.set_timing(False)
    if st == pk.CONVERGED:
        raise RuntimeError("run converged inside the timed region; the step count is not the work done")
    attempts = nw * S * args.steps
    value = attempts / elapsed
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s: {value:.4g} attempts/s")

    avg_ms = sweep_ms / max(launches, 1)
    attempts_per_launch = nw * S
    achieved = LDS_BYTES_PER_ATTEMPT * attempts_per_launch / (avg_ms * 1e-3) / 1e9
    per_walker = S * args.steps / elapsed
    W = g.W
    lnf_final = cfg["lnf_final"]
    converge_attempts = (int(W / lnf_final) // S + 1) * S if cfg["schedule"] == 1 else None

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
                   "attempts_per_step_per_walker": S, "attempts_per_step": nw * S},
        "roofline": {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / LDS_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep", "kernel_avg_ms": avg_ms, "kernel_launches": launches,
                     "bytes_per_attempt": LDS_BYTES_PER_ATTEMPT},
        "per_walker_attempts_per_s": per_walker,
        "sync_point_avg_ms": sync_ms / max(syncs, 1),
        "walkin_s": walkin_s,
    }
    if converge_attempts:
        out["time_to_lnf_final_s_projected"] = walkin_s + converge_attempts / per_walker
        out["attempts_per_walker_to_lnf_final"] = converge_attempts
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg, spins, args.cpu_attempts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
