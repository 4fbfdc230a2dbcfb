"""Benchmark: RVEA generations per second on one MI355X.

One step = one whole generation of the hot path (rvea_step, rvea_select,
rvea_adapt: mating, SBX + polynomial mutation, evaluation, ideal point,
association, APD, per-vector argmin, new population, periodic adaptation)
on the 10,011-vector, d=500, m=3 workload (linear-front multimodal test
problem, N = K = 10,011).  Everything is resident in HBM before timing
starts.  Prints one JSON line.

Also reported, for the kernel that takes the most time: its roofline
(algorithmic bytes or flops per launch over its HIP-event-timed average
launch), and the CPU oracle timed on a bounded sample of generations of the
same workload on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector
TIMING_REPS = 20          # back-to-back launches per timed kernel
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix
WORKLOAD = "large_m3_d500_n10011"


def operator_rows(op, N, K):
    """Gene and velocity rows one reproduction launch reads and writes at
    least: the rows each child (CSO: each pair) uses, counted once per use
    but never beyond the K population rows they come from, and the
    children's rows (genes, plus velocities for the swarms)."""
    P = (N + 1) // 2
    reads = {0: min(2 * P, K), 1: min(4 * N, K), 2: min(2 * N, K) + min(N, K),
             3: 2 * min(2 * P, K), 4: 0}[op]
    writes = {0: N, 1: N, 2: 2 * N, 3: 2 * N, 4: N}[op]
    return reads, writes


def kernel_work(name, run):
    """Algorithmic work of one launch: (unit, amount)."""
    N, K, d, m = run.N, run.K, run.d, run.m
    P = (N + 1) // 2
    if name == "offspring":
        op = int(run.params.op)
        if op == 0:
            # read both parent rows of every pair, write every child row and its objectives
            return "bytes", 2 * P * d * 4 + N * d * 4 + N * m * 4
        reads, writes = operator_rows(op, N, K)
        return "bytes", (reads + writes) * d * 4 + N * m * 4
    if name == "assoc" and getattr(run, "indexed", False):
        # indexed association: per merged row its objectives and take-part
        # flag read, association and APD written, one 8-byte atomic minimum
        # (the candidate lists, about five records per row, stay in cache)
        return "bytes", (K + N) * (4 * m + 1 + 4 + 8 + 8)
    if name == "assoc":
        # every (merged row, vector) pair: an m-term dot product (m fused
        # multiply-adds, 2m flops) and one max
        return "flops", (K + N) * K * (2 * m + 1)
    if name == "rerank":
        return "bytes", (K + N) * (m * 4 + 8 + 4)
    return "bytes", 0


def roofline_of(name, run, avg_ms, launches, traffic=None):
    """Roofline record of one kernel from its per-launch time."""
    unit, work = kernel_work(name, run)
    if unit == "bytes":
        ach = work / (avg_ms * 1e-3) / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=ach / PEAK_HBM_GBS, traffic=traffic, kernel=name,
                    avg_launch_us=avg_ms * 1e3, launches=launches, algorithmic_bytes=work)
    ach = work / (avg_ms * 1e-3) / 1e12
    return dict(bound="alu", achieved=ach, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=ach / PEAK_FP32_TFLOPS, traffic=None, kernel=name,
                avg_launch_us=avg_ms * 1e3, launches=launches, algorithmic_flops=work)


def sweeps_leg(a):
    """The paper's two scaling sweeps (its Tables 3 and 4): Series 1 (m = 3,
    d = 100, n = 2^5..2^14) and Series 2 (n = 100, d = 2^9..2^18), 100
    generations each on the linear-front multimodal problem; per point the
    time per generation (graph-replayed run) and the reproduction and
    association kernels against their rooflines."""
    import torch

    import paper_2404_01159_amd as P
    from workloads import SERIES1, SERIES2

    pts = []
    for c in SERIES1 + SERIES2:
        prm = P.default_params(t_max=c["gens"])
        run = P.Run(c["problem"], c["m"], c["d"], c["N"], c["K"], seed=c["seed"], params=prm)
        run.prepare(c["gens"])
        run.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.run(c["gens"])
        run.synchronize()
        el = time.perf_counter() - t0
        run.step()
        t = run.time_kernels(TIMING_REPS)
        run.select()
        run.adapt()
        run.synchronize()
        off = roofline_of("offspring", run, t["offspring"], TIMING_REPS)
        asc = roofline_of("assoc", run, t["assoc"], TIMING_REPS)
        run.close()
        pts.append(dict(workload=c["name"], series=c["series"], n=c["n"], d=c["d"], N=c["N"],
                        K=c["K"], ms_per_generation=el * 1e3 / c["gens"],
                        generations_per_s=c["gens"] / el,
                        offspring_us=off["avg_launch_us"], offspring_hbm_frac=off["frac"],
                        assoc_us=asc["avg_launch_us"], assoc_bound=asc["bound"],
                        assoc_frac=asc["frac"],
                        rerank_us=None if run.indexed else t["rerank"] * 1e3))
    return dict(workload="Series 1: m=3, d=100, n=2^5..2^14; Series 2: m=3, n=100, "
                         "d=2^9..2^18; N=n, K=the smallest lattice count >= n, 100 generations",
                points=pts)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the PMC runs recorded in
    profiles/traffic.json, or None when that kernel's sources have changed
    since (the record keeps their SHA-256)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def cpu_baseline(cfg, budget_s):
    import oracle as O

    prm = O.params()
    st = O.initial_state(cfg["problem"], cfg["m"], cfg["d"], cfg["N"], cfg["K"], cfg["seed"])
    n = 0
    t0 = time.perf_counter()
    while True:
        O.generation(prm, cfg["problem"], cfg["m"], cfg["d"], cfg["N"], cfg["K"], cfg["seed"],
                     n + 1, st)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= cfg["gens"]:
            break
    return dict(value=n / el, unit="generations/s", cores=O.num_threads(), kind="oracle",
                sample=f"generations 1..{n} of the same workload from its initial state, "
                       f"{el:.1f} s")


def policy_flops(N, E, T):
    """Algorithmic flops of one rollout launch: the three policy products
    (64x32, 64x64, 8x64 per rollout step, on the matrix cores in bfloat16).
    The dynamics A x + B u (2 (32x32 + 32x8) flops per step) are not
    counted: their split-bfloat16 products are extra matrix work of the
    implementation, not of the policy."""
    per_step = 2 * (64 * 32 + 64 * 64 + 8 * 64)
    return N * E * T * per_step


def policy_leg(a):
    """The neuroevolution-shaped workload: 4,096 policies (d = 6,728), m = 2,
    K = 4,096, 16 rollouts x 200 steps per individual, 50 generations."""
    import torch

    import oracle as O
    import paper_2404_01159_amd as P
    from workloads import POLICY_CONFIG as C, lq_system

    S = dict(lq_system(C["seed"], E=C["E"]), T=C["T"], sigma=C["sigma"])
    prm = P.default_params(t_max=C["gens"], lb=C["lb"], ub=C["ub"])
    mk = lambda seed: P.Run(C["problem"], C["m"], C["d"], C["N"], C["K"], seed=seed,
                            params=prm, system=S)
    warm = mk(C["seed"] + 1)
    warm.run(2)
    warm.synchronize()
    warm.close()
    run = mk(C["seed"])
    st0 = run.get_state(genes=False)
    tuning = run.autotune() if not a.no_autotune else None
    run.prepare(C["gens"])
    run.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.run(C["gens"])
    run.synchronize()
    el = time.perf_counter() - t0
    counters = run.counters()
    st = run.get_state(genes=False)
    run.close()
    out = {"workload": "4,096 policies 32-64-64-8 tanh (d=6,728), m=2, K=4,096, 16 rollouts "
                       "x 200 steps, 50 generations",
           "generations_per_s": C["gens"] / el, "ms_per_generation": el * 1e3 / C["gens"],
           "counters": counters, "assoc_tiles": tuning}
    # quality of the final survivors: objectives normalised by lo = 0 and
    # hi = the initial population's largest values (both objectives are sums
    # of squares), hypervolume with reference point ones and expected utility
    # over 100 evenly spread weights
    hi = st0["F"][st0["valid"] == 1].astype("float64").max(axis=0)
    W = weights_simplex(2, 99)
    out["indicators"] = dict(
        normalisation="lo = 0, hi = the initial population's largest objective values",
        hypervolume_initial=P.hypervolume(st0["F"], st0["valid"], [0.0, 0.0], hi),
        hypervolume_final=P.hypervolume(st["F"], st["valid"], [0.0, 0.0], hi),
        expected_utility_final=P.expected_utility(st["F"], W, st["valid"], [0.0, 0.0], hi))
    names = ["offspring", "assoc", "rerank", "adapt", "rollout"]
    run = mk(C["seed"])
    if not a.no_autotune:
        run.autotune()
    run.set_timing(range(5))
    run.run(C["gens"])
    run.synchronize()
    per = {}
    for k in range(5):
        ms, n = run.kernel_time(k)
        if n:
            per[names[k]] = (ms / n, n)
    run.close()
    out["kernels_avg_us"] = {k: v[0] * 1e3 for k, v in per.items()}
    avg_ms, n = per["rollout"]
    ach = policy_flops(C["N"], C["E"], C["T"]) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = dict(bound="mfma", achieved=ach, peak=PEAK_BF16_TFLOPS, unit="TFLOP/s",
                           frac=ach / PEAK_BF16_TFLOPS, traffic=None, kernel="rollout",
                           avg_launch_us=avg_ms * 1e3, launches=n)
    if not a.no_cpu_baseline:
        # the oracle's first generation of the same workload (all 4,096 rollouts)
        op = O.params(lq=S, t_max=C["gens"], lb=C["lb"], ub=C["ub"])
        st = O.initial_state(C["problem"], C["m"], C["d"], C["N"], C["K"], C["seed"], C["lb"],
                             C["ub"], lq=S)
        t0 = time.perf_counter()
        O.generation(op, C["problem"], C["m"], C["d"], C["N"], C["K"], C["seed"], 1, st)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=1.0 / el, unit="generations/s", cores=O.num_threads(),
                                   kind="oracle", sample=f"generation 1 of the same workload, "
                                                         f"{el:.1f} s")
    return out


def weights_simplex(m, H):
    """Das-Dennis weight vectors on the simplex (entries a/H summing to 1),
    each equally likely: the weight set of the expected utility."""
    import itertools

    import numpy as np

    rows = []
    for c in itertools.combinations(range(1, H + m), m - 1):
        prev, a = 0, []
        for ci in c:
            a.append(ci - prev - 1)
            prev = ci
        a.append(H + m - 1 - prev)
        rows.append(a)
    return np.array(rows, np.float64) / H


def indicators_leg(a):
    """Hypervolume (App. C.2) and expected utility of the 105-vector
    workload's final survivors (sphere-front problem, whose front spans
    [0, 1] in every objective: no normalisation), and the time of the
    device hypervolume on the 10,011-vector workload's final population."""
    import torch

    import paper_2404_01159_amd as P
    from workloads import CONFIGS

    out = {}
    c = CONFIGS["small_m3_d12_n105"]
    run = P.Run(c["problem"], c["m"], c["d"], c["N"], c["K"], seed=c["seed"],
                params=P.default_params(t_max=c["gens"]))
    run.run(c["gens"])
    st = run.get_state(genes=False)
    run.close()
    out["small_m3_d12_n105"] = dict(
        generations=c["gens"], hypervolume=P.hypervolume(st["F"], st["valid"]),
        expected_utility=P.expected_utility(st["F"], weights_simplex(3, 13), st["valid"]))
    c = CONFIGS[WORKLOAD]
    run = P.Run(c["problem"], c["m"], c["d"], c["N"], c["K"], seed=c["seed"],
                params=P.default_params(t_max=c["gens"]))
    run.run(c["gens"])
    st = run.get_state(genes=False)
    run.close()
    F = torch.from_numpy(st["F"]).cuda()
    v = torch.from_numpy(st["valid"]).cuda()
    hi = 1.1 * st["F"][st["valid"] == 1].astype("float64").max(axis=0)
    lo = [0.0] * c["m"]
    P.hypervolume(F, v, lo, hi)  # warm
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        hv = P.hypervolume(F, v, lo, hi)
    el = (time.perf_counter() - t0) / reps
    out[WORKLOAD] = dict(generations=c["gens"], rows=c["K"], hypervolume=hv,
                         normalisation="lo = 0, hi = 1.1 x the survivors' largest values",
                         hypervolume_call_ms=el * 1e3)
    return out


def operators_leg(a):
    """The extensibility study (Sec. 4): GA, DE, PSO, CSO and random
    reproduction in the same RVEA.  On the policy workload, 50 generations
    each from the same initial population: generations/s and the final
    survivors' hypervolume and expected utility (normalised as in the policy
    leg).  On the 10,011-vector workload: generations/s and the reproduction
    kernel's time and HBM roofline per operator."""
    import numpy as np
    import torch

    import paper_2404_01159_amd as P
    from workloads import CONFIGS, POLICY_CONFIG as C, lq_system

    out = {"operator_parameters": {"ga": "SBX + PM, eta 20, p_c 1, p_m 1",
                                   "de": "DE/rand/1/bin F 0.5, CR 0.9",
                                   "pso": "inertia 0.5, social 1.5", "cso": "phi 0",
                                   "rand": "uniform in the box"}}
    S = dict(lq_system(C["seed"], E=C["E"]), T=C["T"], sigma=C["sigma"])
    W = weights_simplex(2, 99)
    pol = {}
    hi = None
    for name in ("ga", "de", "pso", "cso", "rand"):
        prm = P.default_params(name, t_max=C["gens"], lb=C["lb"], ub=C["ub"])
        run = P.Run(C["problem"], C["m"], C["d"], C["N"], C["K"], seed=C["seed"], params=prm,
                    system=S)
        st0 = run.get_state(genes=False)
        if hi is None:  # the same initial population for every operator
            hi = st0["F"][st0["valid"] == 1].astype(np.float64).max(axis=0)
        run.prepare(C["gens"])
        run.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.run(C["gens"])
        run.synchronize()
        el = time.perf_counter() - t0
        st = run.get_state(genes=False)
        run.close()
        pol[name] = dict(generations_per_s=C["gens"] / el,
                         hypervolume_final=P.hypervolume(st["F"], st["valid"], [0.0, 0.0], hi),
                         expected_utility_final=P.expected_utility(st["F"], W, st["valid"],
                                                                   [0.0, 0.0], hi))
    out["policy"] = dict(workload="4,096 policies (d=6,728), m=2, K=4,096, 16 rollouts x 200 "
                                  "steps, 50 generations", per_operator=pol)
    c = CONFIGS[WORKLOAD]
    head = {}
    for name in ("ga", "de", "pso", "cso", "rand"):
        prm = P.default_params(name, t_max=c["gens"])
        run = P.Run(c["problem"], c["m"], c["d"], c["N"], c["K"], seed=c["seed"], params=prm)
        run.run(3)
        gens = 20
        run.prepare(gens)
        run.synchronize()
        t0 = time.perf_counter()
        run.run(gens)
        run.synchronize()
        el = time.perf_counter() - t0
        run.step()
        t = run.time_kernels(TIMING_REPS)
        run.select()
        run.adapt()
        run.synchronize()
        r = roofline_of("offspring", run, t["offspring"], TIMING_REPS)
        run.close()
        head[name] = dict(generations_per_s=gens / el, offspring_us=t["offspring"] * 1e3,
                          hbm_gbs=r["achieved"], hbm_frac=r["frac"],
                          algorithmic_bytes=r["algorithmic_bytes"])
    out[WORKLOAD] = head
    return out


def serving_legs(a):
    """Served runs (open loop, Poisson arrivals), the same runs all at once
    (batched capacity), and the same runs one at a time on the plain path."""
    import torch

    import paper_2404_01159_amd as P
    from paper_2404_01159_amd.serve import DeviceBackend, Request, Server, latency_summary
    from workloads import serving_specs

    specs = serving_specs(a.serve_runs, a.serve_rate, seed=0)
    reqs = [Request(s["rid"], s["arrival"], s["problem"], s["m"], s["d"], s["N"], s["K"],
                    s["seed"], s["gens"]) for s in specs]
    out = {"workload": f"{len(reqs)} runs, Poisson {a.serve_rate}/s, m in {{2,3,5,8}}, "
                       "d in [30,2000], K=N in [100,10011], 100 generations each"}
    budget = int(a.serve_budget_gib * (1 << 30))
    if not a.batched_only:
        be = DeviceBackend(budget, max_runs=256)
        srv = Server(be, budget, max_runs=256)
        res = srv.serve(reqs)
        out["open_loop"] = dict(latency_summary(res), arena_gib=a.serve_budget_gib,
                                peak_resident_runs=srv.peak_runs, ticks=srv.ticks)
        del be, srv
    # the same runs arriving faster (Poisson serve_rate_high/s, below the
    # batched capacity): many runs resident at once, in a 16 GiB arena
    if a.serve_rate_high > 0 and not a.batched_only:
        hs = serving_specs(a.serve_runs, a.serve_rate_high, seed=0)
        hreqs = [Request(s["rid"], s["arrival"], s["problem"], s["m"], s["d"], s["N"], s["K"],
                         s["seed"], s["gens"]) for s in hs]
        hb = 16 << 30
        be = DeviceBackend(hb, max_runs=256)
        srv = Server(be, hb, max_runs=256)
        res = srv.serve(hreqs)
        out["open_loop_high_rate"] = dict(latency_summary(res), rate_per_s=a.serve_rate_high,
                                          arena_gib=16, peak_resident_runs=srv.peak_runs,
                                          ticks=srv.ticks)
        del be, srv
    # saturated: every request present at t = 0, large arena
    sat = [Request(r.rid, 0.0, r.problem, r.m, r.d, r.N, r.K, r.seed, r.gens) for r in reqs]
    total = sum(P.footprint(r.problem, r.m, r.d, r.N, r.K, P.default_params()) for r in sat)
    be = DeviceBackend(total + (1 << 26), max_runs=256)
    srv = Server(be, total + (1 << 26), max_runs=256)
    t0 = time.perf_counter()
    res = srv.serve(sat)
    el = time.perf_counter() - t0
    out["batched_all_at_once"] = dict(runs=len(res), runs_per_s=len(res) / el, seconds=el,
                                      ticks=srv.ticks, arena_gib=total / (1 << 30))
    del be, srv
    torch.cuda.synchronize()
    if a.batched_only:
        return out
    # one run at a time, plain single-run path (multi-generation graphs)
    t0 = time.perf_counter()
    for r in sat:
        run = P.Run(r.problem, r.m, r.d, r.N, r.K, seed=r.seed,
                    params=P.default_params(t_max=100))
        run.run(r.gens)
        run.synchronize()
        run.close()
    el1 = time.perf_counter() - t0
    out["one_at_a_time"] = dict(runs=len(sat), runs_per_s=len(sat) / el1, seconds=el1)
    out["batched_over_one_at_a_time"] = out["batched_all_at_once"]["runs_per_s"] / (
        len(sat) / el1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=WORKLOAD)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-kernel events (for profiler runs)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served / batched runs legs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default association tiles")
    ap.add_argument("--no-policy", action="store_true",
                    help="skip the policy-rollout (neuroevolution-shaped) workload")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the population-size and dimension sweeps")
    ap.add_argument("--no-operators", action="store_true",
                    help="skip the reproduction-operator comparison")
    ap.add_argument("--no-indicators", action="store_true",
                    help="skip the hypervolume / expected-utility leg")
    ap.add_argument("--serve-runs", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--serve-rate-high", type=float, default=400.0,
                    help="arrival rate of the second open-loop run (0: skip it)")
    ap.add_argument("--batched-only", action="store_true",
                    help="serving: only the runs all present at once (for profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported by this build",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if a.calibrate_copy:
        n = a.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 5}), flush=True)
        return

    import paper_2404_01159_amd as P
    from workloads import CONFIGS

    cfg = CONFIGS[a.config]
    prm = P.default_params(t_max=max(cfg["gens"], 1))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # warm-up on a separate run of the same shape
    warm = P.Run(cfg["problem"], cfg["m"], cfg["d"], cfg["N"], cfg["K"], seed=cfg["seed"] + 1,
                 params=prm, device="cuda:0")
    warm.run(a.warmup)
    warm.synchronize()
    warm.close()
    del warm

    # timed pass: a fresh run, association tiles autotuned on its first
    # generation (nothing committed), every generation one HIP-graph launch
    run = P.Run(cfg["problem"], cfg["m"], cfg["d"], cfg["N"], cfg["K"], seed=cfg["seed"],
                params=prm, device="cuda:0")
    tuning = run.autotune() if not a.no_autotune else None
    run.prepare(a.steps)  # graph capture outside the timed region
    run.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.run(a.steps)
    run.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gens_per_s = a.steps / el
    st = run.get_state(genes=False)
    counters = run.counters()

    # kernel timing on the same run, one generation further: each hot kernel
    # launched REPS times back to back between two HIP events on the run's
    # stream (a replayed graph cannot carry fresh events, and an event pair
    # around every single launch adds its own dispatch time)
    # the same generations with the association by full scans (identical
    # results): what the vector index gains on this workload
    full_scan = None
    if run.indexed and not a.no_timing:
        fs = P.Run(cfg["problem"], cfg["m"], cfg["d"], cfg["N"], cfg["K"], seed=cfg["seed"],
                   params=prm, device="cuda:0")
        fs.set_index(False)
        if not a.no_autotune:
            fs.autotune()
        fs.prepare(a.steps)
        fs.synchronize()
        t0 = time.perf_counter()
        fs.run(a.steps)
        fs.synchronize()
        fel = time.perf_counter() - t0
        fs.close()
        full_scan = dict(generations_per_s=a.steps / fel, ms_per_generation=fel * 1e3 / a.steps)

    roof = None
    rooflines = {}
    per_kernel = {}
    if not a.no_timing:
        run.step()
        t = run.time_kernels(TIMING_REPS)
        run.select()
        run.adapt()
        run.synchronize()
        # the indexed association has no separate re-rank
        for k in ("offspring", "assoc") + (() if run.indexed else ("rerank",)):
            per_kernel[k] = (t[k], TIMING_REPS)
        dom = max(per_kernel, key=lambda k: per_kernel[k][0])
        for k in ("offspring", "assoc"):
            avg_ms, n = per_kernel[k]
            traffic = measured_traffic(k) if (a.config == WORKLOAD and k == "offspring") else None
            rooflines[k] = roofline_of(k, run, avg_ms, n, traffic)
        roof = rooflines.get(dom) or roofline_of(dom, run, *per_kernel[dom])
    run.close()

    serving = None
    if not a.no_serving:
        serving = serving_legs(a)

    policy = None
    if not a.no_policy:
        policy = policy_leg(a)

    sweeps = None
    if not a.no_sweeps:
        sweeps = sweeps_leg(a)

    indicators = None
    if not a.no_indicators:
        indicators = indicators_leg(a)

    operators = None
    if not a.no_operators:
        operators = operators_leg(a)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(cfg, a.cpu_budget)

    out = {
        "metric": "RVEA generations/s at N=10k,m=3,d=500 vs plain; served runs/s + p50/p99 latency",
        "value": gens_per_s,
        "unit": "generations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 genes and objectives, f64 selection finish",
        "data": "synthetic",
        "config": {"workload": a.config, "problem": "linear front, multimodal distance term",
                   "N": cfg["N"], "K": cfg["K"], "m": cfg["m"], "d": cfg["d"],
                   "generations_timed": a.steps, "survivors_final": int(st["valid"].sum())},
        "roofline": roof,
        "rooflines": rooflines,
        "kernels_avg_us": {k: v[0] * 1e3 for k, v in per_kernel.items()},
        "assoc_tiles": tuning,
        "association_by_full_scan": full_scan,
        "counters": counters,
        "cpu_baseline": cpu,
        "serving": serving,
        "policy": policy,
        "sweeps": sweeps,
        "indicators": indicators,
        "operators": operators,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
