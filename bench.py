"""Benchmark: parallel GOM partial evaluations per second and time-to-optimum on one MI355X,
batched against plain.

Default line (the batched configuration): 256 independent Max-Cut instances with n
log-uniform in [10^3, 10^5] (even positions L x L tori, odd positions random 4- and 8-regular
graphs), weights uniform in [1, 100], populations uniform in [16, 64], univariate and
neighbourhood FOS alternating in pairs, run as lockstep batches (two by default, one a
stream, at the same time) until every torus reaches its total weight or 200 generations: per
generation step, resident-block sweeps for the instances the autotuner leaves there, one class
launch per class position covering every other instance (bit-sliced where admitted), one
finalize and one vertex pass, replayed from captured HIP graphs.

A step is one batched run of the whole mix from fresh initial populations (new seeds per
step).  `value` = attempted partial evaluations (population x FOS sets x generations, summed
over instances and steps) per second of the timed region.  Beside it: the plain loop (the
first timed step's seeds, one instance after another, each alone, with the default schedule),
whether every result is identical (counters and state hashes), time to optimum, the roofline
of the batched sweep kernel (algorithmic bytes of every instance-generation over the summed
launch times, from HIP events recorded by each launch's dispatch in one more run after the
timed region) and the CPU oracle timed on a bounded sample of the mix.

Other modes: --workload NAME (plain GOM on one instance per launch sequence, e.g.
torus100_nbhd_p64), --serve (the serving loop), --ims (interleaved multistart).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "GOM partial evals/sec and time-to-optimum at 1 GPU, batched vs plain (bit-exact)"
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "torus100_nbhd_p64"
WORKLOAD_NAMES = {"torus100_nbhd_p64": "torus100x100_nbhd_pop64_to_optimum_or_500"}


# HBM traffic per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a device
# copy of known size), with the hash of the kernel sources they were taken on.  Reported as
# roofline.traffic only while the sources still hash the same; the summaries and commands are
# in profiles/.  A source change whose gfx950 assembly is identical (hipcc
# --offload-device-only -S, apart from the compilation-unit id) carries the figures over to
# the new hash.
MEASURED_TRAFFIC = {
    # per generation step: 216 k_bcl_gs_sweep dispatches (two batches x 108) x 50284353 bytes
    ("batched_sweeps", "batch256_mix"): {
        "bytes": 10861420248, "source": "706ff9da0b9d659e",
        "profile": "profiles/k_bcl_gs_sweep_batch256_mix.md"},
    ("k_gen_swar_sweep + k_class_sweep", "torus1000_nbhd_p64"): {
        "bytes": 49310592, "source": "706ff9da0b9d659e",
        "profile": "profiles/k_gen_swar_sweep_torus1000_nbhd_p64.md"},
    ("k_uni_swar_sweep", "torus3162_uni_p64"): {
        "bytes": 269255872, "source": "706ff9da0b9d659e",
        "profile": "profiles/k_uni_swar_sweep_torus3162_uni_p64.md"},
    ("k_uni_swar_sweep", "torus1000_uni_p64"): {
        "bytes": 23209750, "source": "706ff9da0b9d659e",
        "profile": "profiles/k_uni_swar_sweep_torus1000_uni_p64.md"},
    ("k_class_sweep", "torus100_nbhd_p64"): {
        "bytes": 934260, "source": "706ff9da0b9d659e",
        "profile": "profiles/k_class_sweep_torus100_nbhd_p64.md"},
}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("gom_kernels.hip", "gom_internal.h"):
        with open(os.path.join(ROOT, "paper_2203_08680_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def class_sweep_bytes(csr, set_ptr, set_vars, class_ptr, class_elems, pop):
    """Algorithmic bytes of each class-sweep launch: the population words of the vertices the
    class's sets touch (N[F_j]: members and their neighbours) read once from O, the members'
    words read from P and written to O, and each member's adjacency (an int32 row pointer plus
    an int32 (neighbour, weight) pair per incident edge)."""
    row_ptr, col, _ = csr
    bp = pop / 8.0
    deg = np.diff(row_ptr).astype(np.int64)
    sizes = np.diff(set_ptr)
    out = []
    for c in range(len(class_ptr) - 1):
        sets = class_elems[class_ptr[c]:class_ptr[c + 1]]
        members = np.concatenate([set_vars[set_ptr[j]:set_ptr[j] + sizes[j]] for j in sets]) \
            if len(sets) < 64 else set_vars[np.concatenate(
                [np.arange(set_ptr[j], set_ptr[j + 1]) for j in sets])]
        starts, counts = row_ptr[members], deg[members]
        idx = np.repeat(starts - np.cumsum(counts) + counts, counts) + np.arange(counts.sum())
        touched = np.unique(np.concatenate([members, col[idx]]))
        out.append(bp * (touched.size + 2 * members.size) + float(np.sum(4 + 8 * counts)))
    return np.array(out)


def native_oracle():
    """Point the oracle at a -march=native build of its unchanged source for this host (the
    portable in-tree build when the compiler refuses).  Returns whether the native one is used."""
    import tempfile
    import oracle
    try:
        oracle.use_native_build(os.path.join(tempfile.gettempdir(),
                                             f"liboracle_native_{os.getpid()}.so"))
        return True
    except Exception as e:
        log(f"cpu baseline: native build failed ({e}); portable build used")
        return False


def cpu_baseline(g, fos_kind, pop, gens, target, fi=False):
    """The oracle, unchanged, on seed 1's first `gens` generations of the same workload, each
    colour class's solutions spread over every host core (up to 16); the oracle builds its own
    FOS (and colouring) from the graph."""
    import oracle
    native = native_oracle()
    workers = max(1, min(16, os.cpu_count() or 1))
    set_ptr, set_vars = oracle.fos(g, fos_kind)
    run = oracle.Run(g, set_ptr, set_vars, pop=pop, seed=1, flags=oracle.FLAG_FI if fi else 0)
    used = run.set_workers(workers)
    t0 = time.perf_counter()
    ran = run.run(target, gens)
    dt = time.perf_counter() - t0
    s = run.state(genes=False)
    run.close()
    return {"value": s["attempted"] / dt, "unit": "evals/s", "cores": used, "kind": "oracle",
            "sample": f"seed 1, first {ran} generations of the benchmark run "
                      f"({s['attempted']} attempted partial evaluations in {dt:.2f} s; each "
                      f"colour class's solutions spread over {used} threads)",
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count(),
            "build": "gcc -O2 -fopenmp -march=native" if native else "in-tree portable build"}


def instance_bytes(inst, pop):
    """Algorithmic bytes of one generation of one instance (every class swept once)."""
    _, class_ptr, class_elems = inst.classes()
    set_ptr, set_vars = inst.fos.sets()
    return float(class_sweep_bytes(inst.graph.csr(), set_ptr, set_vars, class_ptr, class_elems,
                                   pop).sum())


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_mix(items, seeds, count, gens):
    """The oracle, unchanged, built with -march=native on this host, on the first `count`
    instances of the mix for `gens` generations each (the seeds of the first timed step), its
    colour classes' solutions spread over every host core (up to 16)."""
    import oracle
    workers = max(1, min(16, os.cpu_count() or 1))
    native = native_oracle()
    attempted, dt, used = 0, 0.0, 1
    for it, sd in zip(items[:count], seeds[:count]):
        set_ptr, set_vars = oracle.fos(it.graph, it.fos)
        run = oracle.Run(it.graph, set_ptr, set_vars, pop=it.pop, seed=int(sd))
        used = run.set_workers(workers)
        tg = it.graph.total_weight if it.to_total_weight else (1 << 62)
        t0 = time.perf_counter()
        run.run(tg, gens)
        dt += time.perf_counter() - t0
        attempted += run.state(genes=False)["attempted"]
        run.close()
    return {"value": attempted / dt, "unit": "evals/s", "cores": used, "kind": "oracle",
            "sample": f"first {count} instances of the mix (the first timed step's seeds), "
                      f"{gens} generations each: {attempted} attempted partial evaluations in "
                      f"{dt:.2f} s; each colour class's solutions spread over {used} threads "
                      "(results independent of the thread count)",
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count(),
            "build": "gcc -O2 -fopenmp" + (" -march=native" if native else "")}


def write_metrics_log(path, gom, torch, st, target, max_gens):
    """Per-generation metrics of one more run (seed 1), one JSON line per generation: the
    generation, the elitist's and the population's best and mean fitness, the cumulative
    attempted / evaluated / accepted counts and the wall time of the generation (enqueue to
    completion, ns).  Outside the timed region: each generation waits for its read-back."""
    gom.gom_state_reseed(st, 1)
    with open(path, "w") as fh:
        for g in range(max_gens):
            torch.cuda.synchronize()
            t0 = time.perf_counter_ns()
            gom.gom_generation(st)
            s = gom.gom_state_read(st, genes=False)
            ns = time.perf_counter_ns() - t0
            f = np.asarray(s["fitness"])
            fh.write(json.dumps({"g": s["generation"], "elite": s["elite_fitness"],
                                 "best": int(f.max()), "mean": float(f.mean()),
                                 "attempted": s["attempted"], "evaluated": s["evaluated"],
                                 "accepted": s["accepted"], "ns": ns}) + "\n")
            if s["elite_fitness"] >= target:
                break
    log(f"metrics log: {path}")


def write_batch_metrics_log(path, gom, torch, batches, groups, seeds, targets, max_gens):
    """Per-generation metrics of one more batched run (the given seeds), one JSON line per
    generation step: the generation, instances at their target, the sum and the mean of the
    instances' elitist fitnesses, the cumulative attempted / evaluated / accepted counts over
    all instances and the wall time of the step (enqueue to completion, ns).  Outside the
    timed region: each step waits for its read-back, the batches one after another."""
    for batch, g in zip(batches, groups):
        gom.gom_batch_reseed(batch, [seeds[i] for i in g])
    with open(path, "w") as fh:
        for gen in range(1, max_gens + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter_ns()
            res = []
            for batch in batches:
                res.extend(gom.gom_batch_run(batch, gen)[0])
            ns = time.perf_counter_ns() - t0
            states = [gom.gom_state_read(batch.state(p), genes=False)
                      for batch, g in zip(batches, groups) for p in range(len(g))]
            order = [i for g in groups for i in g]
            reached = sum(1 for s_, i in zip(states, order) if s_["elite_fitness"] >= targets[i])
            elites = [s_["elite_fitness"] for s_ in states]
            fh.write(json.dumps({
                "g": gen, "reached": reached, "elite_sum": int(sum(elites)),
                "elite_mean": float(np.mean(elites)),
                "attempted": int(sum(s_["attempted"] for s_ in states)),
                "evaluated": int(sum(s_["evaluated"] for s_ in states)),
                "accepted": int(sum(s_["accepted"] for s_ in states)), "ns": ns}) + "\n")
    log(f"metrics log: {path}")


def copy_calibration(torch, mb):
    """A device copy of a known byte count (3 times), for scaling profiler traffic counters."""
    if not mb:
        return
    nbytes = mb << 20
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes")


def step_seeds(items, k):
    """Seeds of timed step k (k >= 0); warm-up steps use k < 0.  Distinct per instance and
    step."""
    return [(k + 2) * 100_000 + b for b in range(len(items))]


def small_mix_time_to_optimum(torch, gom, count, max_gens):
    """Time to optimum on a mix of small instances that reach it: tori of 6x6 to 12x12 and
    random 4/8-regular graphs of 36 to 144 vertices, batched against the plain loop, with
    identical results."""
    items = workloads.batch_mix(count=count, seed=4, n_lo=36, n_hi=144)
    insts = [gom.Instance(it.graph.n, it.graph.u, it.graph.v, it.graph.w, it.fos)
             for it in items]
    targets = [it.graph.total_weight if it.to_total_weight else (1 << 62) for it in items]
    pops, seeds = [it.pop for it in items], [it.seed for it in items]
    batch = gom.gom_batch_init(insts, pops, seeds, targets)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, tt = gom.gom_batch_run(batch, max_gens)
    t_batch = time.perf_counter() - t0
    plain_t, plain = [], []
    for x, p, sd, tg in zip(insts, pops, seeds, targets):
        st = x.state(pop=p, seed=sd)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        plain.append(gom.gom_run_to_target(st, tg, max_gens))
        plain_t.append(time.perf_counter() - s0)
    same = all((a.generations, a.reached, a.best, a.evaluated, a.accepted) ==
               (b.generations, b.reached, b.best, b.evaluated, b.accepted)
               for a, b in zip(res, plain))
    tori = [b for b, it in enumerate(items) if it.to_total_weight and res[b].reached]
    loop_t = np.cumsum(plain_t) * 1e3
    q = lambda x, p: float(np.percentile(np.asarray(x), p)) if len(x) else None
    return {"workload": f"batch{count}_tori_and_regular_36_144", "max_generations": max_gens,
            "tori_reached": len(tori), "identical_results": same,
            "batched_ms": t_batch * 1e3, "plain_loop_ms": float(loop_t[-1]),
            "batched_p50": q([tt[b] for b in tori], 50), "batched_p99": q([tt[b] for b in tori], 99),
            "plain_loop_p50": q([loop_t[b] for b in tori], 50),
            "plain_loop_p99": q([loop_t[b] for b in tori], 99),
            "plain_alone_p50": q([plain_t[b] * 1e3 for b in tori], 50),
            "plain_alone_p99": q([plain_t[b] * 1e3 for b in tori], 99)}


def batch_groups(insts, k):
    """Instance indices of k batches: dealt round-robin in order of class count (largest
    first), each group in instance order."""
    if k <= 1:
        return [list(range(len(insts)))]
    kc = [len(x.classes()[1]) - 1 for x in insts]
    order = sorted(range(len(insts)), key=lambda i: (-kc[i], i))
    return [sorted(order[g::k]) for g in range(k)]


def run_batch_mode(args, torch, gom):
    """Batched vs plain on the 256-instance mix (the default line).  A step is one batched run
    of the whole mix: fresh initial populations (new seeds), then lockstep generations until
    every instance has reached its target or the generation limit.  The plain leg runs the
    first timed step's seeds one instance after another, each alone; results must be
    identical (counters and state hashes)."""
    n_lo, n_hi = args.batch_n_range
    n_label = "1e3_1e5" if (n_lo, n_hi) == (1e3, 1e5) else f"{n_lo:g}_{n_hi:g}"
    items = workloads.batch_mix(count=args.batch_count, seed=4, n_lo=n_lo, n_hi=n_hi)
    max_gens = args.max_gens or 200
    t0 = time.perf_counter()
    insts = [gom.Instance(it.graph.n, it.graph.u, it.graph.v, it.graph.w, it.fos)
             for it in items]
    targets = [it.graph.total_weight if it.to_total_weight else (1 << 62) for it in items]
    pops = [it.pop for it in items]
    t_setup = time.perf_counter() - t0
    log(f"batch set-up: {len(items)} instances, {sum(x.n for x in insts)} vertices, graphs, "
        f"FOS and colourings in {t_setup:.1f} s")
    # the mix as `batch_streams` batches, each on its own stream (instances dealt round-robin
    # in order of their class counts, so every batch holds a like share of long and short
    # class sequences); each batch runs from its own host thread
    groups = batch_groups(insts, args.batch_streams)
    t0 = time.perf_counter()
    seeds_init = step_seeds(items, 0)
    batches = [gom.gom_batch_init([insts[i] for i in g], [pops[i] for i in g],
                                  [seeds_init[i] for i in g], [targets[i] for i in g])
               for g in groups]
    streams = [torch.cuda.Stream() for _ in groups] if len(groups) > 1 else [None]
    for batch in batches:
        gom.gom_batch_set_graph(batch, args.batch_graph == "on")
    log(f"batch states: {time.perf_counter() - t0:.1f} s ({len(batches)} batches)")
    tuned = (args.batch_narrow is None and args.batch_class_min is None and
             args.batch_class_ppw is None and args.batch_class_form is None)
    for batch in batches:
        if tuned:
            t0 = time.perf_counter()
            chosen = gom.gom_batch_autotune(batch, 2)
            log(f"batch autotune: thresholds {chosen} in {time.perf_counter() - t0:.1f} s")
        else:
            if args.batch_narrow is not None:
                gom.gom_batch_set_narrow(batch, args.batch_narrow)
            if args.batch_class_min is not None:
                gom.gom_batch_set_class_launch(batch, args.batch_class_min)
            if args.batch_class_ppw is not None:
                gom.gom_batch_set_class_positions(batch, args.batch_class_ppw)
            if args.batch_class_form is not None:
                gom.gom_batch_set_class_bitsliced(batch, args.batch_class_form == "bitsliced")
    shapes = [(gom.gom_batch_get_narrow(b), gom.gom_batch_get_class_launch(b)) for b in batches]
    narrow = [x[0][0] for x in shapes]
    sweep_launches = [x[0][1] for x in shapes]
    class_min = [x[1][0] for x in shapes]
    class_insts = sum(x[1][1] for x in shapes)
    class_launches = [x[1][2] for x in shapes]
    class_ppw = [x[1][3] for x in shapes]
    class_bits = all(gom.gom_batch_get_class_bitsliced(b)[0] for b, x in zip(batches, shapes)
                     if x[1][1]) if class_insts else False

    def run_all(k, timing=False):
        """Fresh populations (the seeds of step k) and a run of every batch, the batches at
        once on their streams (one host thread each) or, for the timing pass, one by one."""
        seeds = step_seeds(items, k)
        for batch, g, s in zip(batches, groups, streams):
            gom.gom_batch_reseed(batch, [seeds[i] for i in g], stream=s)
        out = [None] * len(batches)

        def go(j):
            out[j] = gom.gom_batch_run(batches[j], max_gens, stream=streams[j])

        if len(batches) == 1 or timing:
            for j in range(len(batches)):
                go(j)
        else:
            th = [threading.Thread(target=go, args=(j,)) for j in range(len(batches))]
            for x in th:
                x.start()
            for x in th:
                x.join()
        res, tt = [None] * len(items), np.zeros(len(items))
        for j, g in enumerate(groups):
            for pos, i in enumerate(g):
                res[i] = out[j][0][pos]
                tt[i] = out[j][1][pos]
        return res, tt

    def one_step(k):
        return run_all(k)

    for w in range(args.warmup):
        res, _ = one_step(-1 - w)
        log(f"warmup {w}: {sum(r.generations for r in res)} instance-generations")
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        res, tt = one_step(k)
        steps.append((res, tt, time.perf_counter() - s0))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    attempted = sum(r.attempted for res, _, _ in steps for r in res)
    evaluated = sum(r.evaluated for res, _, _ in steps for r in res)
    for k, (res, tt, dt) in enumerate(steps):
        log(f"step {k}: {dt * 1e3:.1f} ms, {sum(r.attempted for r in res)} attempted, "
            f"reached {sum(r.reached for r in res)}")

    # kernel-timing pass after the timed region: the first timed step's seeds again, every
    # sweep launch timed with HIP events recorded by its own dispatch (direct launches)
    for batch in batches:
        gom.gom_batch_timing_enable(batch, True)
        gom.gom_batch_timing_read(batch)
    res_t, _ = run_all(0, timing=True)
    sweep_ms, launches = 0.0, 0
    for batch in batches:  # (summed over the batches, per generation step)
        ms, n = gom.gom_batch_timing_read(batch)
        sweep_ms += ms
        launches = max(launches, n)
        gom.gom_batch_timing_enable(batch, False)
    copy_calibration(torch, args.copy_calib_mb)
    where = {i: (j, pos) for j, g in enumerate(groups) for pos, i in enumerate(g)}
    batch_hash = [gom.gom_state_hash(batches[where[i][0]].state(where[i][1]))
                  for i in range(len(items))]
    same_timed = all((a.generations, a.best, a.evaluated, a.accepted) ==
                     (b.generations, b.best, b.evaluated, b.accepted)
                     for a, b in zip(res_t, steps[0][0]))

    # plain leg: the same seeds, one instance after another, each alone
    seeds0 = step_seeds(items, 0)
    plain, plain_t, plain_hash = [], [], []
    t0 = time.perf_counter()
    for x, p, sd, tg in zip(insts, pops, seeds0, targets):
        if args.no_plain:
            break
        st = x.state(pop=p, seed=sd)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        gom.gom_state_reseed(st, sd)
        plain.append(gom.gom_run_to_target(st, tg, max_gens))
        plain_t.append(time.perf_counter() - s0)
        plain_hash.append(gom.gom_state_hash(st))
        del st
    t_plain = sum(plain_t)
    ev_plain = sum(r.attempted for r in plain)
    same = None if args.no_plain else same_timed and all(
        (a.generations, a.reached, a.best, a.attempted, a.evaluated, a.accepted, ha) ==
        (b.generations, b.reached, b.best, b.attempted, b.evaluated, b.accepted, hb)
        for a, b, ha, hb in zip(steps[0][0], plain, batch_hash, plain_hash))
    log(f"plain: {t_plain * 1e3:.1f} ms for the first step's seeds, identical results: {same}")
    if args.metrics_jsonl:  # one more run (the first timed step's seeds), after the checks
        write_batch_metrics_log(args.metrics_jsonl, gom, torch, batches, groups, seeds0,
                                targets, max_gens)

    value = attempted / total
    plain_value = ev_plain / t_plain if plain else None
    res0, tt0, t_step0 = steps[0]
    tori = [b for b, it in enumerate(items) if it.to_total_weight and res0[b].reached]
    loop_t = np.cumsum(plain_t) * 1e3 if plain else np.zeros(len(items))
    q = lambda x, p: float(np.percentile(np.asarray(x), p)) if len(x) else None

    # roofline of the batched sweep: the algorithmic bytes of every instance-generation the
    # timing pass ran, over the summed sweep time
    roofline = None
    if launches:
        ib = [instance_bytes(x, p) for x, p in zip(insts, pops)]
        total_bytes = float(sum(ib[b] * res_t[b].generations for b in range(len(items))))
        achieved = total_bytes / (sweep_ms / 1e3) / 1e9
        # the counters were taken on the default mix as two batches, every instance in the
        # bit-sliced class launches: only that configuration reports them
        profiled = (args.batch_count == 256 and (n_lo, n_hi) == (1e3, 1e5) and
                    len(batches) == 2 and class_bits and class_insts == len(items))
        meas = MEASURED_TRAFFIC.get(("batched_sweeps", "batch256_mix")) if profiled else None
        traffic = meas["bytes"] if meas and meas["source"] == kernel_source_hash() else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                    "traffic": traffic,
                    "traffic_profile": meas["profile"] if traffic else None,
                    "kernel": ("k_batch_sweep + " +
                               ("k_bcl_gs_sweep" if class_bits else "k_bcl_sweep"))
                              if class_insts else "k_batch_sweep",
                    "bytes_per_launch": round(total_bytes / launches, 1),
                    "avg_launch_us": round(sweep_ms / launches * 1e3, 3), "launches": launches,
                    "timing": "every sweep launch of one more batched run (the first timed "
                              "step's seeds, the batches one after another) after the timed "
                              "region, HIP events recorded by the dispatch; summed over the "
                              "batches per generation step"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_mix(items, seeds0, args.cpu_instances, args.cpu_gens)
        log(f"cpu baseline: {cpu}")
    small = None if args.no_small_mix else small_mix_time_to_optimum(torch, gom, 256, 300)
    if small:
        log(f"small mix: {small}")
    line = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"batch{len(items)}_tori_and_regular_{n_label}",
                   "instances": len(items), "vertices": int(sum(x.n for x in insts)),
                   "pop_range": [16, 64], "max_generations": max_gens,
                   "fos": "univariate and neighbourhood alternating in pairs",
                   "mode": "batched", "batches": len(batches),
                   "batch_streams": "one batch a stream, each run from its own host thread",
                   "narrow_blocks_max_n": narrow, "resident_launches_per_step": sweep_launches,
                   "class_launch_min_n": class_min, "class_launch_instances": class_insts,
                   "class_launches_per_step": class_launches,
                   "class_positions_per_wave": None if class_bits else class_ppw,
                   "class_launch_form": ("bitsliced" if class_bits else "lane_per_solution")
                                        if class_insts else None,
                   "launch_shapes": "autotuned" if tuned else "fixed",
                   "generation_steps": ("hip_graph_chunks_of_4" if args.batch_graph == "on"
                                        else "direct_launches"),
                   "step": "fresh populations (new seeds) and a batched run of the whole mix "
                           "to every target or the generation limit"},
        "evaluated_per_s": evaluated / total,
        "plain": None if not plain else {
            "value": plain_value, "ms": t_plain * 1e3, "seeds": "the first timed step's",
            "schedule": "auto per instance, one instance at a time"},
        "batched_over_plain": value / plain_value if plain else None,
        "identical_results": same,
        "time_to_optimum_ms": {
            "instances_reached": len(tori),
            "batched_p50": q([tt0[b] for b in tori], 50),
            "batched_p99": q([tt0[b] for b in tori], 99),
            "plain_loop_p50": q([loop_t[b] for b in tori], 50) if plain else None,
            "plain_loop_p99": q([loop_t[b] for b in tori], 99) if plain else None,
            "plain_alone_p50": q([plain_t[b] * 1e3 for b in tori], 50) if plain else None,
            "plain_alone_p99": q([plain_t[b] * 1e3 for b in tori], 99) if plain else None,
            "note": None if tori else
            f"no torus of this mix reaches its total weight within {max_gens} generations "
            "in either mode (the pinned method without forced improvement stalls below the "
            "optimum on tori of 16x16 and larger); see time_to_optimum_small_mix"},
        "time_to_optimum_small_mix": small,
        "set_up_s": t_setup,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def run_serve_mode(args, torch, gom):
    """Serving loop on a Poisson stream of jobs: every job alone first (its service time, and
    the result it must reproduce), then the stream at an arrival rate of 0.7 x the plain
    capacity through the serving loop.  Time to solution is from arrival to completion; the
    plain figure is a first-come-first-served queue of the same arrivals with the measured
    solo service times."""
    sizes = tuple(args.serve_sizes.split(","))
    jobs = workloads.serve_stream(count=args.serve_jobs, seed=5, max_gens=args.serve_max_gens,
                                  sizes=sizes)
    t0 = time.perf_counter()
    insts = [gom.Instance(j.graph.n, j.graph.u, j.graph.v, j.graph.w, j.fos) for j in jobs]
    log(f"serve set-up: {len(jobs)} jobs, {sum(x.n for x in insts)} vertices, "
        f"{time.perf_counter() - t0:.1f} s")
    # warm-up: one small job alone and through a server
    w = workloads.torus(16, 1, 9, seed=1)
    wi = gom.Instance(w.n, w.u, w.v, w.w, 1)
    gom.gom_run_to_target(wi.state(pop=16, seed=1), w.total_weight, 4)
    ws = gom.GomServer(64 << 20, max_jobs=4, streams=args.serve_streams)
    ws.submit(wi, 16, 1, w.total_weight, 4)
    while ws.step() != (0, 0):
        pass
    ws.close()
    # plain: each job alone, one after another; a job's service time includes the creation of
    # its state (records, uploads, initial population), which the server does at admission
    solo, service = [], []
    for x, j in zip(insts, jobs):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        st = x.state(pop=j.pop, seed=j.seed)
        r = gom.gom_run_to_target(st, j.target, j.max_gens)
        service.append(time.perf_counter() - s0)
        solo.append((r, gom.gom_state_hash(st)))
        del st
    service = np.array(service)
    capacity = len(jobs) / service.sum()
    rate = args.serve_load * capacity
    arrivals = workloads.poisson_arrivals(len(jobs), rate, seed=5)
    finish, plain_tts = 0.0, []
    for a, sv in zip(arrivals, service):
        finish = max(a, finish) + sv
        plain_tts.append(finish - a)
    log(f"plain: capacity {capacity:.2f} jobs/s, arrival rate {rate:.2f} jobs/s")
    # served: the same arrivals through the serving loop
    arena_bytes = int(args.serve_arena_gb * (1 << 30))
    srv = gom.GomServer(arena_bytes, max_jobs=args.serve_max_active, streams=args.serve_streams)
    srv.set_large(args.serve_large_min)
    start = time.perf_counter()
    nxt, ids, res = 0, {}, {}
    while len(res) < len(jobs):
        now = time.perf_counter() - start
        while nxt < len(jobs) and arrivals[nxt] <= now:
            j = jobs[nxt]
            ids[srv.submit(insts[nxt], j.pop, j.seed, j.target, j.max_gens)] = nxt
            nxt += 1
        a, q = srv.step()
        for r in srv.results():
            res[ids[r["job"]]] = (r, time.perf_counter() - start)
        if a == 0 and q == 0 and nxt < len(jobs):
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - start)))
    makespan = time.perf_counter() - start
    served_tts = [res[k][1] - arrivals[k] for k in range(len(jobs))]

    def same_as_solo(res):
        return all((res[k][0]["generations"], res[k][0]["best"], res[k][0]["evaluated"],
                    res[k][0]["accepted"], res[k][0]["hash"]) ==
                   (solo[k][0].generations, solo[k][0].best, solo[k][0].evaluated,
                    solo[k][0].accepted, solo[k][1]) for k in range(len(jobs)))

    same = same_as_solo(res)
    attempted = sum(r.attempted for r, _ in solo)
    log(f"served: makespan {makespan:.2f} s, identical results: {same}")
    # saturated: every job submitted at once (capacity of the serving loop)
    ids, res2 = {}, {}
    start = time.perf_counter()
    for k, j in enumerate(jobs):
        ids[srv.submit(insts[k], j.pop, j.seed, j.target, j.max_gens)] = k
    while len(res2) < len(jobs):
        srv.step()
        for r in srv.results():
            res2[ids[r["job"]]] = (r, time.perf_counter() - start)
    saturated = time.perf_counter() - start
    same2 = same_as_solo(res2)
    log(f"saturated: all {len(jobs)} jobs in {saturated:.2f} s (alone one after another: "
        f"{service.sum():.2f} s), identical results: {same2}")
    pct = lambda x, q: float(np.percentile(np.array(x) * 1e3, q))
    line = {
        "metric": METRIC, "value": attempted / makespan, "unit": "evals/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": makespan * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"serve{len(jobs)}_tori_and_regular_{'_'.join(sizes)}",
                   "jobs": len(jobs), "max_generations": args.serve_max_gens,
                   "arrival_rate_jobs_per_s": rate, "load": args.serve_load,
                   "arena_bytes": arena_bytes, "streams": args.serve_streams,
                   "max_active_jobs": args.serve_max_active,
                   "large_min_vertices": args.serve_large_min,
                   "mode": "served"},
        "time_to_solution_ms": {"served_p50": pct(served_tts, 50),
                                "served_p99": pct(served_tts, 99),
                                "plain_fifo_p50": pct(plain_tts, 50),
                                "plain_fifo_p99": pct(plain_tts, 99)},
        "plain": {"capacity_jobs_per_s": capacity, "service_ms_total": service.sum() * 1e3,
                  "value": attempted / service.sum()},
        "saturated": {"served_ms": saturated * 1e3, "value": attempted / saturated,
                      "served_over_plain": service.sum() / saturated},
        "identical_results": same and same2,
    }
    print(json.dumps(line), flush=True)


def run_ims_mode(args, torch, gom):
    """The interleaved multi-start scheme on the chosen workload: levels of 16, 32 and 64
    solutions, c_IMS = 4, until some level's elitist reaches the optimum (tori) or the
    generation budget (the workload's generation limit times the number of levels) is spent;
    one run per seed.  Reports time to optimum and evaluations per second."""
    wl = workloads.WORKLOADS[args.workload]
    g = wl.graph()
    target = g.total_weight if wl.to_total_weight else (1 << 62)
    inst = gom.Instance(g.n, g.u, g.v, g.w, wl.fos,
                        lt_bound=wl.lt_bound if wl.fos == 2 else None)
    levels, n_base, c_ims = 3, 16, 4
    budget = (args.max_gens or wl.max_gens) * levels
    gom.gom_ims_run(inst, n_base, c_ims, levels, 999, target, 8, forced_improvement=args.fi)
    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        res, _ = gom.gom_ims_run(inst, n_base, c_ims, levels, k + 1, target, budget,
                                 forced_improvement=args.fi)
        runs.append((res, time.perf_counter() - s0))
        log(f"ims seed {k + 1}: {res}")
    total = time.perf_counter() - t0
    attempted = 0
    sets = inst.fos.info()["n_sets"]
    for res, _ in runs:
        attempted += sum(gen * (n_base << lvl) * sets for lvl, gen in enumerate(res["generations"]))
    tto = [dt * 1e3 for res, dt in runs if res["reached"]]
    line = {
        "metric": METRIC, "value": attempted / total, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": total * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.workload, args.workload),
                   "mode": "ims", "n_base": n_base, "c_ims": c_ims, "levels": levels,
                   "generation_budget": budget, "forced_improvement": bool(args.fi),
                   "target": target if wl.to_total_weight else None},
        "time_to_optimum_ms_median": float(np.median(tto)) if tto else None,
        "reached": len(tto), "best": [res["best"] for res, _ in runs],
        "generations_total": sum(res["total_generations"] for res, _ in runs),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-gens", type=int, default=None,
                    help="generations of the oracle sample for the CPU baseline (default: 10 "
                         "per instance for the batched mix, 40 for a single workload)")
    ap.add_argument("--cpu-instances", type=int, default=8,
                    help="instances of the batched mix in the oracle sample")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched mode: skip the plain loop (no identity check; for profiling)")
    ap.add_argument("--no-small-mix", action="store_true",
                    help="batched mode: skip the time-to-optimum comparison on the mix of "
                         "small instances")
    ap.add_argument("--schedule", choices=("tuned", "auto", "class", "resident", "bitsliced"),
                    default="tuned",
                    help="launch schedule of the generations (results are identical); 'tuned' "
                         "times each allowed schedule on a few generations before the warmup "
                         "and keeps the fastest")
    ap.add_argument("--workload", default=None, choices=sorted(workloads.WORKLOADS),
                    help="plain GOM on this single workload instead of the batched mix")
    ap.add_argument("--batch", action="store_true",
                    help="batched vs plain on the mix (the default when no workload is named)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-n-range", type=float, nargs=2, metavar=("LO", "HI"),
                    default=(1e3, 1e5),
                    help="vertex-count range of the batched mix (log-uniform; default 1e3 1e5)")
    ap.add_argument("--local-search", action="store_true",
                    help="plain mode, univariate FOS: the colouring-parallel local search after "
                         "every generation (the hybrid); reports time to optimum")
    ap.add_argument("--ils", type=int, nargs=2, metavar=("ROUNDS", "FLIPS"), default=None,
                    help="with --local-search: after each search, the iterated local search "
                         "(ROUNDS rounds of FLIPS drawn flips per solution)")
    ap.add_argument("--no-batched", action="store_true",
                    help="plain mode: skip the comparison with the same seeds run as one batch")
    ap.add_argument("--batch-narrow", type=int, default=None,
                    help="batched mode: instances with at most this many vertices sweep with "
                         "256-thread blocks, larger ones 1024 (-1: all 1024; default: "
                         "autotuned)")
    ap.add_argument("--batch-class-min", type=int, default=None,
                    help="batched mode: neighbourhood instances with at least this many "
                         "vertices take the batched class launches (-1: none; default: "
                         "autotuned)")
    ap.add_argument("--batch-streams", type=int, default=2,
                    help="batched mode: split the mix into this many batches, one a stream, "
                         "run at the same time from their own host threads")
    ap.add_argument("--batch-class-form", choices=("bitsliced", "lanes"), default=None,
                    help="batched mode: form of the class launches (bit-sliced where "
                         "available, or lane = solution)")
    ap.add_argument("--batch-class-ppw", type=int, default=None,
                    help="batched mode: class positions per wave of the class launches (1..8)")
    ap.add_argument("--batch-graph", choices=("on", "off"), default="on",
                    help="batched steps as captured HIP graph chunks (default) or direct launches")
    ap.add_argument("--ims", action="store_true",
                    help="interleaved multi-start scheme (levels of 16, 32, 64) on the chosen "
                         "workload")
    ap.add_argument("--serve", action="store_true",
                    help="serving loop on a Poisson stream of jobs instead of the default "
                         "single-instance workload")
    ap.add_argument("--serve-jobs", type=int, default=60)
    ap.add_argument("--serve-max-gens", type=int, default=200)
    ap.add_argument("--serve-sizes", default="small,medium",
                    help="size classes of the job stream: small (10^4 vertices), medium "
                         "(10^5), large (10^6; host set-up of up to 30 s per job)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="arrival rate as a fraction of the measured plain capacity")
    ap.add_argument("--serve-arena-gb", type=float, default=32.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-max-active", type=int, default=256,
                    help="serving: most jobs admitted (running) at once; the others queue")
    ap.add_argument("--serve-large-min", type=int, default=-1,
                    help="jobs with at least this many vertices run one at a time on the "
                         "first stream, small jobs on the others (default -1: every job on "
                         "the least loaded stream)")
    ap.add_argument("--max-gens", type=int, default=None,
                    help="override the workload's generation limit")
    ap.add_argument("--metrics-jsonl", default=None,
                    help="write per-generation metrics of one more run to this file (JSON "
                         "lines; batched mode: totals over the instances)")
    ap.add_argument("--staged", action="store_true",
                    help="plain mode: class sweeps of small general sets take the staged "
                         "evaluation (two rounds of loads per set)")
    ap.add_argument("--fused", action="store_true",
                    help="bit-sliced schedule: the fused generation sweep (one cooperative "
                         "launch per generation) instead of one launch per class")
    ap.add_argument("--bitsliced-min-sets", type=int, default=None,
                    help="plain mode, general FOS: smallest class the bit-sliced schedule "
                         "sweeps with the general bit-sliced sweep (library default 8192)")
    ap.add_argument("--block", type=int, default=0,
                    help="class-launch block size (with --schedule class; 0 = default)")
    ap.add_argument("--fi", action="store_true",
                    help="forced improvement after each generation's classes")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after the timed steps, run a device copy of this many MiB (a known "
                         "byte count for scaling profiler traffic counters)")
    ap.add_argument("--event-period", type=int, default=0,
                    help="inside the timed region, time every k-th sweep launch with HIP "
                         "events recorded by its own dispatch (0: none; reported beside the "
                         "timing pass, which times every launch of one extra run)")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="do not record HIP events around sweep launches (roofline omitted)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent instances would shard across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)
    if args.ils and not args.local_search:
        ap.error("--ils needs --local-search")

    import torch
    from paper_2203_08680_amd import build as gbuild
    from paper_2203_08680_amd import gom
    if not os.path.exists(gom.LIB_PATH):
        gbuild.build()
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.serve:
        run_serve_mode(args, torch, gom)
        return
    if args.ims:
        args.workload = args.workload or DEFAULT_WORKLOAD
        run_ims_mode(args, torch, gom)
        return
    if args.batch or (args.workload is None and not args.local_search):
        args.cpu_gens = args.cpu_gens or 10
        run_batch_mode(args, torch, gom)
        return
    args.cpu_gens = args.cpu_gens or 40
    args.workload = args.workload or DEFAULT_WORKLOAD

    wl = workloads.WORKLOADS[args.workload]
    max_gens = args.max_gens or wl.max_gens
    g = wl.graph()
    target = g.total_weight if wl.to_total_weight else (1 << 62)
    inst = gom.Instance(g.n, g.u, g.v, g.w, wl.fos,
                        lt_bound=wl.lt_bound if wl.fos == 2 else None)
    st = inst.state(pop=wl.pop, seed=1000)
    if args.fi:
        gom.gom_state_set_fi(st, True)
    if args.bitsliced_min_sets is not None:
        gom.gom_state_set_bitsliced_min_sets(st, args.bitsliced_min_sets)
    if args.schedule == "tuned":
        gom.gom_state_autotune(st, 10)
    else:
        gom.gom_state_set_schedule(st, {"auto": gom.GOM_SCHED_AUTO,
                                        "class": gom.GOM_SCHED_CLASS_LAUNCH,
                                        "resident": gom.GOM_SCHED_RESIDENT,
                                        "bitsliced": gom.GOM_SCHED_BITSLICED}[args.schedule])
    if args.block:
        gom.gom_state_set_block(st, args.block)
    if args.fused and gom.gom_state_get_fused(st)[1]:
        gom.gom_state_set_fused(st, True)
    if args.staged:
        gom.gom_state_set_staged(st, True)
    sched = gom.gom_state_get_schedule(st)
    sched_name = {gom.GOM_SCHED_RESIDENT: "resident", gom.GOM_SCHED_BITSLICED: "bitsliced"}.get(
        sched, "class_launch")
    fused = sched_name == "bitsliced" and gom.gom_state_get_fused(st)[0]
    if fused:
        sched_name = "bitsliced_fused"
    info = st.info()
    _, class_ptr, class_elems = inst.classes()
    set_ptr, set_vars = inst.fos.sets()
    cbytes = class_sweep_bytes(inst.graph.csr(), set_ptr, set_vars, class_ptr, class_elems,
                               wl.pop)

    ls_passes = [0]

    def one_run(seed):
        gom.gom_state_reseed(st, seed)
        if not args.local_search:
            return gom.gom_run_to_target(st, target, max_gens)
        # hybrid: a generation, then the colouring-parallel local search, until the target
        # or the generation limit (the search is synchronous, so the check costs nothing more)
        gens = 0
        r = gom.gom_run_to_target(st, target, 0)
        while not r.reached and gens < max_gens:
            gom.gom_generation(st)
            ls_passes[0] += gom.gom_local_search(st)
            if args.ils:
                ls_passes[0] += gom.gom_iterated_local_search(st, 0, args.ils[0], args.ils[1])
            gens += 1
            r = gom.gom_run_to_target(st, target, 0)
        return gom.RunResult(gens, r.reached, r.best, r.attempted, r.evaluated, r.accepted)

    for w in range(args.warmup):
        r = one_run(1000 + w)
        log(f"warmup {w}: generations {r.generations} reached {r.reached}")
    torch.cuda.synchronize()

    if not args.no_kernel_events and args.event_period > 0:
        gom.gom_timing_enable(st, args.event_period)
        gom.gom_timing_read(st)
    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        r = one_run(k + 1)
        runs.append((r, time.perf_counter() - s0))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    if not args.no_kernel_events:
        sampled_ms, sampled_launches = gom.gom_timing_read(st)
        # Kernel-timing pass right after the timed region: one more run of the same workload
        # (seed steps + 1) with every sweep launch timed.  Timing every launch costs several
        # microseconds of wall time per launch, so it stays out of the timed region.  Launches
        # sampled inside the timed region read about 1 us longer than the profiler's average
        # on MI355X (measured; the cause is not established), so they are only reported.
        gom.gom_timing_enable(st, 1)
        one_run(args.steps + 1)
        sweep_ms, launches = gom.gom_timing_read(st)
        gom.gom_timing_enable(st, 0)
    copy_calibration(torch, args.copy_calib_mb)
    for k, (r, dt) in enumerate(runs):
        log(f"step {k} seed {k + 1}: generations {r.generations} reached {r.reached} "
            f"best {r.best}/{target} attempted {r.attempted} evaluated {r.evaluated} "
            f"accepted {r.accepted} time {dt * 1e3:.2f} ms")

    if args.metrics_jsonl:
        write_metrics_log(args.metrics_jsonl, gom, torch, st, target, max_gens)
    attempted = sum(r.attempted for r, _ in runs)
    gens = sum(r.generations for r, _ in runs)
    tto = [dt * 1e3 for r, dt in runs if r.reached]
    value = attempted / total
    batched = None if args.fi or args.no_batched or args.local_search else batched_compare(
        args, torch, gom, inst, wl.pop, target, max_gens, [r for r, _ in runs], value)
    roofline = None
    if not args.no_kernel_events and launches:
        # class launch: every class is swept once per generation, so the mean over launches
        # of the algorithmic bytes is the mean over classes; resident: one launch sweeps
        # every class of a generation
        # (the fused bit-sliced sweep, like the resident one, covers every class per launch)
        whole = sched_name in ("resident", "bitsliced_fused")
        avg_bytes = float(cbytes.sum() if whole else cbytes.mean())
        avg_s = sweep_ms / 1e3 / launches
        achieved = avg_bytes / avg_s / 1e9
        kname = {"resident": "k_resident_sweep",
                 "bitsliced": "k_uni_swar_sweep" if wl.fos == 0 else
                              "k_gen_swar_sweep + k_class_sweep",
                 "bitsliced_fused": "k_uni_swar_fused"}.get(sched_name, "k_class_sweep")
        meas = MEASURED_TRAFFIC.get((kname, args.workload))
        traffic = meas["bytes"] if meas and meas["source"] == kernel_source_hash() else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                    "traffic": traffic,
                    "traffic_profile": meas["profile"] if traffic else None,
                    "kernel": kname,
                    "bytes_per_launch": round(avg_bytes, 1),
                    "avg_launch_us": round(avg_s * 1e6, 3), "launches": launches,
                    "timing": "every sweep launch of one run after the timed region, HIP "
                              "events recorded by the dispatch",
                    "avg_launch_us_sampled_in_timed_region":
                        round(sampled_ms / 1e3 / sampled_launches * 1e6, 3)
                        if sampled_launches else None}
    cpu = None
    if not args.no_cpu_baseline:
        if wl.fos == 2:
            # the oracle's linkage tree is dense UPGMA (n^2 similarities, every pair rescanned
            # per merge): out of reach at 10^4 vertices
            cpu = None
            log("cpu baseline: not run (the oracle's dense linkage-tree build does not scale "
                "to this size)")
        else:
            cpu = cpu_baseline(g, wl.fos, wl.pop, min(args.cpu_gens, max_gens), target,
                               fi=args.fi)
            log(f"cpu baseline: {cpu}")

    line = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES.get(args.workload, args.workload), "n": g.n,
                   "m": g.m,
                   "fos": {0: "univariate", 1: "neighbourhood"}.get(
                       wl.fos, f"linkage_tree_bound{wl.lt_bound}"),
                   "pop": wl.pop, "max_generations": max_gens,
                   "target": target if wl.to_total_weight else None,
                   "classes": info["n_classes"], "seeds": list(range(1, args.steps + 1)),
                   "mode": "plain", "schedule": sched_name,
                   "class_sweep_block": gom.gom_state_get_block(st),
                   "staged_evaluation": bool(args.staged),
                   "forced_improvement": bool(args.fi),
                   "local_search_after_each_generation": bool(args.local_search),
                   "iterated_local_search": ({"rounds": args.ils[0], "flips": args.ils[1]}
                                             if args.ils else None)},
        "time_to_optimum_ms_median": float(np.median(tto)) if tto else None,
        "reached": len(tto), "generations_total": gens,
        "us_per_generation": total * 1e6 / max(gens, 1),
        "us_per_class": total * 1e6 / max(gens, 1) / max(info["n_classes"], 1),
        "roofline": roofline, "cpu_baseline": cpu,
        "batched": batched,
        "local_search_passes": ls_passes[0] if args.local_search else None,
    }
    print(json.dumps(line), flush=True)


def batched_compare(args, torch, gom, inst, pop, target, max_gens, plain, plain_value):
    """The plain runs' seeds again, as one lockstep batch of instances (the batched engine):
    evaluations per second, time to optimum per seed, and whether every result is identical
    to its plain run.  None when the instance does not fit the batched (resident) schedule."""
    seeds = list(range(1, len(plain) + 1))
    try:
        wb = gom.gom_batch_init([inst], [pop], [999], [target])
        gom.gom_batch_run(wb, 2)
        del wb
        b = gom.gom_batch_init([inst] * len(seeds), [pop] * len(seeds), seeds,
                               [target] * len(seeds))
    except gom.GomError as e:
        log(f"batched comparison: not run ({e})")
        return None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, tt = gom.gom_batch_run(b, max_gens)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    same = all((a.generations, a.reached, a.best, a.attempted, a.evaluated, a.accepted) ==
               (p.generations, p.reached, p.best, p.attempted, p.evaluated, p.accepted)
               for a, p in zip(res, plain))
    value = sum(r.attempted for r in res) / dt
    reached = [float(t) for r, t in zip(res, tt) if r.reached]
    log(f"batched: {len(seeds)} seeds in one batch, {dt * 1e3:.1f} ms, identical: {same}")
    return {"value": value, "ms": dt * 1e3, "instances": len(seeds),
            "schedule": "batched_resident", "identical_results": same,
            "batched_over_plain": value / plain_value,
            "time_to_optimum_ms_median": float(np.median(reached)) if reached else None,
            "reached": len(reached)}


if __name__ == "__main__":
    main()
