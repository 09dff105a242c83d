"""GPU parity over whole trajectories: the configured workloads run for their full generation
budgets (or, where the oracle needs minutes per generation, a stated prefix), with the state
hash (every gene, fitness, elitist and counter) compared to the oracle's after EVERY
generation and the full state compared at checkpoints.

One oracle run per workload serves several GPU states in lockstep (one per launch schedule),
since every schedule must follow the same trajectory.  The oracle spreads each colour class's
solutions over host threads; its results do not depend on their number.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from paper_2203_08680_amd import gom

pytestmark = pytest.mark.gpu

KEYS = ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted", "evaluated",
        "accepted")
WORKERS = max(1, min(16, os.cpu_count() or 1))


def assert_same(a, b, where):
    for key in KEYS:
        x, y = np.asarray(a[key]), np.asarray(b[key])
        if not np.array_equal(x, y):
            if key == "genes":
                bad = np.argwhere(x != y)
                raise AssertionError(f"{where}: genes differ at {len(bad)} places, first "
                                     f"(solution, vertex) {bad[:5].tolist()}")
            raise AssertionError(f"{where}: {key} differs: gpu {x} oracle {y}")


def _states(inst, pop, seed, scheds):
    """One state per (schedule, block size[, staged evaluation]); under the bit-sliced
    schedule every class that qualifies takes the bit-sliced sweep, whatever its size."""
    out = []
    for sched, block, *rest in scheds:
        st = inst.state(pop=pop, seed=seed)
        if sched == gom.GOM_SCHED_BITSLICED:
            gom.gom_state_set_bitsliced_min_sets(st, 0)
        gom.gom_state_set_schedule(st, sched)
        if block:
            gom.gom_state_set_block(st, block)
        if rest:
            gom.gom_state_set_staged(st, rest[0])
        out.append((f"sched {sched} block {block} {rest}", st))
    return out


def _trajectory(label, g, kind, pop, seed, gens, scheds, full_every, target=None):
    """Run the oracle and one GPU state per schedule for `gens` generations (or until the
    target), comparing hashes after every generation and full states every `full_every`."""
    print(f"case trajectory {label}: {gens} generations, schedules {scheds}", flush=True)
    ptr, vars_ = oracle.fos(g, kind)
    inst = gom.Instance(g.n, g.u, g.v, g.w, kind)
    states = _states(inst, pop, seed, scheds)
    ref = oracle.Run(g, ptr, vars_, pop=pop, seed=seed, workers=WORKERS)
    h = ref.hash()
    for name, st in states:
        assert gom.gom_state_hash(st) == h, f"{label} {name}: initial state"
    for gen in range(gens):
        ref.generation()
        h = ref.hash()
        full = (gen + 1) % full_every == 0 or gen == gens - 1
        b = ref.state(genes=full) if full else None
        for name, st in states:
            gom.gom_generation(st)
            got = gom.gom_state_hash(st)
            if got != h or full:
                a = gom.gom_state_read(st, genes=full)
                if b is None:
                    b = ref.state(genes=False)
                    a["genes"] = b["genes"] = None
                assert_same(a, b, f"{label} {name} generation {gen}")
                assert got == h, f"{label} {name} generation {gen}: hash differs"
        if target is not None and ref.state(genes=False)["elite_fitness"] >= target:
            print(f"  {label}: target reached after generation {gen}", flush=True)
            break
    return ref


def test_c2_full_trajectory():
    """100x100 torus, neighbourhood FOS, population 64, seed 1: the whole 500-generation run
    of the plain single-instance workload, under the class-launch schedule with 64-thread
    blocks, 256-thread blocks, 64-thread blocks with the staged evaluation, the resident
    schedule and the bit-sliced schedule."""
    g = workloads.torus(100, 1, 100, seed=2)
    scheds = [(gom.GOM_SCHED_CLASS_LAUNCH, 64), (gom.GOM_SCHED_CLASS_LAUNCH, 256),
              (gom.GOM_SCHED_CLASS_LAUNCH, 64, True), (gom.GOM_SCHED_RESIDENT, 0),
              (gom.GOM_SCHED_BITSLICED, 0)]
    _trajectory("torus100 nbhd p64 seed 1", g, 1, 64, 1, 500, scheds, 50,
                target=g.total_weight)


def test_c2_batched_trajectory_checkpoints():
    """The same run and two more seeds as one lockstep batch: every instance's hash equals
    the oracle's at generations 50, 100, ..., 500."""
    print("case batched torus100 nbhd p64 seeds 1-3", flush=True)
    g = workloads.torus(100, 1, 100, seed=2)
    ptr, vars_ = oracle.fos(g, 1)
    inst = gom.Instance(g.n, g.u, g.v, g.w, 1)
    seeds = [1, 2, 3]
    b = gom.gom_batch_init([inst] * 3, [64] * 3, seeds, [g.total_weight] * 3)
    refs = [oracle.Run(g, ptr, vars_, pop=64, seed=s, workers=WORKERS) for s in seeds]
    for stop in range(50, 501, 50):
        gom.gom_batch_run(b, stop)
        for k, ref in enumerate(refs):
            ref.run(g.total_weight, stop)  # (the generation limit is absolute)
            assert gom.gom_state_hash(b.state(k)) == ref.hash(), (seeds[k], stop)
    for k, ref in enumerate(refs):
        assert_same(gom.gom_state_read(b.state(k)), ref.state(), f"batched seed {seeds[k]}")


def test_c3_d3_univariate_200_generations():
    """Random 3-regular graph, n = 10^5, weights +-U{1..50}, univariate FOS, population 32:
    all 200 generations under class launch, the bit-sliced sweep and the resident schedule."""
    g = workloads.configuration_model(100_000, 3, seed=3, weights="signed50")
    scheds = [(gom.GOM_SCHED_CLASS_LAUNCH, 0), (gom.GOM_SCHED_BITSLICED, 0),
              (gom.GOM_SCHED_RESIDENT, 0)]
    _trajectory("cm100k d3 uni p32", g, 0, 32, 1, 200, scheds, 50)


@pytest.mark.parametrize("d,gens", [(3, 20), (6, 20), (12, 5)])
def test_c3_neighbourhood_prefix(d, gens):
    """Random d-regular graphs, n = 10^5, neighbourhood FOS, population 32: the first 20
    generations (degree 3 and 6) or 5 (degree 12, about 270 colour classes and 4 s of oracle
    time per generation) under class launch and the resident schedule."""
    g = workloads.configuration_model(100_000, d, seed=3, weights="signed50")
    scheds = [(gom.GOM_SCHED_CLASS_LAUNCH, 0), (gom.GOM_SCHED_RESIDENT, 0)]
    if d <= 8:  # (degree 12: 13 members, beyond the bit-sliced general sweep)
        scheds.append((gom.GOM_SCHED_BITSLICED, 0))
    _trajectory(f"cm100k d{d} nbhd p32", g, 1, 32, 1, gens, scheds, 10)


def test_torus1000_univariate_5_generations():
    """The 10^6-vertex torus, univariate FOS, population 64: five generations under the
    bit-sliced sweep and class launch, hashes every generation, full states at the end."""
    g = workloads.torus(1000, 1, 100, seed=7)
    scheds = [(gom.GOM_SCHED_BITSLICED, 0), (gom.GOM_SCHED_CLASS_LAUNCH, 0)]
    _trajectory("torus1000 uni p64", g, 0, 64, 1, 5, scheds, 5)


def test_torus1000_neighbourhood_2_generations():
    """The 10^6-vertex torus, neighbourhood FOS, population 64, class launch (the batched-
    entries form with shared draws, and the staged evaluation) and the bit-sliced schedule:
    two generations."""
    g = workloads.torus(1000, 1, 100, seed=7)
    _trajectory("torus1000 nbhd p64", g, 1, 64, 1, 2,
                [(gom.GOM_SCHED_CLASS_LAUNCH, 0), (gom.GOM_SCHED_CLASS_LAUNCH, 0, True),
                 (gom.GOM_SCHED_BITSLICED, 0)], 2)


def test_headline_mix_sampled():
    """The 256-instance mix (tori and 4/8-regular graphs of 10^3-10^5 vertices, univariate and
    neighbourhood FOS, populations 16-64) in the benchmark's launch configuration: two
    batches (instances dealt round-robin by class count), each autotuned, reseeded and run
    on its own stream from its own host thread.  After two generations the state hash of
    each sampled instance (the largest of each FOS kind, every 11th of the rest) equals the
    oracle's, and every instance ran both generations."""
    import threading
    import torch
    print("case headline mix: set-up", flush=True)
    items = workloads.batch_mix()
    insts = [gom.Instance(it.graph.n, it.graph.u, it.graph.v, it.graph.w, it.fos)
             for it in items]
    targets = [it.graph.total_weight if it.to_total_weight else (1 << 62) for it in items]
    kc = [len(x.classes()[1]) - 1 for x in insts]
    order = sorted(range(len(items)), key=lambda i: (-kc[i], i))
    groups = [sorted(order[j::2]) for j in range(2)]
    batches = [gom.gom_batch_init([insts[i] for i in g], [items[i].pop for i in g],
                                  [items[i].seed for i in g], [targets[i] for i in g])
               for g in groups]
    streams = [torch.cuda.Stream() for _ in groups]
    for batch, g, s in zip(batches, groups, streams):
        gom.gom_batch_autotune(batch, 2, stream=s)
        gom.gom_batch_reseed(batch, [items[i].seed for i in g], stream=s)
    print(f"case headline mix: class forms {[gom.gom_batch_get_class_bitsliced(b) for b in batches]}",
          flush=True)
    gens = 2
    out = [None, None]

    def go(j):
        out[j] = gom.gom_batch_run(batches[j], gens, stream=streams[j])

    threads = [threading.Thread(target=go, args=(j,)) for j in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    where = {}
    for j, g in enumerate(groups):
        for b, i in enumerate(g):
            where[i] = (j, b)
            assert out[j][0][b].generations == gens, f"instance {i}"
    sizes = [it.graph.n for it in items]
    sample = set(range(0, len(items), 11))
    for kind in (0, 1):
        sample.add(max((i for i in range(len(items)) if items[i].fos == kind),
                       key=lambda i: sizes[i]))
    for i in sorted(sample):
        it = items[i]
        j, b = where[i]
        print(f"case headline mix: instance {i} (n {it.graph.n}, fos {it.fos}, pop {it.pop})",
              flush=True)
        ptr, vars_ = oracle.fos(it.graph, it.fos)
        ref = oracle.Run(it.graph, ptr, vars_, pop=it.pop, seed=it.seed, workers=WORKERS)
        ref.run(targets[i], gens)
        st = batches[j].state(b)
        if gom.gom_state_hash(st) != ref.hash():
            assert_same(gom.gom_state_read(st), ref.state(), f"mix instance {i}")
            raise AssertionError(f"mix instance {i}: hash differs")
        ref.close()
