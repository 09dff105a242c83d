"""States driven from several host threads at once, each on its own stream.

Calls on different handles may overlap in time; the launchers that raise a kernel's dynamic
LDS limit (resident and large-set sweeps) share that per-device setting between the threads.
Each state must still follow its own oracle run bit for bit.
"""
from __future__ import annotations

import threading

import numpy as np
import pytest

import oracle
import workloads
from paper_2203_08680_amd import gom

pytestmark = pytest.mark.gpu

KEYS = ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted", "evaluated",
        "accepted")


def test_states_on_three_host_threads(cuda):
    import torch
    cases = [
        ("torus32_nbhd_resident", workloads.torus(32, 1, 100, seed=3), 1, 64, 5,
         gom.GOM_SCHED_RESIDENT),
        ("cm4000_d4_uni_resident", workloads.configuration_model(4000, 4, seed=11), 0, 32, 6,
         gom.GOM_SCHED_RESIDENT),
        ("cm2000_d4_nbhd_class", workloads.configuration_model(2000, 4, seed=12), 1, 48, 7,
         gom.GOM_SCHED_CLASS_LAUNCH),
    ]
    gens = 25
    runs = []
    for label, g, kind, pop, seed, sched in cases:
        inst = gom.Instance(g.n, g.u, g.v, g.w, kind)
        st = inst.state(pop=pop, seed=seed)
        gom.gom_state_set_schedule(st, sched)
        ptr, vars_ = oracle.fos(g, kind)
        ref = oracle.Run(g, ptr, vars_, pop=pop, seed=seed)
        runs.append((label, inst, st, ref, torch.cuda.Stream()))
    torch.cuda.synchronize()
    print("case three host threads: " + ", ".join(r[0] for r in runs), flush=True)

    results, errors = {}, []

    def drive(label, st, stream):
        try:
            results[label] = gom.gom_run_to_target(st, 1 << 62, gens, stream=stream)
            stream.synchronize()
        except Exception as e:  # reported on the main thread
            errors.append((label, e))

    threads = [threading.Thread(target=drive, args=(label, st, stream))
               for label, _, st, _, stream in runs]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a host thread did not finish"
    assert not errors, errors
    torch.cuda.synchronize()

    for label, _, st, ref, _ in runs:
        assert ref.run(1 << 62, gens) == gens
        r = results[label]
        assert r.generations == gens
        a, b = gom.gom_state_read(st), ref.state()
        for key in KEYS:
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), f"{label}: {key}"


def test_batches_on_two_host_threads(cuda):
    """Two batches (the benchmark's way of running its mix on two streams), each with graph
    chunks and the bit-sliced class launches, run at the same time from two host threads on
    two streams: every instance equals its solo run, and a second round after a reseed does
    too."""
    import torch
    rng = np.random.default_rng(70)
    gs, kinds, pops = [], [], []
    for k in range(16):
        if k % 2 == 0:
            gs.append(workloads.torus(int(rng.choice([10, 20, 30])), 1, 100, seed=700 + k))
        else:
            d = int(rng.choice([4, 8]))
            n = int(rng.integers(500, 3000))
            gs.append(workloads.configuration_model(n + (n * d) % 2, d, seed=700 + k,
                                                    weights="uniform", w_lo=1, w_hi=100))
        kinds.append(0 if k % 4 < 2 else 1)
        pops.append(int(rng.choice([16, 33, 64])))
    insts = [gom.Instance(g.n, g.u, g.v, g.w, kd) for g, kd in zip(gs, kinds)]
    targets = [g.total_weight if k % 2 == 0 else (1 << 62) for k, g in enumerate(gs)]
    groups = [list(range(0, 16, 2)), list(range(1, 16, 2))]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    batches = []
    for g in groups:
        b = gom.gom_batch_init([insts[i] for i in g], [pops[i] for i in g],
                               [50 + i for i in g], [targets[i] for i in g])
        gom.gom_batch_set_class_launch(b, 0)
        batches.append(b)
    for rnd, gens in ((0, 24), (1, 16)):
        if rnd:
            for b, g, s in zip(batches, groups, streams):
                gom.gom_batch_reseed(b, [90 + i for i in g], stream=s)
        out = [None, None]

        def go(j):
            out[j] = gom.gom_batch_run(batches[j], gens, stream=streams[j])

        th = [threading.Thread(target=go, args=(j,)) for j in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        torch.cuda.synchronize()
        for j, g in enumerate(groups):
            for pos, i in enumerate(g):
                st = insts[i].state(pop=pops[i], seed=(90 if rnd else 50) + i)
                r = gom.gom_run_to_target(st, targets[i], gens)
                got = out[j][0][pos]
                assert (got.generations, got.best, got.attempted, got.evaluated,
                        got.accepted) == (r.generations, r.best, r.attempted, r.evaluated,
                                          r.accepted), (rnd, i)
                assert gom.gom_state_hash(batches[j].state(pos)) == gom.gom_state_hash(st), \
                    (rnd, i)
