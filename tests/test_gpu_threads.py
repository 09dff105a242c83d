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
