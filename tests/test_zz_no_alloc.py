"""gom_state_init_static (state in the library's static device arena, nothing allocated)
against gom_state_init (state in a caller arena): identical states every generation, on two
instances in a row, the second smaller than the first, and the second static state created
only after the first is freed."""
import numpy as np
import pytest

import workloads
from paper_2203_08680_amd import gom

pytestmark = pytest.mark.gpu

KEYS = ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted", "evaluated",
        "accepted")


def _same(a, b, where):
    for key in KEYS:
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), f"{where}: {key}"


def _compare(inst, pop, seed, gens, label):
    st = gom.gom_state_init_static(inst.graph, inst.fos, pop, seed)
    ref = inst.state(pop=pop, seed=seed)
    _same(gom.gom_state_read(st), gom.gom_state_read(ref), f"{label} init")
    for g in range(gens):
        gom.gom_generation(st)
        gom.gom_generation(ref)
        _same(gom.gom_state_read(st), gom.gom_state_read(ref), f"{label} generation {g}")
        assert gom.gom_state_hash(st) == gom.gom_state_hash(ref)
    r1 = gom.gom_run_to_target(st, inst.total_weight, gens + 6)
    r2 = gom.gom_run_to_target(ref, inst.total_weight, gens + 6)
    assert r1 == r2
    _same(gom.gom_state_read(st), gom.gom_state_read(ref), f"{label} run to target")
    return st


def test_static_state_equals_arena_state(cuda):
    print("case static arena: torus100 nbhd p64, then torus10 nbhd p16", flush=True)
    big = workloads.torus(100, 1, 100, seed=2)
    small = workloads.torus(10, 1, 5, seed=1)
    ib = gom.Instance(big.n, big.u, big.v, big.w, 1)
    is_ = gom.Instance(small.n, small.u, small.v, small.w, 1)
    st = _compare(ib, 64, 3, 6, "torus100")
    # the device's static arena is taken until the state is freed
    with pytest.raises(gom.GomError) as e:
        gom.gom_state_init_static(is_.graph, is_.fos, 16, 5)
    assert e.value.code == gom.GOM_E_STATE
    st.close()
    st2 = _compare(is_, 16, 5, 8, "torus10")
    st2.close()


def test_static_state_rejects_oversized(cuda):
    print("case static arena: oversized instance", flush=True)
    g = workloads.torus(1000, 1, 100, seed=7)
    inst = gom.Instance(g.n, g.u, g.v, g.w, 0)
    assert gom.gom_state_bytes(inst.graph, inst.fos, 64) > gom.GOM_STATIC_ARENA_BYTES
    with pytest.raises(gom.GomError) as e:
        gom.gom_state_init_static(inst.graph, inst.fos, 64, 1)
    assert e.value.code == gom.GOM_E_RANGE
    # the failed call leaves the arena free
    small = workloads.torus(10, 1, 5, seed=1)
    i2 = gom.Instance(small.n, small.u, small.v, small.w, 0)
    st = gom.gom_state_init_static(i2.graph, i2.fos, 16, 1)
    st.close()
