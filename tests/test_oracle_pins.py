"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each test ties one oracle function to something outside itself: a library routine (numpy's
Philox), the paper's own formula or worked example (Figures 1-3), closed forms and brute
force, hand-worked generations, an independent whole-class reference that evaluates every
trial in full (tests/class_at_once.py), or an invariant the method guarantees.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads
from class_at_once import ClassAtOnceGomea, initial_population

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------
# Philox
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((1, 2), (5, 6, 7, 8)),
                                     ((2**64 - 1, 12345), (2**64 - 2, 3, 2**63, 9))])
def test_philox4x64_matches_numpy(key, ctr):
    """The shared Philox round template, 4x64 instance, against numpy.random.Philox (which
    increments its counter before producing a block)."""
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
    want = bg.random_raw(4)
    c = list(ctr)
    c[0] = (c[0] + 1) % 2**64
    if c[0] == 0:
        c[1] = (c[1] + 1) % 2**64
    got = oracle.philox4x64(key, c)
    assert [int(x) for x in got] == [int(x) for x in want]


@pytest.mark.parametrize("key,ctr,want", [
    ((0x00000000, 0x00000000), (0x00000000, 0x00000000, 0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0xa4093822, 0x299f31d0), (0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox4x32_known_answers(key, ctr, want):
    """Philox4x32-10 against the published known-answer vectors of the Random123 distribution
    (Salmon, Moraes, Dror & Shaw, SC'11): all-zero key and counter, all-ones, and the
    pi-digit vector.  These fix the 4x32 multipliers and Weyl constants, which the 4x64
    comparison with numpy does not reach."""
    assert tuple(int(x) for x in oracle.philox4x32(key, ctr)) == want


def test_philox4x32_bits_balanced_and_counter_sensitive():
    """4x32 instance (same template): outputs change with every counter word and key word,
    and bits are balanced over many blocks."""
    base = oracle.philox4x32((1, 2), (3, 4, 5, 6))
    for pos in range(4):
        c = [3, 4, 5, 6]
        c[pos] ^= 1
        assert not np.array_equal(oracle.philox4x32((1, 2), c), base)
    assert not np.array_equal(oracle.philox4x32((1, 3), (3, 4, 5, 6)), base)
    ones = 0
    for t in range(2000):
        out = oracle.philox4x32((7, 0), (t, 0, 0, 0))
        ones += sum(bin(int(x)).count("1") for x in out)
    frac = ones / (2000 * 128)
    assert abs(frac - 0.5) < 0.005


# ------------------------------------------------------------------------------------------
# Max-Cut objective
# ------------------------------------------------------------------------------------------
def paper_objective(g, x):
    """Section 6.2 objective with x in {-1, 1}: one half of the sum over pairs i < j of
    w_ij (1 - x_i x_j) (pairs without an edge have w = 0)."""
    s = 2 * np.asarray(x, np.int64) - 1
    total = 0
    for e in range(g.m):
        i, j = sorted((int(g.u[e]), int(g.v[e])))
        total += int(g.w[e]) * (1 - s[i] * s[j])
    assert total % 2 == 0
    return total // 2


def brute_force_max(g):
    best = None
    for bits in itertools.product((0, 1), repeat=g.n):
        f = oracle.maxcut(g, np.array(bits, np.uint8))
        best = f if best is None else max(best, f)
    return best


def test_maxcut_equals_paper_formula():
    rng = np.random.default_rng(0)
    for n, d in ((30, 3), (40, 4), (25, 6)):
        g = workloads.configuration_model(n, d, seed=n, weights="signed50")
        for _ in range(5):
            x = rng.integers(0, 2, n).astype(np.uint8)
            assert oracle.maxcut(g, x) == paper_objective(g, x)


def test_maxcut_closed_forms_brute_force():
    bowtie = workloads.from_edges(5, [(0, 1), (0, 2), (1, 2), (2, 3), (2, 4), (3, 4)])
    assert brute_force_max(bowtie) == 4          # Figure 1 graph, unit weights
    c5 = workloads.from_edges(5, [(i, (i + 1) % 5) for i in range(5)])
    assert brute_force_max(c5) == 4              # odd cycle: all edges but one
    c6 = workloads.from_edges(6, [(i, (i + 1) % 6) for i in range(6)])
    assert brute_force_max(c6) == 6              # even cycle is bipartite
    for n in (4, 5, 6):
        kn = workloads.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
        assert brute_force_max(kn) == (n * n) // 4   # complete graph: floor(n^2 / 4)
    t4 = workloads.torus(4, 1, 9, seed=3)
    assert brute_force_max(t4) == t4.total_weight    # even torus is bipartite


def test_maxcut_symmetries_and_checkerboard():
    g = workloads.torus(10, 1, 5, seed=1)
    assert oracle.maxcut(g, np.zeros(g.n, np.uint8)) == 0
    r, c = np.divmod(np.arange(g.n), 10)
    board = ((r + c) % 2).astype(np.uint8)
    assert oracle.maxcut(g, board) == g.total_weight
    assert oracle.maxcut(g, 1 - board) == g.total_weight
    x = np.random.default_rng(1).integers(0, 2, g.n).astype(np.uint8)
    assert oracle.maxcut(g, x) == oracle.maxcut(g, 1 - x)


# ------------------------------------------------------------------------------------------
# FOS, LMIG and colouring
# ------------------------------------------------------------------------------------------
def test_fos_builders():
    g = workloads.configuration_model(200, 5, seed=4, weights="uniform")
    p, v = oracle.fos(g, 0)
    assert np.array_equal(p, np.arange(g.n + 1)) and np.array_equal(v, np.arange(g.n))
    p, v = oracle.fos(g, 1)
    nb = [set() for _ in range(g.n)]
    for a, b in zip(g.u, g.v):
        nb[a].add(int(b))
        nb[b].add(int(a))
    for x in range(g.n):
        assert v[p[x]:p[x + 1]].tolist() == sorted(nb[x] | {x})


def read_fig123():
    vig, sets, lmig, caption = [], {}, set(), []
    with open(os.path.join(GOLDEN, "fig123_lmig.txt")) as fh:
        for line in fh:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            nums = [int(x) for x in t[1:]]
            if t[0] == "vig":
                vig.append((nums[0] - 1, nums[1] - 1))
            elif t[0] == "set":
                sets[nums[0]] = [x - 1 for x in nums[1:]]
            elif t[0] == "lmig":
                lmig.add(tuple(sorted((nums[0] - 1, nums[1] - 1))))
            elif t[0] == "caption":
                caption.append([x - 1 for x in nums])
    g = workloads.from_edges(5, vig)
    order = sorted(sets)
    ptr = np.zeros(len(order) + 1, np.int32)
    ptr[1:] = np.cumsum([len(sets[j]) for j in order])
    vars_ = np.concatenate([np.asarray(sets[j], np.int32) for j in order])
    return g, ptr, vars_, lmig, caption


def test_lmig_of_figure3():
    g, ptr, vars_, lmig, _ = read_fig123()
    assert len(lmig) == 22
    got = {tuple(p) for p in oracle.lmig_pairwise(g, ptr, vars_).tolist()}
    assert got == lmig


def valid_colouring(pairs, colour):
    return all(colour[a] != colour[b] for a, b in pairs)


def test_colouring_of_figure3():
    """Welsh-Powell with (degree desc, index asc): {F3}, {F6}, {F8}, {F1,F4}, {F2,F5}, {F7};
    k = 6 = chromatic number ({F3..F8} is a 6-clique).  The caption's grouping is another
    valid 6-colouring."""
    g, ptr, vars_, lmig, caption = read_fig123()
    k, col, deg = oracle.colour(g, ptr, vars_)
    assert k == 6
    classes = sorted(sorted(int(j) for j in np.nonzero(col == c)[0]) for c in range(k))
    assert classes == sorted([[2], [5], [7], [0, 3], [1, 4], [6]])
    assert col[2] == 0 and col[5] == 1 and col[7] == 2 and col[0] == col[3] == 3
    assert deg.tolist() == [4, 4, 7, 5, 5, 7, 5, 7]
    assert valid_colouring(lmig, col)
    cap = np.zeros(8, np.int64)
    for c, members in enumerate(caption):
        cap[members] = c
    assert sorted(sum(caption, [])) == list(range(8))
    assert valid_colouring(lmig, cap)
    clique = [2, 3, 4, 5, 6, 7]
    assert all(tuple(sorted(p)) in lmig for p in itertools.combinations(clique, 2))


@pytest.mark.parametrize("n,d,kind", [(40, 3, 0), (40, 3, 1), (30, 5, 1), (24, 8, 1)])
def test_colouring_valid_and_degree_matches_pairwise_lmig(n, d, kind):
    g = workloads.configuration_model(n, d, seed=n * d, weights="uniform")
    ptr, vars_ = oracle.fos(g, kind)
    pairs = oracle.lmig_pairwise(g, ptr, vars_)
    k, col, deg = oracle.colour(g, ptr, vars_)
    pdeg = np.bincount(pairs.ravel(), minlength=len(ptr) - 1)
    assert np.array_equal(pdeg, deg)
    assert valid_colouring(pairs.tolist(), col)
    assert set(col.tolist()) == set(range(k))
    # Welsh-Powell bound: k <= max_i min(d_(i) + 1, i) over the sorted degree sequence.
    ds = sorted(deg.tolist(), reverse=True)
    assert k <= max(min(dd + 1, i + 1) for i, dd in enumerate(ds))


def test_colouring_on_tori():
    g = workloads.torus(10, 1, 5, seed=1)
    ptr, vars_ = oracle.fos(g, 0)
    k, col, _ = oracle.colour(g, ptr, vars_)
    r, c = np.divmod(np.arange(g.n), 10)
    parity = (r + c) % 2
    assert k == 2
    assert len(set(zip(col.tolist(), parity.tolist()))) == 2  # classes = checkerboard parity
    g = workloads.torus(12, 1, 5, seed=1)
    ptr, vars_ = oracle.fos(g, 1)
    k, col, _ = oracle.colour(g, ptr, vars_)
    assert k >= 8
    assert valid_colouring(oracle.lmig_pairwise(g, ptr, vars_).tolist(), col)


# ------------------------------------------------------------------------------------------
# GOM generations
# ------------------------------------------------------------------------------------------
def read_hand_cases():
    cases = []
    with open(os.path.join(GOLDEN, "hand_generations.txt")) as fh:
        for line in fh:
            if not line.startswith("case "):
                continue
            head, start, pop, fit, elite, fe, cnt = [s.split() for s in line.split("|")]
            cases.append({
                "name": head[1], "rule": 1 if head[2] == "always" else 0,
                "w": [int(head[3]), int(head[4])],
                "start": [[int(ch) for ch in s] for s in start],
                "pop": [[int(ch) for ch in s] for s in pop], "fit": [int(x) for x in fit],
                "elite": [int(ch) for ch in elite[0]], "fE": int(fe[0]),
                "evaluated": int(cnt[0]), "accepted": int(cnt[1])})
    return cases


@pytest.mark.parametrize("case", read_hand_cases(), ids=lambda c: f"{c['name']}-{c['rule']}")
def test_hand_worked_generation(case):
    g = workloads.from_edges(3, [(0, 1), (1, 2)], case["w"])
    ptr, vars_ = oracle.fos(g, 0)
    N = len(case["start"])
    run = oracle.Run(g, ptr, vars_, pop=N, seed=1, rule=case["rule"],
                     order=oracle.ORDER_FIXED)
    cp, ce = run.classes()
    assert ce[cp[0]:cp[1]].tolist() == [1] and ce[cp[1]:cp[2]].tolist() == [0, 2]
    start = np.array(case["start"], np.uint8)
    f0 = [oracle.maxcut(g, x) for x in start]
    b = int(np.argmax(f0))
    run.set_state(start, start[b], f0[b], 0, [0, 0, 0])
    run.generation()
    s = run.state()
    assert s["genes"].tolist() == case["pop"]
    assert s["fitness"].tolist() == case["fit"]
    assert s["elite"].tolist() == case["elite"] and s["elite_fitness"] == case["fE"]
    assert (s["evaluated"], s["accepted"]) == (case["evaluated"], case["accepted"])
    assert s["attempted"] == N * 3


@pytest.mark.parametrize("n,d,kind,pop,rule,order", [
    (12, 3, 1, 5, 0, 0), (16, 4, 0, 4, 0, 0), (14, 3, 1, 7, 1, 0), (20, 2, 1, 3, 0, 1),
    (18, 5, 1, 9, 0, 0)])
def test_oracle_equals_class_at_once_reference(n, d, kind, pop, rule, order):
    """The step-at-a-time oracle (partial deltas, one step after another inside a class)
    against the whole-class reference (every pair of a class decided on the class-start
    offspring with the objective evaluated in full, then applied together), every
    generation."""
    g = workloads.configuration_model(n, d, seed=n + 100 * d, weights="signed50")
    ptr, vars_ = oracle.fos(g, kind)
    run = oracle.Run(g, ptr, vars_, pop=pop, seed=n * pop, rule=rule, order=order)
    cp, ce = run.classes()
    classes = [ce[cp[c]:cp[c + 1]].tolist() for c in range(len(cp) - 1)]
    cao = ClassAtOnceGomea(g, ptr, vars_, classes, pop, seed=n * pop, rule=rule, order=order)
    s = run.state()
    assert np.array_equal(s["genes"], cao.P)
    for gen in range(6):
        run.generation()
        cao.generation()
        s = run.state()
        assert np.array_equal(s["genes"], cao.P), gen
        assert s["fitness"].tolist() == cao.f.tolist(), gen
        assert np.array_equal(s["elite"], cao.E) and s["elite_fitness"] == cao.fE
        assert (s["evaluated"], s["accepted"]) == (cao.evaluated, cao.accepted)


@pytest.mark.parametrize("n,d,kind,pop,order", [(12, 3, 1, 5, 0), (16, 4, 0, 4, 0),
                                                 (18, 5, 1, 9, 1)])
def test_stop_after_class_equals_class_at_once(n, d, kind, pop, order):
    """A generation cut after each class position shows the whole-class reference's offspring,
    running fitness and counters after the same group; finishing it equals an uncut
    generation."""
    g = workloads.configuration_model(n, d, seed=n + 100 * d, weights="signed50")
    ptr, vars_ = oracle.fos(g, kind)
    run = oracle.Run(g, ptr, vars_, pop=pop, seed=n * pop, order=order)
    whole = oracle.Run(g, ptr, vars_, pop=pop, seed=n * pop, order=order)
    cp, ce = run.classes()
    k = len(cp) - 1
    classes = [ce[cp[c]:cp[c + 1]].tolist() for c in range(k)]
    for gen in range(4):
        for t in range(k):
            cao = ClassAtOnceGomea(g, ptr, vars_, classes, pop, seed=n * pop, order=order,
                                  P=run.state()["genes"])
            s0 = run.state()
            cao.E, cao.fE, cao.gen = s0["elite"].copy(), s0["elite_fitness"], s0["generation"]
            cao.evaluated, cao.accepted = s0["evaluated"], s0["accepted"]
            cao.generation(stop_after=t)
            probe = oracle.Run(g, ptr, vars_, pop=pop, seed=n * pop, order=order)
            probe.set_state(s0["genes"], s0["elite"], s0["elite_fitness"], s0["generation"],
                            [s0["attempted"], s0["evaluated"], s0["accepted"]])
            probe.stop_after_class(t)
            m = probe.state()
            O, f, ev, ac = cao.mid
            assert np.array_equal(m["genes"], O), (gen, t)
            assert m["fitness"].tolist() == f.tolist(), (gen, t)
            assert (m["evaluated"], m["accepted"]) == (ev, ac), (gen, t)
            assert m["generation"] == s0["generation"]
            probe.generation()
            lit2 = probe.state()
            assert np.array_equal(lit2["genes"], cao.P) and lit2["fitness"].tolist() == cao.f.tolist()
        run.stop_after_class(gen % k)
        with pytest.raises(ValueError):
            run.stop_after_class(k)
        if gen % k > 0:
            with pytest.raises(ValueError):
                run.stop_after_class(gen % k - 1)
        run.generation()
        whole.generation()
        a, b = run.state(), whole.state()
        for key in ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted",
                    "evaluated", "accepted"):
            assert np.array_equal(a[key], b[key]), (gen, key)


def _hash_definition(s):
    """The state hash from its definition, over the bytes the accessors return: the sum
    modulo 2^64 of SplitMix64's output mixer of 256 k + b_k over the canonical string."""
    def le(x, nbytes):
        return list(int(x & ((1 << (8 * nbytes)) - 1)).to_bytes(nbytes, "little"))
    parts = [s["genes"].reshape(-1).astype(np.uint64)]
    parts.append(np.array([b for f in s["fitness"].tolist() for b in le(f, 8)], np.uint64))
    parts.append(s["elite"].astype(np.uint64))
    tail = le(s["elite_fitness"], 8) + le(s["generation"], 4)
    for key in ("attempted", "evaluated", "accepted"):
        tail += le(s[key], 8)
    parts.append(np.array(tail, np.uint64))
    b = np.concatenate(parts)
    z = (np.arange(b.shape[0], dtype=np.uint64) << np.uint64(8)) | b
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        return int(z.sum(dtype=np.uint64))


def test_state_hash_definition():
    """The oracle's state hash equals its definition at the start, mid-generation and after
    generations, and changes when any part of the state changes."""
    g = workloads.torus(6, 1, 9, seed=3)
    ptr, vars_ = oracle.fos(g, 1)
    run = oracle.Run(g, ptr, vars_, pop=7, seed=11)
    seen = set()
    for step in range(5):
        s = run.state()
        assert run.hash() == _hash_definition(s), step
        seen.add(run.hash())
        if step % 2:
            run.generation()
        else:
            run.stop_after_class(0)
    assert len(seen) == 5
    s = run.state()
    genes = s["genes"].copy()
    genes[3, 5] ^= 1
    run.set_state(genes, s["elite"], s["elite_fitness"], s["generation"],
                  [s["attempted"], s["evaluated"], s["accepted"]])
    assert run.hash() == _hash_definition(run.state()) and run.hash() not in seen


def _read_lt_fixture(name):
    n, edges, sets = 0, [], []
    for line in open(os.path.join(GOLDEN, name)):
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "n":
            n = int(t[1])
        elif t[0] == "edge":
            edges.append((int(t[1]), int(t[2]), int(t[3])))
        elif t[0] == "set":
            sets.append([int(x) for x in t[1:]])
    e = np.array(edges, np.int64)
    g = workloads.from_edges(n, e[:, :2], e[:, 2])
    return g, sets


def _lt_sets(ptr, vars_):
    return [vars_[ptr[j]:ptr[j + 1]].tolist() for j in range(len(ptr) - 1)]


@pytest.mark.parametrize("name", ["fig2_linkage_tree.txt", "two_cliques_linkage_tree.txt"])
def test_linkage_tree_fixtures(name):
    """The Fig. 2 tree from weights that must produce it, and a hand-derived tree that
    exercises both tie rules."""
    g, expected = _read_lt_fixture(name)
    ptr, vars_ = oracle.linkage_tree(g, 0)
    assert _lt_sets(ptr, vars_) == expected


def _check_upgma(g, ptr, vars_, bound):
    """Brute-force check of a linkage tree against its definition: every merged set is the
    union of two clusters alive at that point, every merge takes a pair of largest average
    similarity (exact fractions over all allowed pairs, ties by size sum then ids), merge
    similarities never increase (average linkage is reducible), the bound holds, and at the
    end no allowed pair is left."""
    from fractions import Fraction
    n = g.n
    S = np.zeros((n, n), np.int64)
    for a, b, w in zip(g.u, g.v, g.w):
        S[a, b] += abs(int(w))
        S[b, a] += abs(int(w))
    cap = bound if bound else n
    sets = _lt_sets(ptr, vars_)
    assert sets[:n] == [[v] for v in range(n)]
    clusters = {v: [v] for v in range(n)}
    last = None
    for c in range(n, len(sets)):
        alive = sorted(clusters)
        best = None
        for x in range(len(alive)):
            for y in range(x + 1, len(alive)):
                i, j = alive[x], alive[y]
                A, B = clusters[i], clusters[j]
                tot = len(A) + len(B)
                if tot > cap or tot >= n:
                    continue
                key = (-Fraction(int(S[np.ix_(A, B)].sum()), len(A) * len(B)), tot, i, j)
                if best is None or key < best:
                    best = key
        assert best is not None, "a merge was made with no allowed pair"
        i, j = best[2], best[3]
        assert sorted(clusters[i] + clusters[j]) == sets[c], f"merge {c}"
        if last is not None:
            assert -best[0] <= last, "merge similarity increased"
        last = -best[0]
        clusters[c] = sets[c]
        del clusters[i], clusters[j]
        assert len(sets[c]) <= cap
    alive = sorted(clusters)
    for x in range(len(alive)):
        for y in range(x + 1, len(alive)):
            tot = len(clusters[alive[x]]) + len(clusters[alive[y]])
            assert tot > cap or tot >= n, "the tree stopped with an allowed pair left"
    if not bound:
        assert len(sets) == 2 * n - 2


@pytest.mark.parametrize("maker,bound", [
    (lambda: workloads.torus(5, 1, 4, seed=3), 0),
    (lambda: workloads.torus(6, 1, 1, seed=1), 0),          # all weights equal: ties decide
    (lambda: workloads.configuration_model(24, 3, seed=2), 0),
    (lambda: workloads.configuration_model(30, 4, seed=5), 5),
    (lambda: workloads.torus(6, 1, 9, seed=2), 3),
    (lambda: workloads.from_edges(9, [(0, 1), (1, 2), (3, 4), (5, 6), (6, 7)],
                                  [4, -6, 2, 1, 1]), 0),  # disconnected, a negative weight
    (lambda: workloads.from_edges(9, [(0, 1), (1, 2), (3, 4), (5, 6), (6, 7)],
                                  [4, -6, 2, 1, 1]), 4),
])
def test_linkage_tree_is_upgma(maker, bound):
    g = maker()
    ptr, vars_ = oracle.linkage_tree(g, bound)
    _check_upgma(g, ptr, vars_, bound)


def _complete_graph(n, seed, unit=False):
    """K_n with weights +-U{1..9} (or all 1): with univariate sets every pair of sets is
    dependent, so every colour class holds a single set.  With unit weights and n odd a flip
    often leaves the cut unchanged, so neutral steps occur."""
    rng = np.random.default_rng(seed)
    e = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    w = np.ones(e.shape[0], np.int64) if unit else workloads.signed_uniform(rng, e.shape[0], 9)
    return workloads.from_edges(n, e, w)


def _overlapping_sets(n):
    """Singletons, cyclic pairs and triples: on a complete graph all of them conflict."""
    sets = [[u] for u in range(n)] + [sorted([u, (u + 1) % n]) for u in range(n)] + \
        [sorted([u, (u + 2) % n, (u + 3) % n]) for u in range(0, n, 2)]
    ptr = np.zeros(len(sets) + 1, np.int32)
    ptr[1:] = np.cumsum([len(x) for x in sets])
    return ptr, np.concatenate([np.asarray(x, np.int32) for x in sets])


@pytest.mark.parametrize("n,seed", [(6, 6), (6, 10), (8, 38), (8, 42)])
def test_forced_improvement_stops_at_improvement_not_at_acceptance(n, seed):
    """Instances (complete graphs with weights +-1 and overlapping sets, one set per class)
    on which a neutral accepted step precedes the first improving one during forced
    improvement: stopping at the first accepted step would give a different population.  The
    oracle follows the paper's rule (stop at the first step that raises fitness)."""
    rng = np.random.default_rng(seed)
    e = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    g = workloads.from_edges(n, e, rng.choice([-1, 1], size=e.shape[0]))
    ptr, vars_ = _overlapping_sets(n)
    pop = 4 + seed % 3
    run = oracle.Run(g, ptr, vars_, pop=pop, seed=seed, flags=oracle.FLAG_FI)
    cp, ce = run.classes()
    assert np.all(np.diff(cp) == 1)
    classes = [ce[cp[c]:cp[c + 1]].tolist() for c in range(len(cp) - 1)]
    cao = ClassAtOnceGomea(g, ptr, vars_, classes, pop, seed=seed, fi=True)
    wrong = ClassAtOnceGomea(g, ptr, vars_, classes, pop, seed=seed, fi=True,
                            fi_stop_on_accept=True)
    readings_differ = False
    for gen in range(10):
        run.generation()
        cao.generation()
        wrong.generation()
        s = run.state()
        assert np.array_equal(s["genes"], cao.P), gen
        assert s["fitness"].tolist() == cao.f.tolist(), gen
        assert (s["evaluated"], s["accepted"]) == (cao.evaluated, cao.accepted), gen
        readings_differ |= not np.array_equal(cao.P, wrong.P)
    assert readings_differ


@pytest.mark.parametrize("n,pop,rule,seed", [(7, 5, 0, 1), (8, 6, 1, 2), (9, 4, 0, 3),
                                             (6, 8, 0, 4)])
def test_forced_improvement_equals_serial_with_one_set_per_class(n, pop, rule, seed):
    """With one set per class, the class-by-class forced improvement is the serial procedure
    of Section 4 (the whole-class reference stops at the first improving step)."""
    g = _complete_graph(n, seed)
    ptr, vars_ = oracle.fos(g, 0)
    run = oracle.Run(g, ptr, vars_, pop=pop, seed=seed, rule=rule, flags=oracle.FLAG_FI)
    cp, ce = run.classes()
    assert np.all(np.diff(cp) == 1)
    classes = [ce[cp[c]:cp[c + 1]].tolist() for c in range(len(cp) - 1)]
    cao = ClassAtOnceGomea(g, ptr, vars_, classes, pop, seed=seed, rule=rule, fi=True)
    plain = oracle.Run(g, ptr, vars_, pop=pop, seed=seed, rule=rule)
    differs = False
    for gen in range(8):
        run.generation()
        cao.generation()
        plain.generation()
        s = run.state()
        assert np.array_equal(s["genes"], cao.P), gen
        assert s["fitness"].tolist() == cao.f.tolist(), gen
        assert (s["evaluated"], s["accepted"]) == (cao.evaluated, cao.accepted), gen
        assert np.array_equal(s["elite"], cao.E) and s["elite_fitness"] == cao.fE
        differs |= not np.array_equal(s["genes"], plain.state()["genes"])
    assert differs, "forced improvement never changed anything"


@pytest.mark.parametrize("n,d,kind,pop", [(40, 3, 1, 10), (60, 4, 0, 12), (50, 5, 1, 7)])
def test_forced_improvement_invariants(n, d, kind, pop):
    """On graphs with several sets per class: full re-evaluation agrees with every partial
    delta (debug flag), fitness never falls, and each solution that made no accepted GOM step
    ends either fitter than it started or equal to the elitist."""
    g = workloads.configuration_model(n, d, seed=n + d, weights="signed50")
    ptr, vars_ = oracle.fos(g, kind)
    run = oracle.Run(g, ptr, vars_, pop=pop, seed=5, flags=oracle.FLAG_FI | oracle.FLAG_DEBUG)
    ref = oracle.Run(g, ptr, vars_, pop=pop, seed=5)
    for gen in range(10):
        s0 = run.state()
        ref.set_state(s0["genes"], s0["elite"], s0["elite_fitness"], s0["generation"],
                      [s0["attempted"], s0["evaluated"], s0["accepted"]])
        ref.generation()
        run.generation()
        s1, r1 = run.state(), ref.state()
        assert s1["debug_mismatches"] == 0
        assert np.all(s1["fitness"] >= s0["fitness"]), gen
        for i in range(pop):
            if r1["fitness"][i] == s0["fitness"][i] and \
                    np.array_equal(r1["genes"][i], s0["genes"][i]):
                # no accepted step without FI (same draws), so FI ran for solution i
                assert s1["fitness"][i] > s0["fitness"][i] or \
                    np.array_equal(s1["genes"][i], s0["elite"]), (gen, i)
            else:
                assert np.array_equal(s1["genes"][i], r1["genes"][i]), (gen, i)


def test_ims_generation_order():
    """The interleaving of the multi-start scheme against a hand-derived order, and each
    level's population size and seed."""
    spec = {}
    for line in open(os.path.join(GOLDEN, "ims_order.txt")):
        t = line.split()
        if t and not t[0].startswith("#"):
            spec[t[0]] = [int(x) for x in t[1:]]
    g = workloads.torus(6, 1, 9, seed=2)
    ptr, vars_ = oracle.fos(g, 0)
    runs, order = oracle.ims_run(g, ptr, vars_, n_base=4, c_ims=spec["c"][0],
                                 max_levels=spec["levels"][0], seed=7, target=1 << 62,
                                 max_total_generations=len(spec["order"]))
    assert order == spec["order"]
    assert [r.N for r in runs] == [4, 8, 16]
    for lvl, r in enumerate(runs, start=1):
        alone = oracle.Run(g, ptr, vars_, pop=4 << (lvl - 1), seed=7 + lvl - 1)
        for _ in range(order.count(lvl)):
            alone.generation()
        assert np.array_equal(alone.state()["genes"], r.state()["genes"]), lvl


def test_ims_stops_at_target():
    """The scheme stops after the step in which some level's elitist reaches the target."""
    g = workloads.torus(6, 1, 9, seed=2)
    ptr, vars_ = oracle.fos(g, 1)
    runs, order = oracle.ims_run(g, ptr, vars_, n_base=4, c_ims=4, max_levels=3, seed=3,
                                 target=g.total_weight, max_total_generations=500)
    best = [r.state(genes=False)["elite_fitness"] for r in runs]
    assert max(best) >= g.total_weight and len(order) < 500
    # one step earlier no level had reached it: rerun with the budget cut before the last step
    last_step = len(order) - 1
    while last_step > 0 and order[last_step] != 1:
        last_step -= 1
    runs2, order2 = oracle.ims_run(g, ptr, vars_, n_base=4, c_ims=4, max_levels=3, seed=3,
                                   target=g.total_weight, max_total_generations=last_step)
    assert max(r.state(genes=False)["elite_fitness"] for r in runs2) < g.total_weight


def test_initial_population_rule():
    g = workloads.torus(12, 1, 3, seed=2)
    ptr, vars_ = oracle.fos(g, 0)
    run = oracle.Run(g, ptr, vars_, pop=6, seed=99)
    assert np.array_equal(run.state()["genes"], initial_population(g.n, 6, 99))
    s = run.state()
    assert s["fitness"].tolist() == [oracle.maxcut(g, x) for x in s["genes"]]
    b = int(np.argmax(s["fitness"]))
    assert np.array_equal(s["elite"], s["genes"][b]) and s["elite_fitness"] == s["fitness"][b]


@pytest.mark.parametrize("kind", [0, 1])
def test_partial_delta_equals_full_reevaluation(kind):
    """Debug mode re-evaluates the whole solution after every step and counts mismatches
    with the partially updated fitness (Section 2.2)."""
    for n, d in ((60, 3), (50, 6)):
        g = workloads.configuration_model(n, d, seed=d, weights="signed50")
        ptr, vars_ = oracle.fos(g, kind)
        run = oracle.Run(g, ptr, vars_, pop=8, seed=3, flags=oracle.FLAG_DEBUG)
        run.run(1 << 62, 8)
        s = run.state()
        assert s["debug_mismatches"] == 0
        assert s["evaluated"] > 0 and s["accepted"] > 0
        assert s["fitness"].tolist() == [oracle.maxcut(g, x) for x in s["genes"]]


def test_order_within_class_is_irrelevant():
    """Reverse the visiting order of solutions and sets inside every class: same result."""
    g = workloads.configuration_model(300, 4, seed=5, weights="signed50")
    ptr, vars_ = oracle.fos(g, 1)
    a = oracle.Run(g, ptr, vars_, pop=12, seed=4)
    b = oracle.Run(g, ptr, vars_, pop=12, seed=4, flags=oracle.FLAG_REVERSE)
    a.run(1 << 62, 10)
    b.run(1 << 62, 10)
    sa, sb = a.state(), b.state()
    for key in ("genes", "fitness", "elite", "evaluated", "accepted"):
        assert np.array_equal(sa[key], sb[key])


def test_univariate_trajectory_independent_of_donor_draws():
    """With single-variable sets any differing donor carries the flipped gene, so changing
    every donor draw (salted donor key) leaves the univariate trajectory unchanged; with the
    neighbourhood FOS it changes."""
    g = workloads.configuration_model(400, 4, seed=8, weights="signed50")
    for kind, same in ((0, True), (1, False)):
        ptr, vars_ = oracle.fos(g, kind)
        a = oracle.Run(g, ptr, vars_, pop=16, seed=6)
        b = oracle.Run(g, ptr, vars_, pop=16, seed=6, donor_salt=0x5DEECE66D)
        a.run(1 << 62, 8)
        b.run(1 << 62, 8)
        assert np.array_equal(a.state()["genes"], b.state()["genes"]) == same


def test_monotone_fitness_and_bounds():
    g = workloads.configuration_model(16, 3, seed=7, weights="uniform", w_lo=1, w_hi=20)
    ptr, vars_ = oracle.fos(g, 1)
    run = oracle.Run(g, ptr, vars_, pop=10, seed=2)
    best = brute_force_max(g)
    prev = run.state()
    for _ in range(10):
        run.generation()
        s = run.state()
        assert (s["fitness"] >= prev["fitness"]).all()
        assert s["elite_fitness"] >= prev["elite_fitness"]
        assert s["elite_fitness"] <= best
        assert s["elite_fitness"] == oracle.maxcut(g, s["elite"])
        prev = s


def test_converged_population_is_fixed_point():
    g = workloads.torus(6, 1, 5, seed=1)
    ptr, vars_ = oracle.fos(g, 1)
    run = oracle.Run(g, ptr, vars_, pop=5, seed=2)
    x = np.random.default_rng(3).integers(0, 2, g.n).astype(np.uint8)
    run.set_state(np.tile(x, (5, 1)), x, oracle.maxcut(g, x), 0, [0, 0, 0])
    run.run(1 << 62, 4)
    s = run.state()
    assert (s["genes"] == x).all() and s["evaluated"] == 0 and s["accepted"] == 0


def test_checkpoint_resume_reproduces_run():
    g = workloads.configuration_model(500, 3, seed=2, weights="signed50")
    ptr, vars_ = oracle.fos(g, 1)
    a = oracle.Run(g, ptr, vars_, pop=9, seed=5)
    a.run(1 << 62, 4)
    snap = a.state()
    b = oracle.Run(g, ptr, vars_, pop=9, seed=5)
    b.set_state(snap["genes"], snap["elite"], snap["elite_fitness"], snap["generation"],
                [snap["attempted"], snap["evaluated"], snap["accepted"]])
    a.run(1 << 62, 9)
    b.run(1 << 62, 9)
    sa, sb = a.state(), b.state()
    for key in ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted",
                "evaluated", "accepted"):
        assert np.array_equal(sa[key], sb[key])


def test_small_torus_reaches_total_weight():
    """Observed (not guaranteed by the method): a 6x6 torus is solved to its bipartite
    optimum, and the optimum genotype is a checkerboard."""
    g = workloads.torus(6, 1, 9, seed=5)
    ptr, vars_ = oracle.fos(g, 1)
    run = oracle.Run(g, ptr, vars_, pop=16, seed=1)
    run.run(g.total_weight, 200)
    s = run.state()
    assert s["elite_fitness"] == g.total_weight
    r, c = np.divmod(np.arange(g.n), 6)
    board = ((r + c) % 2).astype(np.uint8)
    assert np.array_equal(s["elite"], board) or np.array_equal(s["elite"], 1 - board)


def test_target_checked_before_first_generation():
    g = workloads.torus(6, 1, 9, seed=5)
    ptr, vars_ = oracle.fos(g, 0)
    run = oracle.Run(g, ptr, vars_, pop=4, seed=1)
    assert run.run(run.state()["elite_fitness"], 50) == 0


# ------------------------------------------------------------------------------------------
# Colouring-parallel local search (the hybrid named as future work in the paper's conclusion)
# ------------------------------------------------------------------------------------------
LS_GRAPHS = [
    ("torus6_w9", lambda: workloads.torus(6, 1, 9, seed=2)),
    ("torus8_unit", lambda: workloads.torus(8, 1, 1, seed=3)),          # many zero gains
    ("cm40_d3_signed", lambda: workloads.configuration_model(40, 3, seed=4)),
    ("cm60_d5_signed", lambda: workloads.configuration_model(60, 5, seed=5)),
]


def _ls_run(g, pop, seed, gens):
    ptr, vars_ = oracle.fos(g, 0)
    ref = oracle.Run(g, ptr, vars_, pop=pop, seed=seed)
    for _ in range(gens):
        ref.generation()
    return ref


def _gain(g, x, u):
    """Change of the cut when vertex u flips, from the objective itself."""
    y = x.copy()
    y[u] ^= 1
    return oracle.maxcut(g, y) - oracle.maxcut(g, x)


@pytest.mark.parametrize("label,maker", LS_GRAPHS, ids=[c[0] for c in LS_GRAPHS])
def test_local_search_ends_at_local_optima(label, maker):
    """After an unlimited search every solution is a local optimum (no single flip raises
    the cut, checked with the objective), its fitness is the full evaluation, no fitness fell,
    and the elitist is the best solution if that one is strictly better than before."""
    g = maker()
    ref = _ls_run(g, 8, 3, 2)
    before = ref.state()
    passes = ref.local_search(10_000)
    after = ref.state()
    assert 1 <= passes < 10_000  # strict improvements only: the search ends
    for i in range(8):
        x = after["genes"][i]
        assert after["fitness"][i] == oracle.maxcut(g, x)
        assert after["fitness"][i] >= before["fitness"][i]
        assert all(_gain(g, x, u) <= 0 for u in range(g.n))
    best = int(after["fitness"].max())
    assert after["elite_fitness"] == max(best, before["elite_fitness"])
    if best > before["elite_fitness"]:
        b = int(np.argmax(after["fitness"]))  # lowest index among the best
        assert np.array_equal(after["elite"], after["genes"][b])
    for key in ("generation", "attempted", "evaluated", "accepted"):
        assert after[key] == before[key]


def _literal_local_search(g, classes, genes, max_passes):
    """A literal reading: per pass, per class in ascending index, per solution, first the
    gains of every variable of the class (from the objective), then every improving flip at
    once.  Returns (genes, passes)."""
    x = genes.copy()
    cp, ce = classes
    passes = 0
    while passes < max_passes:
        any_flip = False
        for c in range(len(cp) - 1):
            members = [int(u) for u in ce[cp[c]:cp[c + 1]]]  # univariate: set j = {j}
            for i in range(x.shape[0]):
                gains = [_gain(g, x[i], u) for u in members]
                for u, d in zip(members, gains):
                    if d > 0:
                        x[i, u] ^= 1
                        any_flip = True
        passes += 1
        if not any_flip:
            break
    return x, passes


@pytest.mark.parametrize("label,maker", LS_GRAPHS, ids=[c[0] for c in LS_GRAPHS])
@pytest.mark.parametrize("max_passes", [1, 2, 3, 50])
def test_local_search_equals_literal_reading(label, maker, max_passes):
    """The oracle's search (flips inside a class one after another) equals the literal
    reading (a class's gains first, then its flips together) pass by pass, in genes and in
    the number of passes."""
    g = maker()
    ref = _ls_run(g, 6, 5, 1)
    start = ref.state()["genes"]
    want, want_passes = _literal_local_search(g, ref.classes(), start, max_passes)
    got_passes = ref.local_search(max_passes)
    assert got_passes == want_passes
    assert np.array_equal(ref.state()["genes"], want)


def test_local_search_second_search_is_idle_and_needs_univariate():
    g = workloads.torus(6, 1, 9, seed=2)
    ref = _ls_run(g, 5, 2, 3)
    assert ref.local_search(10_000) < 10_000
    s1 = ref.state()
    assert ref.local_search(10_000) == 1
    s2 = ref.state()
    for key in ("genes", "fitness", "elite", "elite_fitness"):
        assert np.array_equal(np.asarray(s1[key]), np.asarray(s2[key]))
    ptr, vars_ = oracle.fos(g, 1)
    nb = oracle.Run(g, ptr, vars_, pop=4, seed=1)
    with pytest.raises(ValueError):
        nb.local_search()


# ------------------------------------------------------------------------------------------
# Iterated local search (perturbation, search, keep-or-revert per solution)
# ------------------------------------------------------------------------------------------
def _perturbation_vars(seed, gen, i, r, flips, n_sets, classes, ptr, vars_):
    """The variables a round's perturbation flips in solution i, from the draw's definition:
    word t mod 4 of Philox4x32(key = seed, counter = (gen, 0xFFFFFFFE, i, 16 r + t // 4))
    scaled to a class position, then that position's set."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    _, ce = classes
    out = []
    for t in range(flips):
        word = int(oracle.philox4x32(key, (gen, 0xFFFFFFFE, i, 16 * r + t // 4))[t % 4])
        q = (word * n_sets) >> 32
        out.append(int(vars_[ptr[int(ce[q])]]))
    return out


@pytest.mark.parametrize("flips,round0,gens", [(1, 0, 0), (1, 3, 1), (5, 2, 0), (9, 0, 2)])
def test_iterated_local_search_perturbation_follows_the_draw(flips, round0, gens):
    """With no search passes a round is the perturbation and the acceptance alone: every
    solution either carries exactly the drawn flips (when that does not lower its cut,
    checked with the objective) or is unchanged."""
    g = workloads.configuration_model(30, 3, seed=6)
    ptr, vars_ = oracle.fos(g, 0)
    seed = (7 << 32) | 11
    ref = oracle.Run(g, ptr, vars_, pop=24, seed=seed)
    for _ in range(gens):
        ref.generation()
    before = ref.state()
    assert ref.iterated_local_search(round0, 1, flips, max_passes=0) == 0
    after = ref.state()
    changed = 0
    for i in range(24):
        x = before["genes"][i].copy()
        for u in _perturbation_vars(seed, int(before["generation"]), i, round0, flips,
                                    g.n, ref.classes(), ptr, vars_):
            x[u] ^= 1
        want = x if oracle.maxcut(g, x) >= oracle.maxcut(g, before["genes"][i]) \
            else before["genes"][i]
        assert np.array_equal(after["genes"][i], want)
        assert after["fitness"][i] == oracle.maxcut(g, want)
        changed += not np.array_equal(want, before["genes"][i])
    assert changed > 0


def _literal_iterated_local_search(g, ref, genes, elite_f, seed, gen, round0, rounds, flips,
                                   max_passes):
    ptr, vars_ = ref.set_ptr, ref.set_vars
    x = genes.copy()
    total = 0
    for r in range(round0, round0 + rounds):
        cand = x.copy()
        for i in range(x.shape[0]):
            for u in _perturbation_vars(seed, gen, i, r, flips, g.n, ref.classes(), ptr,
                                        vars_):
                cand[i, u] ^= 1
        cand, p = _literal_local_search(g, ref.classes(), cand, max_passes)
        total += p
        for i in range(x.shape[0]):
            if oracle.maxcut(g, cand[i]) >= oracle.maxcut(g, x[i]):
                x[i] = cand[i]
        fit = [oracle.maxcut(g, xi) for xi in x]
        elite_f = max(elite_f, max(fit))
    return x, total, elite_f


@pytest.mark.parametrize("label,maker", LS_GRAPHS, ids=[c[0] for c in LS_GRAPHS])
@pytest.mark.parametrize("rounds,flips,max_passes", [(1, 3, 50), (4, 2, 50), (3, 7, 1),
                                                     (2, 64, 2)])
def test_iterated_local_search_equals_literal_reading(label, maker, rounds, flips,
                                                      max_passes):
    """The oracle's iterated search equals a literal reading built on the literal local
    search (a class's gains first, then its flips together), in genes, summed passes and
    elitist fitness."""
    g = maker()
    ref = _ls_run(g, 6, 9, 1)
    s0 = ref.state()
    want, want_passes, want_ef = _literal_iterated_local_search(
        g, ref, s0["genes"], int(s0["elite_fitness"]), 9, int(s0["generation"]), 1, rounds,
        flips, max_passes)
    assert ref.iterated_local_search(1, rounds, flips, max_passes) == want_passes
    s1 = ref.state()
    assert np.array_equal(s1["genes"], want)
    assert s1["elite_fitness"] == want_ef


@pytest.mark.parametrize("label,maker", LS_GRAPHS, ids=[c[0] for c in LS_GRAPHS])
def test_iterated_local_search_invariants(label, maker):
    """From local optima: every solution stays a local optimum (unlimited passes), no solution
    gets worse, fitness is the full evaluation, the elitist is the best when that one is
    strictly better, and the generation and GOM counters do not change."""
    g = maker()
    ref = _ls_run(g, 8, 4, 2)
    ref.local_search()
    before = ref.state()
    ref.iterated_local_search(0, 6, 3)
    after = ref.state()
    for i in range(8):
        x = after["genes"][i]
        assert after["fitness"][i] == oracle.maxcut(g, x)
        assert after["fitness"][i] >= before["fitness"][i]
        assert all(_gain(g, x, u) <= 0 for u in range(g.n))
    best = int(after["fitness"].max())
    assert after["elite_fitness"] == max(best, before["elite_fitness"])
    if best > before["elite_fitness"]:
        assert np.array_equal(after["elite"], after["genes"][int(np.argmax(after["fitness"]))])
    for key in ("generation", "attempted", "evaluated", "accepted"):
        assert after[key] == before[key]


def test_iterated_local_search_zero_flips_and_round_ranges():
    """Zero-flip rounds are the plain search followed by idle one-pass rounds; rounds a..b
    then b..c equal rounds a..c; the FOS must be univariate and the arguments in range."""
    g = workloads.torus(6, 1, 9, seed=2)
    a, b = _ls_run(g, 5, 2, 3), _ls_run(g, 5, 2, 3)
    p = b.local_search()
    assert a.iterated_local_search(0, 3, 0) == p + 2
    for key in ("genes", "fitness", "elite", "elite_fitness"):
        assert np.array_equal(np.asarray(a.state()[key]), np.asarray(b.state()[key]))
    c, d = _ls_run(g, 5, 2, 3), _ls_run(g, 5, 2, 3)
    pc = c.iterated_local_search(2, 5, 4)
    pd = d.iterated_local_search(2, 2, 4) + d.iterated_local_search(4, 3, 4)
    assert pc == pd
    assert np.array_equal(c.state()["genes"], d.state()["genes"])
    for args in ((-1, 1, 1), (0, -1, 1), (0, 1, 65), (0, 1, -1), ((1 << 27), 1, 1)):
        with pytest.raises(ValueError):
            c.iterated_local_search(*args)
    ptr, vars_ = oracle.fos(g, 1)
    with pytest.raises(ValueError):
        oracle.Run(g, ptr, vars_, pop=4, seed=1).iterated_local_search(0, 1, 1)


@pytest.mark.parametrize("kind,pop,flags", [(1, 33, 0), (0, 64, oracle.FLAG_DEBUG),
                                             (1, 17, oracle.FLAG_FI | oracle.FLAG_DEBUG)])
def test_oracle_workers_do_not_change_the_run(kind, pop, flags):
    """Solutions of a class spread over several worker threads: the same states and hashes as
    one worker, every generation (a class's solutions write only their own offspring)."""
    g = workloads.torus(20, 1, 100, seed=5)
    ptr, vars_ = oracle.fos(g, kind)
    runs = [oracle.Run(g, ptr, vars_, pop=pop, seed=9, flags=flags, workers=w) for w in (1, 3, 8)]
    for gen in range(8):
        for r in runs:
            r.generation()
        states = [r.state() for r in runs]
        for s in states[1:]:
            for key in ("genes", "fitness", "elite", "elite_fitness", "generation", "attempted",
                        "evaluated", "accepted", "debug_mismatches"):
                assert np.array_equal(np.asarray(s[key]), np.asarray(states[0][key])), (gen, key)
        assert len({r.hash() for r in runs}) == 1
        assert states[0]["debug_mismatches"] == 0
