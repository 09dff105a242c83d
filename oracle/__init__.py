"""ctypes wrapper around the CPU oracle (oracle/gom_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package's smoke check and the benchmark's
CPU-baseline leg.  The product path never imports it.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

NEUTRAL_PAPER, NEUTRAL_ALWAYS = 0, 1
ORDER_RANDOM, ORDER_FIXED = 0, 1
FLAG_DEBUG, FLAG_REVERSE, FLAG_FI = 1, 2, 4

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def use_native_build(path: str) -> str:
    """Compile a copy of the oracle with -march=native at `path` and load it instead of the
    in-tree portable library (for timing on the host that runs it).  Must come before the
    first use of the oracle in the process."""
    global _lib
    if _lib is not None:
        raise RuntimeError("use_native_build: the oracle library is already loaded")
    _build.build(out=path, native=True)
    lib(path)
    return path


def lib(path: str | None = None):
    """Load oracle/liboracle.so (or `path`), compiling it first only when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
    L = C.CDLL(path)
    L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.or_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    L.or_maxcut.restype = C.c_int64
    L.or_maxcut.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _i32p, _u8p]
    L.or_fos_build.restype = C.c_int64
    L.or_fos_build.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, C.c_int, _i32p, C.c_void_p]
    L.or_lmig_pairwise.restype = C.c_int64
    L.or_lmig_pairwise.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, C.c_int32, _i32p, _i32p,
                                   C.c_int64, _i32p]
    L.or_colour.restype = C.c_int32
    L.or_colour.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, C.c_int32, _i32p, _i32p, _i32p,
                            _i64p]
    L.or_new.restype = C.c_void_p
    L.or_new.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _i32p, C.c_int32, _i32p, _i32p,
                         C.c_int32, C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_int]
    L.or_free.argtypes = [C.c_void_p]
    L.or_generation.argtypes = [C.c_void_p]
    L.or_run.restype = C.c_int32
    L.or_run.argtypes = [C.c_void_p, C.c_int64, C.c_int32]
    L.or_num_classes.restype = C.c_int32
    L.or_num_classes.argtypes = [C.c_void_p]
    L.or_get_classes.argtypes = [C.c_void_p, _i32p, _i32p]
    L.or_get.argtypes = [C.c_void_p, C.c_void_p, _i64p, C.c_void_p, C.POINTER(C.c_int64),
                         C.POINTER(C.c_int32), _i64p]
    L.or_set.argtypes = [C.c_void_p, _u8p, _u8p, C.c_int64, C.c_int32, _i64p]
    L.or_linkage_tree.restype = C.c_int32
    L.or_linkage_tree.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _i32p, C.c_int32, _i32p,
                                  _i32p]
    L.or_stop_after_class.restype = C.c_int32
    L.or_stop_after_class.argtypes = [C.c_void_p, C.c_int32]
    L.or_local_search.restype = C.c_int32
    L.or_local_search.argtypes = [C.c_void_p, C.c_int32]
    L.or_iterated_local_search.restype = C.c_int32
    L.or_iterated_local_search.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                           C.c_int32]
    L.or_hash.restype = C.c_uint64
    L.or_hash.argtypes = [C.c_void_p]
    L.or_set_workers.restype = C.c_int32
    L.or_set_workers.argtypes = [C.c_void_p, C.c_int32]
    _lib = L
    return L


def philox4x32(key, ctr):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(key, np.uint32), np.asarray(ctr, np.uint32), out)
    return out


def philox4x64(key, ctr):
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(np.asarray(key, np.uint64), np.asarray(ctr, np.uint64), out)
    return out


def maxcut(g, x) -> int:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    return int(lib().or_maxcut(g.n, g.m, g.u, g.v, g.w, x))


def fos(g, kind: int):
    """(set_ptr, set_vars) for FOS kind 0 (univariate) or 1 (neighbourhood)."""
    ptr = np.zeros(g.n + 1, np.int32)
    total = lib().or_fos_build(g.n, g.m, g.u, g.v, kind, ptr, None)
    vars_ = np.zeros(max(total, 1), np.int32)
    lib().or_fos_build(g.n, g.m, g.u, g.v, kind, ptr,
                       vars_.ctypes.data_as(C.c_void_p))
    return ptr, vars_[:total]


def linkage_tree(g, bound: int = 0):
    """UPGMA linkage tree on |w| (bound 0 = unbounded): (set_ptr, set_vars)."""
    n = g.n
    ptr = np.zeros(2 * n, np.int32)
    vars_ = np.zeros(n * n, np.int32)
    k = lib().or_linkage_tree(n, g.m, g.u, g.v, g.w, int(bound), ptr, vars_)
    if k < 0:
        raise ValueError("or_linkage_tree failed")
    return ptr[:k + 1].copy(), vars_[:ptr[k]].copy()


def lmig_pairwise(g, set_ptr, set_vars):
    set_ptr = np.ascontiguousarray(set_ptr, np.int32)
    set_vars = np.ascontiguousarray(set_vars, np.int32)
    nsets = set_ptr.shape[0] - 1
    cap = nsets * (nsets - 1) // 2 + 1
    pairs = np.zeros(2 * cap, np.int32)
    cnt = lib().or_lmig_pairwise(g.n, g.m, g.u, g.v, nsets, set_ptr, set_vars, cap, pairs)
    return pairs[: 2 * cnt].reshape(-1, 2)


def colour(g, set_ptr, set_vars):
    """Welsh-Powell colouring: (k, colour[nsets], lmig_degree[nsets])."""
    set_ptr = np.ascontiguousarray(set_ptr, np.int32)
    set_vars = np.ascontiguousarray(set_vars, np.int32)
    nsets = set_ptr.shape[0] - 1
    col = np.zeros(nsets, np.int32)
    deg = np.zeros(nsets, np.int64)
    k = lib().or_colour(g.n, g.m, g.u, g.v, nsets, set_ptr, set_vars, col, deg)
    if k < 1:
        raise RuntimeError("oracle colouring failed")
    return int(k), col, deg


class Run:
    """One oracle run of parallel GOM (Algorithm 3) on graph g with the given FOS."""

    def __init__(self, g, set_ptr, set_vars, pop: int, seed: int, rule: int = NEUTRAL_PAPER,
                 order: int = ORDER_RANDOM, flags: int = 0, donor_salt: int = 0,
                 workers: int = 1):
        self._L = lib()
        self.g = g
        self.set_ptr = np.ascontiguousarray(set_ptr, np.int32)
        self.set_vars = np.ascontiguousarray(set_vars, np.int32)
        self.N = pop
        h = self._L.or_new(g.n, g.m, g.u, g.v, g.w, self.set_ptr.shape[0] - 1, self.set_ptr,
                           self.set_vars, pop, seed, donor_salt, rule, order, flags)
        if not h:
            raise RuntimeError("or_new failed")
        self._h = h
        if workers != 1:
            self.set_workers(workers)

    def set_workers(self, workers: int) -> int:
        """Spread the solutions of each colour class over `workers` threads (results do not
        change).  Returns the number in use."""
        r = int(self._L.or_set_workers(self._h, int(workers)))
        if r < 0:
            raise MemoryError("or_set_workers: out of memory")
        return r

    def close(self):
        if self._h:
            self._L.or_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def generation(self):
        self._L.or_generation(self._h)

    def run(self, target: int, max_gens: int) -> int:
        return int(self._L.or_run(self._h, target, max_gens))

    def stop_after_class(self, pos: int):
        """Run the generation (starting one if none is open) up to class-order position pos
        and leave it open; state() then shows the offspring and running fitness."""
        if self._L.or_stop_after_class(self._h, int(pos)) != 0:
            raise ValueError(f"class position {pos} out of range or already passed")

    def hash(self) -> int:
        return int(self._L.or_hash(self._h))

    def local_search(self, max_passes: int = 1 << 30) -> int:
        """Colouring-parallel local search on the population (univariate FOS, between
        generations): improving single-bit flips a colour class at a time until a pass flips
        nothing or max_passes passes ran.  Returns the passes run."""
        r = self._L.or_local_search(self._h, int(max_passes))
        if r < 0:
            raise ValueError("local search needs a univariate FOS and no open generation")
        return r

    def iterated_local_search(self, round0: int, rounds: int, flips: int,
                              max_passes: int = 1 << 30) -> int:
        """Iterated local search, rounds round0 .. round0 + rounds - 1: per round and solution
        `flips` random single-bit flips, the local search, and the result kept when it is not
        worse.  Returns the passes summed over the rounds."""
        r = self._L.or_iterated_local_search(self._h, int(round0), int(rounds), int(flips),
                                             int(max_passes))
        if r < 0:
            raise ValueError("iterated local search needs a univariate FOS, no open "
                             "generation and arguments in range")
        return r

    def classes(self):
        k = self._L.or_num_classes(self._h)
        cp = np.zeros(k + 1, np.int32)
        ce = np.zeros(self.set_ptr.shape[0] - 1, np.int32)
        self._L.or_get_classes(self._h, cp, ce)
        return cp, ce

    def state(self, genes: bool = True):
        n = self.g.n
        G = np.zeros((self.N, n), np.uint8) if genes else None
        f = np.zeros(self.N, np.int64)
        E = np.zeros(n, np.uint8)
        fE = C.c_int64()
        gen = C.c_int32()
        cnt = np.zeros(4, np.int64)
        self._L.or_get(self._h, G.ctypes.data_as(C.c_void_p) if genes else None, f,
                       E.ctypes.data_as(C.c_void_p), C.byref(fE), C.byref(gen), cnt)
        return {"genes": G, "fitness": f, "elite": E, "elite_fitness": int(fE.value),
                "generation": int(gen.value), "attempted": int(cnt[0]),
                "evaluated": int(cnt[1]), "accepted": int(cnt[2]),
                "debug_mismatches": int(cnt[3])}

    def set_state(self, genes, elite, elite_fitness: int, generation: int, counters):
        self._L.or_set(self._h, np.ascontiguousarray(genes, np.uint8).reshape(-1),
                       np.ascontiguousarray(elite, np.uint8), int(elite_fitness),
                       int(generation), np.asarray(counters[:3], np.int64))


def ims_run(g, set_ptr, set_vars, n_base: int, c_ims: int, max_levels: int, seed: int,
            target: int, max_total_generations: int, rule: int = NEUTRAL_PAPER,
            flags: int = 0):
    """Interleaved Multi-start Scheme (Section 6.3) over oracle runs.  Population P_i (i =
    1, 2, ...) has n_base * 2^(i-1) solutions and seed `seed + i - 1`; a step runs one
    generation of P_1, and whenever P_i has then completed a multiple of c_ims generations
    it continues with one generation of P_(i+1) (created at its first generation), up to
    max_levels populations.  The run stops after the step in which some population's elitist
    reaches `target`, or as soon as max_total_generations generations have run.
    Returns (runs, order): the Run of every level created and the list of levels (1-based)
    in the order their generations ran."""
    runs, order = [], []
    total = 0

    def reached():
        return any(r.state(genes=False)["elite_fitness"] >= target for r in runs)

    def step(i):
        nonlocal total
        if total >= max_total_generations:
            return
        if len(runs) < i:
            runs.append(Run(g, set_ptr, set_vars, pop=n_base << (i - 1), seed=seed + i - 1,
                            rule=rule, flags=flags))
            if runs[-1].state(genes=False)["elite_fitness"] >= target:
                return
        runs[i - 1].generation()
        order.append(i)
        total += 1
        gens = runs[i - 1].state(genes=False)["generation"]
        if gens % c_ims == 0 and i < max_levels:
            step(i + 1)

    while total < max_total_generations and not (runs and reached()):
        step(1)
    return runs, order
