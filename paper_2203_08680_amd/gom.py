"""Thin ctypes binding of libgom (include/gom.h): the same entry-point names, argument
marshalling only.  Every step of the optimisation runs inside libgom's HIP kernels; PyTorch
provides the device arena (a uint8 tensor) and the stream.  There is no CPU fallback: if
libgom.so is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgom.so")

GOM_OK, GOM_E_ARG, GOM_E_GRAPH, GOM_E_RANGE, GOM_E_NOMEM, GOM_E_DEVICE, GOM_E_STATE = (
    0, -1, -2, -3, -4, -5, -6)
GOM_FOS_UNIVARIATE, GOM_FOS_NEIGHBOURHOOD = 0, 1
GOM_NEUTRAL_PAPER, GOM_NEUTRAL_ALWAYS = 0, 1
GOM_ORDER_RANDOM, GOM_ORDER_FIXED = 0, 1
GOM_MAX_POP = 64
GOM_SCHED_AUTO, GOM_SCHED_CLASS_LAUNCH, GOM_SCHED_RESIDENT, GOM_SCHED_BITSLICED = 0, 1, 2, 3

EXPORTED = (
    "gom_last_error", "gom_version", "mc_graph_load", "mc_graph_info", "mc_graph_csr",
    "mc_graph_free", "gom_fos_build", "gom_fos_from_sets", "gom_fos_build_lt", "gom_fos_info",
    "gom_fos_get",
    "gom_fos_free", "gom_colour", "gom_colour_get", "gom_state_bytes", "gom_state_init",
    "gom_state_init_static", "gom_state_reseed", "gom_generation", "gom_run_to_target", "gom_state_read", "gom_state_write",
    "gom_timing_enable", "gom_timing_read", "gom_state_set_schedule", "gom_state_get_schedule",
    "gom_state_autotune", "gom_debug_stop_after_class", "gom_state_hash", "gom_state_set_fi",
    "gom_state_get_fi", "gom_state_set_block", "gom_state_get_block", "gom_state_set_fused",
    "gom_state_get_fused", "gom_state_set_grid_limit", "gom_state_set_bitsliced_min_sets", "gom_state_set_staged", "gom_local_search",
    "gom_iterated_local_search",
    "gom_ims_bytes",
    "gom_ims_run",
    "gom_state_info", "gom_state_free", "gom_batch_bytes", "gom_batch_init", "gom_batch_run",
    "gom_batch_set_graph", "gom_batch_reseed", "gom_batch_timing_enable",
    "gom_batch_timing_read", "gom_batch_set_narrow", "gom_batch_get_narrow",
    "gom_batch_autotune", "gom_batch_set_class_launch", "gom_batch_get_class_launch",
    "gom_batch_set_class_positions", "gom_batch_set_class_bitsliced",
    "gom_batch_get_class_bitsliced",
    "gom_batch_state", "gom_batch_free", "gom_server_create", "gom_server_submit",
    "gom_server_step", "gom_server_results", "gom_server_info", "gom_server_free",
    "gom_server_set_large",
)


class GomError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgom error {code}: {msg}")
        self.code = code


class gom_result(C.Structure):
    _fields_ = [("generations", C.c_int32), ("reached", C.c_int32), ("best", C.c_int64),
                ("attempted", C.c_int64), ("evaluated", C.c_int64), ("accepted", C.c_int64)]


GOM_IMS_MAX_LEVELS = 8


class gom_ims_result(C.Structure):
    _fields_ = [("levels", C.c_int32), ("steps", C.c_int32), ("total_generations", C.c_int32),
                ("reached", C.c_int32), ("best", C.c_int64), ("best_level", C.c_int32),
                ("generations", C.c_int32 * GOM_IMS_MAX_LEVELS), ("evaluated", C.c_int64),
                ("accepted", C.c_int64)]


class gom_job_result(C.Structure):
    _fields_ = [("job", C.c_int64), ("generations", C.c_int32), ("reached", C.c_int32),
                ("best", C.c_int64), ("attempted", C.c_int64), ("evaluated", C.c_int64),
                ("accepted", C.c_int64), ("hash", C.c_uint64), ("submit_ms", C.c_double),
                ("admit_ms", C.c_double), ("done_ms", C.c_double), ("status", C.c_int32)]


_lib = None
_vp = C.c_void_p
_i32, _i64, _u64, _sz = C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
_P = C.POINTER


def lib() -> C.CDLL:
    """Load libgom.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_08680_amd.build "
                           "(or __graft_entry__.build()); there is no fallback path")
    # torch first: its bundled HIP runtime is then the one libgom binds to (same soname), so
    # the process holds a single runtime and the arena/stream handles are valid in libgom.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    sig = {
        "gom_last_error": (C.c_char_p, []),
        "gom_version": (C.c_int, []),
        "mc_graph_load": (C.c_int, [_i32, _i64, _vp, _vp, _vp, _P(_vp)]),
        "mc_graph_info": (C.c_int, [_vp, _P(_i32), _P(_i64), _P(_i64), _P(_i32)]),
        "mc_graph_csr": (C.c_int, [_vp, _vp, _vp, _vp]),
        "mc_graph_free": (None, [_vp]),
        "gom_fos_build": (C.c_int, [_vp, C.c_int, _P(_vp)]),
        "gom_fos_from_sets": (C.c_int, [_vp, _i32, _vp, _vp, _P(_vp)]),
        "gom_fos_info": (C.c_int, [_vp, _P(_i32), _P(_i64), _P(_i32)]),
        "gom_fos_get": (C.c_int, [_vp, _vp, _vp]),
        "gom_fos_free": (None, [_vp]),
        "gom_colour": (C.c_int, [_vp, _vp, _P(_i32)]),
        "gom_colour_get": (C.c_int, [_vp, _vp, _vp, _vp]),
        "gom_state_bytes": (C.c_int, [_vp, _vp, _i32, _P(_sz)]),
        "gom_state_init": (C.c_int, [_vp, _vp, _i32, _u64, C.c_int, C.c_int, _vp, _sz, _vp,
                                     _P(_vp)]),
        "gom_state_reseed": (C.c_int, [_vp, _u64, _vp]),
        "gom_generation": (C.c_int, [_vp, _vp]),
        "gom_run_to_target": (C.c_int, [_vp, _i64, _i32, _vp, _P(gom_result)]),
        "gom_state_read": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _P(_i64), _P(_i32), _vp]),
        "gom_state_write": (C.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _vp]),
        "gom_timing_enable": (C.c_int, [_vp, C.c_int]),
        "gom_timing_read": (C.c_int, [_vp, _P(C.c_double), _P(_i64)]),
        "gom_state_set_schedule": (C.c_int, [_vp, C.c_int]),
        "gom_state_get_schedule": (C.c_int, [_vp, _P(C.c_int)]),
        "gom_state_autotune": (C.c_int, [_vp, _i32, _vp, _P(C.c_int)]),
        "gom_fos_build_lt": (C.c_int, [_vp, _i32, _P(_vp)]),
        "gom_state_set_fi": (C.c_int, [_vp, C.c_int]),
        "gom_state_set_block": (C.c_int, [_vp, C.c_int]),
        "gom_ims_bytes": (C.c_int, [_vp, _vp, _i32, _i32, _P(_sz)]),
        "gom_ims_run": (C.c_int, [_vp, _vp, _i32, _i32, _i32, _u64, C.c_int, C.c_int, _i64,
                                  _i32, _vp, _sz, _vp, _vp, _vp]),
        "gom_state_get_block": (C.c_int, [_vp, _P(C.c_int)]),
        "gom_state_set_fused": (C.c_int, [_vp, C.c_int]),
        "gom_state_set_grid_limit": (C.c_int, [_vp, _i32]),
        "gom_state_set_bitsliced_min_sets": (C.c_int, [_vp, _i32]),
        "gom_state_set_staged": (C.c_int, [_vp, C.c_int]),
        "gom_state_get_fused": (C.c_int, [_vp, _P(C.c_int), _P(C.c_int)]),
        "gom_state_get_fi": (C.c_int, [_vp, _P(C.c_int)]),
        "gom_debug_stop_after_class": (C.c_int, [_vp, _i32, _vp]),
        "gom_state_hash": (C.c_int, [_vp, _vp, _P(C.c_uint64)]),
        "gom_state_info": (C.c_int, [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_i32), _P(_i32)]),
        "gom_state_free": (None, [_vp]),
        "gom_batch_bytes": (C.c_int, [_i32, _vp, _vp, _vp, _P(_sz)]),
        "gom_batch_init": (C.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, _vp, _sz,
                                     _vp, _P(_vp)]),
        "gom_batch_run": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
        "gom_batch_set_graph": (C.c_int, [_vp, C.c_int]),
        "gom_batch_reseed": (C.c_int, [_vp, _vp, _vp]),
        "gom_state_init_static": (C.c_int, [_vp, _vp, _i32, _u64, C.c_int, C.c_int, _vp,
                                            _P(_vp)]),
        "gom_batch_timing_enable": (C.c_int, [_vp, C.c_int]),
        "gom_batch_timing_read": (C.c_int, [_vp, _P(C.c_double), _P(_i64)]),
        "gom_batch_set_narrow": (C.c_int, [_vp, _i64, _vp]),
        "gom_batch_get_narrow": (C.c_int, [_vp, _P(_i64), _P(_i32)]),
        "gom_batch_autotune": (C.c_int, [_vp, _i32, _vp, _P(_i64), _P(_i64)]),
        "gom_batch_set_class_launch": (C.c_int, [_vp, _i64, _vp]),
        "gom_batch_get_class_launch": (C.c_int, [_vp, _P(_i64), _P(_i32), _P(_i32), _P(_i32)]),
        "gom_batch_set_class_positions": (C.c_int, [_vp, _i32]),
        "gom_batch_set_class_bitsliced": (C.c_int, [_vp, C.c_int, _vp]),
        "gom_batch_get_class_bitsliced": (C.c_int, [_vp, _P(C.c_int), _P(C.c_int)]),
        "gom_local_search": (C.c_int, [_vp, _i32, _vp, _P(_i32)]),
        "gom_iterated_local_search": (C.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _P(_i32)]),
        "gom_batch_state": (C.c_int, [_vp, _i32, _P(_vp)]),
        "gom_batch_free": (None, [_vp]),
        "gom_server_create": (C.c_int, [_vp, _sz, _i32, _i32, _P(_vp)]),
        "gom_server_submit": (C.c_int, [_vp, _vp, _vp, _i32, _u64, _i64, _i32, C.c_int, C.c_int,
                                        _P(_i64)]),
        "gom_server_step": (C.c_int, [_vp, _P(_i32), _P(_i32)]),
        "gom_server_set_large": (C.c_int, [_vp, _i64]),
        "gom_server_results": (C.c_int, [_vp, _vp, _i32, _P(_i32)]),
        "gom_server_info": (C.c_int, [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_sz)]),
        "gom_server_free": (None, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != GOM_OK:
        raise GomError(rc, lib().gom_last_error().decode())


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------------------------------
# Graph
# ------------------------------------------------------------------------------------------
class McGraph:
    """Owned mc_graph handle."""

    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mc_graph_free(self.handle)
            self.handle = None

    def info(self):
        n, m, W, dmax = _i32(), _i64(), _i64(), _i32()
        _check(lib().mc_graph_info(self.handle, C.byref(n), C.byref(m), C.byref(W),
                                   C.byref(dmax)))
        return {"n": n.value, "m": m.value, "total_weight": W.value, "max_degree": dmax.value}

    def csr(self):
        inf = self.info()
        rp = np.zeros(inf["n"] + 1, np.int32)
        col = np.zeros(2 * inf["m"], np.int32)
        w = np.zeros(2 * inf["m"], np.int32)
        _check(lib().mc_graph_csr(self.handle, _ptr(rp), _ptr(col), _ptr(w)))
        return rp, col, w


def mc_graph_load(n_vertices: int, u, v, w=None) -> McGraph:
    u = np.ascontiguousarray(u, np.int32)
    v = np.ascontiguousarray(v, np.int32)
    if u.shape != v.shape:
        raise ValueError("u and v differ in length")
    wa = None if w is None else np.ascontiguousarray(w, np.int32)
    if wa is not None and wa.shape != u.shape:
        raise ValueError("w differs in length from u")
    h = _vp()
    _check(lib().mc_graph_load(int(n_vertices), int(u.shape[0]), _ptr(u), _ptr(v),
                               None if wa is None else _ptr(wa), C.byref(h)))
    return McGraph(h.value)


# ------------------------------------------------------------------------------------------
# FOS and colouring
# ------------------------------------------------------------------------------------------
class GomFos:
    """Owned gom_fos handle."""

    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gom_fos_free(self.handle)
            self.handle = None

    def info(self):
        s, mem, mx = _i32(), _i64(), _i32()
        _check(lib().gom_fos_info(self.handle, C.byref(s), C.byref(mem), C.byref(mx)))
        return {"n_sets": s.value, "n_members": mem.value, "max_set": mx.value}

    def sets(self):
        inf = self.info()
        ptr = np.zeros(inf["n_sets"] + 1, np.int32)
        vars_ = np.zeros(inf["n_members"], np.int32)
        _check(lib().gom_fos_get(self.handle, _ptr(ptr), _ptr(vars_)))
        return ptr, vars_


def gom_fos_build(g: McGraph, kind: int) -> GomFos:
    h = _vp()
    _check(lib().gom_fos_build(g.handle, int(kind), C.byref(h)))
    return GomFos(h.value)


def gom_fos_build_lt(g: McGraph, bound: int = 0) -> GomFos:
    """Fixed linkage tree by UPGMA on |w| (bound > 0: bounded; 0: full tree)."""
    h = _vp()
    _check(lib().gom_fos_build_lt(g.handle, int(bound), C.byref(h)))
    return GomFos(h.value)


def gom_fos_from_sets(g: McGraph, ptr, vars_) -> GomFos:
    ptr = np.ascontiguousarray(ptr, np.int32)
    vars_ = np.ascontiguousarray(vars_, np.int32)
    h = _vp()
    _check(lib().gom_fos_from_sets(g.handle, int(ptr.shape[0] - 1), _ptr(ptr), _ptr(vars_),
                                   C.byref(h)))
    return GomFos(h.value)


def gom_colour(g: McGraph, f: GomFos) -> int:
    k = _i32()
    _check(lib().gom_colour(g.handle, f.handle, C.byref(k)))
    return k.value


def gom_colour_get(f: GomFos, k: int):
    """(colour_of_set, class_ptr, class_elems)."""
    S = f.info()["n_sets"]
    col = np.zeros(S, np.int32)
    cp = np.zeros(k + 1, np.int32)
    ce = np.zeros(S, np.int32)
    _check(lib().gom_colour_get(f.handle, _ptr(col), _ptr(cp), _ptr(ce)))
    return col, cp, ce


# ------------------------------------------------------------------------------------------
# State
# ------------------------------------------------------------------------------------------
def gom_state_bytes(g: McGraph, f: GomFos, pop: int) -> int:
    b = _sz()
    _check(lib().gom_state_bytes(g.handle, f.handle, int(pop), C.byref(b)))
    return b.value


class GomState:
    """Owned gom_state handle plus the torch tensor that holds its device arena."""

    def __init__(self, handle: int, arena, n: int, pop: int):
        self.handle = handle
        self.arena = arena
        self.n = n
        self.pop = pop

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_borrowed", False):
            self.handle = None
            return
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gom_state_free(self.handle)
            self.handle = None

    def info(self):
        n, pop, s, k, mx = _i32(), _i32(), _i32(), _i32(), _i32()
        _check(lib().gom_state_info(self.handle, C.byref(n), C.byref(pop), C.byref(s),
                                    C.byref(k), C.byref(mx)))
        return {"n": n.value, "pop": pop.value, "n_sets": s.value, "n_classes": k.value,
                "max_class": mx.value}


def gom_state_init(g: McGraph, f: GomFos, pop: int, seed: int,
                   neutral_rule: int = GOM_NEUTRAL_PAPER, class_order: int = GOM_ORDER_RANDOM,
                   device=None, stream=None) -> GomState:
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    nbytes = gom_state_bytes(g, f, pop)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-arena.data_ptr()) % 256
    h = _vp()
    with torch.cuda.device(dev):
        _check(lib().gom_state_init(g.handle, f.handle, int(pop), int(seed) & (2**64 - 1),
                                    int(neutral_rule), int(class_order),
                                    arena.data_ptr() + off, nbytes, _stream_handle(stream),
                                    C.byref(h)))
    return GomState(h.value, arena, g.info()["n"], pop)


GOM_STATIC_ARENA_BYTES = 64 << 20


def gom_state_init_static(g: McGraph, f: GomFos, pop: int, seed: int,
                          neutral_rule: int = GOM_NEUTRAL_PAPER,
                          class_order: int = GOM_ORDER_RANDOM, stream=None) -> GomState:
    """gom_state_init in the library's static device arena: no device memory is allocated.
    One such state per device at a time (free it before creating the next)."""
    h = _vp()
    _check(lib().gom_state_init_static(g.handle, f.handle, int(pop), int(seed) & (2**64 - 1),
                                       int(neutral_rule), int(class_order),
                                       _stream_handle(stream), C.byref(h)))
    return GomState(h.value, None, g.info()["n"], pop)


def gom_state_reseed(s: GomState, seed: int, stream=None):
    _check(lib().gom_state_reseed(s.handle, int(seed) & (2**64 - 1), _stream_handle(stream)))


def gom_generation(s: GomState, stream=None):
    _check(lib().gom_generation(s.handle, _stream_handle(stream)))


@dataclass
class RunResult:
    generations: int
    reached: bool
    best: int
    attempted: int
    evaluated: int
    accepted: int


def gom_run_to_target(s: GomState, target: int, max_generations: int,
                      stream=None) -> RunResult:
    r = gom_result()
    _check(lib().gom_run_to_target(s.handle, int(target), int(max_generations),
                                   _stream_handle(stream), C.byref(r)))
    return RunResult(r.generations, bool(r.reached), r.best, r.attempted, r.evaluated,
                     r.accepted)


def gom_state_read(s: GomState, genes: bool = True, stream=None) -> dict:
    G = np.zeros((s.pop, s.n), np.uint8) if genes else None
    f = np.zeros(s.pop, np.int64)
    E = np.zeros(s.n, np.uint8)
    fE, gen = _i64(), _i32()
    cnt = np.zeros(3, np.int64)
    _check(lib().gom_state_read(s.handle, _stream_handle(stream),
                                _ptr(G) if genes else None, _ptr(f), _ptr(E), C.byref(fE),
                                C.byref(gen), _ptr(cnt)))
    return {"genes": G, "fitness": f, "elite": E, "elite_fitness": fE.value,
            "generation": gen.value, "attempted": int(cnt[0]), "evaluated": int(cnt[1]),
            "accepted": int(cnt[2])}


def gom_state_write(s: GomState, genes, elite, elite_fitness: int, generation: int, counters,
                    stream=None):
    genes = np.ascontiguousarray(genes, np.uint8).reshape(s.pop, s.n)
    elite = np.ascontiguousarray(elite, np.uint8).reshape(s.n)
    cnt = np.ascontiguousarray(np.asarray(counters[:3], np.int64))
    _check(lib().gom_state_write(s.handle, _stream_handle(stream), _ptr(genes), _ptr(elite),
                                 int(elite_fitness), int(generation), _ptr(cnt)))


def gom_timing_enable(s: GomState, period: int = 1):
    """Time every `period`-th sweep launch with HIP events (0 = off)."""
    _check(lib().gom_timing_enable(s.handle, int(period)))


def gom_timing_read(s: GomState):
    """(summed class-sweep milliseconds, launches) since the last read."""
    ms, n = C.c_double(), _i64()
    _check(lib().gom_timing_read(s.handle, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def gom_state_set_schedule(s: GomState, schedule: int):
    _check(lib().gom_state_set_schedule(s.handle, int(schedule)))


def gom_state_get_schedule(s: GomState) -> int:
    v = C.c_int()
    _check(lib().gom_state_get_schedule(s.handle, C.byref(v)))
    return v.value


def gom_state_autotune(s: GomState, trial_generations: int = 3, stream=None) -> int:
    """Time each allowed schedule on real generations and keep the fastest; returns it."""
    v = C.c_int()
    _check(lib().gom_state_autotune(s.handle, int(trial_generations), _stream_handle(stream),
                                    C.byref(v)))
    return v.value


def gom_debug_stop_after_class(s: GomState, class_position: int, stream=None) -> None:
    """Run the next generation up to class-order position class_position and leave it open."""
    _check(lib().gom_debug_stop_after_class(s.handle, int(class_position),
                                            _stream_handle(stream)))


def gom_local_search(s: GomState, max_passes: int = 1 << 30, stream=None) -> int:
    """Colouring-parallel local search on the population (univariate FOS, between
    generations); returns the passes run."""
    n = _i32()
    _check(lib().gom_local_search(s.handle, int(max_passes), _stream_handle(stream),
                                  C.byref(n)))
    return int(n.value)


def gom_iterated_local_search(s: GomState, round0: int, rounds: int, flips: int,
                              max_passes: int = 1 << 30, stream=None) -> int:
    """Iterated local search (univariate FOS, between generations): rounds round0 ..
    round0 + rounds - 1 of drawn single-bit flips, the local search, and keep-unless-worse per
    solution; returns the search passes summed over the rounds."""
    n = _i32()
    _check(lib().gom_iterated_local_search(s.handle, int(round0), int(rounds), int(flips),
                                           int(max_passes), _stream_handle(stream),
                                           C.byref(n)))
    return int(n.value)


def gom_state_hash(s: GomState, stream=None) -> int:
    """64-bit hash of the state (genes, fitness, elitist, generation, counters)."""
    v = C.c_uint64()
    _check(lib().gom_state_hash(s.handle, _stream_handle(stream), C.byref(v)))
    return int(v.value)


def gom_state_set_fused(s: GomState, enabled: bool) -> None:
    """Whole generations of the bit-sliced schedule as one fused launch (when available)."""
    _check(lib().gom_state_set_fused(s.handle, 1 if enabled else 0))


def gom_state_get_fused(s: GomState):
    """(in use, available)."""
    e, a = C.c_int(), C.c_int()
    _check(lib().gom_state_get_fused(s.handle, C.byref(e), C.byref(a)))
    return bool(e.value), bool(a.value)


def gom_state_set_grid_limit(s: GomState, blocks: int) -> None:
    """Grid cap of the per-class sweeps (results do not depend on it)."""
    _check(lib().gom_state_set_grid_limit(s.handle, int(blocks)))


def gom_state_set_bitsliced_min_sets(s: GomState, sets: int) -> None:
    """Smallest class the bit-sliced schedule sweeps with the general bit-sliced sweep."""
    _check(lib().gom_state_set_bitsliced_min_sets(s.handle, int(sets)))


def gom_state_set_staged(s: GomState, enabled: bool) -> None:
    """Staged evaluation of small general sets in the class sweeps (results identical)."""
    _check(lib().gom_state_set_staged(s.handle, 1 if enabled else 0))


def gom_state_set_block(s: GomState, threads: int) -> None:
    """Block size of the class-launch sweeps (64..512, a multiple of 64)."""
    _check(lib().gom_state_set_block(s.handle, int(threads)))


def gom_state_get_block(s: GomState) -> int:
    v = C.c_int()
    _check(lib().gom_state_get_block(s.handle, C.byref(v)))
    return v.value


def gom_state_set_fi(s: GomState, enabled: bool = True) -> None:
    """Forced improvement after each generation's classes (off by default)."""
    _check(lib().gom_state_set_fi(s.handle, int(bool(enabled))))


def gom_state_get_fi(s: GomState) -> bool:
    v = C.c_int()
    _check(lib().gom_state_get_fi(s.handle, C.byref(v)))
    return bool(v.value)


def gom_version() -> int:
    return int(lib().gom_version())


# ------------------------------------------------------------------------------------------
# Convenience: one object for a whole instance set-up (graph + FOS + colouring)
# ------------------------------------------------------------------------------------------
class Instance:
    """A loaded graph with its coloured FOS, ready to create states from."""

    def __init__(self, n: int, u, v, w, fos_kind: int | None = None, sets=None,
                 lt_bound: int | None = None):
        """FOS: explicit `sets` (ptr, vars), a linkage tree when lt_bound is given (0 = full
        tree), else the built-in kind."""
        self.graph = mc_graph_load(n, u, v, w)
        if sets is not None:
            self.fos = gom_fos_from_sets(self.graph, sets[0], sets[1])
        elif lt_bound is not None:
            self.fos = gom_fos_build_lt(self.graph, lt_bound)
        else:
            self.fos = gom_fos_build(self.graph, fos_kind)
        self.k = gom_colour(self.graph, self.fos)
        inf = self.graph.info()
        self.n, self.m, self.total_weight = inf["n"], inf["m"], inf["total_weight"]

    def classes(self):
        return gom_colour_get(self.fos, self.k)

    def state(self, pop: int, seed: int, neutral_rule: int = GOM_NEUTRAL_PAPER,
              class_order: int = GOM_ORDER_RANDOM, device=None, stream=None) -> GomState:
        return gom_state_init(self.graph, self.fos, pop, seed, neutral_rule, class_order,
                              device, stream)


# ------------------------------------------------------------------------------------------
# Batches of independent instances
# ------------------------------------------------------------------------------------------
class GomBatch:
    """Owned gom_batch handle plus the torch tensor holding its device arena."""

    def __init__(self, handle: int, arena, instances, pops):
        self.handle = handle
        self.arena = arena
        self.instances = instances  # keep the graphs/FOS alive with the batch
        self.pops = list(pops)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gom_batch_free(self.handle)
            self.handle = None

    def state(self, index: int) -> "GomState":
        h = _vp()
        _check(lib().gom_batch_state(self.handle, int(index), C.byref(h)))
        st = GomState.__new__(GomState)
        st.handle, st.arena, st.n, st.pop = h.value, None, self.instances[index].n, \
            self.pops[index]
        st._borrowed = True
        return st


def _handles(objs):
    arr = (C.c_void_p * len(objs))(*[o.handle for o in objs])
    return arr


def gom_batch_bytes(instances, pops) -> int:
    b = _sz()
    pops = np.ascontiguousarray(pops, np.int32)
    _check(lib().gom_batch_bytes(len(instances), _handles([x.graph for x in instances]),
                                 _handles([x.fos for x in instances]), _ptr(pops), C.byref(b)))
    return b.value


def gom_batch_init(instances, pops, seeds, targets, neutral_rule: int = GOM_NEUTRAL_PAPER,
                   class_order: int = GOM_ORDER_RANDOM, device=None, stream=None) -> GomBatch:
    """instances: list of Instance (graph + coloured FOS)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    pops = np.ascontiguousarray(pops, np.int32)
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    targets = np.ascontiguousarray(targets, np.int64)
    nbytes = gom_batch_bytes(instances, pops)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-arena.data_ptr()) % 256
    h = _vp()
    with torch.cuda.device(dev):
        _check(lib().gom_batch_init(len(instances), _handles([x.graph for x in instances]),
                                    _handles([x.fos for x in instances]), _ptr(pops),
                                    _ptr(seeds), _ptr(targets), int(neutral_rule),
                                    int(class_order), arena.data_ptr() + off, nbytes,
                                    _stream_handle(stream), C.byref(h)))
    return GomBatch(h.value, arena, list(instances), pops)


def gom_batch_run(b: GomBatch, max_generations: int, stream=None):
    """(list of RunResult, numpy array of time-to-target milliseconds, -1 if not reached)."""
    n = len(b.instances)
    res = (gom_result * n)()
    tt = np.zeros(n, np.float64)
    _check(lib().gom_batch_run(b.handle, int(max_generations), _stream_handle(stream), res,
                               _ptr(tt)))
    out = [RunResult(r.generations, bool(r.reached), r.best, r.attempted, r.evaluated,
                     r.accepted) for r in res]
    return out, tt


def gom_batch_reseed(b: GomBatch, seeds, stream=None) -> None:
    """Fresh initial populations for every instance (seeds[b]); the step budget restarts."""
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    if seeds.shape[0] != len(b.instances):
        raise ValueError("gom_batch_reseed: one seed per instance")
    _check(lib().gom_batch_reseed(b.handle, _ptr(seeds), _stream_handle(stream)))


def gom_batch_timing_enable(b: GomBatch, enabled: bool = True) -> None:
    _check(lib().gom_batch_timing_enable(b.handle, 1 if enabled else 0))


def gom_batch_timing_read(b: GomBatch):
    """(summed sweep milliseconds, timed sweep launches) since the previous read."""
    ms, n = C.c_double(), _i64()
    _check(lib().gom_batch_timing_read(b.handle, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def gom_batch_set_narrow(b: GomBatch, narrow_max_n: int, stream=None) -> None:
    """Instances with at most narrow_max_n vertices sweep with 256-thread blocks, larger ones
    with 1024 (-1: all 1024)."""
    _check(lib().gom_batch_set_narrow(b.handle, int(narrow_max_n), _stream_handle(stream)))


def gom_batch_get_narrow(b: GomBatch):
    """(block-size threshold, sweep launches per step)."""
    t, n = _i64(), _i32()
    _check(lib().gom_batch_get_narrow(b.handle, C.byref(t), C.byref(n)))
    return t.value, n.value


def gom_batch_autotune(b: GomBatch, trial_steps: int = 2, stream=None):
    """Time trial generation steps under each class-launch threshold, then each block-size
    threshold, and keep the fastest; returns (block-size threshold, class-launch threshold).
    The trial steps are ordinary steps of the run."""
    c, m = _i64(), _i64()
    _check(lib().gom_batch_autotune(b.handle, int(trial_steps), _stream_handle(stream),
                                    C.byref(c), C.byref(m)))
    return c.value, m.value


def gom_batch_set_class_launch(b: GomBatch, min_n: int, stream=None) -> None:
    """Eligible instances with at least min_n vertices take the batched class launches
    (-1: none)."""
    _check(lib().gom_batch_set_class_launch(b.handle, int(min_n), _stream_handle(stream)))


def gom_batch_get_class_launch(b: GomBatch):
    """(threshold, instances selected, class launches per step, positions per wave)."""
    m, n, k, w = _i64(), _i32(), _i32(), _i32()
    _check(lib().gom_batch_get_class_launch(b.handle, C.byref(m), C.byref(n), C.byref(k),
                                            C.byref(w)))
    return m.value, n.value, k.value, w.value


def gom_batch_set_class_bitsliced(b: GomBatch, enabled: bool, stream=None) -> None:
    """Bit-sliced form of the batched class launches (on by default where available)."""
    _check(lib().gom_batch_set_class_bitsliced(b.handle, 1 if enabled else 0,
                                               _stream_handle(stream)))


def gom_batch_get_class_bitsliced(b: GomBatch):
    """(in use, available) of the bit-sliced form of the batched class launches."""
    en, av = C.c_int(), C.c_int()
    _check(lib().gom_batch_get_class_bitsliced(b.handle, C.byref(en), C.byref(av)))
    return bool(en.value), bool(av.value)


def gom_batch_set_class_positions(b: GomBatch, positions_per_wave: int) -> None:
    """Consecutive class positions per wave of the class launches (1..8)."""
    _check(lib().gom_batch_set_class_positions(b.handle, int(positions_per_wave)))


def gom_batch_set_graph(b: GomBatch, enabled: bool = True) -> None:
    """Run gom_batch_run's chunks of 4 steps as a captured HIP graph (default) or as separate
    launches."""
    _check(lib().gom_batch_set_graph(b.handle, 1 if enabled else 0))


# ------------------------------------------------------------------------------------------
# Serving loop
# ------------------------------------------------------------------------------------------
class GomServer:
    """Owned gom_server handle, its device arena (a torch tensor) and the instances of the
    jobs submitted to it (kept alive until their results have been taken)."""

    def __init__(self, arena_bytes: int, max_jobs: int = 256, streams: int = 4, device=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=dev)
        off = (-self.arena.data_ptr()) % 256
        self._jobs = {}
        h = _vp()
        torch.cuda.synchronize(dev)  # the arena's allocation is ordered before the server's work
        with torch.cuda.device(dev):
            _check(lib().gom_server_create(self.arena.data_ptr() + off, int(arena_bytes),
                                           int(max_jobs), int(streams), C.byref(h)))
        self.handle = h.value

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gom_server_free(self.handle)
            self.handle = None

    def submit(self, inst: "Instance", pop: int, seed: int, target: int, max_generations: int,
               neutral_rule: int = GOM_NEUTRAL_PAPER,
               class_order: int = GOM_ORDER_RANDOM) -> int:
        j = _i64()
        _check(lib().gom_server_submit(self.handle, inst.graph.handle, inst.fos.handle,
                                       int(pop), int(seed) & (2**64 - 1), int(target),
                                       int(max_generations), int(neutral_rule),
                                       int(class_order), C.byref(j)))
        self._jobs[j.value] = inst
        return j.value

    def set_large(self, large_min_n: int) -> None:
        """Jobs with at least large_min_n vertices run one at a time on the first stream
        (-1: no size-aware placement)."""
        _check(lib().gom_server_set_large(self.handle, int(large_min_n)))

    def step(self):
        """Admit what fits, retire or continue finished chunks; returns (active, queued)
        without waiting for running chunks."""
        a, q = _i32(), _i32()
        _check(lib().gom_server_step(self.handle, C.byref(a), C.byref(q)))
        return a.value, q.value

    def results(self, capacity: int = 1024):
        buf = (gom_job_result * capacity)()
        n = _i32()
        _check(lib().gom_server_results(self.handle, buf, int(capacity), C.byref(n)))
        out = []
        for r in buf[:n.value]:
            out.append({"job": r.job, "generations": r.generations, "reached": bool(r.reached),
                        "best": r.best, "attempted": r.attempted, "evaluated": r.evaluated,
                        "accepted": r.accepted, "hash": r.hash, "submit_ms": r.submit_ms,
                        "admit_ms": r.admit_ms, "done_ms": r.done_ms, "status": r.status})
            self._jobs.pop(r.job, None)
        return out

    def info(self):
        a, q, b, fb = _i32(), _i32(), _i32(), _sz()
        _check(lib().gom_server_info(self.handle, C.byref(a), C.byref(q), C.byref(b),
                                     C.byref(fb)))
        return {"active": a.value, "queued": q.value, "streams": b.value,
                "free_bytes": fb.value}


# ------------------------------------------------------------------------------------------
# Interleaved multi-start scheme
# ------------------------------------------------------------------------------------------
def gom_ims_run(inst: "Instance", n_base: int, c_ims: int, max_levels: int, seed: int,
                target: int, max_total_generations: int, neutral_rule: int = GOM_NEUTRAL_PAPER,
                forced_improvement: bool = False, device=None, stream=None):
    """(result dict, list of the levels' GomState, None for levels not created)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    b = _sz()
    _check(lib().gom_ims_bytes(inst.graph.handle, inst.fos.handle, int(n_base),
                               int(max_levels), C.byref(b)))
    arena = torch.empty(b.value + 256, dtype=torch.uint8, device=dev)
    off = (-arena.data_ptr()) % 256
    res = gom_ims_result()
    hs = (C.c_void_p * int(max_levels))()
    with torch.cuda.device(dev):
        _check(lib().gom_ims_run(inst.graph.handle, inst.fos.handle, int(n_base), int(c_ims),
                                 int(max_levels), int(seed) & (2**64 - 1), int(neutral_rule),
                                 int(bool(forced_improvement)), int(target),
                                 int(max_total_generations), arena.data_ptr() + off, b.value,
                                 _stream_handle(stream), C.byref(res), hs))
    states = []
    for lvl in range(int(max_levels)):
        h = hs[lvl]
        if not h:
            states.append(None)
            continue
        st = GomState.__new__(GomState)
        st.handle, st.arena, st.n, st.pop = h, arena, inst.n, n_base << lvl
        st._borrowed = False
        states.append(st)
    out = {"levels": res.levels, "steps": res.steps, "total_generations": res.total_generations,
           "reached": bool(res.reached), "best": res.best, "best_level": res.best_level,
           "generations": list(res.generations)[:res.levels], "evaluated": res.evaluated,
           "accepted": res.accepted}
    return out, states
