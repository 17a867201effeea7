"""ctypes binding of libcoralai.so: one Python function per C entry point,
same names, argument marshalling only.  Every step of the update runs in the
HIP library; PyTorch only supplies device memory (the caller-owned arenas)
and streams.  There is no CPU fallback: if the library is missing the import
of this module's functions raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoralai.so")

CORALAI_FP32 = 0
CORALAI_BF16 = 1
CORALAI_OK = 0
CORALAI_E_INVALID = -1
CORALAI_E_NOMEM = -2
CORALAI_E_GENOME = -3
CORALAI_E_NUMERIC = -4
CORALAI_E_HIP = -5
CORALAI_E_BUSY = -6
ERR_GENOME_RANGE, ERR_GENOME_UNSET, ERR_LEDGER, ERR_NONFINITE, ERR_MASS = 1, 2, 4, 8, 16
WORLD_ENERGY_FLOWS = 1

EXPORTED = [
    "coralai_world_bytes", "coralai_world_create", "coralai_world_destroy", "coralai_set_state",
    "coralai_get_state", "coralai_set_genomes", "coralai_get_genomes", "coralai_step",
    "coralai_radiate", "coralai_sync", "coralai_get_stats", "coralai_batch_bytes",
    "coralai_batch_create", "coralai_batch_set_worlds", "coralai_batch_step", "coralai_batch_sync",
    "coralai_batch_destroy", "coralai_autotune", "coralai_set_tuning", "coralai_last_error",
    "coralai_version", "coralai_debug_buckets", "coralai_debug_actuators",
    "coralai_debug_set_weights", "coralai_debug_get_weights", "coralai_debug_physics",
    "coralai_set_profiling", "coralai_get_profile", "coralai_batch_autotune",
    "coralai_batch_set_tuning", "coralai_debug_set_act_segments",
    "coralai_debug_set_weights_noalloc", "coralai_set_daylight", "coralai_get_energy_ledger",
    "coralai_set_physics_variant", "coralai_get_lineage", "coralai_get_births",
    "coralai_genetic_distance", "coralai_merge", "coralai_set_step_count", "coralai_set_genome_ext",
    "coralai_get_genome_ext", "coralai_set_structural_mutation",
]
# coralai_genome_ext (46 words): masks, then direct-connection, added-node in and out weights
GENOME_EXT_DTYPE = np.dtype([("conn_mask", np.uint32), ("node_mask", np.uint32), ("node_act", np.uint32),
                             ("reserved", np.uint32), ("conn_w", np.float32, (10,)),
                             ("node_in", np.float32, (16,)), ("node_out", np.float32, (16,))])
assert GENOME_EXT_DTYPE.itemsize == 46 * 4
PHASES = ["bucket", "act", "physics", "finalize", "radiate"]


class coralai_world_desc(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32), ("n_weight_layers", ct.c_int32),
                ("hidden", ct.c_int32), ("genome_capacity", ct.c_int32), ("precision", ct.c_int32),
                ("seed", ct.c_uint64), ("rho_invest", ct.c_float), ("rho_liquidate", ct.c_float),
                ("kappa_flow", ct.c_float), ("flags", ct.c_int32)]


class coralai_stats(ct.Structure):
    _fields_ = [("mass_quanta", ct.c_int64), ("mass_fp64", ct.c_double), ("steps", ct.c_int64),
                ("live_genomes", ct.c_int32), ("takeovers", ct.c_int32), ("hits", ct.c_int32),
                ("dropped_hits", ct.c_int32), ("error_word", ct.c_uint32), ("reserved", ct.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CoralaiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("coralai error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib() -> ct.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcoralai.so is not built (run paper_2406_09654_amd/build.py): %s"
                              % LIB_PATH)
        L = ct.CDLL(LIB_PATH)
        P, I32, U64, SZ = ct.c_void_p, ct.c_int32, ct.c_uint64, ct.c_size_t
        D, S = ct.POINTER(coralai_world_desc), ct.POINTER(coralai_stats)
        sig = {
            "coralai_world_bytes": (SZ, [D]),
            "coralai_world_create": (ct.c_int, [D, P, SZ, P, ct.POINTER(P)]),
            "coralai_world_destroy": (ct.c_int, [P]),
            "coralai_set_state": (ct.c_int, [P, P, P, P, P, P, ct.c_int]),
            "coralai_get_state": (ct.c_int, [P, P, P, P, P, P, ct.c_int]),
            "coralai_set_genomes": (ct.c_int, [P, I32, P, P]),
            "coralai_get_genomes": (ct.c_int, [P, I32, P, P]),
            "coralai_step": (ct.c_int, [P, I32, S]),
            "coralai_radiate": (ct.c_int, [P, ct.c_double, ct.c_float, U64, S]),
            "coralai_sync": (ct.c_int, [P]),
            "coralai_get_stats": (ct.c_int, [P, S]),
            "coralai_batch_bytes": (SZ, [I32]),
            "coralai_batch_create": (ct.c_int, [I32, P, SZ, P, ct.POINTER(P)]),
            "coralai_batch_set_worlds": (ct.c_int, [P, ct.POINTER(P), I32]),
            "coralai_batch_step": (ct.c_int, [P, I32]),
            "coralai_batch_sync": (ct.c_int, [P]),
            "coralai_batch_destroy": (ct.c_int, [P]),
            "coralai_autotune": (ct.c_int, [P, ct.POINTER(I32), ct.POINTER(I32), ct.POINTER(I32)]),
            "coralai_set_tuning": (ct.c_int, [P, I32, I32, I32]),
            "coralai_batch_autotune": (ct.c_int, [P, ct.POINTER(I32), ct.POINTER(I32), ct.POINTER(I32)]),
            "coralai_batch_set_tuning": (ct.c_int, [P, I32, I32, I32]),
            "coralai_last_error": (ct.c_char_p, []),
            "coralai_version": (ct.c_char_p, []),
            "coralai_debug_buckets": (ct.c_int, [P, P, P, P]),
            "coralai_debug_actuators": (ct.c_int, [P, P]),
            "coralai_debug_set_weights": (ct.c_int, [P, I32, P]),
            "coralai_debug_get_weights": (ct.c_int, [P, I32, P]),
            "coralai_debug_physics": (ct.c_int, [P, P, P, P]),
            "coralai_debug_set_act_segments": (ct.c_int, [P, I32]),
            "coralai_debug_set_weights_noalloc": (ct.c_int, [P, I32, P]),
            "coralai_set_daylight": (ct.c_int, [P, I32, ct.c_int64, I32]),
            "coralai_get_energy_ledger": (ct.c_int, [P, P, P, P, P]),
            "coralai_set_physics_variant": (ct.c_int, [P, I32, ct.c_float]),
            "coralai_get_lineage": (ct.c_int, [P, I32, P, P, P, P]),
            "coralai_get_births": (ct.c_int, [P, I32, P, P, P, P, P]),
            "coralai_merge": (ct.c_int, [P, ct.c_double, U64, S]),
            "coralai_set_step_count": (ct.c_int, [P, ct.c_int64]),
            "coralai_set_genome_ext": (ct.c_int, [P, I32, P, P]),
            "coralai_get_genome_ext": (ct.c_int, [P, I32, P, P]),
            "coralai_set_structural_mutation": (ct.c_int, [P, ct.c_double, ct.c_double]),
            "coralai_genetic_distance": (ct.c_int, [P, I32, P, I32, P, ct.c_float, ct.c_float, ct.c_float, P]),
            "coralai_set_profiling": (ct.c_int, [P, ct.c_int]),
            "coralai_get_profile": (ct.c_int, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != CORALAI_OK:
        raise CoralaiError(rc, coralai_last_error())
    return rc


def _host(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ct.c_void_p)


# ---------------------------------------------------------------- 1:1 entry points

def coralai_last_error() -> str:
    return lib().coralai_last_error().decode()


def coralai_version() -> str:
    return lib().coralai_version().decode()


def coralai_world_bytes(desc: coralai_world_desc) -> int:
    return int(lib().coralai_world_bytes(ct.byref(desc)))


def coralai_world_create(desc: coralai_world_desc, arena_ptr: int, arena_bytes: int,
                         stream_ptr: int) -> ct.c_void_p:
    h = ct.c_void_p()
    _check(lib().coralai_world_create(ct.byref(desc), ct.c_void_p(arena_ptr), arena_bytes,
                                      ct.c_void_p(stream_ptr), ct.byref(h)))
    return h


def coralai_world_destroy(h) -> None:
    _check(lib().coralai_world_destroy(h))


def coralai_set_state(h, E, I, C, G, R, on_device: int = 0) -> None:
    ptrs = [_host(a) if not on_device else ct.c_void_p(a) for a in (E, I, C, G, R)]
    _check(lib().coralai_set_state(h, *ptrs, on_device))


def coralai_get_state(h, E, I, C, G, R, on_device: int = 0) -> None:
    ptrs = [None if a is None else (_host(a) if not on_device else ct.c_void_p(a))
            for a in (E, I, C, G, R)]
    _check(lib().coralai_get_state(h, *ptrs, on_device))


def coralai_set_genomes(h, slots: np.ndarray, params: np.ndarray) -> None:
    _check(lib().coralai_set_genomes(h, int(slots.size), _host(slots), _host(params)))


def coralai_get_genomes(h, slots: np.ndarray, out: np.ndarray) -> None:
    _check(lib().coralai_get_genomes(h, int(slots.size), _host(slots), _host(out)))


def coralai_step(h, n_steps: int, stats: coralai_stats | None = None) -> None:
    _check(lib().coralai_step(h, n_steps, ct.byref(stats) if stats is not None else None))


def coralai_radiate(h, rate: float, sigma: float, step_index: int,
                    stats: coralai_stats | None = None) -> None:
    _check(lib().coralai_radiate(h, rate, sigma, step_index,
                                 ct.byref(stats) if stats is not None else None))


def coralai_merge(h, rate: float, step_index: int, stats: coralai_stats | None = None) -> None:
    _check(lib().coralai_merge(h, rate, step_index, ct.byref(stats) if stats is not None else None))


def coralai_set_genome_ext(h, slots: np.ndarray, ext: np.ndarray) -> None:
    assert ext.dtype == GENOME_EXT_DTYPE and ext.size == slots.size
    _check(lib().coralai_set_genome_ext(h, int(slots.size), _host(slots), _host(ext)))


def coralai_get_genome_ext(h, slots: np.ndarray, out: np.ndarray) -> None:
    assert out.dtype == GENOME_EXT_DTYPE and out.size == slots.size
    _check(lib().coralai_get_genome_ext(h, int(slots.size), _host(slots), _host(out)))


def coralai_set_structural_mutation(h, p_conn: float, p_node: float) -> None:
    _check(lib().coralai_set_structural_mutation(h, p_conn, p_node))


def coralai_set_step_count(h, steps: int) -> None:
    _check(lib().coralai_set_step_count(h, steps))


def coralai_set_daylight(h, period: int, inject_quanta: int, remove_num: int) -> None:
    _check(lib().coralai_set_daylight(h, period, inject_quanta, remove_num))


def coralai_set_physics_variant(h, explore_mode: int, kappa_energy: float) -> None:
    _check(lib().coralai_set_physics_variant(h, explore_mode, kappa_energy))


def coralai_get_lineage(h, slots: np.ndarray, parents: np.ndarray, parents2: np.ndarray,
                        births: np.ndarray) -> None:
    _check(lib().coralai_get_lineage(h, int(slots.size), _host(slots), _host(parents), _host(parents2),
                                     _host(births)))


def coralai_get_births(h, max_births: int, cells, parents, parents2, slots) -> int:
    n = ct.c_int32(0)
    _check(lib().coralai_get_births(h, max_births, _host(cells), _host(parents), _host(parents2),
                                    _host(slots), ct.byref(n)))
    return int(n.value)


def coralai_genetic_distance(h, slots_a: np.ndarray, slots_b: np.ndarray, c1: float, c2: float, c3: float,
                             out_ptr: int) -> None:
    _check(lib().coralai_genetic_distance(h, int(slots_a.size), _host(slots_a), int(slots_b.size),
                                          _host(slots_b), c1, c2, c3, ct.c_void_p(out_ptr)))


def coralai_get_energy_ledger(h) -> dict:
    v = np.zeros(4, np.int64)
    p = [ct.c_void_p(v.ctypes.data + 8 * k) for k in range(4)]
    _check(lib().coralai_get_energy_ledger(h, *p))
    return {"injected_last": int(v[0]), "removed_last": int(v[1]),
            "injected_total": int(v[2]), "removed_total": int(v[3])}


def coralai_sync(h) -> None:
    _check(lib().coralai_sync(h))


def coralai_get_stats(h, stats: coralai_stats) -> None:
    _check(lib().coralai_get_stats(h, ct.byref(stats)))


def coralai_autotune(h) -> tuple[int, int, int]:
    a, w, p = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(lib().coralai_autotune(h, ct.byref(a), ct.byref(w), ct.byref(p)))
    return a.value, w.value, p.value


def coralai_set_tuning(h, act_cells: int, act_waves: int, phys_tile: int) -> None:
    _check(lib().coralai_set_tuning(h, act_cells, act_waves, phys_tile))


def coralai_batch_autotune(b) -> tuple[int, int, int]:
    a, w, p = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(lib().coralai_batch_autotune(b, ct.byref(a), ct.byref(w), ct.byref(p)))
    return a.value, w.value, p.value


def coralai_batch_set_tuning(b, act_cells: int, act_waves: int, phys_tile: int) -> None:
    _check(lib().coralai_batch_set_tuning(b, act_cells, act_waves, phys_tile))


def coralai_batch_bytes(max_worlds: int) -> int:
    return int(lib().coralai_batch_bytes(max_worlds))


def coralai_batch_create(max_worlds: int, arena_ptr: int, arena_bytes: int, stream_ptr: int):
    h = ct.c_void_p()
    _check(lib().coralai_batch_create(max_worlds, ct.c_void_p(arena_ptr), arena_bytes,
                                      ct.c_void_p(stream_ptr), ct.byref(h)))
    return h


def coralai_batch_set_worlds(b, handles) -> None:
    arr = (ct.c_void_p * max(1, len(handles)))(*[x.value for x in handles])
    _check(lib().coralai_batch_set_worlds(b, arr, len(handles)))


def coralai_batch_step(b, n_steps: int) -> None:
    _check(lib().coralai_batch_step(b, n_steps))


def coralai_batch_sync(b) -> None:
    _check(lib().coralai_batch_sync(b))


def coralai_batch_destroy(b) -> None:
    _check(lib().coralai_batch_destroy(b))


def coralai_debug_buckets(h, counts, offsets, perm) -> None:
    _check(lib().coralai_debug_buckets(h, _host(counts), _host(offsets), _host(perm)))


def coralai_debug_actuators(h, act) -> None:
    _check(lib().coralai_debug_actuators(h, _host(act)))


def coralai_debug_set_weights(h, slot: int, flat) -> None:
    _check(lib().coralai_debug_set_weights(h, slot, _host(flat)))


def coralai_debug_set_weights_noalloc(h, slot: int, flat) -> None:
    _check(lib().coralai_debug_set_weights_noalloc(h, slot, _host(flat)))


def coralai_debug_get_weights(h, slot: int, flat) -> None:
    _check(lib().coralai_debug_get_weights(h, slot, _host(flat)))


def coralai_debug_physics(h, i1, flows8, explore) -> None:
    _check(lib().coralai_debug_physics(h, _host(i1), _host(flows8), _host(explore)))


def coralai_debug_set_act_segments(h, n_segments: int) -> None:
    _check(lib().coralai_debug_set_act_segments(h, n_segments))


def coralai_set_profiling(h, on: bool) -> None:
    _check(lib().coralai_set_profiling(h, 1 if on else 0))


def coralai_get_profile(h) -> dict:
    ms = np.zeros(len(PHASES), np.float64)
    n = np.zeros(len(PHASES), np.int64)
    _check(lib().coralai_get_profile(h, _host(ms), _host(n)))
    return {PHASES[k]: (float(ms[k]), int(n[k])) for k in range(len(PHASES))}
