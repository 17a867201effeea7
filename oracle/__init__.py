"""FP64 CPU oracle of the Coralai per-step update -- test infrastructure only.

Only the tests, the smoke check and the bench's CPU-baseline leg import this
package.  It wraps the plain C oracle (coralai_oracle.c) through ctypes and
shares no code with the HIP library: the two meet only in the seeded inputs
of the ``workloads`` package.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "coralai_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
N_PARAM = 56
N_IN = 54
N_OUT = 14
# near-tie report per target: logit gap, |v - I1|, v_win - v_second, magnitude, decided flag
N_MARGIN = 5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP over cells)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(ct.Structure):
    _fields_ = [("width", ct.c_int32), ("height", ct.c_int32),
                ("n_weight_layers", ct.c_int32), ("hidden", ct.c_int32),
                ("rho_invest", ct.c_double), ("rho_liquidate", ct.c_double),
                ("kappa_flow", ct.c_double), ("day_period", ct.c_int32),
                ("night_num", ct.c_int32), ("day_inject", ct.c_int64),
                ("cycle_step", ct.c_int64), ("explore_mode", ct.c_int32),
                ("pad_desc", ct.c_int32), ("kappa_energy", ct.c_double)]


class Record(ct.Structure):
    _fields_ = [("e1", ct.c_int64), ("i1", ct.c_int64), ("flow", ct.c_int64 * 8),
                ("explore_dir", ct.c_int32), ("explore_pos", ct.c_int32),
                ("logit_gap", ct.c_double), ("runner_dir", ct.c_int32), ("exact", ct.c_int32),
                ("eflow", ct.c_int64 * 8)]


RECORD_DTYPE = np.dtype([("e1", np.int64), ("i1", np.int64), ("flow", np.int64, (8,)),
                         ("explore_dir", np.int32), ("explore_pos", np.int32),
                         ("logit_gap", np.float64), ("runner_dir", np.int32),
                         ("exact", np.int32), ("eflow", np.int64, (8,))])
assert RECORD_DTYPE.itemsize == ct.sizeof(Record)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ct.CDLL(_LIB)
        P = ct.c_void_p
        L.orc_net_size.restype = ct.c_int64
        L.orc_net_size.argtypes = [P]
        L.orc_cppn.argtypes = [P] + [ct.c_double] * 4 + [P]
        L.orc_cppn_to_net.argtypes = [P, P, P]
        L.orc_nets_for.argtypes = [P, ct.c_int64, P, P]
        L.orc_sense.argtypes = [P, P, P, P, P, ct.c_int64, P]
        L.orc_forward.argtypes = [P, P, P, P]
        L.orc_kernel_dir.restype = ct.c_int
        L.orc_kernel_dir.argtypes = [ct.c_int, ct.c_int]
        L.orc_step_rows.restype = ct.c_int64
        L.orc_step_rows.argtypes = [P, P, P, P, P, P, P, ct.c_int32, ct.c_int32, ct.c_int32,
                                    P, P, P, P, P, P, P, P, P]
        L.orc_physics_from_records.restype = ct.c_int64
        L.orc_physics_from_records.argtypes = [P] * 9
        L.orc_buckets.restype = ct.c_int
        L.orc_buckets.argtypes = [ct.c_int64, P, ct.c_int32, P, P, P]
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_uniform.restype = ct.c_double
        L.orc_uniform.argtypes = [ct.c_uint64]
        L.orc_mutation_normals.argtypes = [ct.c_uint64, ct.c_uint64, ct.c_uint64, P]
        L.orc_hit_threshold.restype = ct.c_uint64
        L.orc_hit_threshold.argtypes = [ct.c_double]
        L.orc_radiate.restype = ct.c_int64
        L.orc_radiate.argtypes = [ct.c_int64, P, ct.c_int32, P, ct.c_uint64, ct.c_uint64,
                                  ct.c_uint64, ct.c_double, P, P, ct.c_int64, P]
        L.orc_merge.restype = ct.c_int64
        L.orc_merge.argtypes = [ct.POINTER(_Desc), P, P, ct.c_int32, P, ct.c_uint64, ct.c_uint64,
                                ct.c_uint64, P, P, P, P, ct.c_int64, P]
        L.orc_cppn_to_net_x.restype = None
        L.orc_cppn_to_net_x.argtypes = [ct.POINTER(_Desc), P, P, P]
        L.orc_nets_for_x.restype = None
        L.orc_nets_for_x.argtypes = [ct.POINTER(_Desc), ct.c_int64, P, P, P]
        L.orc_radiate_x.restype = ct.c_int64
        L.orc_radiate_x.argtypes = [ct.c_int64, P, ct.c_int32, P, P, ct.c_uint64, ct.c_uint64, ct.c_uint64,
                                    ct.c_double, ct.c_uint64, ct.c_uint64, P, P, ct.c_int64, P]
        L.orc_merge_x.restype = ct.c_int64
        L.orc_merge_x.argtypes = [ct.POINTER(_Desc), P, P, ct.c_int32, P, P, ct.c_uint64, ct.c_uint64,
                                  ct.c_uint64, P, P, P, P, ct.c_int64, P]
        L.orc_genetic_distance_x.restype = ct.c_double
        L.orc_genetic_distance_x.argtypes = [P, P, P, P, ct.c_double, ct.c_double, ct.c_double]
        L.orc_genetic_distance.restype = ct.c_double
        L.orc_genetic_distance.argtypes = [P, P, ct.c_double]
        L.orc_mass.restype = ct.c_int64
        L.orc_mass.argtypes = [ct.c_int64, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


@dataclass
class Desc:
    width: int
    height: int
    n_weight_layers: int = 2
    hidden: int = 32
    rho_invest: float = 0.1
    rho_liquidate: float = 0.1
    kappa_flow: float = 0.25
    day_period: int = 0          # day / night cycle: 0 = none
    night_num: int = 0
    day_inject: int = 0
    cycle_step: int = 0          # steps completed before the step
    explore_mode: int = 0        # 0: softmax split of the exploration budget, 1: all to the maximal
    kappa_energy: float = 0.0    # > 0: energy moves along the flow directions

    @classmethod
    def from_spec(cls, spec) -> "Desc":
        # the constants are float32 in the world descriptor; the oracle widens
        # exactly those values to FP64
        f = lambda v: float(np.float32(v))
        return cls(spec.width, spec.height, spec.n_weight_layers, spec.hidden,
                   f(spec.rho_invest), f(spec.rho_liquidate), f(spec.kappa_flow))

    def c(self) -> _Desc:
        return _Desc(self.width, self.height, self.n_weight_layers, self.hidden,
                     self.rho_invest, self.rho_liquidate, self.kappa_flow, self.day_period,
                     self.night_num, self.day_inject, self.cycle_step, self.explore_mode, 0,
                     self.kappa_energy)

    @property
    def n(self) -> int:
        return self.width * self.height

    def widths(self) -> list[int]:
        return [N_IN] + [self.hidden] * (self.n_weight_layers - 1) + [N_OUT]


def net_size(d: Desc) -> int:
    return int(lib().orc_net_size(ct.byref(d.c())))


def cppn(params: np.ndarray, x1: float, y1: float, x2: float, y2: float) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros(2, dtype=np.float64)
    lib().orc_cppn(_p(p), x1, y1, x2, y2, _p(out))
    return out


def cppn_to_net(d: Desc, params: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros(net_size(d), dtype=np.float64)
    lib().orc_cppn_to_net(ct.byref(d.c()), _p(p), _p(out))
    return out


def nets_for(d: Desc, params: np.ndarray) -> np.ndarray:
    """Flat FP64 networks [n_genomes, net_size] for an array of CPPN params
    (cppn_to_net of each, genomes spread over the OpenMP threads)."""
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, N_PARAM))
    out = np.zeros((p.shape[0], net_size(d)), dtype=np.float64)
    if p.shape[0]:
        lib().orc_nets_for(ct.byref(d.c()), p.shape[0], _p(p), _p(out))
    return out


def unflatten(d: Desc, net: np.ndarray) -> list[tuple[np.ndarray, np.ndarray]]:
    """Flat network -> [(W_l [out, in], b_l [out])]."""
    L = d.widths()
    out, k = [], 0
    for l in range(d.n_weight_layers):
        w = net[k:k + L[l + 1] * L[l]].reshape(L[l + 1], L[l])
        k += L[l + 1] * L[l]
        b = net[k:k + L[l + 1]]
        k += L[l + 1]
        out.append((w, b))
    return out


def forward(d: Desc, net: np.ndarray, u: np.ndarray) -> np.ndarray:
    a = np.zeros(N_OUT, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    n = np.ascontiguousarray(net, dtype=np.float64)
    lib().orc_forward(ct.byref(d.c()), _p(n), _p(uu), _p(a))
    return a


def kernel_dir(r: int, p: int) -> int:
    return int(lib().orc_kernel_dir(r, p))


@dataclass
class State:
    E: np.ndarray   # int64 [H, W]
    I: np.ndarray   # int64 [H, W]
    C: np.ndarray   # float64 [4, H, W]
    G: np.ndarray   # int32 [H, W]
    R: np.ndarray   # uint8 [H, W]

    @classmethod
    def from_init(cls, init) -> "State":
        return cls(init.E.astype(np.int64).copy(), init.I.astype(np.int64).copy(),
                   init.C.astype(np.float64).copy(), init.G.astype(np.int32).copy(),
                   init.R.astype(np.uint8).copy())

    def copy(self) -> "State":
        return State(self.E.copy(), self.I.copy(), self.C.copy(), self.G.copy(), self.R.copy())


def sense(d: Desc, s: State, i: int) -> np.ndarray:
    u = np.zeros(N_IN, dtype=np.float64)
    E = np.ascontiguousarray(s.E, dtype=np.int64)
    I = np.ascontiguousarray(s.I, dtype=np.int64)
    C = np.ascontiguousarray(s.C, dtype=np.float64)
    R = np.ascontiguousarray(s.R, dtype=np.uint8)
    lib().orc_sense(ct.byref(d.c()), _p(E), _p(I), _p(C), _p(R), int(i), _p(u))
    return u


def step(d: Desc, s: State, nets: np.ndarray, rows: tuple[int, int] | None = None,
         want_act: bool = False, want_records: bool = False, want_margins: bool = False):
    """One step (or the rows [y0, y1) of it).  Returns (State, info dict)."""
    H, W = d.height, d.width
    N = H * W
    y0, y1 = rows if rows is not None else (0, H)
    E = np.ascontiguousarray(s.E, dtype=np.int64)
    I = np.ascontiguousarray(s.I, dtype=np.int64)
    C = np.ascontiguousarray(s.C, dtype=np.float64)
    G = np.ascontiguousarray(s.G, dtype=np.int32)
    R = np.ascontiguousarray(s.R, dtype=np.uint8)
    nets = np.ascontiguousarray(nets, dtype=np.float64)
    E2 = E.copy()
    I2 = I.copy()
    C2 = C.copy()
    G2 = G.copy()
    R2 = R.copy()
    act = np.full((N, N_OUT), np.nan) if want_act else None
    rec = np.zeros(N, dtype=RECORD_DTYPE) if want_records else None
    mar = np.full((N, N_MARGIN), np.nan) if want_margins else None
    nul = ct.c_void_p(0)
    eio = np.zeros(2, np.int64)
    tk = lib().orc_step_rows(ct.byref(d.c()), _p(E), _p(I), _p(C), _p(G), _p(R), _p(nets),
                             int(nets.shape[0]), int(y0), int(y1), _p(E2), _p(I2), _p(C2),
                             _p(G2), _p(R2), _p(act) if act is not None else nul,
                             _p(rec) if rec is not None else nul,
                             _p(mar) if mar is not None else nul, _p(eio))
    if tk < 0:
        raise ValueError("genome id outside the network table")
    info = {"takeovers": int(tk), "injected": int(eio[0]), "removed": int(eio[1])}
    if act is not None:
        info["act"] = act.reshape(H, W, N_OUT)
    if rec is not None:
        info["records"] = rec.reshape(H, W)
    if mar is not None:
        info["margins"] = mar.reshape(H, W, N_MARGIN)
    return State(E2, I2, C2, G2, R2), info


def physics_from_records(d: Desc, i1, flow8, explore_dir, G, R):
    """Physics alone from records: I1 [N], flows [N, 8] (absolute direction),
    explore direction [N]; returns (I2, G2, R2, takeovers)."""
    N = d.n
    i1 = np.ascontiguousarray(i1, dtype=np.int64).ravel()
    f8 = np.ascontiguousarray(flow8, dtype=np.int64).reshape(N, 8)
    ed = np.ascontiguousarray(explore_dir, dtype=np.int32).ravel()
    G = np.ascontiguousarray(G, dtype=np.int32).ravel()
    R = np.ascontiguousarray(R, dtype=np.uint8).ravel()
    I2 = np.zeros(N, np.int64)
    G2 = np.zeros(N, np.int32)
    R2 = np.zeros(N, np.uint8)
    tk = lib().orc_physics_from_records(ct.byref(d.c()), _p(i1), _p(f8), _p(ed), _p(G), _p(R),
                                        _p(I2), _p(G2), _p(R2))
    shp = (d.height, d.width)
    return I2.reshape(shp), G2.reshape(shp), R2.reshape(shp), int(tk)


def buckets(G: np.ndarray, cap: int):
    G = np.ascontiguousarray(G, dtype=np.int32).ravel()
    counts = np.zeros(cap, np.int32)
    offsets = np.zeros(cap + 1, np.int32)
    perm = np.zeros(G.size, np.int32)
    if lib().orc_buckets(G.size, _p(G), cap, _p(counts), _p(offsets), _p(perm)) != 0:
        raise ValueError("genome id outside [0, cap)")
    return counts, offsets, perm


def philox(counter, key) -> np.ndarray:
    c = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(o))
    return o


def uniform(o: int) -> float:
    return float(lib().orc_uniform(int(o)))


def mutation_normals(seed: int, i: int, s: int) -> np.ndarray:
    z = np.zeros(N_PARAM, np.float64)
    lib().orc_mutation_normals(int(seed), int(i), int(s), _p(z))
    return z


def hit_threshold(rate: float) -> int:
    return int(lib().orc_hit_threshold(float(rate)))


def radiate(G: np.ndarray, cap: int, params: np.ndarray, seed: int, step_index: int,
            rate: float, sigma: float, max_hits: int = 1 << 20):
    """Radiation after step ``step_index``: returns (G', params', hits list, dropped)."""
    shp = G.shape
    G2 = np.ascontiguousarray(G, dtype=np.int32).ravel().copy()
    P = np.ascontiguousarray(params, dtype=np.float64).copy()
    assert P.shape == (cap, N_PARAM)
    hc = np.zeros(max_hits, np.int64)
    hs = np.zeros(max_hits, np.int32)
    dropped = ct.c_int64(0)
    T = hit_threshold(rate)
    nh = lib().orc_radiate(G2.size, _p(G2), cap, _p(P), int(seed), int(step_index), T,
                           float(sigma), _p(hc), _p(hs), max_hits, ct.byref(dropped))
    k = min(nh, max_hits)
    return G2.reshape(shp), P, (hc[:k].copy(), hs[:k].copy()), int(dropped.value)


def merge(d: Desc, G: np.ndarray, R: np.ndarray, cap: int, params: np.ndarray, seed: int,
          step_index: int, rate: float, max_hits: int = 1 << 20):
    """Merging (NEAT crossover) after step ``step_index``: returns
    (G', params', (cells, slots, a, b), dropped)."""
    shp = G.shape
    G2 = np.ascontiguousarray(G, dtype=np.int32).ravel().copy()
    R2 = np.ascontiguousarray(R, dtype=np.uint8).ravel()
    assert G2.size == R2.size == d.width * d.height
    P = np.ascontiguousarray(params, dtype=np.float64).copy()
    assert P.shape == (cap, N_PARAM)
    hc = np.zeros(max_hits, np.int64)
    hs = np.zeros(max_hits, np.int32)
    ha = np.zeros(max_hits, np.int32)
    hb = np.zeros(max_hits, np.int32)
    dropped = ct.c_int64(0)
    dc = d.c()
    nh = lib().orc_merge(ct.byref(dc), _p(G2), _p(R2), cap, _p(P), int(seed), int(step_index),
                         hit_threshold(rate), _p(hc), _p(hs), _p(ha), _p(hb), max_hits,
                         ct.byref(dropped))
    k = min(nh, max_hits)
    return (G2.reshape(shp), P, (hc[:k].copy(), hs[:k].copy(), ha[:k].copy(), hb[:k].copy()),
            int(dropped.value))


# Structural genes of a genome (NEAT over the bounded superset of the CPPN;
# see orc_ext): direct connections input m -> output o at 5 o + m, added
# nodes splitting hidden j -> output o at 2 j + o.
EXT_DTYPE = np.dtype([("conn_mask", np.uint32), ("node_mask", np.uint32), ("node_act", np.uint32),
                      ("pad", np.uint32), ("conn_w", np.float64, (10,)), ("node_in", np.float64, (16,)),
                      ("node_out", np.float64, (16,))])
assert EXT_DTYPE.itemsize == 16 + 42 * 8


def empty_ext(n: int) -> np.ndarray:
    return np.zeros(n, EXT_DTYPE)


def cppn_to_net_x(d: Desc, p: np.ndarray, e) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    e = np.ascontiguousarray(np.asarray(e, EXT_DTYPE).reshape(1))
    out = np.zeros(net_size(d))
    dc = d.c()
    lib().orc_cppn_to_net_x(ct.byref(dc), _p(p), _p(e), _p(out))
    return out


def nets_for_x(d: Desc, params: np.ndarray, exts: np.ndarray) -> np.ndarray:
    params = np.ascontiguousarray(params, dtype=np.float64)
    exts = np.ascontiguousarray(exts, EXT_DTYPE)
    assert len(exts) == len(params)
    out = np.zeros((len(params), net_size(d)))
    dc = d.c()
    lib().orc_nets_for_x(ct.byref(dc), len(params), _p(params), _p(exts), _p(out))
    return out


def radiate_x(G: np.ndarray, cap: int, params: np.ndarray, ext: np.ndarray, seed: int, step_index: int,
              rate: float, sigma: float, p_conn: float, p_node: float, max_hits: int = 1 << 20):
    """Radiation with NEAT's structural mutations: (G', params', ext', hits, dropped)."""
    shp = G.shape
    G2 = np.ascontiguousarray(G, dtype=np.int32).ravel().copy()
    P = np.ascontiguousarray(params, dtype=np.float64).copy()
    X = np.ascontiguousarray(ext, EXT_DTYPE).copy()
    assert P.shape == (cap, N_PARAM) and X.shape == (cap,)
    hc = np.zeros(max_hits, np.int64)
    hs = np.zeros(max_hits, np.int32)
    dropped = ct.c_int64(0)
    nh = lib().orc_radiate_x(G2.size, _p(G2), cap, _p(P), _p(X), int(seed), int(step_index), hit_threshold(rate),
                             float(sigma), hit_threshold(p_conn), hit_threshold(p_node), _p(hc), _p(hs),
                             max_hits, ct.byref(dropped))
    k = min(nh, max_hits)
    return G2.reshape(shp), P, X, (hc[:k].copy(), hs[:k].copy()), int(dropped.value)


def merge_x(d: Desc, G: np.ndarray, R: np.ndarray, cap: int, params: np.ndarray, ext: np.ndarray, seed: int,
            step_index: int, rate: float, max_hits: int = 1 << 20):
    """Merging with structural genes: (G', params', ext', (cells, slots, a, b), dropped)."""
    shp = G.shape
    G2 = np.ascontiguousarray(G, dtype=np.int32).ravel().copy()
    R2 = np.ascontiguousarray(R, dtype=np.uint8).ravel()
    P = np.ascontiguousarray(params, dtype=np.float64).copy()
    X = np.ascontiguousarray(ext, EXT_DTYPE).copy()
    hc = np.zeros(max_hits, np.int64)
    hs = np.zeros(max_hits, np.int32)
    ha = np.zeros(max_hits, np.int32)
    hb = np.zeros(max_hits, np.int32)
    dropped = ct.c_int64(0)
    dc = d.c()
    nh = lib().orc_merge_x(ct.byref(dc), _p(G2), _p(R2), cap, _p(P), _p(X), int(seed), int(step_index),
                           hit_threshold(rate), _p(hc), _p(hs), _p(ha), _p(hb), max_hits, ct.byref(dropped))
    k = min(nh, max_hits)
    return (G2.reshape(shp), P, X, (hc[:k].copy(), hs[:k].copy(), ha[:k].copy(), hb[:k].copy()),
            int(dropped.value))


def genetic_distance_x(pa, ea, pb, eb, c1: float = 1.0, c2: float = 1.0, c3: float = 0.4) -> float:
    """NEAT compatibility distance with structural genes."""
    pa = np.ascontiguousarray(pa, dtype=np.float64)
    pb = np.ascontiguousarray(pb, dtype=np.float64)
    ea = np.ascontiguousarray(np.asarray(ea, EXT_DTYPE).reshape(1))
    eb = np.ascontiguousarray(np.asarray(eb, EXT_DTYPE).reshape(1))
    return float(lib().orc_genetic_distance_x(_p(pa), _p(ea), _p(pb), _p(eb), float(c1), float(c2), float(c3)))


def mass(E: np.ndarray, I: np.ndarray) -> int:
    E = np.ascontiguousarray(E, dtype=np.int64).ravel()
    I = np.ascontiguousarray(I, dtype=np.int64).ravel()
    return int(lib().orc_mass(E.size, _p(E), _p(I)))


def genetic_distance(a: np.ndarray, b: np.ndarray, c3: float = 1.0) -> float:
    """NEAT compatibility distance of two genomes' CPPN parameters."""
    pa = np.ascontiguousarray(a, dtype=np.float64)
    pb = np.ascontiguousarray(b, dtype=np.float64)
    return float(lib().orc_genetic_distance(_p(pa), _p(pb), float(c3)))


def births(G_before: np.ndarray, hits) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """The phylogeny's new edges of one radiation call: (cell, parent slot,
    new slot) of every hit that received a slot, from the genome map before
    the call and radiate()'s hit list."""
    cells, slots = hits
    took = slots >= 0
    cells = cells[took].astype(np.int64)
    return cells, np.asarray(G_before).ravel()[cells].astype(np.int32), slots[took].astype(np.int32)
