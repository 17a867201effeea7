"""Convenience wrappers over the C ABI: a World owns its torch-allocated
device arena and its library handle; a Batch groups worlds for the batched
form.  All compute happens in libcoralai.so."""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def make_desc(width: int, height: int, n_weight_layers: int = 2, hidden: int = 32,
              genome_capacity: int = 16, precision: int = 0, seed: int = 0,
              rho_invest: float = 0.1, rho_liquidate: float = 0.1,
              kappa_flow: float = 0.25, flags: int = 0) -> B.coralai_world_desc:
    return B.coralai_world_desc(width, height, n_weight_layers, hidden, genome_capacity,
                                precision, seed, rho_invest, rho_liquidate, kappa_flow, flags)


def desc_from_spec(spec) -> B.coralai_world_desc:
    return make_desc(spec.width, spec.height, spec.n_weight_layers, spec.hidden,
                     spec.genome_capacity, spec.precision, spec.seed, spec.rho_invest,
                     spec.rho_liquidate, spec.kappa_flow)


class World:
    def __init__(self, desc: B.coralai_world_desc, stream: torch.cuda.Stream | None = None,
                 device: str = "cuda", sync: bool = True):
        """sync=False allocates the arena in the stream's order instead of
        waiting for the whole device (the arena then belongs to that stream)."""
        self.desc = desc
        self.nbytes = B.coralai_world_bytes(desc)
        if self.nbytes == 0:
            raise ValueError("invalid world description")
        self.stream = stream
        if sync or stream is None:
            self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
            torch.cuda.synchronize()
        else:
            with torch.cuda.stream(stream):
                self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        sp = stream.cuda_stream if stream is not None else 0
        self.h = B.coralai_world_create(desc, self.arena.data_ptr(), self.nbytes, sp)
        self.W, self.H = desc.width, desc.height
        self.N = self.W * self.H

    @classmethod
    def from_init(cls, init, stream=None, precision: int | None = None,
                  sync: bool = True, flags: int = 0) -> "World":
        d = desc_from_spec(init.spec)
        d.flags = flags
        if precision is not None:
            d.precision = precision
        w = cls(d, stream, sync=sync)
        w.set_state(init.E, init.I, init.C, init.G, init.R)
        w.set_genomes(init.slots, init.params)
        return w

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            B.coralai_world_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, E, I, C, G, R) -> None:
        c = lambda a, t: np.ascontiguousarray(a, dtype=t)
        B.coralai_set_state(self.h, c(E, np.int64), c(I, np.int64), c(C, np.float32),
                            c(G, np.int32), c(R, np.uint8), 0)

    def get_state_device(self) -> dict:
        """Copy of the current state into new device tensors (stream-ordered)."""
        H, W = self.H, self.W
        ctx = torch.cuda.stream(self.stream) if self.stream is not None else _nullctx()
        with ctx:
            out = {"E": torch.empty((H, W), dtype=torch.int64, device="cuda"),
                   "I": torch.empty((H, W), dtype=torch.int64, device="cuda"),
                   "C": torch.empty((4, H, W), dtype=torch.float32, device="cuda"),
                   "G": torch.empty((H, W), dtype=torch.int32, device="cuda"),
                   "R": torch.empty((H, W), dtype=torch.uint8, device="cuda")}
        B.coralai_get_state(self.h, *(out[k].data_ptr() for k in ("E", "I", "C", "G", "R")), 1)
        return out

    def get_state(self) -> dict:
        H, W = self.H, self.W
        E = np.empty((H, W), np.int64)
        I = np.empty((H, W), np.int64)
        C = np.empty((4, H, W), np.float32)
        G = np.empty((H, W), np.int32)
        R = np.empty((H, W), np.uint8)
        B.coralai_get_state(self.h, E, I, C, G, R, 0)
        return {"E": E, "I": I, "C": C, "G": G, "R": R}

    def set_genomes(self, slots, params) -> None:
        B.coralai_set_genomes(self.h, np.ascontiguousarray(slots, dtype=np.int32),
                              np.ascontiguousarray(params, dtype=np.float32))

    def get_genomes(self, slots) -> np.ndarray:
        s = np.ascontiguousarray(slots, dtype=np.int32)
        out = np.empty((s.size, 56), np.float32)
        B.coralai_get_genomes(self.h, s, out)
        return out

    def step(self, n: int = 1, stats: bool = False) -> dict | None:
        if stats:
            st = B.coralai_stats()
            B.coralai_step(self.h, n, st)
            return st.as_dict()
        B.coralai_step(self.h, n, None)
        return None

    def radiate(self, rate: float, sigma: float, step_index: int, stats: bool = True):
        if stats:
            st = B.coralai_stats()
            B.coralai_radiate(self.h, rate, sigma, step_index, st)
            return st.as_dict()
        B.coralai_radiate(self.h, rate, sigma, step_index, None)
        return None

    def merge(self, rate: float, step_index: int, stats: bool = True):
        """Merging (NEAT crossover of a cell's genome and the one it faces)."""
        if stats:
            st = B.coralai_stats()
            B.coralai_merge(self.h, rate, step_index, st)
            return st.as_dict()
        B.coralai_merge(self.h, rate, step_index, None)
        return None

    def set_step_count(self, steps: int) -> None:
        """Completed-step count (the day / night phase) of a resumed world."""
        B.coralai_set_step_count(self.h, steps)

    def set_daylight(self, period: int, inject_quanta: int, remove_num: int) -> None:
        """Day / night cycle: period in steps (0 = off), energy quanta added per
        cell per step at noon, fraction (over 65536) of a cell's energy removed
        per step at midnight."""
        B.coralai_set_daylight(self.h, period, inject_quanta, remove_num)

    def set_physics_variant(self, explore_mode: int, kappa_energy: float) -> None:
        """explore_mode 0: softmax split of the exploration budget, 1: all to
        the maximal explore actuator; kappa_energy > 0: that fraction of a
        cell's energy moves along the same directions (needs the world created
        with flags=WORLD_ENERGY_FLOWS)."""
        B.coralai_set_physics_variant(self.h, explore_mode, kappa_energy)

    def lineage(self, slots) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(parent slot, second parent slot, birth step) of each slot; parent -1
        for genomes the caller set, second parent -1 unless born by merging."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        parents = np.empty(s.size, np.int32)
        parents2 = np.empty(s.size, np.int32)
        births = np.empty(s.size, np.int64)
        B.coralai_get_lineage(self.h, s, parents, parents2, births)
        return parents, parents2, births

    def births(self) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """(cell, parent slot, second parent slot, new slot) of each birth of the
        last radiation or merging call."""
        one = lambda: np.empty(1, np.int32)
        n = B.coralai_get_births(self.h, 0, one(), one(), one(), one())
        cells, parents, parents2, slots = (np.empty(max(n, 1), np.int32) for _ in range(4))
        B.coralai_get_births(self.h, n, cells, parents, parents2, slots)
        return cells[:n], parents[:n], parents2[:n], slots[:n]

    def set_genome_ext(self, slots, ext) -> None:
        """NEAT structural genes of the slots (records of B.GENOME_EXT_DTYPE)."""
        s = np.ascontiguousarray(slots, dtype=np.int32)
        e = np.ascontiguousarray(np.asarray(ext).astype(B.GENOME_EXT_DTYPE))
        B.coralai_set_genome_ext(self.h, s, e)

    def genome_ext(self, slots) -> np.ndarray:
        s = np.ascontiguousarray(slots, dtype=np.int32)
        out = np.zeros(s.size, B.GENOME_EXT_DTYPE)
        B.coralai_get_genome_ext(self.h, s, out)
        return out

    def set_structural_mutation(self, p_conn: float, p_node: float) -> None:
        """Probabilities of NEAT's add-connection and add-node at each radiation hit."""
        B.coralai_set_structural_mutation(self.h, p_conn, p_node)

    def genetic_distance(self, slots_a, slots_b, c3: float = 1.0, c1: float = 1.0, c2: float = 1.0) -> np.ndarray:
        """NEAT compatibility distance matrix [len(a), len(b)], computed on the GPU."""
        a = np.ascontiguousarray(slots_a, dtype=np.int32)
        b = np.ascontiguousarray(slots_b, dtype=np.int32)
        out = torch.empty((a.size, b.size), dtype=torch.float32, device="cuda")
        ctx = torch.cuda.stream(self.stream) if self.stream is not None else _nullctx()
        with ctx:
            torch.cuda.current_stream().synchronize()
        B.coralai_genetic_distance(self.h, a, b, c1, c2, c3, out.data_ptr())
        return out.cpu().numpy()

    def energy_ledger(self) -> dict:
        return B.coralai_get_energy_ledger(self.h)

    def sync(self) -> None:
        B.coralai_sync(self.h)

    def stats(self) -> dict:
        st = B.coralai_stats()
        B.coralai_get_stats(self.h, st)
        return st.as_dict()

    def autotune(self) -> tuple[int, int, int]:
        """(act_cells, act_waves, phys_tile) chosen by timing on the current state."""
        return B.coralai_autotune(self.h)

    def set_tuning(self, act_cells: int, act_waves: int, phys_tile: int) -> None:
        """Fix the launch choices (same order as autotune returns them)."""
        B.coralai_set_tuning(self.h, act_cells, act_waves, phys_tile)

    def set_profiling(self, on: bool) -> None:
        B.coralai_set_profiling(self.h, on)

    def profile(self) -> dict:
        """{phase: (summed ms, launches)} of the steps timed since profiling began."""
        return B.coralai_get_profile(self.h)

    # parity hooks
    def debug_buckets(self):
        cap = self.desc.genome_capacity
        counts = np.empty(cap, np.int32)
        offsets = np.empty(cap + 1, np.int32)
        perm = np.empty(self.N, np.int32)
        B.coralai_debug_buckets(self.h, counts, offsets, perm)
        return counts, offsets, perm

    def debug_actuators(self) -> np.ndarray:
        act = np.empty((self.N, 14), np.float32)
        B.coralai_debug_actuators(self.h, act)
        return act.reshape(self.H, self.W, 14)

    def debug_set_weights(self, slot: int, flat) -> None:
        B.coralai_debug_set_weights(self.h, slot, np.ascontiguousarray(flat, dtype=np.float32))

    def debug_set_weights_noalloc(self, slot: int, flat) -> None:
        B.coralai_debug_set_weights_noalloc(self.h, slot, np.ascontiguousarray(flat, dtype=np.float32))

    def debug_get_weights(self, slot: int, size: int) -> np.ndarray:
        out = np.zeros(size, np.float32)
        B.coralai_debug_get_weights(self.h, slot, out)
        return out

    def debug_set_act_segments(self, n_segments: int) -> None:
        B.coralai_debug_set_act_segments(self.h, n_segments)

    def debug_physics(self, i1, flows8, explore) -> None:
        B.coralai_debug_physics(self.h, np.ascontiguousarray(i1, dtype=np.int64).ravel(),
                                np.ascontiguousarray(flows8, dtype=np.uint32).reshape(-1, 8),
                                np.ascontiguousarray(explore, dtype=np.uint8).ravel())


class Batch:
    def __init__(self, max_worlds: int, stream: torch.cuda.Stream | None = None,
                 device: str = "cuda"):
        self.nbytes = B.coralai_batch_bytes(max_worlds)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        torch.cuda.synchronize()
        self.h = B.coralai_batch_create(max_worlds, self.arena.data_ptr(), self.nbytes,
                                        stream.cuda_stream if stream is not None else 0)
        self.worlds: list[World] = []

    def set_worlds(self, worlds: list[World]) -> None:
        self.worlds = list(worlds)
        B.coralai_batch_set_worlds(self.h, [w.h for w in worlds])

    def step(self, n: int = 1) -> None:
        B.coralai_batch_step(self.h, n)

    def autotune(self) -> tuple[int, int, int]:
        return B.coralai_batch_autotune(self.h)

    def set_tuning(self, act_cells: int, act_waves: int, phys_tile: int) -> None:
        B.coralai_batch_set_tuning(self.h, act_cells, act_waves, phys_tile)

    def sync(self) -> None:
        B.coralai_batch_sync(self.h)

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            B.coralai_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
