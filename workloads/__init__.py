"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *draws* inputs: initial substrates, genome maps and CPPN
parameters.  It holds none of the update rule's arithmetic (no sensing, no
network, no physics, no random draws the method itself makes), so the CPU
oracle and the HIP path can both consume it without sharing method code.

The paper (System Design; Experiment) fixes the channels but no initial
conditions; the recipes below are the readings recorded in the design notes:

* plain method, 64x64: E, I ~ U(0,1), comm = 0, rotation = 0, GenomeIndex =
  16 Voronoi patches, 16 CPPNs with N(0,1) parameters;
* 1024x1024: energy = 64 periodic Gaussian blobs (sigma 16, peak 1) plus
  U(0, 0.1), infrastructure U(0,1), 256 genomes over 256 patches;
* 4096x4096: E, I ~ U(0,1), 4096 genomes drawn Zipf(s=1.1) over 65536
  Voronoi patches, 54-64-64-14 networks;
* batched worlds and the Poisson serving stream built from the above.

Mass values are stored in an integer ledger of 2**-24 units (quanta); the
conversion of a drawn real value x to the ledger is floor(x * 2**24).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

QUANTUM_BITS = 24
N_CPPN_PARAMS = 56          # A (8x5) then B (2x8), row-major


@dataclass
class WorldSpec:
    """Shape and physics constants of one world (mirrors coralai_world_desc)."""
    width: int
    height: int
    n_weight_layers: int = 2
    hidden: int = 32
    genome_capacity: int = 16
    precision: int = 0              # 0 = FP32 networks, 1 = BF16 networks
    seed: int = 0
    rho_invest: float = 0.1
    rho_liquidate: float = 0.1
    kappa_flow: float = 0.25


@dataclass
class WorldInit:
    """A seeded initial state plus the genomes it references."""
    spec: WorldSpec
    E: np.ndarray                   # int64 [H, W] quanta
    I: np.ndarray                   # int64 [H, W] quanta
    C: np.ndarray                   # float32 [4, H, W]
    G: np.ndarray                   # int32 [H, W]
    R: np.ndarray                   # uint8 [H, W] in 0..7
    slots: np.ndarray               # int32 [n] genome slot ids
    params: np.ndarray              # float32 [n, 56] CPPN parameters
    meta: dict = field(default_factory=dict)


def to_ledger(x: np.ndarray) -> np.ndarray:
    """Real mass values -> int64 quanta, floor(x * 2**24)."""
    return np.floor(np.asarray(x, dtype=np.float64) * float(1 << QUANTUM_BITS)).astype(np.int64)


def voronoi_labels(width: int, height: int, n_seeds: int, rng: np.random.Generator) -> np.ndarray:
    """Nearest-seed labels on a periodic grid.

    Seeds are uniform on the torus [0,W)x[0,H); cell (x, y) is represented by
    its centre (x+0.5, y+0.5); distance is the torus distance.  Returns int32
    [H, W] labels in 0..n_seeds-1.
    """
    from scipy.spatial import cKDTree

    seeds = rng.random((n_seeds, 2)) * np.array([width, height], dtype=np.float64)
    # cKDTree's periodic box requires data strictly inside [0, box)
    seeds = np.minimum(seeds, np.nextafter(np.array([width, height], dtype=np.float64), 0))
    tree = cKDTree(seeds, boxsize=[width, height])
    ys, xs = np.mgrid[0:height, 0:width]
    pts = np.stack([xs.ravel() + 0.5, ys.ravel() + 0.5], axis=1)
    _, idx = tree.query(pts, k=1, workers=-1)
    return idx.astype(np.int32).reshape(height, width)


def periodic_blobs(width: int, height: int, n_blobs: int, sigma: float, peak: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Sum of periodic Gaussian blobs, centres uniform on the torus. float64 [H, W]."""
    centres = rng.random((n_blobs, 2)) * np.array([width, height], dtype=np.float64)
    xs = np.arange(width, dtype=np.float64) + 0.5
    ys = np.arange(height, dtype=np.float64) + 0.5
    # each blob is separable, exp(-dx^2 / 2s^2) exp(-dy^2 / 2s^2): the sum over
    # blobs of the outer products is one matrix product
    dx = np.abs(xs[None, :] - centres[:, :1])
    dx = np.minimum(dx, width - dx)
    dy = np.abs(ys[None, :] - centres[:, 1:])
    dy = np.minimum(dy, height - dy)
    gx = np.exp(-dx * dx / (2.0 * sigma * sigma))
    gy = np.exp(-dy * dy / (2.0 * sigma * sigma))
    return peak * (gy.T @ gx)


def zipf_choice(n_draws: int, n_ranks: int, s: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. draws from the truncated Zipf law P(k) ~ k**-s, k = 1..n_ranks; returns k-1."""
    k = np.arange(1, n_ranks + 1, dtype=np.float64)
    p = k ** (-s)
    p /= p.sum()
    return rng.choice(n_ranks, size=n_draws, p=p).astype(np.int32)


def cppn_params(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal((n, N_CPPN_PARAMS)).astype(np.float32)


def _finish(spec: WorldSpec, E, I, G, n_genomes, rng, R=None, C=None, meta=None) -> WorldInit:
    H, W = spec.height, spec.width
    if C is None:
        C = np.zeros((4, H, W), dtype=np.float32)
    if R is None:
        R = np.zeros((H, W), dtype=np.uint8)
    params = cppn_params(n_genomes, rng)
    return WorldInit(spec=spec, E=E, I=I, C=C, G=G.astype(np.int32), R=R.astype(np.uint8),
                     slots=np.arange(n_genomes, dtype=np.int32), params=params, meta=meta or {})


def plain_world(width: int = 64, height: int = 64, n_genomes: int = 16, seed: int = 0,
                hidden: int = 32, n_weight_layers: int = 2, precision: int = 0,
                capacity: int | None = None, random_rotation: bool = False,
                random_comm: bool = False) -> WorldInit:
    """The plain-method world: E, I ~ U(0,1), comm 0, rotation 0, Voronoi genomes."""
    rng = np.random.default_rng(seed)
    spec = WorldSpec(width, height, n_weight_layers, hidden,
                     capacity if capacity is not None else n_genomes, precision, seed)
    E = to_ledger(rng.random((height, width)))
    I = to_ledger(rng.random((height, width)))
    G = voronoi_labels(width, height, n_genomes, rng)
    R = rng.integers(0, 8, size=(height, width), dtype=np.uint8) if random_rotation else None
    C = rng.random((4, height, width)).astype(np.float32) if random_comm else None
    return _finish(spec, E, I, G, n_genomes, rng, R=R, C=C)


def blob_world(width: int = 1024, height: int = 1024, n_genomes: int = 256, seed: int = 0,
               n_blobs: int = 64, precision: int = 0, hidden: int = 32,
               n_weight_layers: int = 2, capacity: int | None = None) -> WorldInit:
    """1024^2-style world: blob energy + U(0,0.1), infrastructure U(0,1)."""
    rng = np.random.default_rng(seed)
    spec = WorldSpec(width, height, n_weight_layers, hidden,
                     capacity if capacity is not None else n_genomes, precision, seed)
    e = periodic_blobs(width, height, n_blobs, 16.0, 1.0, rng) + 0.1 * rng.random((height, width))
    E = to_ledger(e)
    I = to_ledger(rng.random((height, width)))
    G = voronoi_labels(width, height, n_genomes, rng)
    return _finish(spec, E, I, G, n_genomes, rng)


def zipf_world(width: int = 4096, height: int = 4096, n_genomes: int = 4096,
               n_patches: int = 65536, zipf_s: float = 1.1, seed: int = 0,
               precision: int = 1, hidden: int = 64, n_weight_layers: int = 3,
               capacity: int = 1 << 17) -> WorldInit:
    """4096^2-style world: uniform E, I; Zipf genomes over Voronoi patches."""
    rng = np.random.default_rng(seed)
    spec = WorldSpec(width, height, n_weight_layers, hidden, capacity, precision, seed)
    E = to_ledger(rng.random((height, width)))
    I = to_ledger(rng.random((height, width)))
    patch = voronoi_labels(width, height, n_patches, rng)
    patch_genome = zipf_choice(n_patches, n_genomes, zipf_s, rng)
    G = patch_genome[patch]
    return _finish(spec, E, I, G, n_genomes, rng, meta={"n_patches": n_patches})


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def config_plain_64() -> WorldInit:
    """64x64, FP32, 16 genomes, 54-32-14, seed 0, no mutation (100 steps)."""
    return plain_world(64, 64, 16, seed=0)


def config_blobs_1024(precision: int = 0) -> WorldInit:
    """1024x1024, 256 genomes, blob energy; run in FP32 and in BF16."""
    return blob_world(1024, 1024, 256, seed=0, precision=precision)


def config_zipf_4096(precision: int = 1, width: int = 4096, height: int = 4096,
                     n_patches: int = 65536) -> WorldInit:
    """4096x4096, 4096 Zipf genomes, 54-64-64-14, radiation 1e-4, sigma 0.1."""
    return zipf_world(width, height, 4096, n_patches=n_patches, seed=0, precision=precision)


RADIATION_RATE = 1e-4
RADIATION_SIGMA = 0.1


def batched_world_specs(n_worlds: int = 512, seed: int = 7) -> list[tuple[int, int, int]]:
    """(side, n_genomes, world_seed) for the batched form: side ~ U{64,96,...,512},
    genomes ~ U{8..128}, world seed 1000 + w."""
    rng = np.random.default_rng(seed)
    sides = np.arange(64, 513, 32)
    out = []
    for w in range(n_worlds):
        side = int(rng.choice(sides))
        ng = int(rng.integers(8, 129))
        out.append((side, ng, 1000 + w))
    return out


def batched_world(side: int, n_genomes: int, world_seed: int, precision: int = 1) -> WorldInit:
    return plain_world(side, side, n_genomes, seed=world_seed, precision=precision)


@dataclass
class Request:
    rid: int
    arrival_s: float
    side: int
    n_genomes: int
    n_steps: int
    seed: int


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def poisson_requests(n_requests: int, rate_per_s: float, seed: int = 3,
                     side_range=(128, 2048), genome_range=(16, 1024),
                     step_range=(10, 1000)) -> list[Request]:
    """Poisson arrivals; side, genome count and step count log-uniform."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        out.append(Request(r, t, _log_uniform_int(rng, *side_range),
                           _log_uniform_int(rng, *genome_range),
                           _log_uniform_int(rng, *step_range), 5000 + r))
    return out


def request_world(req: Request, precision: int = 0) -> WorldInit:
    """A serving request's state: blob energy scaled with area (at least 1 blob)."""
    n_blobs = max(1, int(round(64 * (req.side / 1024.0) ** 2)))
    return blob_world(req.side, req.side, req.n_genomes, seed=req.seed, n_blobs=n_blobs,
                      precision=precision)
