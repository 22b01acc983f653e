"""Seeded synthetic workloads: inverse-temperature ladders and run shapes.

This module only describes inputs (lattice model and size, replica count, the
beta ladder, seeds, the sweep/exchange/record schedule).  It holds none of the
method's arithmetic, so both the GPU binding and the CPU oracle tests can take
their inputs from here.  All random content of a run (initial spins, EA
couplings, flip and swap draws) is generated inside each implementation from
the seeds, by its own Philox4x32-10.

The paper's own workload is a 2D Ising lattice with J = 1 and no field
(Sec. 4.2); the shapes below are the synthetic configurations this project is
measured on.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ISING2D = 0
EA3D = 1


def beta_geometric(b0: float, b1: float, R: int) -> np.ndarray:
    """beta_k = b0 * (b1/b0)^(k/(R-1)), slot 0 = b0 (FP64, computed once)."""
    if R == 1:
        return np.array([b0], dtype=np.float64)
    k = np.arange(R, dtype=np.float64)
    return np.array([b0 * (b1 / b0) ** (kk / (R - 1)) for kk in k], dtype=np.float64)


def beta_linear(b0: float, b1: float, R: int) -> np.ndarray:
    """beta_k = b0 + k (b1 - b0)/(R-1), slot 0 = b0."""
    if R == 1:
        return np.array([b0], dtype=np.float64)
    return np.array([b0 + k * (b1 - b0) / (R - 1) for k in range(R)], dtype=np.float64)


@dataclass
class Workload:
    name: str
    model: int
    L: int
    R: int
    beta: np.ndarray
    sweeps: int
    exchange_every: int
    record_every: int
    seed: int
    coupling_seed: int = 0
    J: float = 1.0
    h: float = 0.0
    stream_id: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return 3 if self.model == EA3D else 2

    @property
    def sites(self) -> int:
        return self.L ** self.dim

    @property
    def attempts_per_sweep(self) -> int:
        return self.R * self.sites


def ising16() -> Workload:
    """2D Ising 16x16, R=8, beta geometric 0.20..0.60, 1000 sweeps, exchange every 10."""
    return Workload("ising2d_L16_R8", ISING2D, 16, 8, beta_geometric(0.20, 0.60, 8),
                    sweeps=1000, exchange_every=10, record_every=1, seed=1)


def ising1024() -> Workload:
    """2D Ising 1024x1024, R=64, beta linear 0.30..0.55 (spans beta_c), 10^4 sweeps."""
    return Workload("ising2d_L1024_R64", ISING2D, 1024, 64, beta_linear(0.30, 0.55, 64),
                    sweeps=10_000, exchange_every=10, record_every=1, seed=2)


def ea32() -> Workload:
    """3D +-J EA spin glass 32^3, R=128, beta geometric 0.5..3.0, 5000 sweeps, exchange every sweep."""
    return Workload("ea3d_L32_R128", EA3D, 32, 128, beta_geometric(0.5, 3.0, 128),
                    sweeps=5_000, exchange_every=1, record_every=1, seed=3, coupling_seed=3)


HOT_PATH = {w.name: w for w in (ising16(), ising1024(), ea32())}


def paper_shape(L: int = 300) -> Workload:
    """The shape of the paper's speed-up runs (Sec. 4.2): a 2D Ising L x L
    lattice (the paper's is 300 x 300; 256 and 512 are kept as power-of-two
    neighbours), 1500 replicas on the paper's temperature ladder T_k = 1 + 3k/R
    (Sec. 3), no swaps.  The paper's run length is 3*10^5 attempts per replica,
    i.e. ceil(3*10^5 / L^2) sweeps."""
    R = 1500
    beta = np.array([1.0 / (1.0 + 3.0 * k / R) for k in range(R)], dtype=np.float64)
    return Workload("paper_shape_L%d_R1500" % L, ISING2D, L, R, beta,
                    sweeps=-(-300_000 // (L * L)), exchange_every=0, record_every=10, seed=6)


# every single-configuration workload bench.py can run
WORKLOADS = dict(HOT_PATH, **{w.name: w for w in (paper_shape(300), paper_shape(256), paper_shape(512))})


def batched2048(seed: int = 4, n: int = 2048):
    """Independent 2D Ising PT instances run together: L uniform in {32, 64, 128,
    256}, R uniform in {16, 32, 64}, beta linear over [0.30, 0.55], field h
    uniform in [-0.1, 0.1]; 2000 sweeps with an exchange step every 5.  Instance
    i uses Philox stream_id i under the common seed."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice([32, 64, 128, 256], size=n)
    Rs = rng.choice([16, 32, 64], size=n)
    hs = rng.uniform(-0.1, 0.1, size=n)
    return [Workload("batched_%d" % i, ISING2D, int(Ls[i]), int(Rs[i]),
                     beta_linear(0.30, 0.55, int(Rs[i])), sweeps=2000, exchange_every=5,
                     record_every=0, seed=seed, h=float(hs[i]), stream_id=i)
            for i in range(n)]


def served_jobs(seed: int = 5, n: int = 10_000):
    """A stream of independent PT jobs for the served form.  With probability
    0.2 a job is a 3D +-J EA instance with L uniform in {8, 16, 32} and beta
    geometric over [0.5, 3.0]; otherwise a 2D Ising instance with L = 2^k, k the
    rounded value of U[4, 10] (L from 16 to 1024), beta linear over [0.30, 0.55],
    J = 1, h = 0.  R is uniform in [8, 128] and the sweep count log-uniform in
    [10^3, 10^5]; every job exchanges every 10 sweeps and records E, M every 100.
    Job i uses Philox stream_id i under the common seed (EA couplings from
    coupling_seed = seed + i)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        ea = rng.random() < 0.2
        R = int(rng.integers(8, 129))
        sweeps = int(round(10 ** rng.uniform(3.0, 5.0)))
        if ea:
            L = int(rng.choice([8, 16, 32]))
            w = Workload("served_%d" % i, EA3D, L, R, beta_geometric(0.5, 3.0, R), sweeps=sweeps,
                         exchange_every=10, record_every=100, seed=seed, coupling_seed=seed + i,
                         stream_id=i)
        else:
            L = 2 ** int(round(rng.uniform(4.0, 10.0)))
            w = Workload("served_%d" % i, ISING2D, L, R, beta_linear(0.30, 0.55, R), sweeps=sweeps,
                         exchange_every=10, record_every=100, seed=seed, stream_id=i)
        out.append(w)
    return out


def poisson_arrivals(rate: float, n: int, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from the start) of a Poisson process of the given
    rate: cumulative sums of exponential gaps, from their own generator."""
    rng = np.random.default_rng([seed, 1])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
