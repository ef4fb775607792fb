"""Seeded synthetic workloads (positions, charges, slab parameters).

This module only draws random numbers and holds parameter sets; it contains
none of the method's arithmetic, so both the GPU path and the CPU oracle can
take their inputs from it.  Charges are listed positives first.

Workloads (uniform electrolyte slabs standing in for the paper's implicit-
solvent electrolytes and water slabs):
  small_fp64  N=500 1:1, 20x20x5, no dielectric jump, alpha=1, r_c=4, P=100
  dielectric  N=10,000 1:1, 50x50x10, gamma=0.9/0.9, M=8, alpha=0.5, r_c=6, P=200
  replicas    64 slabs, N log-uniform in [1e3, 5e4], 2:1, density 0.05,
              H=10, gamma uniform in [-0.95, 0.95], M=8, alpha=0.5, r_c=6, P=200
  large_md    N=1e6 1:1, 800x800x40, gamma=+0.95/-0.95, M=10, alpha=0.3,
              r_c=10, P=500, 100 velocity-Verlet steps, dt=1e-3
  gradient    N=20,000 1:1, 60x60x12, gamma=0.8/0.8, M=8, alpha=0.5, r_c=6, P=300
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Workload:
    name: str
    N: int
    Lx: float
    Ly: float
    H: float
    gamma_top: float
    gamma_bot: float
    alpha: float
    r_c: float
    P: int
    M: int
    seed: int
    valence: tuple = (1, -1)      # (cation, anion); N splits to keep the charge neutral
    margin: float = 0.5           # distance of the sampled z range from the walls
    precision: str = "fp64"
    steps: int = 0
    dt: float = 1e-3
    extra: dict = field(default_factory=dict)

    def slab_kwargs(self, **over):
        d = dict(Lx=self.Lx, Ly=self.Ly, H=self.H, gamma_top=self.gamma_top, gamma_bot=self.gamma_bot,
                 alpha=self.alpha, r_c=self.r_c, P=self.P, M=self.M)
        d.update(over)
        return d

    def with_(self, **kw):
        return replace(self, **kw)


def charges(N, valence=(1, -1)):
    zp, zm = valence
    # n_plus * zp + n_minus * zm = 0
    n_plus = N * (-zm) // (zp - zm)
    q = np.empty(N)
    q[:n_plus] = zp
    q[n_plus:] = zm
    return q


def positions(rng, N, Lx, Ly, H, margin):
    x = rng.uniform(0.0, Lx, N)
    y = rng.uniform(0.0, Ly, N)
    z = rng.uniform(margin, H - margin, N)
    return np.ascontiguousarray(np.stack([x, y, z], axis=1))


def thinned_positions(rng, N, Lx, Ly, H, margin, dmin, max_rounds=500):
    """Uniform positions as positions(), then every particle closer than dmin
    to another one (minimum image in x and y) is redrawn until none is: the
    start of runs with a short-range repulsion."""
    from scipy.spatial import cKDTree
    pos = positions(rng, N, Lx, Ly, H, margin)
    if N < 2:
        return pos
    box = [Lx, Ly, 4.0 * H]   # z is not periodic: its period exceeds every distance
    for _ in range(max_rounds):
        pos[:, 0] %= Lx
        pos[:, 1] %= Ly
        pairs = cKDTree(pos, boxsize=box).query_pairs(dmin, output_type="ndarray")
        if len(pairs) == 0:
            return pos
        redo = np.unique(pairs[:, 1])
        pos[redo] = positions(rng, len(redo), Lx, Ly, H, margin)
    raise RuntimeError("could not place the particles at the requested minimum distance")


def sample(w: Workload):
    """(pos (N,3), q (N,)) for a workload, from numpy's default_rng(seed);
    with extra["dmin"] the positions are thinned to that minimum distance."""
    rng = np.random.default_rng(w.seed)
    if w.extra.get("dmin"):
        pos = thinned_positions(rng, w.N, w.Lx, w.Ly, w.H, w.margin, w.extra["dmin"])
    else:
        pos = positions(rng, w.N, w.Lx, w.Ly, w.H, w.margin)
    return pos, charges(w.N, w.valence)


SMALL_FP64 = Workload("small_fp64", 500, 20.0, 20.0, 5.0, 0.0, 0.0, 1.0, 4.0, 100, 0, seed=0)
DIELECTRIC = Workload("dielectric", 10_000, 50.0, 50.0, 10.0, 0.9, 0.9, 0.5, 6.0, 200, 8, seed=1)
LARGE_MD = Workload("large_md", 1_000_000, 800.0, 800.0, 40.0, 0.95, -0.95, 0.3, 10.0, 500, 10, seed=3,
                    precision="fp32", steps=100, dt=1e-3)
GRADIENT = Workload("gradient", 20_000, 60.0, 60.0, 12.0, 0.8, 0.8, 0.5, 6.0, 300, 8, seed=4)


def replicas(n_sys=64, seed=2, density=0.05, H=10.0):
    """The 64-replica batch: per replica N (multiple of 3, 2:1 salt), box
    side from the density, contrasts uniform in [-0.95, 0.95]."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_sys):
        N = 3 * int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e4))) / 3))
        L = math.sqrt(N / (density * H))
        gt, gb = rng.uniform(-0.95, 0.95, 2)
        out.append(Workload(f"replica{r}", N, L, L, H, float(gt), float(gb), 0.5, 6.0, 200, 8,
                            seed=int(rng.integers(0, 2**31)), valence=(2, -1), precision="fp32"))
    return out


def small_random(seed, N, L=10.0, H=4.0, gamma_top=0.0, gamma_bot=0.0, alpha=1.0, r_c=4.0, P=20, M=0,
                 valence=(1, -1), margin=0.3):
    return Workload(f"rand{seed}", N, L, L, H, gamma_top, gamma_bot, alpha, r_c, P, M, seed=seed,
                    valence=valence, margin=margin)
