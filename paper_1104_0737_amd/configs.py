"""Synthetic workloads: lattice shapes, link spread, kappa, sources, SAP setup.

They stand in for the paper's measurement (Sec. 3.1: 32^3 x 64, 12 local
sources at one site, SAP on 8^4 domains), whose gauge configurations are not
available; random SU(3) fields of the same shape replace them.  Seeds: system
k uses gauge seed 1000k+1, source seed 1000k+2 and R~ seed 1000k+3.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import inputs

ANTIPERIODIC_T = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))


@dataclass
class System:
    name: str
    dims: tuple
    eps: float
    kappa: float
    L: int
    block: tuple
    ncy: int = 4
    nmr: int = 4
    tol: float = 1e-10
    source: str = "point"        # "point" | "z2"
    site: int | None = None      # point-source site (None: drawn from seed)
    comp0: int = 0
    seed: int = 1
    phases: tuple = ANTIPERIODIC_T
    extra: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))

    def gauge(self) -> np.ndarray:
        return inputs.gauge_field(self.dims, self.eps, 1000 * self.seed + 1)

    def src_site(self) -> int:
        if self.site is not None:
            return self.site
        return inputs.source_site(self.V, 1000 * self.seed + 2)

    def sources(self) -> np.ndarray:
        if self.source == "z2":
            return inputs.z2_sources(self.V, self.L, 1000 * self.seed + 2)
        return inputs.point_sources(self.V, self.L, self.src_site(), self.comp0)


def c1() -> System:
    """8^4, L=4 point sources (components 0..3 at site 0), FP64, tol 1e-12."""
    return System("c1", (8, 8, 8, 8), 0.3, 0.11, 4, (4, 4, 4, 4), tol=1e-12,
                  site=0, seed=1)


def c2() -> System:
    """16^3x32, L=12 point sources at a seeded site, all-FP64, tol 1e-10."""
    return System("c2", (16, 16, 16, 32), 0.25, 0.1235, 12, (8, 8, 8, 8), seed=2)


def c3() -> System:
    """The c1 system solved with FP32 / FP16-storage SAP, tol 1e-10."""
    s = c1()
    s.name, s.tol = "c3", 1e-10
    return s


def c4(L: int = 12, block_index: int = 0) -> System:
    """32^3x64 (the paper's shape), 12 point sources split into 12/L blocks."""
    return System("c4", (32, 32, 32, 64), 0.2, 0.1240, L, (8, 8, 8, 8), seed=4,
                  comp0=block_index * L)


def c5_systems() -> list:
    """48 independent systems of uneven size for the batched form."""
    out = []
    groups = (((8, 8, 8, 8), 4, (4, 4, 4, 4)),
              ((12, 12, 12, 12), 6, (6, 6, 6, 6)),
              ((16, 16, 16, 32), 12, (8, 8, 8, 8)))
    for g, (dims, L, blk) in enumerate(groups):
        for k in range(16):
            j = 16 * g + k
            rng = np.random.default_rng(5000 + 10 * j + 1)
            eps = float(rng.uniform(0.15, 0.3))
            kappa = float(rng.uniform(0.11, 0.123))
            s = System(f"c5.{j}", dims, eps, kappa, L, blk,
                       source="z2" if k < 8 else "point")
            s.extra["seeds"] = (5000 + 10 * j + 1, 5000 + 10 * j + 2, 5000 + 10 * j + 3)
            out.append(s)
    return out


def c5_gauge(s: System) -> np.ndarray:
    """Links of a batched system: drawn after its eps and kappa from the same RNG."""
    rng = np.random.default_rng(s.extra["seeds"][0])
    rng.uniform(0.15, 0.3)
    rng.uniform(0.11, 0.123)
    V = s.V
    g = rng.standard_normal((V * 4, 9))
    return inputs._su3_from_normals(g, s.eps).reshape(V, 4, 3, 3)


def c5_sources(s: System) -> np.ndarray:
    seed = s.extra["seeds"][1]
    if s.source == "z2":
        return inputs.z2_sources(s.V, s.L, seed)
    return inputs.point_sources(s.V, s.L, inputs.source_site(s.V, seed), 0)
