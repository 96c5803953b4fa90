"""Seeded synthetic workloads (inputs only; no solver arithmetic here).

Each workload fixes the mesh, order, frequency and load data of one
benchmark configuration.  Random draws use numpy's PCG64 generator with the
stated seed, so the oracle, the tests and the benchmark all see the same
numbers.  The paper's Gaussian-beam and seismic inputs are replaced by plane
waves (which have exact solutions) and Gaussian point sources (the paper's
source model); see the design notes for why.
"""
from dataclasses import dataclass, field

import numpy as np


def plane_wave_direction(seed):
    """Unit propagation direction d = g/|g|, g ~ N(0, I_3) from seed."""
    g = np.random.default_rng(seed).standard_normal(3)
    return g / np.linalg.norm(g)


def source_centres(seed, count, lo=0.1, hi=0.9):
    """count point-source centres, uniform in [lo, hi]^3 from seed."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(count, 3))


@dataclass
class Workload:
    name: str
    N: int
    p: int
    omega: float
    dp: int = 1
    nu_pre: int = 1
    nu_post: int = 1
    theta: float = 0.2
    tol: float = 1e-8
    precision: str = "fp64"           # "fp64" or "mixed"
    direction: np.ndarray = None      # plane-wave impedance data, or None
    sources: np.ndarray = None        # [nrhs, 3] centres, one source per rhs
    sigma: float = 0.02
    nrhs: int = 1
    extra: dict = field(default_factory=dict)


def plane_wave_4():
    return Workload("plane-wave N=4 p=2 omega=2pi V(1,1) fp64", N=4, p=2, omega=2 * np.pi,
                    nu_pre=1, nu_post=1, tol=1e-10, direction=plane_wave_direction(0))


def plane_wave_16():
    return Workload("plane-wave N=16 p=3 omega=8pi V(2,2) fp64", N=16, p=3, omega=8 * np.pi,
                    nu_pre=2, nu_post=2, tol=1e-8, direction=plane_wave_direction(1))


def plane_wave_32_mixed():
    return Workload("plane-wave N=32 p=4 omega=16pi V(2,2) mixed", N=32, p=4,
                    omega=16 * np.pi, nu_pre=2, nu_post=2, tol=1e-8, precision="mixed",
                    direction=plane_wave_direction(2))


def plane_wave_32():
    """The 32^3, p = 4 plane wave solved in FP64 throughout, for the
    time-to-tolerance comparison with the mixed-precision path."""
    return Workload("plane-wave N=32 p=4 omega=16pi V(2,2) fp64", N=32, p=4,
                    omega=16 * np.pi, nu_pre=2, nu_post=2, tol=1e-8,
                    direction=plane_wave_direction(2))


def point_sources_24():
    return Workload("point-sources N=24 p=3 omega=12pi 32 rhs mixed", N=24, p=3,
                    omega=12 * np.pi, nu_pre=2, nu_post=2, tol=1e-8, precision="mixed",
                    sources=source_centres(3, 32), sigma=0.02, nrhs=32)


ALL = {"plane_wave_4": plane_wave_4, "plane_wave_16": plane_wave_16,
       "plane_wave_32_mixed": plane_wave_32_mixed, "plane_wave_32": plane_wave_32,
       "point_sources_24": point_sources_24}
