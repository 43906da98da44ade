"""Seeded synthetic inputs and workload presets shared by tests, bench and oracle checks.

Holds no arithmetic of the discretisation: only random vectors from seeds,
closed-form fields evaluated at caller-supplied coordinates, and the
parameters of the benchmark workloads.  The workloads stand in for the
paper's flows (Sec. 6-7): periodic unit cubes at degrees 3-5 and the channel
box 2 pi x 2 x pi with hyperbolic wall grading (Sec. 7.1), with random or
manufactured data instead of simulation snapshots.
"""
import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def uniform(seed, n, lo=-1.0, hi=1.0):
    """fp64 samples of U[lo, hi) from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


# -- closed-form fields (x, y, z are arrays of physical coordinates) -----------
def sin3(x, y, z):
    return np.sin(TWO_PI * x) * np.sin(TWO_PI * y) * np.sin(TWO_PI * z)


def poisson_rhs_sin3(x, y, z):
    """f = -Laplace(sin3) = 3 (2 pi)^2 sin3."""
    return 3.0 * TWO_PI ** 2 * sin3(x, y, z)


def helm_exact(x, y, z):
    return np.sin(TWO_PI * x) * np.cos(TWO_PI * y) * np.sin(TWO_PI * z)


def helm_rhs(mu, nu):
    """f = mu u - nu Laplace u for u = sin(2pi x) cos(2pi y) sin(2pi z)."""
    return lambda x, y, z: (mu + nu * 3.0 * TWO_PI ** 2) * helm_exact(x, y, z)


def channel_exact(x, y, z):
    return (1.0 - y ** 2) * np.sin(x) * np.cos(2.0 * z)


def channel_rhs(mu, nu):
    """f = mu u - nu Laplace u for u = (1 - y^2) sin x cos 2z (zero on y = +-1)."""
    return lambda x, y, z: (mu * (1.0 - y ** 2) + nu * (2.0 + 5.0 * (1.0 - y ** 2))) * np.sin(x) * np.cos(2.0 * z)


def taylor_green(x, y, z):
    """Taylor-Green vortex of unit amplitude on the unit cube, shape (3, m)."""
    return np.stack([np.sin(TWO_PI * x) * np.cos(TWO_PI * y) * np.cos(TWO_PI * z),
                     -np.cos(TWO_PI * x) * np.sin(TWO_PI * y) * np.cos(TWO_PI * z),
                     np.zeros_like(x)])


def parabolic(x, y, z):
    """Laminar channel profile (1 - y^2, 0, 0), shape (3, m)."""
    return np.stack([1.0 - y ** 2, np.zeros_like(y), np.zeros_like(y)])


# -- workload presets ------------------------------------------------------------
@dataclass
class Workload:
    name: str
    degree: int
    cells: tuple
    lengths: tuple = (1.0, 1.0, 1.0)
    y0: float = 0.0
    periodic: tuple = (True, True, True)
    y_tanh_gamma: float = 0.0
    store_qp_metric: bool = False
    mass_coeff: float = 0.0
    diff_coeff: float = 1.0
    penalty_scale: float = 1.0
    conv_points: int = 0
    neumann: tuple = (False,) * 6      # per side x-, x+, y-, y+, z-, z+ (non-periodic directions)
    curve_amp: float = 0.0             # amplitude of the curved-cell deformation (0: affine cells)
    extra: dict = field(default_factory=dict)

    @property
    def ndofs(self):
        n = self.degree + 1
        return self.cells[0] * self.cells[1] * self.cells[2] * n ** 3


# Poisson on the periodic unit cube with tau = (k+1)^2/h, i.e. a penalty scale
# of 1/3 in tau_e = s (k+1)^2 (A_int/2)/V = 3 s (k+1)^2/h.
POISSON_C0 = Workload("poisson_periodic_4c_k3", 3, (4, 4, 4), penalty_scale=1.0 / 3.0)
HELMHOLTZ_C1 = Workload("helmholtz_periodic_32c_k4", 4, (32, 32, 32), mass_coeff=1000.0, diff_coeff=0.01)
POISSON_C2 = Workload("poisson_periodic_64c_k3", 3, (64, 64, 64), penalty_scale=1.0 / 3.0)
CONVECTIVE_C3 = Workload("convective_periodic_32c_k5", 5, (32, 32, 32), conv_points=9)
CHANNEL_C4 = Workload("channel_48x32x48_k4", 4, (48, 32, 48), lengths=(TWO_PI, 2.0, math.pi), y0=-1.0,
                      periodic=(True, False, True), y_tanh_gamma=1.8, store_qp_metric=True,
                      mass_coeff=1000.0, diff_coeff=0.01)
CHANNEL_C4_SMALL = Workload("channel_32x24x32_k4", 4, (32, 24, 32), lengths=(TWO_PI, 2.0, math.pi), y0=-1.0,
                            periodic=(True, False, True), y_tanh_gamma=1.8, store_qp_metric=True,
                            mass_coeff=1000.0, diff_coeff=0.01)
# pressure Poisson operator of the channel: the velocity is Dirichlet on the
# walls, so the pressure is Neumann there (Sec. 3.2); singular (constants)
CHANNEL_PRESSURE_C4 = Workload("channel_pressure_48x32x48_k4", 4, (48, 32, 48), lengths=(TWO_PI, 2.0, math.pi),
                               y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.8, store_qp_metric=True,
                               mass_coeff=0.0, diff_coeff=1.0, neumann=(False, False, True, True, False, False))
# the channel Helmholtz operator on curved (iso-parametric) cells: the box
# deformation of amplitude 0.02 also curves the walls
CHANNEL_CURVED_C4 = Workload("channel_curved_48x32x48_k4", 4, (48, 32, 48), lengths=(TWO_PI, 2.0, math.pi),
                             y0=-1.0, periodic=(True, False, True), y_tanh_gamma=1.8, store_qp_metric=True,
                             mass_coeff=1000.0, diff_coeff=0.01, curve_amp=0.02)

# the periodic Poisson apply at degrees 2..7 on meshes of 17-24M DoF (every
# fp64 working set above the 256 MB Infinity Cache): cost per DoF against k
DEGREE_SWEEP = [Workload(f"poisson_periodic_{c}c_k{k}", k, (c, c, c), penalty_scale=1.0 / 3.0)
                for k, c in ((2, 88), (3, 64), (4, 56), (5, 48), (6, 40), (7, 32))]
# degree 5 on 32^3 cells (7.08M DoF, the convective workload's mesh)
POISSON_32C_K5 = Workload("poisson_periodic_32c_k5", 5, (32, 32, 32), penalty_scale=1.0 / 3.0)

WORKLOADS = {w.name: w for w in (POISSON_C0, HELMHOLTZ_C1, POISSON_C2, CONVECTIVE_C3, CHANNEL_C4,
                                 CHANNEL_C4_SMALL, CHANNEL_PRESSURE_C4, CHANNEL_CURVED_C4, POISSON_32C_K5,
                                 *DEGREE_SWEEP)}


def scaled(w, cells, name=None):
    """Same workload at a different cell count (for oracle-sized parity cases)."""
    import dataclasses
    return dataclasses.replace(w, cells=tuple(cells), name=name or f"{w.name}@{cells}")
