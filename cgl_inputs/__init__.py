"""Seeded synthetic workloads for the complex Ginzburg--Landau stepper.

This module is shared by the FP64 CPU oracle and by the GPU library's tests
and benchmark.  It holds only problem *data*: coefficient sets, grid node
coordinates, time steps and seeded initial states.  None of the method's
arithmetic (finite-difference operators, exponentials, mode products,
nonlinear flows, time steppers) lives here.

Model: the cubic-quintic CGL equation of eq. (cqCGL) in the paper's
introduction, with coefficients alpha_1..4, beta_1..4.  Grids are Cartesian
products of 1-D grids (Section 3.1); the state tensor is stored with index 1
fastest, i.e. the column-stacking ``vec`` of eq. (kronsumv)/(Tucker).

Grid-node conventions (the paper's concrete FD grids are 4th-order; the
workloads use 2nd-order central differences):

* Dirichlet: interior nodes x_j = a + j h, j = 1..n, h = (b-a)/(n+1), as in the
  Dirichlet experiment of Section 4.1.1.
* Neumann: vertex grid x_j = a + j h, j = 0..n-1, h = (b-a)/(n-1): the boundary
  nodes are unknowns, as with the semi-internal nodes of Section 4.2.

Every random draw uses ``numpy.random.default_rng(seed)`` (PCG64) and is
made once on the host in FP64.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

DIRICHLET = 0
NEUMANN = 1
PERIODIC = 2


@dataclasses.dataclass(frozen=True)
class Coeffs:
    """Coefficients of eq. (cqCGL): (a1 + i b1) Lap u + a2 u + (a3 + i b3)|u|^2 u
    + (a4 + i b4)|u|^4 u."""
    a1: float
    b1: float
    a2: float
    a3: float
    b3: float
    a4: float = 0.0
    b4: float = 0.0

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.a1, self.b1, self.a2, self.a3, self.b3, self.a4, self.b4)

    @property
    def cubic(self) -> bool:
        return self.a4 == 0.0 and self.b4 == 0.0


@dataclasses.dataclass(frozen=True)
class Problem:
    """One CGL instance: grid, boundary type, domain, coefficients, time step."""
    name: str
    n: Tuple[int, ...]
    bc: int
    a: float
    b: float
    coeffs: Coeffs
    tau: float
    steps: int
    method: str  # "strang", "lawson4", "split4", "lawson2", ...
    seed: int
    #: condition at the right end of every direction (None: the same as ``bc``)
    bc_hi: int | None = None
    #: finite-difference order of the operators (2 or 4)
    order: int = 2
    #: initial datum: "" (the recipe of the grid's dimension), "noise"
    #: (standard normal / 5000, real, as in the experiments of Sections 4.1-4.2)
    #: or "necklace" (the necklace ring of Section 4.3, no random draw)
    init: str = ""

    @property
    def d(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


# --- the five workloads -----------------------------------------------------

#: 2-D cubic CGL, Dirichlet, 64x64 interior grid on (-10,10)^2, Strang, tau=1e-2.
C0 = Problem("c0_cubic2d_64_dirichlet_strang", (64, 64), DIRICHLET, -10.0, 10.0,
             Coeffs(1.0, 1.5, 0.5, -1.0, 1.0), 1e-2, 100, "strang", 0)

#: cubic-quintic coefficient set of the 3-D workloads.
CQ = Coeffs(1.0, 0.8, -0.1, 1.2, 1.0, -0.1, -0.5)

#: 3-D cubic-quintic CGL, Neumann, 128^3 vertex grid on (-15,15)^3, Lawson4, tau=5e-3.
C1 = Problem("c1_cq3d_128_neumann_lawson4", (128, 128, 128), NEUMANN, -15.0, 15.0,
             CQ, 5e-3, 400, "lawson4", 1)

#: 3-D cubic-quintic CGL, Dirichlet, 256^3 interior grid on (-15,15)^3, tau=2e-3.
C2 = Problem("c2_cq3d_256_dirichlet", (256, 256, 256), DIRICHLET, -15.0, 15.0,
             CQ, 2e-3, 200, "strang", 2)

#: the paper's Table 1 setting: 2-D cubic CGL on (0,100)^2, 256^2 interior
#: grid, homogeneous Dirichlet, 4th-order FD, a1=1, b1=2, a2=1, a3=-1, b3=0.2,
#: small random initial datum, T = 6 (tau = T / steps).
PAPER_CUBIC = Coeffs(1.0, 2.0, 1.0, -1.0, 0.2)
T1 = Problem("t1_cubic2d_256_dirichlet_fd4", (256, 256), DIRICHLET, 0.0, 100.0,
             PAPER_CUBIC, 6.0 / 100, 100, "split4", 10, order=4, init="noise")

#: the paper's Table 3 setting: 3-D cubic CGL on (0,100)^3, 128^3 semi-internal
#: grid per direction (Dirichlet at 0, Neumann at 100), 4th-order FD, T = 10.
T3 = Problem("t3_cubic3d_128_dn_fd4", (128, 128, 128), DIRICHLET, 0.0, 100.0,
             PAPER_CUBIC, 10.0 / 50, 50, "split4", 11, bc_hi=NEUMANN, order=4, init="noise")

#: the paper's Table 2 setting: the Table 1 equation with periodic
#: boundaries, 256^2 Fourier grid on (0,100)^2, T = 6.
T2 = Problem("t2_cubic2d_256_periodic", (256, 256), PERIODIC, 0.0, 100.0,
             PAPER_CUBIC, 6.0 / 200, 200, "split4", 12, init="noise")

#: the paper's Table 4 setting: 3-D cubic-quintic CGL on (-12,12)^3 with
#: periodic boundaries, 128^3 Fourier grid, a1 = b1 = 1/2, a2 = -1/2,
#: a3 = 2.52, b3 = 1, a4 = -1, b4 = -0.11, necklace-ring datum, T = 5.
PAPER_CQ = Coeffs(0.5, 0.5, -0.5, 2.52, 1.0, -1.0, -0.11)
T4 = Problem("t4_cq3d_128_periodic", (128, 128, 128), PERIODIC, -12.0, 12.0,
             PAPER_CQ, 5.0 / 300, 300, "lawson4", 13, init="necklace")

#: batched sweep: 512 2-D cubic instances (see ``batched_sweep``).
C3_BATCH = 512
C3_SIZES = (64, 96, 128, 160, 192)
C3_TAU = 1e-2
C3_STEPS = 500
C3_SEED = 3

#: surrogate: 128^2 2-D cubic, jump of 50 Lawson4 steps.
C4_N = 128
C4_JUMP = 50
C4_TRAIN_SEED = 4
C4_EVAL_SEED = 5


def nodes(n: int, a: float, b: float, bc: int, bc_hi: int | None = None) -> np.ndarray:
    """1-D grid nodes for ``n`` unknowns on (a, b) (see module docstring).
    With ``bc_hi`` the two ends may differ: a Dirichlet end is not a node, a
    Neumann end is one (DN: x_j = a + j h, j = 1..n, h = (b-a)/n)."""
    if bc_hi is not None and bc_hi != bc:
        if bc == DIRICHLET and bc_hi == NEUMANN:
            h = (b - a) / n
            return a + h * np.arange(1, n + 1, dtype=np.float64)
        if bc == NEUMANN and bc_hi == DIRICHLET:
            h = (b - a) / n
            return a + h * np.arange(0, n, dtype=np.float64)
        raise ValueError("bc must be DIRICHLET or NEUMANN")
    if bc == PERIODIC:
        return a + (b - a) * np.arange(0, n, dtype=np.float64) / n
    if bc == DIRICHLET:
        h = (b - a) / (n + 1)
        return a + h * np.arange(1, n + 1, dtype=np.float64)
    if bc == NEUMANN:
        h = (b - a) / (n - 1)
        return a + h * np.arange(0, n, dtype=np.float64)
    raise ValueError("bc must be DIRICHLET or NEUMANN")


def mesh(p: Problem) -> List[np.ndarray]:
    """Coordinate arrays of shape p.n (index 1 first; 'ij' indexing)."""
    axes = [nodes(nm, p.a, p.b, p.bc) for nm in p.n]
    return list(np.meshgrid(*axes, indexing="ij"))


def random_phase_2d(rng: np.random.Generator, x: np.ndarray, y: np.ndarray,
                    L: float = 20.0) -> np.ndarray:
    """Smooth random phase: 4 low Fourier modes with wave numbers (p, q) drawn
    from {0,1,2}^2 minus (0,0), N(0,1) amplitudes and U(0, 2 pi) shifts."""
    pairs = [(p, q) for p in range(3) for q in range(3) if (p, q) != (0, 0)]
    pick = rng.choice(len(pairs), size=4, replace=False)
    amp = rng.standard_normal(4)
    shift = rng.uniform(0.0, 2.0 * np.pi, size=4)
    theta = np.zeros_like(x)
    for m in range(4):
        p, q = pairs[pick[m]]
        theta += amp[m] * np.cos(2.0 * np.pi * (p * x + q * y) / L + shift[m])
    return theta


def gaussian_phase_2d(n: Sequence[int], a: float, b: float, bc: int, seed: int,
                      noise: float = 0.1) -> np.ndarray:
    """u0 = (1 + noise xi) exp(-(x^2+y^2)) exp(i theta), xi ~ U(-1,1) per point."""
    rng = np.random.default_rng(seed)
    x, y = [np.asarray(c) for c in np.meshgrid(nodes(n[0], a, b, bc),
                                               nodes(n[1], a, b, bc), indexing="ij")]
    xi = rng.uniform(-1.0, 1.0, size=x.shape)
    theta = random_phase_2d(rng, x, y, L=(b - a))
    return ((1.0 + noise * xi) * np.exp(-(x * x + y * y)) * np.exp(1j * theta)).astype(np.complex128)


def vortex_ring_3d(n: Sequence[int], a: float, b: float, bc: int, seed: int,
                   radius: float = 5.0, width: float = 2.5, charge: int = 1,
                   noise: float = 0.01) -> np.ndarray:
    """Gaussian vortex ring of amplitude 1: (1 + noise xi) exp(-((rho-R)^2+z^2)/w^2) e^{i k atan2(y,x)}."""
    rng = np.random.default_rng(seed)
    x, y, z = np.meshgrid(nodes(n[0], a, b, bc), nodes(n[1], a, b, bc),
                          nodes(n[2], a, b, bc), indexing="ij")
    xi = rng.uniform(-1.0, 1.0, size=x.shape)
    rho = np.sqrt(x * x + y * y)
    env = np.exp(-((rho - radius) ** 2 + z * z) / (width * width))
    return ((1.0 + noise * xi) * env * np.exp(1j * charge * np.arctan2(y, x))).astype(np.complex128)


def necklace_ring(n: Sequence[int], a: float, b: float, bc: int, delta: float = 1.2,
                  rho0: float = 6.0, omega: float = 2.5, eta: int = 5,
                  kappa: int = 3) -> np.ndarray:
    """The necklace ring of Section 4.3: delta sech(sqrt((rho - rho0)^2 + z^2) / omega)
    cos(eta theta) exp(i kappa theta), rho = sqrt(x^2 + y^2), theta = atan2(y, x)."""
    x, y, z = np.meshgrid(nodes(n[0], a, b, bc), nodes(n[1], a, b, bc), nodes(n[2], a, b, bc),
                          indexing="ij")
    rho = np.sqrt(x * x + y * y)
    theta = np.arctan2(y, x)
    r = np.sqrt((rho - rho0) ** 2 + z * z)
    return (delta / np.cosh(r / omega) * np.cos(eta * theta) * np.exp(1j * kappa * theta)).astype(
        np.complex128)


def initial_state(p: Problem) -> np.ndarray:
    """Seeded u0 of shape p.n (complex128)."""
    if p.init == "noise":
        rng = np.random.default_rng(p.seed)
        return (rng.standard_normal(p.n) / 5000.0).astype(np.complex128)
    if p.init == "necklace":
        return necklace_ring(p.n, p.a, p.b, p.bc)
    if p.d == 2:
        return gaussian_phase_2d(p.n, p.a, p.b, p.bc, p.seed)
    if p.d == 3:
        return vortex_ring_3d(p.n, p.a, p.b, p.bc, p.seed)
    if p.d == 1:
        rng = np.random.default_rng(p.seed)
        x = nodes(p.n[0], p.a, p.b, p.bc)
        xi = rng.uniform(-1.0, 1.0, size=x.shape)
        return ((1.0 + 0.1 * xi) * np.exp(-x * x) * np.exp(1j * 0.5 * x)).astype(np.complex128)
    raise ValueError("d must be 1, 2 or 3")


def flat(u: np.ndarray) -> np.ndarray:
    """Column-stacking vec(U): index 1 fastest (the layout the library uses)."""
    return np.ascontiguousarray(u.reshape(-1, order="F"))


def unflat(v: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    return np.asarray(v).reshape(tuple(shape), order="F")


def scaled(p: Problem, n: Tuple[int, ...], steps: int | None = None,
           name: str | None = None) -> Problem:
    """The same workload on a smaller grid (for oracle-sized parity cases)."""
    return dataclasses.replace(p, n=tuple(n), steps=p.steps if steps is None else steps,
                               name=name or f"{p.name}@{'x'.join(map(str, n))}")


def batched_sweep(count: int = C3_BATCH, seed: int = C3_SEED,
                  sizes: Sequence[int] = C3_SIZES, fixed_n: int | None = None) -> List[Problem]:
    """Batched sweep of independent 2-D cubic instances.

    Per instance: n1, n2 uniform over ``sizes`` (or both ``fixed_n``),
    a1 ~ U(0.5,2), b1 ~ U(-2,2), a2 ~ U(-0.5,0.5), a3 ~ U(-1.5,-0.5),
    b3 ~ U(0.5,2); Dirichlet on (-10,10)^2; the Gaussian-plus-noise u0 of the
    2-D workload with seed 1000*seed + j.
    """
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        if fixed_n is None:
            n1, n2 = (int(v) for v in rng.choice(np.asarray(sizes), size=2))
        else:
            n1 = n2 = int(fixed_n)
        c = Coeffs(float(rng.uniform(0.5, 2.0)), float(rng.uniform(-2.0, 2.0)),
                   float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-1.5, -0.5)),
                   float(rng.uniform(0.5, 2.0)))
        out.append(Problem(f"c3_inst{j}", (n1, n2), DIRICHLET, -10.0, 10.0, c,
                           C3_TAU, C3_STEPS, "lawson4", 1000 * seed + j))
    return out


def coeff_ranges() -> Dict[str, Tuple[float, float]]:
    """Ranges of the batched sweep's coefficients (used to standardise the
    surrogate's coefficient planes)."""
    return {"a1": (0.5, 2.0), "b1": (-2.0, 2.0), "a2": (-0.5, 0.5),
            "a3": (-1.5, -0.5), "b3": (0.5, 2.0)}


def random_complex(shape: Sequence[int], seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain seeded complex Gaussian test data (for kernel-level parity)."""
    rng = np.random.default_rng(seed)
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex128)
