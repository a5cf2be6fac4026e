"""Seeded synthetic inputs and workload definitions.

Shared by the tests, the benchmark and the smoke check; holds none of the
step's arithmetic (no sub-step, no sweep, no observable).  Every state is
numpy complex128 of shape (Nz, Ny, Nx) on the node grid x_i = (i-(N-1)/2) dx,
normalised so that dx*dy*dz*sum|psi|^2 = 1 where the workload says
"normalised".

The paper's own input files are not available, so these stand in for them:
the workloads below carry the grid sizes, traps, couplings and initial-state
shapes of the target configurations (a Gaussian, a Thomas-Fermi profile with
noise, a ground-state-like profile with phase noise).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def axis(n: int, d: float) -> np.ndarray:
    """Node coordinates of one axis, symmetric about 0."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * d


def mesh(grid, dx):
    """Broadcastable (z, y, x) coordinate arrays for grid (Nx, Ny, Nz)."""
    nx, ny, nz = grid
    x = axis(nx, dx[0])[None, None, :]
    y = axis(ny, dx[1])[None, :, None]
    z = axis(nz, dx[2])[:, None, None]
    return x, y, z


def normalise(psi: np.ndarray, dx) -> np.ndarray:
    """Scale psi (in place) to dx*dy*dz*sum|psi|^2 = 1: defines a normalised input."""
    s = float(np.vdot(psi, psi).real) * dx[0] * dx[1] * dx[2]
    psi *= 1.0 / math.sqrt(s)
    return psi


def gaussian(grid, dx, omega) -> np.ndarray:
    """exp(-(gamma x^2 + nu y^2 + lambda z^2)/2), normalised."""
    x, y, z = mesh(grid, dx)
    g, n, l = omega
    psi = np.exp(-0.5 * (g * x * x + n * y * y + l * z * z)).astype(np.complex128)
    return normalise(psi, dx)


def separable_gaussian(grid, dx, omega, dtype=np.complex64) -> np.ndarray:
    """The same normalised Gaussian as `gaussian`, built from three 1D
    factors (outer products, no 3D exponential) in the requested dtype --
    fast enough to make one per served request."""
    f = [np.exp(-0.5 * w * axis(n, d) ** 2) for n, d, w in zip(grid, dx, omega)]
    f = [v / math.sqrt(float(np.dot(v, v)) * d) for v, d in zip(f, dx)]
    zy = np.multiply.outer(f[2], f[1])
    return np.multiply.outer(zy, f[0]).astype(dtype)


def mu_thomas_fermi(omega, g: float) -> float:
    """Thomas-Fermi chemical potential 1/2 (15 g gamma nu lambda / (4 pi))^(2/5)."""
    return 0.5 * (15.0 * g * omega[0] * omega[1] * omega[2] / (4.0 * math.pi)) ** 0.4


def thomas_fermi(grid, dx, omega, g: float, noise: float = 0.0, seed: int = 0,
                 floor: float = 0.0) -> np.ndarray:
    """sqrt(max(0, (mu_TF - V)/g)) + complex Gaussian noise of std `noise` per
    component, normalised.  `floor` adds a small Gaussian tail so the state
    has no exact zeros (optional).  Built one z plane at a time (the noise
    of plane k is drawn after that of plane k-1: real parts, then imaginary
    parts), so large grids need no grid-sized temporaries."""
    nx, ny, nz = grid
    x = axis(nx, dx[0])[None, :]
    y = axis(ny, dx[1])[:, None]
    z = axis(nz, dx[2])
    vxy = 0.5 * (omega[0] ** 2 * x * x + omega[1] ** 2 * y * y)
    mu = mu_thomas_fermi(omega, g)
    rng = np.random.default_rng(seed) if noise else None
    psi = np.empty((nz, ny, nx), dtype=np.complex128)
    for k in range(nz):
        V = vxy + 0.5 * omega[2] ** 2 * z[k] * z[k]
        amp = np.sqrt(np.maximum(0.0, (mu - V) / g))
        if floor:
            amp = amp + floor * np.exp(-V / max(mu, 1e-300))
        plane = psi[k]
        plane.real = amp
        plane.imag = 0.0
        if noise:
            plane.real += noise * rng.standard_normal((ny, nx))
            plane.imag += noise * rng.standard_normal((ny, nx))
    return normalise(psi, dx)


def phase_noise(psi: np.ndarray, amplitude: float, seed: int) -> np.ndarray:
    """psi * exp(i theta), theta ~ U(-amplitude, amplitude) per point (in
    place), drawn one z plane at a time."""
    rng = np.random.default_rng(seed)
    for k in range(psi.shape[0]):
        psi[k] *= np.exp(1j * rng.uniform(-amplitude, amplitude, psi.shape[1:]))
    return psi


def random_state(grid, dx, seed: int) -> np.ndarray:
    """Complex standard-normal values per point, normalised (parity inputs)."""
    rng = np.random.default_rng(seed)
    shape = (grid[2], grid[1], grid[0])
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return normalise(psi, dx)


def smooth_random_state(grid, dx, omega, seed: int) -> np.ndarray:
    """A Gaussian envelope times a random complex field: smooth on the scale
    of the trap but with every mode excited."""
    psi = gaussian(grid, dx, omega) * (1.0 + 0.3 * random_state(grid, dx, seed) *
                                       math.sqrt(dx[0] * dx[1] * dx[2] * grid[0] * grid[1] * grid[2]))
    return normalise(psi, dx)


def sine_mode(grid, modes) -> np.ndarray:
    """prod_a sin(pi m_a (i_a + 1) / (N_a + 1)): unnormalised lattice sine mode."""
    nx, ny, nz = grid
    mx, my, mz = modes
    sx = np.sin(math.pi * mx * (np.arange(nx) + 1) / (nx + 1))
    sy = np.sin(math.pi * my * (np.arange(ny) + 1) / (ny + 1))
    sz = np.sin(math.pi * mz * (np.arange(nz) + 1) / (nz + 1))
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).astype(np.complex128)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    grid: tuple          # (Nx, Ny, Nz)
    dx: tuple
    dt: float
    omega: tuple         # (gamma, nu, lambda)
    g: float
    mode: str            # "imag" | "real"
    steps: int
    g_after: float | None = None   # real-time quench: g for the timed steps
    description: str = ""

    @property
    def points(self) -> int:
        return self.grid[0] * self.grid[1] * self.grid[2]


# Smallest case: imaginary time, 32^3, dx 0.25, dt = 0.1 dx^2, trap (1, 1.4, 2),
# g = 10, normalised Gaussian start, 200 steps.
SMALL_IMAG = Workload(
    name="imag-32^3", grid=(32, 32, 32), dx=(0.25,) * 3, dt=0.1 * 0.25 ** 2,
    omega=(1.0, 1.4, 2.0), g=10.0, mode="imag", steps=200,
    description="imaginary time, 32^3, dx 0.25, dt 0.1 dx^2, trap (1, 1.4, 2), g 10, Gaussian start")

# Real-time quench: 240x200x160, dx 0.1, dt = 0.005 dx^2, trap (0.5, 1, 1.5),
# ground state at g = 22 with 1e-3 phase noise, then g -> 11 for 1000 steps.
QUENCH = Workload(
    name="real-240x200x160-quench", grid=(240, 200, 160), dx=(0.1,) * 3, dt=0.005 * 0.1 ** 2,
    omega=(0.5, 1.0, 1.5), g=22.0, g_after=11.0, mode="real", steps=1000,
    description="real time, 240x200x160, dx 0.1, dt 5e-5, trap (0.5, 1, 1.5), g 22 -> 11")

# Large real-time run: 512x512x384, dx 0.05, trap (1, 1.2, 4), g 2000,
# Thomas-Fermi start with 1e-4 Gaussian noise, 500 steps; dt = 0.005 dx^2.
LARGE_REAL = Workload(
    name="real-512x512x384", grid=(512, 512, 384), dx=(0.05,) * 3, dt=0.005 * 0.05 ** 2,
    omega=(1.0, 1.2, 4.0), g=2000.0, mode="real", steps=500,
    description="real time, 512x512x384, dx 0.05, dt 1.25e-5, trap (1, 1.2, 4), g 2000, TF + 1e-4 noise")

WORKLOADS = {w.name: w for w in (SMALL_IMAG, QUENCH, LARGE_REAL)}

# Batch of independent imaginary-time ground-state solves of uneven sizes:
# grids drawn from five shapes, traps uniform in [0.5, 3] per axis, g
# log-uniform in [1, 1000], dx 0.2, dt = 0.1 dx^2, Gaussian start per solve.
BATCH_GRIDS = ((48, 48, 48), (64, 64, 64), (96, 64, 48), (128, 96, 64), (160, 160, 160))


def batch_imag_specs(n: int = 256, seed: int = 3, dx: float = 0.2, grids=BATCH_GRIDS) -> list:
    """Seeded specs of a batch of imaginary-time solves (dicts with grid,
    dx, dt, trap, g)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        grid = tuple(grids[int(rng.integers(len(grids)))])
        trap = tuple(float(v) for v in rng.uniform(0.5, 3.0, 3))
        g = float(np.exp(rng.uniform(0.0, np.log(1000.0))))
        out.append({"grid": grid, "dx": dx, "dt": 0.1 * dx * dx, "trap": trap, "g": g})
    return out


def quench_relaxation_start(w: Workload) -> np.ndarray:
    """Where the quench workload's ground state is relaxed from: the
    Thomas-Fermi profile of its trap and g = 22 with a small Gaussian tail
    (real, no noise).  The benchmark relaxes it in imaginary time with the
    library itself, then applies phase_noise(psi, 1e-3, 2)."""
    return thomas_fermi(w.grid, w.dx, w.omega, w.g, floor=1e-3)


def initial_state(w: Workload, seed: int | None = None) -> np.ndarray:
    """The documented starting state of a workload (host, complex128).

    The quench workload starts from its imaginary-time ground state, which
    the method itself produces; the parity tests stand in for it with the
    Thomas-Fermi profile of the same trap and g (with a small Gaussian tail)
    times the 1e-3 phase noise, which is what this returns.  The benchmark's
    quench leg instead relaxes quench_relaxation_start in imaginary time on
    the GPU and adds the same phase noise."""
    if w is SMALL_IMAG or w.name == SMALL_IMAG.name:
        return gaussian(w.grid, w.dx, w.omega)
    if w.name == QUENCH.name:
        psi = thomas_fermi(w.grid, w.dx, w.omega, w.g, floor=1e-3)
        return phase_noise(psi, 1e-3, 2 if seed is None else seed)
    if w.name == LARGE_REAL.name:
        return thomas_fermi(w.grid, w.dx, w.omega, w.g, noise=1e-4, seed=5 if seed is None else seed)
    raise KeyError(w.name)
