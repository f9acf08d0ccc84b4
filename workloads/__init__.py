"""Seeded synthetic inputs for the stencil workloads.

This module only draws random numbers and lays out physical inputs (initial
fields, velocity models, source wavelets, positions).  It holds none of the
stencil arithmetic: both the FP64 oracle and the GPU path consume what it
returns, so neither depends on the other.

Workloads follow the shapes of the paper's Devito benchmarks (Section 6.1:
heat diffusion and the isotropic acoustic wave, 2D/3D, space orders 2/4/8,
FP32 fields).  The paper names no dataset; every input is synthetic.

Recipe readings where the paper is silent:
  * velocity: depth (slowest axis) is split into 8 equal layers with
    v_j = 1500 + 3000*j/7 m/s, each point scaled by (1 + 0.05*U[-1,1)).
  * dt: half the leapfrog stability limit of the 3D space-order-8 star,
    dt = 0.5 * 2h / (v_max * sqrt(3 * S8)), S8 = 2048/315 being the largest
    magnitude of that operator's symbol; a literal Courant number of 0.5 is
    unstable for this stencil.
  * source: unit Ricker wavelet, f0 = 10 Hz, t0 = 1/f0, injected after each
    sweep as dt^2 * v_s^2 * w(n*dt) at one grid point.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20240402
# Largest |symbol| of the centred 8th-order second difference, used only to
# pick the timestep of the wave workloads (recipe constant, see module doc).
S8_SYMBOL_MAX = 2048.0 / 315.0


def seed_for(config_index: int) -> int:
    return SEED_BASE + int(config_index)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


# ----------------------------------------------------------------------------
# storage rounding
# ----------------------------------------------------------------------------

_STORAGE = ("f32", "bf16", "f16", "f64")


def round_to_storage(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round an FP64 array to the storage dtype (round to nearest even) and
    return the rounded values as FP64."""
    a = np.asarray(a, dtype=np.float64)
    if dtype == "f64":
        return a.copy()
    if dtype == "f32":
        return a.astype(np.float32).astype(np.float64)
    if dtype == "f16":
        return a.astype(np.float16).astype(np.float64)
    if dtype == "bf16":
        import torch

        t = torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16)
        return t.to(torch.float64).numpy()
    raise ValueError(f"unknown storage dtype {dtype!r}; expected one of {_STORAGE}")


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def uniform_field(rng: np.random.Generator, shape) -> np.ndarray:
    """U[0,1) interior values in FP64."""
    return rng.random(tuple(int(s) for s in shape), dtype=np.float64)


def gaussian_bump(shape, sigma: float, amplitude: float = 1.0) -> np.ndarray:
    """amplitude * exp(-|x-c|^2 / (2 sigma^2)) with c at the box centre (n-1)/2."""
    shape = tuple(int(s) for s in shape)
    out = np.zeros(shape, dtype=np.float64)
    axes = [np.arange(n, dtype=np.float64) - (n - 1) / 2.0 for n in shape]
    r2 = np.zeros(shape, dtype=np.float64)
    for d, ax in enumerate(axes):
        sh = [1] * len(shape)
        sh[d] = shape[d]
        r2 = r2 + (ax.reshape(sh) ** 2)
    out[...] = amplitude * np.exp(-r2 / (2.0 * sigma * sigma))
    return out


def layered_velocity(rng: np.random.Generator, shape, layers: int = 8,
                     vmin: float = 1500.0, vmax: float = 4500.0,
                     noise: float = 0.05) -> np.ndarray:
    """Layered velocity (m/s): depth = axis 0, `layers` equal-thickness bands,
    each point scaled by (1 + noise*U[-1,1))."""
    shape = tuple(int(s) for s in shape)
    nz = shape[0]
    z = np.arange(nz)
    j = np.minimum((z * layers) // nz, layers - 1)
    vj = vmin + (vmax - vmin) * j / (layers - 1)
    sh = [nz] + [1] * (len(shape) - 1)
    v = np.broadcast_to(vj.reshape(sh).astype(np.float64), shape).copy()
    v *= 1.0 + noise * (2.0 * rng.random(shape, dtype=np.float64) - 1.0)
    return v


def wave_dt(vmax: float, h: float, ndim: int = 3, fraction: float = 0.5,
            symbol_max: float = S8_SYMBOL_MAX) -> float:
    """Timestep at `fraction` of the leapfrog stability limit
    dt_crit = 2h / (vmax * sqrt(ndim * symbol_max))."""
    return fraction * 2.0 * h / (vmax * math.sqrt(ndim * symbol_max))


def ricker(t: np.ndarray, f0: float = 10.0, t0: float | None = None) -> np.ndarray:
    """Unit-amplitude Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2)."""
    if t0 is None:
        t0 = 1.0 / f0
    a = (math.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def source_amplitudes(wavelet: np.ndarray, dt: float, v_at_source: float) -> np.ndarray:
    """Per-step injected amount dt^2 * v_s^2 * w(t_n), FP64."""
    return (dt * dt) * (v_at_source ** 2) * np.asarray(wavelet, dtype=np.float64)


def beta_from_velocity(v: np.ndarray, dt: float, h: float) -> np.ndarray:
    """Coefficient field (dt * v / h)^2 carried by the wave sweep, FP64."""
    return (dt * np.asarray(v, dtype=np.float64) / h) ** 2


def embed(interior: np.ndarray, halo: int) -> np.ndarray:
    """Dense buffer with a zero halo of width `halo` around `interior`."""
    interior = np.asarray(interior, dtype=np.float64)
    out = np.zeros(tuple(s + 2 * halo for s in interior.shape), dtype=np.float64)
    sl = tuple(slice(halo, halo + s) for s in interior.shape)
    out[sl] = interior
    return out


def interior_of(buf: np.ndarray, halo: int) -> np.ndarray:
    sl = tuple(slice(halo, s - halo) for s in buf.shape)
    return buf[sl]


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

@dataclass
class HeatProblem:
    name: str
    ndim: int
    shape: tuple
    radius: int
    halo: int
    alpha: float
    nsteps: int
    seed: int
    u0: np.ndarray  # interior, FP64 (not yet rounded)


@dataclass
class WaveProblem:
    name: str
    shape: tuple
    radius: int
    halo: int
    h: float
    dt: float
    nsteps: int
    seed: int
    velocity: np.ndarray          # interior, m/s, FP64
    src: np.ndarray               # [nsrc, 3] interior coordinates (z, y, x)
    src_amp: np.ndarray           # [nsteps, nsrc] FP64 amounts added after each sweep
    rec: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int64))
    extra: dict = field(default_factory=dict)

    @property
    def beta(self) -> np.ndarray:
        return beta_from_velocity(self.velocity, self.dt, self.h)


def heat2d_c1(n: int = 256, nsteps: int = 100) -> HeatProblem:
    """2D 5-point heat / Jacobi, Dirichlet-zero halo of 1, alpha = 0.2."""
    seed = seed_for(0)
    rng = rng_for(seed)
    return HeatProblem("heat2d_so2", 2, (n, n), 1, 1, 0.2, nsteps, seed,
                       uniform_field(rng, (n, n)))


def heat3d_c2(n: int = 512, nsteps: int = 50, sigma: float = 16.0) -> HeatProblem:
    """3D 13-point heat (space order 4), halo 2, alpha = 0.05, U[0,1) plus a
    unit Gaussian bump of width sigma cells at the centre."""
    seed = seed_for(1)
    rng = rng_for(seed)
    shape = (n, n, n)
    u0 = uniform_field(rng, shape)
    u0 += gaussian_bump(shape, sigma)
    return HeatProblem("heat3d_so4", 3, shape, 2, 2, 0.05, nsteps, seed, u0)


def wave3d_c3(n: int = 512, nsteps: int = 400, h: float = 10.0, f0: float = 10.0,
              shape: tuple | None = None) -> WaveProblem:
    """3D acoustic wave, space order 8 (radius 4, halo 4), layered velocity,
    Ricker source at the interior centre floor(n_d/2)."""
    seed = seed_for(2)
    rng = rng_for(seed)
    shape = tuple(shape) if shape is not None else (n, n, n)
    v = layered_velocity(rng, shape)
    dt = wave_dt(float(v.max()), h)
    src = np.array([[s // 2 for s in shape]], dtype=np.int64)
    vs = float(v[tuple(src[0])])
    w = ricker(np.arange(nsteps) * dt, f0)
    amp = source_amplitudes(w, dt, vs).reshape(nsteps, 1)
    return WaveProblem("wave3d_so8", shape, 4, 4, h, dt, nsteps, seed, v, src, amp)


@dataclass
class BatchProblem:
    name: str
    shots: list  # list[WaveProblem]
    nsteps: int
    seed: int


def batch_c4(nshots: int = 32, nmin: int = 128, nmax: int = 384, nsteps: int = 200,
             h: float = 10.0, f0: float = 10.0) -> BatchProblem:
    """Independent so-8 wave shots of seeded uneven cubic sizes, one source
    each, placed uniformly at least 2r = 8 cells from the interior faces."""
    seed = seed_for(3)
    rng = rng_for(seed)
    sizes = rng.integers(nmin, nmax + 1, size=nshots)
    shots = []
    for i, n in enumerate(sizes):
        n = int(n)
        srng = rng_for(seed * 1000 + i)
        shape = (n, n, n)
        v = layered_velocity(srng, shape)
        dt = wave_dt(float(v.max()), h)
        src = srng.integers(8, n - 8, size=3).reshape(1, 3).astype(np.int64)
        vs = float(v[tuple(src[0])])
        w = ricker(np.arange(nsteps) * dt, f0)
        amp = source_amplitudes(w, dt, vs).reshape(nsteps, 1)
        shots.append(WaveProblem(f"shot{i}", shape, 4, 4, h, dt, nsteps,
                                 seed * 1000 + i, v, src, amp))
    return BatchProblem("batch_so8", shots, nsteps, seed)


@dataclass
class InversionProblem:
    name: str
    shape: tuple
    radius: int
    halo: int
    h: float
    dt: float
    nsteps: int
    checkpoint_every: int
    seed: int
    v0: np.ndarray        # background velocity (interior)
    v_true: np.ndarray    # true velocity (interior)
    src: np.ndarray       # [1,3]
    wavelet: np.ndarray   # [nsteps] unit Ricker samples w(n dt)
    rec: np.ndarray       # [nrec,3]

    @property
    def m0(self) -> np.ndarray:
        return 1.0 / (self.v0 ** 2)

    @property
    def m_true(self) -> np.ndarray:
        return 1.0 / (self.v_true ** 2)


def receiver_line(n: int, nrec: int = 64, depth: int = 8) -> np.ndarray:
    """nrec receivers at z = depth, y = floor(n/2), x_j = round(32 + j (n-64)/(nrec-1))."""
    xs = [int(round(32 + j * (n - 64) / (nrec - 1))) for j in range(nrec)]
    return np.array([[depth, n // 2, x] for x in xs], dtype=np.int64)


def inversion_c5(n: int = 256, nsteps: int = 500, nrec: int = 64, h: float = 10.0,
                 f0: float = 20.0, checkpoint_every: int = 25,
                 anomaly_sigma: float = 12.0, anomaly: float = 0.05,
                 anomaly_depth: int = 16) -> InversionProblem:
    """so-8 wave gradient workload: layered background, a +5% Gaussian
    velocity anomaly (sigma 12 cells) centred `anomaly_depth` cells below the
    source and receiver plane with its horizontal centre seeded within n/16
    of the source, a surface receiver line and a source at (8, n/2, n/2).

    500 steps at the stability-derived dt last 0.24 s; a wavefield started
    near the surface only reaches a few tens of cells in that time, so the
    perturbation sits where it is illuminated (a centred anomaly would leave
    the data, and the misfit, unchanged)."""
    seed = seed_for(4)
    rng = rng_for(seed)
    shape = (n, n, n)
    v0 = layered_velocity(rng, shape)
    depth = min(8, n - 1)
    off = rng.uniform(-n / 16.0, n / 16.0, size=2)
    c = np.array([depth + anomaly_depth, n // 2 + off[0], n // 2 + off[1]], dtype=np.float64)
    axes = [np.arange(n, dtype=np.float64) - c[d] for d in range(3)]
    r2 = (axes[0].reshape(n, 1, 1) ** 2 + axes[1].reshape(1, n, 1) ** 2
          + axes[2].reshape(1, 1, n) ** 2)
    v_true = v0 * (1.0 + anomaly * np.exp(-r2 / (2.0 * anomaly_sigma ** 2)))
    dt = wave_dt(float(max(v0.max(), v_true.max())), h)
    src = np.array([[depth, n // 2, n // 2]], dtype=np.int64)
    rec = receiver_line(n, nrec, depth=depth)
    w = ricker(np.arange(nsteps) * dt, f0)
    return InversionProblem("adjoint_so8", shape, 4, 4, h, dt, nsteps, checkpoint_every,
                            seed, v0, v_true, src, w, rec)


def damping_profiles(shape, width, gmax):
    """Per-axis absorbing-layer profiles (an input of the damped wave): on
    each axis, gmax * ((width - d) / width)^2 at distance d < width points
    from the nearer end, 0 inside."""
    out = []
    for n in shape:
        d = np.minimum(np.arange(n), np.arange(n)[::-1]).astype(np.float64)
        out.append(np.where(d < width, gmax * ((width - d) / width) ** 2, 0.0))
    return out

