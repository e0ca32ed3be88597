"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only draws and shapes problem inputs: velocity models,
source/receiver positions, the source time function, noise draws,
perturbation directions, initial network weights and shuffle orders.
It holds none of the method's arithmetic (no time stepping, adjoint,
misfit, sponge, normalisation or network evaluation), so neither side
of a parity test can inherit a mistake from the other through it.

Recipes (paper Sec. 2 problem statement; Sec. 4.1 workload shape):
  * wave speed: flat layers times (1 + 0.05 r), r a standardised
    Gaussian random field with correlation exp(-d^2 / (2 l^2));
    the small 2D case uses 4 layers and one Gaussian anomaly instead.
  * start model: the true model smoothed by a Gaussian filter.
  * source: Ricker wavelet (the paper's Sec. 4.1 source time function
    with sigma_t = 1/(sqrt(2) pi f0), delayed by 1.5/f0) times a spatial
    Gaussian of std 50 m (Sec. 4.1 smooths its sources with a narrow
    Gaussian of std 0.05 in a 1 km box), truncated at 3 std and normalised
    to unit sum, acting on the vertical velocity; wavelet values carry the
    1/dx^d of a cell volume.
  * receivers: vertical-velocity faces at depth index 2 on a regular
    surface grid.
  * dt = CFL * dx / max(c_true) with CFL = 0.4.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy import ndimage

CFL = 0.4


@dataclasses.dataclass
class Problem:
    """One seeded workload. Arrays are float64 (cast as needed by the user)."""
    name: str
    nz: int
    ny: int
    nx: int
    dx: float
    dt: float
    nt: int
    sponge: int
    c_ref: float                 # speed that sets the sponge strength (max of c_true)
    c_true: np.ndarray           # [nz, ny, nx]
    c_start: np.ndarray          # [nz, ny, nx]
    src: np.ndarray              # [S, 3] int32 (k, j, i) of the v_z face carrying the force
    rec: np.ndarray              # [R, 3] int32 (k, j, i) of the v_z faces sampled
    wavelet: np.ndarray          # [S, T] force density b_z^n (already divided by dx^d)
    f0: np.ndarray               # [S] peak frequencies
    noise: np.ndarray            # [S, T, R] standard normal draws for the data noise
    src_w: np.ndarray = None     # [2R+1, 2R+1 | 1, 2R+1] spatial weights of every source
    noise_level: float = 0.01    # sigma = noise_level * max|d_clean|
    periodic: int = 0

    @property
    def src_radius(self) -> int:
        return 0 if self.src_w is None else (self.src_w.shape[0] - 1) // 2

    @property
    def dims(self) -> int:
        return 2 if self.ny == 1 else 3

    @property
    def n(self) -> int:
        return self.nz * self.ny * self.nx


def ricker(f0: float, dt: float, nt: int) -> np.ndarray:
    """Ricker wavelet r(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
    tau = t - 1.5/f0, sampled at t = n dt, n = 0..nt-1."""
    t = np.arange(nt, dtype=np.float64) * dt
    tau = t - 1.5 / f0
    a = (math.pi * f0 * tau) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def grf(shape: Tuple[int, ...], corr_cells: float, seed: int) -> np.ndarray:
    """Standardised stationary Gaussian random field: white N(0,1) noise
    smoothed with a periodic Gaussian of std corr/sqrt(2) so the correlation
    is exp(-d^2/(2 corr^2)); rescaled to zero mean and unit std."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    sig = [corr_cells / math.sqrt(2.0) if s > 1 else 0.0 for s in shape]
    r = ndimage.gaussian_filter(w, sigma=sig, mode="wrap")
    r -= r.mean()
    sd = r.std()
    return r / sd if sd > 0 else r


def layered(nz: int, ny: int, nx: int, speeds) -> np.ndarray:
    speeds = np.asarray(speeds, dtype=np.float64)
    layer = (np.arange(nz) * len(speeds)) // nz
    return np.broadcast_to(speeds[layer][:, None, None], (nz, ny, nx)).copy()


def smooth(c: np.ndarray, sigma_cells: float) -> np.ndarray:
    sig = [sigma_cells if s > 1 else 0.0 for s in c.shape]
    return ndimage.gaussian_filter(c, sigma=sig, mode="nearest")


def _surface_grid(first: int, step: int, count: int, k: int = 2) -> np.ndarray:
    a = first + step * np.arange(count)
    jj, ii = np.meshgrid(a, a, indexing="ij")
    return np.stack([np.full(jj.size, k), jj.ravel(), ii.ravel()], axis=1).astype(np.int32)


SOURCE_STD_M = 50.0


def source_weights(dx: float, dims: int, std_m: float = SOURCE_STD_M) -> np.ndarray:
    """Gaussian of std `std_m` sampled on the v_z faces around the source face,
    truncated at 3 std, normalised to unit sum; shape (2R+1, 2R+1 | 1, 2R+1)."""
    sc = std_m / dx
    R = int(math.ceil(3.0 * sc))
    k = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-k * k / (2.0 * sc * sc))
    gy = g if dims == 3 else np.ones(1)
    w = g[:, None, None] * gy[None, :, None] * g[None, None, :]
    return w / w.sum()


def _finish(name, nz, ny, nx, dx, nt, c_true, c_start, src, f0, rec, sponge=16,
            noise_seed=1, dt=None, periodic=0, src_std=SOURCE_STD_M) -> Problem:
    c_ref = float(c_true.max())
    if dt is None:
        dt = CFL * dx / c_ref
    d = 2 if ny == 1 else 3
    wav = np.stack([ricker(f, dt, nt) for f in f0]) / dx ** d
    rng = np.random.default_rng(noise_seed)
    noise = rng.standard_normal((len(src), nt, len(rec)))
    src_w = source_weights(dx, d, src_std) if src_std and src_std > 0 else None
    return Problem(name=name, nz=nz, ny=ny, nx=nx, dx=dx, dt=dt, nt=nt, sponge=sponge,
                   c_ref=c_ref, c_true=c_true, c_start=c_start,
                   src=np.asarray(src, dtype=np.int32), rec=np.asarray(rec, dtype=np.int32),
                   wavelet=wav, f0=np.asarray(f0, dtype=np.float64), noise=noise,
                   src_w=src_w, periodic=periodic)


def problem_2d_small(nt: int = 500) -> Problem:
    """128 x 128 2D box, dx 10 m, 4 layers of 32 cells (1.5/2.0/2.5/3.0 km/s)
    with a +5 % Gaussian anomaly (std 8 cells, centre uniform in [40, 88]^2,
    seed 0), one 15 Hz Ricker at (k, i) = (4, 64), 32 receivers at k = 2,
    i = 16 + 3 r; start model smoothed with std 8 cells."""
    nz = nx = 128
    c = layered(nz, 1, nx, [1500.0, 2000.0, 2500.0, 3000.0])
    rng = np.random.default_rng(0)
    za, xa = rng.uniform(40.0, 88.0, size=2)
    kk, ii = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    bump = np.exp(-((kk - za) ** 2 + (ii - xa) ** 2) / (2.0 * 8.0 ** 2))
    c = c * (1.0 + 0.05 * bump[:, None, :])
    c_start = smooth(c, 8.0)
    rec = np.stack([np.full(32, 2), np.zeros(32, int), 16 + 3 * np.arange(32)], axis=1)
    return _finish("2d-128x128-500", nz, 1, nx, 10.0, nt, c, c_start,
                   [[4, 0, 64]], [15.0], rec)


def problem_3d(nz: int, ny: int, nx: int, nt: int, dx: float = 20.0, f0: float = 8.0,
               corr: float = 10.0, smooth_cells: float = 10.0, rec_first: Optional[int] = None,
               rec_step: int = 3, rec_count: Optional[int] = None, sponge: int = 16,
               name: Optional[str] = None, model_seed: int = 0) -> Problem:
    """3D box: 8 flat layers at linspace(1500, 4500, 8) m/s times (1 + 0.05 r),
    r a GRF with correlation length `corr` cells (seed `model_seed`); one
    Ricker at (4, ny/2, nx/2); receivers on a regular surface grid at k = 2."""
    c = layered(nz, ny, nx, np.linspace(1500.0, 4500.0, 8))
    c = c * (1.0 + 0.05 * grf((nz, ny, nx), corr, model_seed))
    c_start = smooth(c, smooth_cells)
    if rec_first is None:
        rec_first = sponge + 1 if sponge else 1
    if rec_count is None:
        span = min(ny, nx) - rec_first - (sponge + 1 if sponge else 1)
        rec_count = max(1, min(64, span // rec_step + 1))
    rec = _surface_grid(rec_first, rec_step, rec_count)
    src = [[4, ny // 2, nx // 2]]
    return _finish(name or f"3d-{nz}x{ny}x{nx}-{nt}", nz, ny, nx, dx, nt, c, c_start,
                   src, [f0], rec, sponge=sponge)


def problem_256(nt: int = 2000) -> Problem:
    """The 256^3 x 2000-step gradient workload: dx 20 m, 8 Hz Ricker at
    (4, 128, 128), 64 x 64 receivers at (j, i) = 33 + 3 (a, b)."""
    return problem_3d(256, 256, 256, nt, rec_first=33, rec_step=3, rec_count=64,
                      name=f"3d-256^3-{nt}")


def problem_384(nt: int = 3000) -> Problem:
    """The 384^3 x 3000-step Hessian-vector workload (8 layers of 48 cells),
    receivers at 33 + 5 (a, b)."""
    return problem_3d(384, 384, 384, nt, rec_first=33, rec_step=5, rec_count=64,
                      name=f"3d-384^3-{nt}")


def problem_multisource(nt: int = 4000, nz: int = 256, ny: int = 512, nx: int = 512,
                        nsrc: int = 8) -> Problem:
    """512 x 512 (y, x) x 256 (z) box with 8 Ricker sources at 6..10 Hz,
    positions uniform inside the non-sponge area shrunk by 8 cells (seed 3),
    depth index 4; receivers at 32 + 7 (a, b)."""
    c = layered(nz, ny, nx, np.linspace(1500.0, 4500.0, 8))
    c = c * (1.0 + 0.05 * grf((nz, ny, nx), 10.0, 0))
    c_start = smooth(c, 10.0)
    rng = np.random.default_rng(3)
    lo = 16 + 8
    src = np.stack([np.full(nsrc, 4), rng.integers(lo, ny - lo, nsrc),
                    rng.integers(lo, nx - lo, nsrc)], axis=1)
    rec = _surface_grid(32, 7, 64)
    return _finish(f"3d-{nz}x{ny}x{nx}-{nt}-s{nsrc}", nz, ny, nx, 20.0, nt, c, c_start, src,
                   list(np.linspace(6.0, 10.0, nsrc)), rec)


def direction_grf(shape, corr_cells: float, seed: int = 2) -> np.ndarray:
    """Standardised GRF used as a perturbation direction (delta c = c * r)."""
    return grf(shape, corr_cells, seed)


def ae_init(in_dim: int = 2048, hidden: int = 512, latent: int = 32, seed: int = 4
            ) -> Dict[str, np.ndarray]:
    """Initial autoencoder parameters, U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for
    weights and biases, drawn in the fixed order W1 b1 W2 b2 W3 b3 W4 b4.
    Weights are stored input-major: W[fan_in, fan_out]."""
    rng = np.random.default_rng(seed)
    dims = [(in_dim, hidden), (hidden, latent), (latent, hidden), (hidden, in_dim)]
    out = {}
    for li, (fi, fo) in enumerate(dims, start=1):
        bound = 1.0 / math.sqrt(fi)
        out[f"W{li}"] = rng.uniform(-bound, bound, size=(fi, fo))
        out[f"b{li}"] = rng.uniform(-bound, bound, size=(fo,))
    return out


def shuffles(nsamples: int, epochs: int, seed: int = 5) -> np.ndarray:
    """One random permutation of range(nsamples) per epoch, int32 [epochs, nsamples]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(nsamples).astype(np.int32) for _ in range(epochs)])


def random_state(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) draws (test vectors for dot-product checks)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)


def smooth_random_state(nf: int, nz: int, ny: int, nx: int, seed: int,
                        corr: float = 3.0) -> np.ndarray:
    """Wave-like test states: per field a GRF times a random amplitude spread
    over six decades, so per-patch scales vary as in a real wavefield."""
    rng = np.random.default_rng(seed)
    out = np.empty((nf, nz, ny, nx))
    for f in range(nf):
        out[f] = grf((nz, ny, nx), corr, int(rng.integers(1 << 30)))
    env = np.exp(rng.uniform(np.log(1e-6), 0.0, size=(1, nz // 8 + 1, ny // 8 + 1, nx // 8 + 1)))
    env = np.repeat(np.repeat(np.repeat(env, 8, axis=1), 8, axis=2), 8, axis=3)
    return out * env[:, :nz, :ny, :nx]


def smooth_random_window(nlev: int, nsrc: int, nz: int, ny: int, nx: int, seed: int) -> np.ndarray:
    """Levels [nlev][nsrc][nz][ny][nx] float32 of a wave-like e field for the time
    codec: per source three GRFs (correlation 3 cells) oscillating in time at
    periods of about 14 to 60 levels with random phases, times a per-8^3-block
    amplitude spread over four decades and a per-source scale of 1e-9..1e-6."""
    rng = np.random.default_rng(seed)
    t = np.arange(nlev, dtype=np.float32)
    out = np.empty((nlev, nsrc, nz, ny, nx), np.float32)
    for s in range(nsrc):
        modes = [grf((nz, ny, nx), 3.0, int(rng.integers(1 << 30))).astype(np.float32) for _ in range(3)]
        om = rng.uniform(0.1, 0.45, 3)
        ph = rng.uniform(0.0, 2.0 * np.pi, 3)
        env = np.exp(rng.uniform(np.log(1e-4), 0.0, size=(nz // 8 + 1, ny // 8 + 1, nx // 8 + 1)))
        env = np.repeat(np.repeat(np.repeat(env, 8, axis=0), 8, axis=1), 8, axis=2)[:nz, :ny, :nx]
        env = (env * 10.0 ** rng.uniform(-9, -6)).astype(np.float32)
        for q in range(nlev):
            acc = np.zeros((nz, ny, nx), np.float32)
            for k in range(3):
                acc += np.float32(np.cos(om[k] * t[q] + ph[k])) * modes[k]
            out[q, s] = acc * env
    return out


def white_noise(shape, seed: int) -> np.ndarray:
    """Standard normal draws (the noise of one prior draw), float64."""
    return np.random.default_rng(seed).standard_normal(shape)


def keep_rows(ndraws: int, nstates: int, npatches: int, keep: float, seed: int) -> List[List[np.ndarray]]:
    """For each draw and each captured state, the sorted patch indices kept
    (each patch independently with probability `keep`): the random
    write-or-discard choice of the training-data generation."""
    rng = np.random.default_rng(seed)
    return [[np.flatnonzero(rng.random(npatches) < keep).astype(np.int32) for _ in range(nstates)]
            for _ in range(ndraws)]
