"""Synthetic templates, particles and starting rotations (see package doc)."""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

ROOT_SEED = 250901180


def seed_rng(config: int, kind: int, index: int, stream: int) -> np.random.Generator:
    """Independent generator per (config, kind, index, stream).

    kind 0 = template (stream 0: blob centres/amplitudes); kind 1 = particle
    (stream 1: rotation g*, 2: noise, 3: starting rotations).
    """
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(config, kind, index, stream))
    return np.random.default_rng(ss)


# ------------------------------------------------------------ rotations ----

def haar_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed unit quaternions (w, x, y, z): normalised Gaussians."""
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    q = np.atleast_2d(q)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def euler_zyz_to_matrix(e: np.ndarray) -> np.ndarray:
    """R_z(a) R_y(b) R_z(g) for Euler triples [..., 3]."""
    e = np.asarray(e, dtype=np.float64)
    a, b, g = e[..., 0], e[..., 1], e[..., 2]
    ca, sa, cb, sb, cg, sg = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(g), np.sin(g)
    R = np.empty(e.shape[:-1] + (3, 3))
    R[..., 0, 0] = ca * cb * cg - sa * sg
    R[..., 0, 1] = -ca * cb * sg - sa * cg
    R[..., 0, 2] = ca * sb
    R[..., 1, 0] = sa * cb * cg + ca * sg
    R[..., 1, 1] = -sa * cb * sg + ca * cg
    R[..., 1, 2] = sa * sb
    R[..., 2, 0] = -sb * cg
    R[..., 2, 1] = sb * sg
    R[..., 2, 2] = cb
    return R


def matrix_to_euler_zyz(R: np.ndarray) -> np.ndarray:
    """ZYZ Euler triples [..., 3] of rotation matrices [..., 3, 3]."""
    R = np.asarray(R, dtype=np.float64)
    beta = np.arccos(np.clip(R[..., 2, 2], -1.0, 1.0))
    sb = np.hypot(R[..., 0, 2], R[..., 1, 2])
    regular = sb > 1e-12
    alpha = np.where(regular, np.arctan2(R[..., 1, 2], R[..., 0, 2]),
                     np.arctan2(R[..., 1, 0], R[..., 0, 0]))
    gamma = np.where(regular, np.arctan2(R[..., 2, 1], -R[..., 2, 0]), 0.0)
    return np.stack([alpha, beta, gamma], axis=-1)


# ---------------------------------------------------------------- blobs ----

@dataclass
class Blobs:
    centres: np.ndarray      # [J, 3]
    amps: np.ndarray         # [J]
    sigma: float


def blob_template(rng: np.random.Generator, n_blobs: int, sigma: float = 0.1,
                  radius: float = 0.8) -> Blobs:
    """Random blob template: centres uniform in a ball, amplitudes U[0.5, 1]."""
    d = rng.standard_normal((n_blobs, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n_blobs) ** (1.0 / 3.0)
    amps = rng.uniform(0.5, 1.0, n_blobs)
    return Blobs(centres=d * r[:, None], amps=amps, sigma=sigma)


def render_blobs(blobs: Blobs, N: int, rot: np.ndarray | None = None) -> np.ndarray:
    """Sample sum_j A_j exp(-|x - R c_j|^2 / 2 sigma^2) on the N^3 grid (FP64).

    The Gaussian is separable, so the volume is sum_j A_j gx_j (x) gy_j (x) gz_j.
    """
    c = blobs.centres if rot is None else blobs.centres @ np.asarray(rot).T
    x = (np.arange(N) - (N - 1) / 2.0) * (2.0 / N)
    s2 = 2.0 * blobs.sigma ** 2
    gx = np.exp(-(x[None, :] - c[:, 0:1]) ** 2 / s2) * blobs.amps[:, None]
    gy = np.exp(-(x[None, :] - c[:, 1:2]) ** 2 / s2)
    gz = np.exp(-(x[None, :] - c[:, 2:3]) ** 2 / s2)
    gyz = (gy[:, :, None] * gz[:, None, :]).reshape(len(c), N * N)
    return (gx.T @ gyz).reshape(N, N, N)


# ---------------------------------------------------------- wedge / noise ----

def wedge_mask(N: int, tilt_deg: float = 60.0) -> np.ndarray:
    """rfftn-layout mask of sampled Fourier points: |k_z| <= tan(tilt) |k_x|."""
    kx = np.fft.fftfreq(N)[:, None, None]
    kz = np.fft.rfftfreq(N)[None, None, :]
    t = np.tan(np.radians(tilt_deg))
    m = np.abs(kz) <= t * np.abs(kx) + 1e-12
    return np.broadcast_to(m, (N, N, N // 2 + 1))


def apply_wedge(vol: np.ndarray, tilt_deg: float = 60.0) -> np.ndarray:
    N = vol.shape[0]
    F = np.fft.rfftn(vol, axes=(0, 1, 2))
    return np.fft.irfftn(F * wedge_mask(N, tilt_deg), s=vol.shape, axes=(0, 1, 2))


def add_noise(vol: np.ndarray, snr: float, rng: np.random.Generator) -> np.ndarray:
    """White noise with variance var(vol) / snr (SNR over all voxels)."""
    if snr is None or not np.isfinite(snr):
        return vol
    sigma = np.sqrt(np.var(vol) / snr)
    return vol + sigma * rng.standard_normal(vol.shape)


# -------------------------------------------------------------- workload ----

@dataclass
class Workload:
    """A synthetic alignment workload (one template, B particles)."""
    config: int
    N: int
    L_max: int
    bands: Tuple[int, ...]
    steps: int
    restarts: int
    n_blobs: int
    snr: float
    tilt_deg: float
    batch: int
    name: str = ""
    extra: dict = field(default_factory=dict)

    def template(self) -> Blobs:
        return blob_template(seed_rng(self.config, 0, 0, 0), self.n_blobs)

    def template_volume(self) -> np.ndarray:
        return render_blobs(self.template(), self.N).astype(np.float32)

    def truth(self, i: int) -> np.ndarray:
        """Planted rotation g*_i of particle i (matrix)."""
        return quat_to_matrix(haar_quaternions(seed_rng(self.config, 1, i, 1), 1))[0]

    def particle(self, i: int, wedge: bool = True, noise: bool = True) -> np.ndarray:
        vol = render_blobs(self.template(), self.N, self.truth(i))
        if wedge and self.tilt_deg is not None:
            vol = apply_wedge(vol, self.tilt_deg)
        if noise:
            vol = add_noise(vol, self.snr, seed_rng(self.config, 1, i, 2))
        return vol.astype(np.float32)

    def particles(self, idx, **kw) -> np.ndarray:
        return np.stack([self.particle(int(i), **kw) for i in idx])

    def starts(self, i: int) -> np.ndarray:
        """Starting rotations of particle i as ZYZ Euler triples [P, 3]."""
        q = haar_quaternions(seed_rng(self.config, 1, i, 3), self.restarts)
        return matrix_to_euler_zyz(quat_to_matrix(q))


def make_particles(w: Workload, idx, **kw) -> np.ndarray:
    return w.particles(idx, **kw)


def random_starts(w: Workload, idx) -> np.ndarray:
    return np.stack([w.starts(int(i)) for i in idx])


# One 32^3 particle, 20-blob template, SNR 0.1, L=8, bands 4 -> 8, 32 starts.
CONFIG1 = Workload(config=1, N=32, L_max=8, bands=(4, 8), steps=20, restarts=32,
                   n_blobs=20, snr=0.1, tilt_deg=60.0, batch=1,
                   name="1x32^3 L8 bands(4,8) P32 T20")
# 1000 particles at 64^3, 50-blob template, SNR 0.05, L=32, bands 8..32.
CONFIG2 = Workload(config=2, N=64, L_max=32, bands=(8, 16, 24, 32), steps=20,
                   restarts=64, n_blobs=50, snr=0.05, tilt_deg=60.0, batch=1000,
                   name="1000x64^3 L32 bands(8,16,24,32) P64 T20")
