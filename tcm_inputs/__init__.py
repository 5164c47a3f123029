"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *describes* workloads: wavelet samples, wave-speed models,
source and receiver positions.  It holds none of the method's arithmetic
(no (c dt/dx)^2 coefficient, no stencil, no trigger logic); each side
derives those from the arrays produced here.

Workloads (all dx = 1, thresholds absolute = relative * max|w|):

* ``c1``  64^3, c = 1, Courant 0.5, Ricker at (32,32,32), 100 steps, tau = 0.
* ``c2``  512^3 two-layer model (1500 m/s above z = 256, 3000 below),
          Courant 0.5 at 3000 m/s, Ricker 100 Hz at (256,256,64), 2000 steps,
          trigger 1e-6 / retire 1e-7 of the source peak.
* ``c3``  virtual 4096^3 smoothed-lognormal model (seed 3), Courant 0.5 at
          4500 m/s, Ricker 100 Hz at the centre, 3000 steps, 64 GB pool cap.
* ``c4``  64 shots of uneven size (edges 96..384), per-shot lognormal models.
* ``c5``  256^3 lognormal model (seed 5), source (128,128,16), 1000 steps,
          128 receivers on z = 240, +2 % Gaussian anomaly for the observed data.

The paper's own scenario (sphere + cube scatterer, Section "Numerical
stability") is not fully specified and its data are not public; these
synthetic pulse workloads stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "ricker", "Wavelet", "two_layer_dense", "LayeredMedia", "LatticeMedia",
    "lognormal_lattice", "lattice_to_dense", "Workload", "c1", "c2", "c3",
    "c4_shots", "c5", "c5_receivers", "c5_true_lattice", "random_media",
]


# --------------------------------------------------------------------------
# Source wavelet
# --------------------------------------------------------------------------
@dataclass
class Wavelet:
    w64: np.ndarray          # FP64 samples r(n dt)
    w32: np.ndarray          # the same, rounded once to FP32
    f: float                 # peak frequency
    t0: float                # delay
    dt: float

    @property
    def nsamples(self) -> int:
        return int(self.w64.size)

    @property
    def peak(self) -> float:
        return float(np.max(np.abs(self.w32.astype(np.float64))))


def ricker(f: float, dt: float, amp: float = 1.0, t0: Optional[float] = None) -> Wavelet:
    """Ricker wavelet r(t) = amp (1 - 2a) exp(-a), a = (pi f (t - t0))^2.

    t0 = 1.5 / f so that the first sample is ~1e-8 of the peak; the wavelet
    is sampled at t = n dt for n = 0 .. ceil(2 t0 / dt) (inclusive).
    """
    if t0 is None:
        t0 = 1.5 / f
    ns = int(math.ceil(2.0 * t0 / dt)) + 1
    t = np.arange(ns, dtype=np.float64) * dt
    a = (math.pi * f * (t - t0)) ** 2
    w = amp * (1.0 - 2.0 * a) * np.exp(-a)
    return Wavelet(w64=w, w32=w.astype(np.float32), f=f, t0=t0, dt=dt)


# --------------------------------------------------------------------------
# Wave-speed models
# --------------------------------------------------------------------------
@dataclass
class LayeredMedia:
    """Horizontal layers: c = c_layer[k] for z_top[k] <= z < z_top[k+1]."""
    z_top: np.ndarray        # int32, ascending, z_top[0] == 0
    c_layer: np.ndarray      # float32

    def dense(self, nx: int, ny: int, nz: int) -> np.ndarray:
        c = np.empty((nz, ny, nx), dtype=np.float32)
        bounds = list(self.z_top.tolist()) + [nz]
        for k in range(len(self.z_top)):
            c[bounds[k]:bounds[k + 1]] = self.c_layer[k]
        return c

    @property
    def cmax(self) -> float:
        return float(np.max(self.c_layer))


def two_layer_dense(nx, ny, nz, z_split, c_top, c_bottom) -> np.ndarray:
    return LayeredMedia(np.array([0, z_split], np.int32),
                        np.array([c_top, c_bottom], np.float32)).dense(nx, ny, nz)


@dataclass
class LatticeMedia:
    """Wave speed given on a coarse lattice with power-of-two spacing S.

    The fine-grid value at cell (x, y, z) is the trilinear interpolation of
    the eight surrounding lattice values, evaluated in FP64 in the fixed
    order below and rounded once to FP32.  Every operand is an IEEE double
    and every operation is a single rounded +, - or *, so any conforming
    implementation (NumPy here, a GPU kernel elsewhere) gives the same bits.

        i = x // S, fx = (x - i S) / S           (exact: S is a power of two)
        cX(j, k) = L[k, j, i] (1 - fx) + L[k, j, i+1] fx
        cY(k)    = cX(j, k) (1 - fy) + cX(j+1, k) fy
        c        = float32( cY(k) (1 - fz) + cY(k+1) fz )
    """
    lattice: np.ndarray      # float64, shape (LZ, LY, LX), x fastest
    spacing: int

    @property
    def log2_spacing(self) -> int:
        s = int(self.spacing)
        assert s > 0 and (s & (s - 1)) == 0
        return s.bit_length() - 1

    @property
    def cmax(self) -> float:
        return float(np.max(self.lattice))


def lognormal_lattice(shape: Tuple[int, int, int], seed: int, sigma: float = 16.0,
                      spacing: int = 8, s: float = 0.25, cmin: float = 1500.0,
                      cmax: float = 4500.0) -> LatticeMedia:
    """Gaussian-smoothed lognormal wave speed on a lattice of spacing ``spacing``.

    g is white noise on a lattice with spacing ``spacing`` cells, smoothed by
    a Gaussian kernel of standard deviation ``sigma`` cells (periodic FFT
    convolution), normalised to zero mean and unit variance;
    c = clip(exp(mu + s g), cmin, cmax) with mu = ln sqrt(cmin cmax).
    ``shape`` is the fine grid (nx, ny, nz).
    """
    nx, ny, nz = shape
    S = int(spacing)
    lx, ly, lz = nx // S + 2, ny // S + 2, nz // S + 2
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((lz, ly, lx))
    sig = sigma / S
    kz = np.fft.fftfreq(lz)[:, None, None]
    ky = np.fft.fftfreq(ly)[None, :, None]
    kx = np.fft.rfftfreq(lx)[None, None, :]
    filt = np.exp(-2.0 * (math.pi * sig) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    g = np.fft.irfftn(np.fft.rfftn(white) * filt, s=(lz, ly, lx), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    mu = math.log(math.sqrt(cmin * cmax))
    lat = np.clip(np.exp(mu + s * g), cmin, cmax).astype(np.float64)
    return LatticeMedia(lattice=np.ascontiguousarray(lat), spacing=S)


def lattice_to_dense(media: LatticeMedia, shape: Tuple[int, int, int],
                     origin: Tuple[int, int, int] = (0, 0, 0),
                     extent: Optional[Tuple[int, int, int]] = None) -> np.ndarray:
    """Evaluate a LatticeMedia on a (sub-)box of the fine grid -> float32 (z, y, x)."""
    nx, ny, nz = shape
    x0, y0, z0 = origin
    sx, sy, sz = extent if extent is not None else (nx - x0, ny - y0, nz - z0)
    S = float(media.spacing)
    L = media.lattice
    x = np.arange(x0, x0 + sx)
    y = np.arange(y0, y0 + sy)
    z = np.arange(z0, z0 + sz)
    ix, iy, iz = x // media.spacing, y // media.spacing, z // media.spacing
    fx = (x - ix * media.spacing).astype(np.float64) / S
    fy = (y - iy * media.spacing).astype(np.float64) / S
    fz = (z - iz * media.spacing).astype(np.float64) / S
    out = np.empty((sz, sy, sx), dtype=np.float32)
    gx0, gx1 = 1.0 - fx, fx
    gy0, gy1 = (1.0 - fy)[:, None], fy[:, None]
    for kk in range(sz):
        k = iz[kk]
        fzk = fz[kk]

        def cy(kl):
            p00 = L[kl, iy][:, ix]
            p01 = L[kl, iy][:, ix + 1]
            p10 = L[kl, iy + 1][:, ix]
            p11 = L[kl, iy + 1][:, ix + 1]
            cx0 = p00 * gx0 + p01 * gx1
            cx1 = p10 * gx0 + p11 * gx1
            return cx0 * gy0 + cx1 * gy1

        c = cy(k) * (1.0 - fzk) + cy(k + 1) * fzk
        out[kk] = c.astype(np.float32)
    return out


def random_media(shape: Tuple[int, int, int], seed: int, cmin: float = 0.5,
                 cmax: float = 1.0) -> np.ndarray:
    """Uncorrelated random wave speed in [cmin, cmax) (float32, (z, y, x))."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.uniform(cmin, cmax, size=(nz, ny, nx)).astype(np.float32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]          # (nx, ny, nz)
    dx: float
    dt: float
    steps: int
    source: Tuple[int, int, int]
    wavelet: Wavelet
    trigger: float                       # absolute
    retire: float                        # absolute
    media_kind: str                      # "dense" | "layered" | "lattice"
    c_dense: Optional[np.ndarray] = None
    layered: Optional[LayeredMedia] = None
    lattice: Optional[LatticeMedia] = None
    pool_bytes: int = 0
    receivers: Optional[np.ndarray] = None   # (nrec, 3) int32 x,y,z
    extra: dict = field(default_factory=dict)

    def dense_c(self) -> np.ndarray:
        nx, ny, nz = self.shape
        if self.media_kind == "dense":
            return self.c_dense
        if self.media_kind == "layered":
            return self.layered.dense(nx, ny, nz)
        return lattice_to_dense(self.lattice, self.shape)

    @property
    def cells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def c1(steps: int = 100) -> Workload:
    n = 64
    w = ricker(f=0.1, dt=0.5)
    c = np.ones((n, n, n), dtype=np.float32)
    return Workload("c1", (n, n, n), 1.0, 0.5, steps, (32, 32, 32), w, 0.0, 0.0,
                    "dense", c_dense=c)


def c2(steps: int = 2000, trigger_rel: float = 1e-6, retire_rel: float = 1e-7,
       n: int = 512) -> Workload:
    dt = 0.5 / 3000.0
    w = ricker(f=100.0, dt=dt)
    lay = LayeredMedia(np.array([0, n // 2], np.int32), np.array([1500.0, 3000.0], np.float32))
    return Workload("c2", (n, n, n), 1.0, dt, steps, (n // 2, n // 2, n // 8), w,
                    trigger_rel * w.peak, retire_rel * w.peak, "layered", layered=lay)


def c3(steps: int = 3000, n: int = 4096, pool_bytes: int = 64_000_000_000,
       spacing: int = 16) -> Workload:
    dt = 0.5 / 4500.0
    w = ricker(f=100.0, dt=dt)
    lat = lognormal_lattice((n, n, n), seed=3, sigma=16.0, spacing=spacing)
    return Workload("c3", (n, n, n), 1.0, dt, steps, (n // 2, n // 2, n // 2), w,
                    1e-6 * w.peak, 1e-7 * w.peak, "lattice", lattice=lat,
                    pool_bytes=pool_bytes)


def c4_shots(nshots: int = 64, steps: int = 1500, seed: int = 4,
             edge_lo: int = 96, edge_hi: int = 384) -> List[Workload]:
    dt = 0.5 / 4500.0
    w = ricker(f=100.0, dt=dt)
    rng = np.random.default_rng(seed)
    shots = []
    for i in range(nshots):
        nx, ny, nz = (int(v) for v in rng.integers(edge_lo, edge_hi + 1, size=3))
        src = tuple(int(rng.integers(16, e - 16)) for e in (nx, ny, nz))
        lat = lognormal_lattice((nx, ny, nz), seed=4000 + i, sigma=16.0, spacing=8)
        shots.append(Workload(f"c4[{i}]", (nx, ny, nz), 1.0, dt, steps, src, w,
                              1e-6 * w.peak, 1e-7 * w.peak, "lattice", lattice=lat))
    return shots


def c5_receivers() -> np.ndarray:
    """16 x 8 receivers on the plane z = 240: x = 8 + 16 i, y = 16 + 32 j."""
    rec = [(8 + 16 * i, 16 + 32 * j, 240) for j in range(8) for i in range(16)]
    return np.array(rec, dtype=np.int32)


def c5(steps: int = 1000, n: int = 256) -> Workload:
    dt = 0.5 / 4500.0
    w = ricker(f=100.0, dt=dt)
    lat = lognormal_lattice((n, n, n), seed=5, sigma=16.0, spacing=8)
    rec = c5_receivers() if n == 256 else None
    return Workload("c5", (n, n, n), 1.0, dt, steps, (n // 2, n // 2, 16), w,
                    0.0, 0.0, "lattice", lattice=lat, receivers=rec,
                    extra={"checkpoint_every": 50})


def c5_true_lattice(base: LatticeMedia, center=(128, 128, 128), radius=12.0,
                    amp=0.02) -> LatticeMedia:
    """Perturbed model for the observed data: c (1 + amp exp(-|x - xa|^2 / (2 r^2)))
    applied at the lattice nodes (node (i,j,k) sits at cell (i S, j S, k S))."""
    S = base.spacing
    lz, ly, lx = base.lattice.shape
    z = (np.arange(lz) * S)[:, None, None]
    y = (np.arange(ly) * S)[None, :, None]
    x = (np.arange(lx) * S)[None, None, :]
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    lat = base.lattice * (1.0 + amp * np.exp(-r2 / (2.0 * radius ** 2)))
    return LatticeMedia(lattice=np.ascontiguousarray(lat), spacing=S)
