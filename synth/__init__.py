"""Seeded synthetic inputs for the photo-switching optoacoustic reconstruction.

This module only *draws inputs*: grid and sampling constants, the banded
spatial impulse response of the focused transducer (beam weight times the
electrical pulse at the propagation delay), the depth fluence profile, the
photo-physics constants of each species, nonnegative tube phantoms, unit
Gaussian noise and the power-iteration start vector.  It contains none of the
reconstruction arithmetic (no photo-switching matrix, no acoustic contraction,
no prox, no solver): both the FP64 oracle and the GPU path consume what it
returns, and neither side imports the other.

Paper context (arXiv 2510.23739):
  * the acoustic model integrates the initial pressure over a semicircle
    around the focal spot weighted by the transducer's spatial response, then
    convolves with the electrical impulse response (Sec. 2.1.4, eqs.
    q-above-1d, q-below-1d, acoustic-temporal-conv).  Here that response is
    synthesised per voxel offset as  w(dx,dy,z) * g'(t*dt - tau(dx,dy,z)),
    a Gaussian beam times a derivative-of-Gaussian pulse at the signed
    semicircle delay, stored as a band of `width` taps starting at `t0`;
  * photo-physics constants follow Table "tab:photophysics" (extinction
    coefficients of species A and B, in 1/(uM mm));
  * the fluence map is the depth profile exp(-mu_eff z) standing in for the
    diffusion solve of Sec. 2.1.3 (precomputed once, as in the paper).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# physical constants of the synthetic scanner
# ----------------------------------------------------------------------------
PITCH_M = 20e-6          # voxel pitch in x, y and z (m)
DT_S = 8e-9              # A-scan sampling interval, 125 MHz (s)
C0_M_S = 1500.0          # speed of sound (m/s)
F_CENTER_HZ = 25e6       # pulse centre frequency (Hz)
MU_EFF_PER_MM = 2.0      # effective attenuation of the fluence (1/mm)
BAND_HALF_SIGMAS = 6.0   # pulse support kept in the band: |u| <= 6 s
SIR_WIDTH = 12           # stored band width (taps)
SNR_DB = 20.0            # measurement SNR on mean power

# Extinction coefficients in 1/(uM mm): a = eps_OFF, b = eps_ON - eps_OFF
# (species 0 and 1 from the paper's photo-physics table; species 2 invented
# between them).  Switching time constants in pulses.
_SPECIES_A = (1.0e-4, 1.0e-4, 1.0e-4)
_SPECIES_B = (4.9e-3, 3.9e-3, 4.4e-3)
_TAU = {1: (2.0,), 2: (2.0, 6.0), 3: (2.0, 5.0, 12.0)}


@dataclasses.dataclass(frozen=True)
class Config:
    """One reconstruction workload (grid, species, pulses, samples, footprint)."""

    name: str
    nx: int
    ny: int
    nz: int
    n_species: int
    n_pulses: int
    nt: int
    f: int                 # lateral footprint (odd); R = (f-1)//2
    k1: int                # outer (FISTA) iterations
    k2: int = 20           # inner (dual TV) iterations
    seed: int = 0
    gamma: float = 0.0     # 0: fluence-independent switching rate, 1: paper's k*Phi*t

    @property
    def r(self) -> int:
        return (self.f - 1) // 2

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def c_shape(self) -> Tuple[int, int, int, int]:
        return (self.n_species, self.ny, self.nx, self.nz)

    @property
    def y_shape(self) -> Tuple[int, int, int, int]:
        return (self.n_pulses, self.ny, self.nx, self.nt)

    def crop(self, nx: int, ny: int, name: str | None = None) -> "Config":
        """Same depth/pulse/sample/footprint geometry on a smaller lateral grid."""
        return dataclasses.replace(self, nx=nx, ny=ny,
                                   name=name or f"{self.name}-crop{nx}x{ny}")


# The five workloads: tiny FP64-checkable, FP32 GPU, mixed precision, the
# batched uneven family (see c4_instance) and the largest single solve.
C1 = Config("C1", 32, 32, 16, 2, 8, 64, 7, k1=20, k2=20, seed=1000)
C2 = Config("C2", 128, 128, 64, 3, 32, 256, 31, k1=100, k2=20, seed=2000)
C3 = Config("C3", 256, 256, 96, 3, 32, 384, 41, k1=200, k2=20, seed=3000)
C5 = Config("C5", 320, 320, 128, 3, 40, 512, 51, k1=300, k2=50, seed=5000)
CONFIGS = {"C1": C1, "C2": C2, "C3": C3, "C5": C5}


def c4_instance(i: int) -> Config:
    """Instance i (0..15) of the batched uneven family: lateral side in
    [64,192], depth in [48,96], pulses in [16,48], 2-3 species, samples in
    [256,384] rounded to a multiple of 32, footprint 31, 100 iterations."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(4000 + i).spawn(4)[2]))
    side = int(rng.integers(64, 193))
    nz = int(rng.integers(48, 97))
    k = int(rng.integers(16, 49))
    s = int(rng.integers(2, 4))
    nt = int(round(int(rng.integers(256, 385)) / 32.0)) * 32
    return Config(f"C4[{i}]", side, side, nz, s, k, nt, 31, k1=100, k2=20, seed=4000 + i)


def streams(seed: int) -> List[np.random.Generator]:
    """Independent PCG64 streams: [phantom, noise, shapes, power-iteration]."""
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(4)]


# ----------------------------------------------------------------------------
# transducer spatial impulse response, banded
# ----------------------------------------------------------------------------
def pulse_sigma_s() -> float:
    """Width s of the derivative-of-Gaussian pulse whose spectrum peaks at the
    centre frequency (the spectrum of u*exp(-u^2/2s^2) peaks at 1/(2 pi s))."""
    return 1.0 / (2.0 * math.pi * F_CENTER_HZ)


def pulse(u: np.ndarray) -> np.ndarray:
    """Electrical impulse response g'(u) = -(u/s) exp(1/2 - u^2/(2 s^2));
    unit peak magnitude (reached at u = -s and u = +s)."""
    s = pulse_sigma_s()
    return -(u / s) * np.exp(0.5 - u * u / (2.0 * s * s))


def focal_depth_vox(nz: int) -> float:
    """Focal plane at mid-depth, in voxel units (z_F = (Nz-1)/2)."""
    return 0.5 * (nz - 1)


def delay_s(dx: np.ndarray, dy: np.ndarray, iz: np.ndarray, nz: int, nt: int) -> np.ndarray:
    """Signed semicircle delay: arrival at the focal time t_F = (Nt/2) dt,
    earlier above the focal plane and later below it by the distance to the
    focal spot over c0 (sign of 0 taken as +1)."""
    dz = (iz - focal_depth_vox(nz)) * PITCH_M
    rho2 = (dx * dx + dy * dy) * PITCH_M * PITCH_M
    sgn = np.where(dz >= 0.0, 1.0, -1.0)
    return (nt // 2) * DT_S + sgn * np.sqrt(rho2 + dz * dz) / C0_M_S


def beam_sigma_vox(iz: np.ndarray, nz: int, f: int) -> np.ndarray:
    """Lateral beam width: 1 voxel at the focus, growing linearly to R/2 at the
    deepest/shallowest plane."""
    r = (f - 1) // 2
    sigma0, sigma_e = 1.0, max(r / 2.0, 1.0)
    zf = focal_depth_vox(nz)
    span = max(zf, (nz - 1) - zf)
    if span <= 0:
        return np.full_like(np.asarray(iz, dtype=np.float64), sigma0)
    return sigma0 + (sigma_e - sigma0) * np.abs(iz - zf) / span


def sir_table(nz: int, f: int, nt: int, width: int = SIR_WIDTH) -> Tuple[np.ndarray, np.ndarray]:
    """Banded spatial impulse response h[z][jdy][jdx][t].

    Offsets are (dy, dx) = (jdy - R, jdx - R) with voxel = scan + offset.
    Returns (t0 int32 [nz,f,f], taps float32 [nz,f,f,width]); the response is
    taps[..., j] at sample t0 + j and zero everywhere else.  Taps beyond the
    pulse support |t dt - tau| <= 6 s are stored as exact zeros.
    """
    r = (f - 1) // 2
    iz = np.arange(nz, dtype=np.float64)[:, None, None]
    d = np.arange(-r, r + 1, dtype=np.float64)
    dy = d[None, :, None]
    dx = d[None, None, :]
    tau = delay_s(dx, dy, iz, nz, nt)                       # [nz,f,f]
    s = pulse_sigma_s()
    half = BAND_HALF_SIGMAS * s
    t0 = np.ceil((tau - half) / DT_S - 1e-9).astype(np.int64)
    sig = beam_sigma_vox(iz, nz, f)
    w = np.exp(-(dx * dx + dy * dy) / (2.0 * sig * sig))     # [nz,f,f]
    j = np.arange(width, dtype=np.float64)
    u = (t0[..., None] + j) * DT_S - tau[..., None]          # [nz,f,f,width]
    taps = np.where(np.abs(u) <= half, w[..., None] * pulse(u), 0.0)
    return t0.astype(np.int32), taps.astype(np.float32)


def random_table(nz: int, f: int, nt: int, width: int, rng: np.random.Generator,
                 t0_lo: int = -4, t0_hi: int | None = None) -> Tuple[np.ndarray, np.ndarray]:
    """An asymmetric random banded table (no dx/dy/z symmetry, arbitrary start
    samples including ones that run off either end of the A-scan)."""
    if t0_hi is None:
        t0_hi = nt - 2
    t0 = rng.integers(t0_lo, t0_hi, size=(nz, f, f)).astype(np.int32)
    taps = rng.standard_normal((nz, f, f, width)).astype(np.float32)
    return t0, taps


# ----------------------------------------------------------------------------
# inputs of the factorised acoustic operator: the spatial response image on
# the voxel grid, the sampled electrical impulse response and the geometry of
# the delay shells
# ----------------------------------------------------------------------------
def spr_table(nz: int, f: int) -> np.ndarray:
    """Spatial response image eta[z][jdy][jdx] (float32): the lateral beam
    weight exp(-(dx^2 + dy^2) / 2 sigma(z)^2) of the banded table, without
    the pulse."""
    r = (f - 1) // 2
    iz = np.arange(nz, dtype=np.float64)[:, None, None]
    d = np.arange(-r, r + 1, dtype=np.float64)
    sig = beam_sigma_vox(iz, nz, f)
    w = np.exp(-(d[None, :, None] ** 2 + d[None, None, :] ** 2) / (2.0 * sig * sig))
    return w.astype(np.float32)


def eir_taps() -> Tuple[np.ndarray, int]:
    """Electrical impulse response sampled at DT_S over its kept support
    |u| <= 6 s: v[j] = pulse((j - origin) dt); returns (v float32, origin)."""
    half = int(math.floor(BAND_HALF_SIGMAS * pulse_sigma_s() / DT_S + 1e-9))
    u = np.arange(-half, half + 1, dtype=np.float64) * DT_S
    return pulse(u).astype(np.float32), half


def shell_geometry(nz: int, nt: int) -> Tuple[float, float, int]:
    """(dr, z_focus, t_focus): radius step per sample in voxel pitches
    (c0 dt / pitch), focal depth in voxel units and the focal sample Nt/2."""
    return C0_M_S * DT_S / PITCH_M, focal_depth_vox(nz), nt // 2


# ----------------------------------------------------------------------------
# optics and photo-physics constants
# ----------------------------------------------------------------------------
def phi_depth(nz: int) -> np.ndarray:
    """Fluence exp(-mu_eff z) at voxel depths z = iz * pitch, float32 [nz]."""
    z_mm = np.arange(nz, dtype=np.float64) * PITCH_M * 1e3
    return np.exp(-MU_EFF_PER_MM * z_mm).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class Species:
    a: Tuple[float, ...]     # eps_OFF per species
    b: Tuple[float, ...]     # eps_ON - eps_OFF per species
    tau: Tuple[float, ...]   # switching time constant (pulses)
    gamma: float             # exponent of the fluence in the switching rate


def species(n_species: int, gamma: float = 0.0) -> Species:
    return Species(_SPECIES_A[:n_species], _SPECIES_B[:n_species], _TAU[n_species], gamma)


# ----------------------------------------------------------------------------
# phantom, noise, start vectors
# ----------------------------------------------------------------------------
def _segment_dist2(px, py, pz, a, b):
    ab = b - a
    l2 = float(ab @ ab)
    apx, apy, apz = px - a[0], py - a[1], pz - a[2]
    if l2 == 0.0:
        u = 0.0
    else:
        u = np.clip((apx * ab[0] + apy * ab[1] + apz * ab[2]) / l2, 0.0, 1.0)
    qx, qy, qz = apx - u * ab[0], apy - u * ab[1], apz - u * ab[2]
    return qx * qx + qy * qy + qz * qz


def phantom(cfg: Config, rng: np.random.Generator | None = None) -> np.ndarray:
    """Nonnegative tube phantom, float32 [S][Ny][Nx][Nz].

    Per species 3 + ceil(Nx/32) straight tubes with Gaussian cross-section
    (radius 1-2.5 voxels, amplitude 0.5-1.5); species may overlap.
    """
    if rng is None:
        rng = streams(cfg.seed)[0]
    c = np.zeros(cfg.c_shape, dtype=np.float64)
    iy, ix, iz = np.meshgrid(np.arange(cfg.ny, dtype=np.float64),
                             np.arange(cfg.nx, dtype=np.float64),
                             np.arange(cfg.nz, dtype=np.float64), indexing="ij")
    n_tubes = 3 + math.ceil(cfg.nx / 32)
    lo = np.array([0.1 * cfg.nx, 0.1 * cfg.ny, 0.2 * cfg.nz])
    hi = np.array([0.9 * cfg.nx, 0.9 * cfg.ny, 0.8 * cfg.nz])
    for s in range(cfg.n_species):
        for _ in range(n_tubes):
            p0 = rng.uniform(lo, hi)
            p1 = rng.uniform(lo, hi)
            sig = rng.uniform(1.0, 2.5)
            amp = rng.uniform(0.5, 1.5)
            d2 = _segment_dist2(ix, iy, iz, p0, p1)
            c[s] += amp * np.exp(-d2 / (2.0 * sig * sig))
    return c.astype(np.float32)


def unit_noise(shape, rng: np.random.Generator) -> np.ndarray:
    """Standard normal noise, float32 (scaled to the SNR by the caller)."""
    return rng.standard_normal(shape).astype(np.float32)


def noise_sigma(clean_rms: float, snr_db: float = SNR_DB) -> float:
    """Noise standard deviation for a given SNR on mean power."""
    return clean_rms * 10.0 ** (-snr_db / 20.0)


def power_start(n: int, rng: np.random.Generator) -> np.ndarray:
    """Gaussian start vector of the power iteration, float32 [n]."""
    return rng.standard_normal(n).astype(np.float32)


def inputs(cfg: Config):
    """Everything a reconstruction of `cfg` needs except the measurements:
    (c_true, t0, taps, phi, species, unit_noise, v0)."""
    g_ph, g_noise, _, g_pow = streams(cfg.seed)
    t0, taps = sir_table(cfg.nz, cfg.f, cfg.nt)
    c_true = phantom(cfg, g_ph)
    n0 = unit_noise(cfg.y_shape, g_noise)
    v0 = power_start(int(np.prod(cfg.c_shape)), g_pow).reshape(cfg.c_shape)
    return c_true, t0, taps, phi_depth(cfg.nz), species(cfg.n_species, cfg.gamma), n0, v0
