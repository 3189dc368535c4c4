"""Seeded synthetic exit-wave series, detector masks and loss weights.

Shared by the tests, the benchmark and the smoke check as the ONE source of
inputs for both the GPU library and the CPU oracle. It holds none of the
spectral method's arithmetic (no mean, window, transform or power): it only
draws series of the shape and structure of the paper's workloads.

Bit-identity across devices: every value is built from integer counter hashes
(keyed by seed, probe, frame, pixel and term), lookups into tables built once on
the host in float64, and IEEE additions and multiplications applied one torch op
at a time in a fixed order. Running the same call on the CPU and on the GPU
therefore yields identical bits, so the oracle can regenerate any pixel subset
of a series that lives only in GPU memory.

Signal model (per probe p, frame n, pixel k):

    psi = 1 + sum_j a * exp(i (2 pi f_j n / Q + 2 pi phi_j / Q)) + noise

with Q = 2^20 phase steps per cycle. Frequencies come either from a uniform
energy band ("uniform": E ~ U(e_lo, e_hi) meV per term) or from a per-probe set
of Lorentzian lines ("lines": each term picks one of the probe's lines and draws
its energy from that line's Cauchy distribution). Noise: real and imaginary
parts drawn from a table of 2^16 standard normals scaled by sigma.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import philox  # noqa: F401  (the fused producer's CPU twin)

PHASE_BITS = 20
Q = 1 << PHASE_BITS
NOISE_BITS = 16
TAN_BITS = 16
MASK32 = 0xFFFFFFFF
_HC = 0x45D9F3B  # multiplier of the integer finaliser below (< 2^31: no int64 overflow)
PLANCK_EV_S = 6.62607015e-34 / 1.602176634e-19

_TABLES: dict = {}


def _hash32(x: torch.Tensor) -> torch.Tensor:
    """32-bit integer finaliser on int64 tensors holding values in [0, 2^32)."""
    x = ((x >> 16) ^ x) * _HC & MASK32
    x = ((x >> 16) ^ x) * _HC & MASK32
    return (x >> 16) ^ x


def _key(*parts) -> torch.Tensor:
    """Chain-hash integer keys (python ints or int64 tensors)."""
    h = None
    for p in parts:
        t = p if isinstance(p, torch.Tensor) else torch.tensor(int(p) & MASK32, dtype=torch.int64)
        h = _hash32(t & MASK32) if h is None else _hash32((h ^ (t & MASK32)) & MASK32)
    return h


def _tables(dtype: torch.dtype, device) -> dict:
    key = (dtype, str(device))
    if key not in _TABLES:
        q = np.arange(Q, dtype=np.float64) * (2.0 * np.pi / Q)
        rdt = torch.float32 if dtype == torch.complex64 else torch.float64
        normals = np.random.Generator(np.random.PCG64(0x7ACA3)).standard_normal(1 << NOISE_BITS)
        u = (np.arange(1 << TAN_BITS, dtype=np.float64) + 0.5) / (1 << TAN_BITS)
        _TABLES[key] = {
            "cos": torch.from_numpy(np.cos(q)).to(rdt).to(device),
            "sin": torch.from_numpy(np.sin(q)).to(rdt).to(device),
            "normal": torch.from_numpy(normals).to(rdt).to(device),
            "cauchy": torch.from_numpy(np.tan(np.pi * (u - 0.5))).to(torch.float64).to(device),
        }
    return _TABLES[key]


@dataclasses.dataclass(frozen=True)
class SeriesSpec:
    n_probe: int
    n_frames: int
    ny: int
    nx: int
    dt_fs: float = 5.0
    dtype: str = "c64"            # "c64" or "c128"
    seed: int = 1
    model: str = "uniform"        # "uniform" or "lines"
    n_terms: int = 3              # sinusoids per pixel
    amplitude: float = 1e-3       # per-term amplitude
    e_lo_mev: float = 5.0         # uniform band (model "uniform")
    e_hi_mev: float = 100.0
    n_lines: int = 6              # Lorentzian lines per probe (model "lines")
    line_lo_mev: float = 10.0
    line_hi_mev: float = 90.0
    hwhm_lo_mev: float = 0.5
    hwhm_hi_mev: float = 3.0
    noise_sigma: float = 1e-5
    elastic: complex = 1.0

    @property
    def n_k(self) -> int:
        return self.ny * self.nx

    @property
    def torch_dtype(self) -> torch.dtype:
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    @property
    def real_dtype(self) -> torch.dtype:
        return torch.float32 if self.dtype == "c64" else torch.float64

    @property
    def nbytes(self) -> int:
        return self.n_probe * self.n_frames * self.n_k * (8 if self.dtype == "c64" else 16)


def _unit(h: torch.Tensor) -> torch.Tensor:
    """Map a 32-bit hash to [0, 1) in float64 (exact: h < 2^32)."""
    return h.to(torch.float64) * (1.0 / 4294967296.0)


def _term_params(spec: SeriesSpec, p: int, kidx: torch.Tensor, device):
    """Integer frequency and phase steps [n_terms, K] for probe p and pixels kidx."""
    tab = _tables(spec.torch_dtype, device)
    cyc_per_mev = 1e-3 / PLANCK_EV_S * spec.dt_fs * 1e-15 * Q   # phase steps per frame per meV
    freqs, phases = [], []
    if spec.model == "lines":
        lines = []
        for l in range(spec.n_lines):
            uc = float(_unit(_key(spec.seed, 0x11, p, l)))
            uw = float(_unit(_key(spec.seed, 0x12, p, l)))
            lines.append((spec.line_lo_mev + (spec.line_hi_mev - spec.line_lo_mev) * uc,
                          spec.hwhm_lo_mev + (spec.hwhm_hi_mev - spec.hwhm_lo_mev) * uw))
        centres = torch.tensor([c for c, _ in lines], dtype=torch.float64, device=device)
        widths = torch.tensor([w for _, w in lines], dtype=torch.float64, device=device)
    for j in range(spec.n_terms):
        hk = _key(spec.seed, 0x21, p, j, kidx)
        if spec.model == "uniform":
            e = spec.e_lo_mev + _unit(hk) * (spec.e_hi_mev - spec.e_lo_mev)
        elif spec.model == "lines":
            which = _hash32(hk ^ 0x5BD1E995) % spec.n_lines
            cauchy = tab["cauchy"][_hash32(hk ^ 0x27D4EB2F) >> (32 - TAN_BITS)]
            e = centres[which] + widths[which] * cauchy
            e = torch.clamp(e, -400.0, 400.0)
        else:
            raise ValueError(f"unknown model {spec.model!r}")
        f = torch.floor(e * cyc_per_mev + 0.5).to(torch.int64) & (Q - 1)
        ph = _key(spec.seed, 0x31, p, j, kidx) & (Q - 1)
        freqs.append(f)
        phases.append(ph)
    if not freqs:
        empty = torch.empty((0, kidx.numel()), dtype=torch.int64, device=device)
        return empty, empty
    return torch.stack(freqs), torch.stack(phases)


def generate(spec: SeriesSpec, probes=None, frames=None, pixels=None, device="cpu") -> torch.Tensor:
    """Series values psi[p, n, k] for the requested probes, frame range and pixels.

    probes: iterable of probe indices (default all); frames: (start, stop) range
    (default all); pixels: 1-D int64 tensor/array of flattened pixel indices
    (default all, in which case the result has shape [P', F', ny, nx]).
    """
    probes = list(range(spec.n_probe)) if probes is None else [int(p) for p in probes]
    f0, f1 = (0, spec.n_frames) if frames is None else (int(frames[0]), int(frames[1]))
    full = pixels is None
    kidx = (torch.arange(spec.n_k, dtype=torch.int64, device=device) if full
            else torch.as_tensor(np.asarray(pixels), dtype=torch.int64).to(device))
    tab = _tables(spec.torch_dtype, device)
    rdt = spec.real_dtype
    amp = torch.tensor(spec.amplitude, dtype=rdt, device=device)
    sig = torch.tensor(spec.noise_sigma, dtype=rdt, device=device)
    out = torch.empty((len(probes), f1 - f0, kidx.numel()), dtype=spec.torch_dtype, device=device)
    n = torch.arange(f0, f1, dtype=torch.int64, device=device)[:, None]
    for i, p in enumerate(probes):
        fr, ph = _term_params(spec, p, kidx, device)
        re = torch.full((f1 - f0, kidx.numel()), float(np.real(spec.elastic)), dtype=rdt, device=device)
        im = torch.full((f1 - f0, kidx.numel()), float(np.imag(spec.elastic)), dtype=rdt, device=device)
        for j in range(spec.n_terms):
            idx = (fr[j][None, :] * n + ph[j][None, :]) & (Q - 1)
            re = re + tab["cos"][idx] * amp
            im = im + tab["sin"][idx] * amp
            del idx
        if spec.noise_sigma != 0.0:
            hn = _key(spec.seed, 0x41, p, n, kidx[None, :])
            re = re + tab["normal"][hn & ((1 << NOISE_BITS) - 1)] * sig
            im = im + tab["normal"][hn >> (32 - NOISE_BITS)] * sig
            del hn
        out[i] = torch.complex(re, im)
    if full:
        out = out.view(len(probes), f1 - f0, spec.ny, spec.nx)
    return out


def generate_into(spec: SeriesSpec, dst: torch.Tensor, probes=None, frame_chunk=256) -> None:
    """Fill dst [P', n_frames, ny, nx] (e.g. on the GPU) frame chunk by chunk."""
    probes = list(range(spec.n_probe)) if probes is None else list(probes)
    for i, p in enumerate(probes):
        for f0 in range(0, spec.n_frames, frame_chunk):
            f1 = min(spec.n_frames, f0 + frame_chunk)
            dst[i, f0:f1] = generate(spec, [p], (f0, f1), device=dst.device)[0]


# ------------------------------------------------------------------ non-stationary series

def perturb(psi, kind: str, amount: float, tau: float = 16.0) -> torch.Tensor:
    """A copy of a series psi [P, n_frames, ny, nx] with a non-stationary part of the
    kinds the paper discusses (values formed in float64, rounded to psi's dtype):

    "offset":    frame 0 shifted by ``amount`` (a snapshot taken before the
                 trajectory settled);
    "transient": amount * exp(-n / tau) added to frame n (thermalisation, Sec. III.A);
    "drift":     a centre-of-mass drift: phase ramp exp(2 pi i f(kx) n) with a
                 Doppler frequency f(kx) = amount * (kx - nx/2) / (nx/2) cycles per
                 frame, linear in the transverse wave-vector (Sec. III.B).
    """
    x = np.asarray(psi.numpy(), dtype=np.complex128).copy()
    P, NT, ny, nx = x.shape
    n = np.arange(NT, dtype=np.float64)
    if kind == "offset":
        x[:, 0] += amount
    elif kind == "transient":
        x += (amount * np.exp(-n / tau))[None, :, None, None]
    elif kind == "drift":
        f = amount * (np.arange(nx, dtype=np.float64) - nx // 2) / (nx / 2)
        x *= np.exp(2j * np.pi * n[:, None] * f[None, :])[None, :, None, :]
    else:
        raise ValueError(f"unknown perturbation {kind!r}")
    return torch.from_numpy(x.astype(np.complex64 if psi.dtype == torch.complex64 else np.complex128))


# ------------------------------------------------------------------ masks

def disk_mask(ny, nx, radius, center=None, inner=0.0):
    """1 where inner <= d < radius, d = distance of the pixel index from center
    (default (ny//2, nx//2)), else 0; float64 [ny, nx]."""
    cy, cx = (ny // 2, nx // 2) if center is None else center
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    d = np.hypot(iy - cy, ix - cx)
    return ((d >= inner) & (d < radius)).astype(np.float64)


def standard_masks(ny, nx, scale=1.0):
    """Four detectors in pixel units times ``scale``: central disk r < 30,
    annulus 60 <= d < 100, and disks r < 30 displaced by +60 px along x and y."""
    cy, cx = ny // 2, nx // 2
    r, a0, a1, off = 30 * scale, 60 * scale, 100 * scale, int(round(60 * scale))
    return np.stack([
        disk_mask(ny, nx, r),
        disk_mask(ny, nx, a1, inner=a0),
        disk_mask(ny, nx, r, center=(cy, cx + off)),
        disk_mask(ny, nx, r, center=(cy + off, cx)),
    ])


def loss_weights(n_det, n_bins, seed=4, scales=(1.0, 0.5, 0.25, 0.125)):
    """a_j(m) = c_j u_j(m), u ~ U[0, 1) (PCG64)."""
    u = np.random.Generator(np.random.PCG64(seed)).random((n_det, n_bins))
    return np.asarray(scales[:n_det], dtype=np.float64)[:, None] * u


# ------------------------------------------------------------------ workloads

def config_plain_1probe() -> SeriesSpec:
    """1 probe, 256 frames at 5 fs, 64 x 64, complex128, 3 uniform-band tones."""
    return SeriesSpec(1, 256, 64, 64, 5.0, "c128", 1, "uniform", 3, 1e-3)


def config_realistic(n_probe=64, n_frames=2048, ny=256, nx=256, seed=2) -> SeriesSpec:
    """64 probes, 2048 frames, 256 x 256 complex64, 6 Lorentzian lines per probe,
    8 tones per pixel of amplitude 1e-3/sqrt(8)."""
    return SeriesSpec(n_probe, n_frames, ny, nx, 5.0, "c64", seed, "lines", 8, 1e-3 / math.sqrt(8))


def config_precision(n_frames=512) -> SeriesSpec:
    return SeriesSpec(1, n_frames, 64, 64, 5.0, "c128", 3, "uniform", 3, 1e-3)


def config_gradient(n_probe=16, n_frames=1024, ny=128, nx=128) -> SeriesSpec:
    return SeriesSpec(n_probe, n_frames, ny, nx, 5.0, "c64", 4, "lines", 8, 1e-3 / math.sqrt(8))


def config_streaming(n_probe=256, n_frames=4096, ny=1024, nx=1024) -> SeriesSpec:
    return SeriesSpec(n_probe, n_frames, ny, nx, 5.0, "c64", 5, "lines", 8, 1e-3 / math.sqrt(8))
