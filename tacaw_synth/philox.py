"""Counter-based synthetic exit waves for the fused producer (CPU twin).

The library's producer kernel (tacaw_synth_frames) writes synthetic exit waves
straight into a plan's ring; this module computes the same values on the CPU,
bit for bit, so the oracle can check any pixel subset of a series that only
ever existed in GPU memory. Like the rest of tacaw_synth it holds none of the
spectral method's arithmetic.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key go
through ten rounds of two 32 x 32 -> 64-bit products and xors, the key bumped by
the Weyl constants between rounds.

Signal model (per probe p, frame n, pixel k; complex64):
  psi = e0 + sum_j a (x_j(n) + i y_j(n)) + sigma (g_r + i g_i)
Term j of pixel k rotates by the quantised frequency f_j (Q = 2^20 steps per
cycle): (x, y) <- (x c - y s, x s + y c) with (c, s) = (cos, sin)(2 pi f_j / Q)
from a table, restarted every 64 frames from the tabulated phase
(f_j n + phi_j) mod Q, so that a frame's value depends only on its 64-frame
block. Every product and sum is one IEEE float32 operation in a fixed order.
f_j and phi_j come from Philox((p, k, j, 0), (seed, 0x21)); the frequency is
drawn from the probe's Lorentzian lines (centre and half width from
Philox((p, l, 0, 0), (seed, 0x11))) or from a uniform band. Noise indices come
from Philox((p, n >> 2, k, 0), (seed, 0x41)), word n & 3 (the low 12 bits of its
two 16-bit halves index a table of 2^12 standard normals).
"""

from __future__ import annotations

import dataclasses

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
Q = 1 << 20
BLOCK = 64            # frames between restarts of the rotation recurrence
NORMALS = 1 << 12     # entries of the noise table
STREAM_LINES, STREAM_TERMS, STREAM_NOISE = 0x11, 0x21, 0x41
PLANCK_EV_S = 6.62607015e-34 / 1.602176634e-19


def philox4x32_10(ctr, key):
    """Philox4x32-10 on uint32 arrays: ctr = (c0, c1, c2, c3) (broadcastable),
    key = (k0, k1) python ints. Returns four uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & MASK32 for x in ctr]
    c = list(np.broadcast_arrays(*c))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return [x.astype(np.uint32) for x in c]


@dataclasses.dataclass(frozen=True)
class ProducerSpec:
    n_probe: int
    n_frames: int
    ny: int
    nx: int
    seed: int = 5
    n_terms: int = 8
    amplitude: float = 1e-3 / np.sqrt(8)
    noise_sigma: float = 1e-5
    elastic: complex = 1.0
    n_lines: int = 6            # 0: frequencies from the uniform band
    e_lo_mev: float = 5.0
    e_hi_mev: float = 100.0
    line_lo_mev: float = 10.0
    line_hi_mev: float = 90.0
    hwhm_lo_mev: float = 0.5
    hwhm_hi_mev: float = 3.0
    dt_fs: float = 5.0
    dtype: str = "c64"

    @property
    def n_k(self) -> int:
        return self.ny * self.nx

    @property
    def nbytes(self) -> int:
        return self.n_probe * self.n_frames * self.n_k * 8


_TAB: dict = {}


def tables():
    """cos/sin of 2 pi q / Q (float32, computed in float64), 2^12 standard normals
    (float32, PCG64 seed 0x7ACA5) and tan(pi (u - 1/2)) at u = (i + 1/2) / 2^16
    (float64): the producer's inputs, identical on both sides."""
    if not _TAB:
        q = np.arange(Q, dtype=np.float64) * (2.0 * np.pi / Q)
        u = (np.arange(1 << 16, dtype=np.float64) + 0.5) / (1 << 16)
        _TAB.update(
            cos=np.cos(q).astype(np.float32), sin=np.sin(q).astype(np.float32),
            normal=np.random.Generator(np.random.PCG64(0x7ACA5)).standard_normal(NORMALS)
            .astype(np.float32),
            tan=np.tan(np.pi * (u - 0.5)))
    return _TAB


def _unit(r):
    return r.astype(np.float64) * (1.0 / 4294967296.0)


def term_params(spec: ProducerSpec, p: int, pixels: np.ndarray):
    """Integer frequency and phase steps [n_terms, K] of probe p at the pixels."""
    tab = tables()
    k = np.asarray(pixels, dtype=np.uint64)
    cyc_per_mev = 1e-3 / PLANCK_EV_S * spec.dt_fs * 1e-15 * Q
    if spec.n_lines > 0:
        l_idx = np.arange(spec.n_lines, dtype=np.uint64)
        r = philox4x32_10((p, l_idx, 0, 0), (spec.seed, STREAM_LINES))
        centre = spec.line_lo_mev + (spec.line_hi_mev - spec.line_lo_mev) * _unit(r[0])
        hwhm = spec.hwhm_lo_mev + (spec.hwhm_hi_mev - spec.hwhm_lo_mev) * _unit(r[1])
    f = np.empty((spec.n_terms, k.size), dtype=np.int64)
    ph = np.empty((spec.n_terms, k.size), dtype=np.int64)
    for j in range(spec.n_terms):
        r = philox4x32_10((p, k, j, 0), (spec.seed, STREAM_TERMS))
        if spec.n_lines > 0:
            line = (r[0] % np.uint32(spec.n_lines)).astype(np.int64)
            e = centre[line] + hwhm[line] * tab["tan"][(r[1] >> np.uint32(16)).astype(np.int64)]
            e = np.minimum(np.maximum(e, -400.0), 400.0)
        else:
            e = spec.e_lo_mev + (spec.e_hi_mev - spec.e_lo_mev) * _unit(r[0])
        f[j] = np.floor(e * cyc_per_mev + 0.5).astype(np.int64) & (Q - 1)
        ph[j] = (r[2] & np.uint32(Q - 1)).astype(np.int64)
    return f, ph


def generate(spec: ProducerSpec, probes=None, frames=None, pixels=None) -> np.ndarray:
    """complex64 values [P', F', K] of the probes, frame range and pixels (default all)."""
    tab = tables()
    probes = range(spec.n_probe) if probes is None else probes
    f0, f1 = (0, spec.n_frames) if frames is None else frames
    pix = np.arange(spec.n_k) if pixels is None else np.asarray(pixels)
    K = pix.size
    a = np.float32(spec.amplitude)
    sig = np.float32(spec.noise_sigma)
    e_re, e_im = np.float32(np.real(spec.elastic)), np.float32(np.imag(spec.elastic))
    b0, b1 = f0 // BLOCK, (f1 + BLOCK - 1) // BLOCK
    nb = b1 - b0
    out = np.empty((len(probes), f1 - f0, K), dtype=np.complex64)
    for i, p in enumerate(probes):
        f, ph = term_params(spec, p, pix)
        c, s = tab["cos"][f], tab["sin"][f]                         # [T, K]
        anchors = (np.arange(b0, b1, dtype=np.int64) * BLOCK)[:, None, None]
        idx = (f[None] * anchors + ph[None]) & (Q - 1)              # [nb, T, K]
        x, y = tab["cos"][idx], tab["sin"][idx]
        re = np.empty((nb, BLOCK, K), dtype=np.float32)
        im = np.empty((nb, BLOCK, K), dtype=np.float32)
        for u in range(BLOCK):
            r_ = np.full((nb, K), e_re, dtype=np.float32)
            i_ = np.full((nb, K), e_im, dtype=np.float32)
            for j in range(spec.n_terms):
                r_ = r_ + x[:, j] * a
                i_ = i_ + y[:, j] * a
            re[:, u], im[:, u] = r_, i_
            x, y = x * c - y * s, x * s + y * c
        n = np.arange(b0 * BLOCK, b1 * BLOCK, dtype=np.uint64)
        if spec.noise_sigma != 0.0:
            w = philox4x32_10((p, (n >> np.uint64(2))[:, None], pix.astype(np.uint64)[None, :], 0),
                              (spec.seed, STREAM_NOISE))
            word = np.choose((n & np.uint64(3)).astype(np.int64)[:, None], w)
            g_r = tab["normal"][(word & np.uint32(NORMALS - 1)).astype(np.int64)]
            g_i = tab["normal"][((word >> np.uint32(16)) & np.uint32(NORMALS - 1)).astype(np.int64)]
            re = re.reshape(nb * BLOCK, K) + g_r * sig
            im = im.reshape(nb * BLOCK, K) + g_i * sig
        else:
            re, im = re.reshape(nb * BLOCK, K), im.reshape(nb * BLOCK, K)
        lo = f0 - b0 * BLOCK
        out[i].real = re[lo:lo + f1 - f0]
        out[i].imag = im[lo:lo + f1 - f0]
    return out
