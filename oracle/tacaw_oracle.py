"""Plain FP64 reference of the TACAW spectral reduction (test infrastructure only).

What it computes (paper, Sec. I Eq. 1 and Sec. II.B):

* the exit-wave series of each probe is cut into chunks ("trajectory chunks",
  Sec. II.B.2 "Welch method") of length L whose starts advance by the
  remainder-less quotient L // nu; only full chunks are used;
* each chunk is multiplied by a window (Hann by default, Sec. II.B.2 and
  Sec. III.A), Fourier transformed along time with the forward kernel
  exp(-i omega t) (Sec. III.B, the drift example's transform), and its squared
  modulus is taken (Eq. 1, without the quantum-statistics factor);
* the chunk spectra are averaged, (1/N) sum_i I_i (Eq. 2), and united over scan
  positions; the result is normalised "per voxel" (Sec. II.B.2, Normalization);
* detector spectra are mask-weighted sums over reciprocal space (DetectorSet,
  Sec. II.B.1 and the detector paragraph of App. B).

Readings where the paper is silent (each is also listed in the design notes):

* the elastic time-mean is removed before the window (GLOBAL: mean over the
  frames that enter at least one chunk; PER_SEGMENT: mean of each chunk;
  NONE: the paper's own behaviour, which keeps the zero-loss peak);
* Hann is the periodic (DFT-even) window, the only variant for which the
  zero-loss peak stays in bins 0 and +-1 as Sec. III.A states;
* per-chunk power is |X|^2 / (L * sum_t w(t)^2), so summing over all bins gives
  the window-weighted mean |psi - mu|^2 ("per voxel" probabilities);
* spectra are averaged over chunks and (by default) over probes;
* the "window width" parameter r stretches the Hann lobe about the chunk
  centre: w_r(t) = 1/2 + 1/2 cos(2 pi (t - L/2) / (r L)) for |t - L/2| <= r L/2,
  else 0 (r = 1 is the periodic Hann);
* frequency bins are in FFT order, bin m at nu_m = m / (L dt) for m < L/2 and
  (m - L) / (L dt) otherwise; an injected exp(+2 pi i nu t) lands at +nu.

Parity status: every function below is pinned by tests against closed forms,
brute force, library special cases (scipy.signal.welch) or the worked numbers
the paper prints (segment count, energy sampling, energy-ROI bin count). None is
"parity unpinned"; the absolute physical scale of the spectra is fixed by the
normalisation reading above, not by a printed value.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "PLANCK_EV_S",
    "hop_from_overlap",
    "segment_count",
    "segment_starts",
    "frames_used",
    "window",
    "window_width_derivative",
    "frequency_axis_thz",
    "energy_axis_mev",
    "energy_sampling_mev",
    "energy_range_mev",
    "energy_roi_bins",
    "dft_matrix",
    "probe_mean",
    "segment_spectra",
    "tacaw_spectra",
    "tacaw_spectra_fft",
    "detector_spectra",
    "detector_loss",
    "spectra_vjp",
    "detector_loss_vjp",
    "quantum_factor",
]

# Planck constant in eV*s (exact SI value h = 6.62607015e-34 J s divided by the
# exact elementary charge 1.602176634e-19 C).
PLANCK_EV_S = 6.62607015e-34 / 1.602176634e-19

MEAN_MODES = ("global", "per_segment", "none")
PROBE_REDUCE = ("mean", "sum")


# --------------------------------------------------------------------------
# Chunking (Sec. II.B.2, "Welch method: trajectory chunk overlap & windowing")
# --------------------------------------------------------------------------

def hop_from_overlap(seg_len: int, overlap: int) -> int:
    """Chunk start advance s_{n+1} - s_n = L / nu with remainder-less division."""
    if seg_len <= 0 or overlap <= 0:
        raise ValueError("segment length and overlap must be positive")
    return seg_len // overlap


def segment_count(n_frames: int, seg_len: int, hop: int) -> int:
    """Number of full chunks of length L starting at 0, H, 2H, ... inside n_frames."""
    if hop <= 0 or seg_len <= 0:
        raise ValueError("segment length and hop must be positive")
    if n_frames < seg_len:
        return 0
    return (n_frames - seg_len) // hop + 1


def segment_starts(n_frames: int, seg_len: int, hop: int) -> list[int]:
    return [s * hop for s in range(segment_count(n_frames, seg_len, hop))]


def frames_used(n_frames: int, seg_len: int, hop: int) -> int:
    """Frames that belong to at least one full chunk (the tail beyond is dropped)."""
    ns = segment_count(n_frames, seg_len, hop)
    return 0 if ns == 0 else (ns - 1) * hop + seg_len


# --------------------------------------------------------------------------
# Windows (Sec. II.B.2 and Sec. III.A; Tukey alpha as the summed taper
# fraction, alpha = 1 Hann, alpha = 0 rectangular)
# --------------------------------------------------------------------------

def window(kind: str, seg_len: int, param: float | None = None) -> np.ndarray:
    """Window values w(t), t = 0..L-1, float64.

    kind: "hann" (periodic), "rect", "tukey" (param = alpha, periodic form),
    "hann_width" (param = r, see module docstring).
    """
    L = int(seg_len)
    t = np.arange(L, dtype=np.float64)
    if kind == "hann":
        return 0.5 - 0.5 * np.cos(2.0 * np.pi * t / L)
    if kind == "rect":
        return np.ones(L)
    if kind == "tukey":
        alpha = 0.5 if param is None else float(param)
        if alpha <= 0.0:
            return np.ones(L)
        # Periodic window of length L = symmetric window of length L + 1 with
        # its last sample dropped; the two tapers together span alpha * L.
        n = np.arange(L + 1, dtype=np.float64)
        span = alpha * L / 2.0
        w = np.ones(L + 1)
        rise = n < span
        w[rise] = 0.5 * (1.0 - np.cos(np.pi * n[rise] / span))
        fall = n > L - span
        w[fall] = 0.5 * (1.0 - np.cos(np.pi * (L - n[fall]) / span))
        return w[:L]
    if kind == "hann_width":
        r = 1.0 if param is None else float(param)
        d = t - L / 2.0
        half = r * L / 2.0
        w = np.where(np.abs(d) <= half, 0.5 + 0.5 * np.cos(2.0 * np.pi * d / (r * L)), 0.0)
        return w
    raise ValueError(f"unknown window {kind!r}")


def window_width_derivative(seg_len: int, r: float) -> np.ndarray:
    """d w_r(t) / d r of the width-r Hann window."""
    L = int(seg_len)
    t = np.arange(L, dtype=np.float64)
    d = t - L / 2.0
    phase = 2.0 * np.pi * d / (r * L)
    inside = np.abs(d) <= r * L / 2.0
    return np.where(inside, 0.5 * np.sin(phase) * phase / r, 0.0)


# --------------------------------------------------------------------------
# Axes (App. B, trajectory paragraph: energies span -h/(2 tau) .. h/(2 tau);
# sampling h / (L tau); Sec. III.A worked numbers)
# --------------------------------------------------------------------------

def frequency_axis_thz(seg_len: int, dt_fs: float) -> np.ndarray:
    """nu_m in THz for bins m = 0..L-1 in FFT order."""
    L = int(seg_len)
    m = np.arange(L)
    signed = np.where(m < (L + 1) // 2, m, m - L).astype(np.float64)
    return signed / (L * dt_fs * 1e-15) / 1e12


def energy_axis_mev(seg_len: int, dt_fs: float) -> np.ndarray:
    return frequency_axis_thz(seg_len, dt_fs) * 1e12 * PLANCK_EV_S * 1e3


def energy_sampling_mev(seg_len: int, dt_fs: float) -> float:
    return PLANCK_EV_S / (seg_len * dt_fs * 1e-15) * 1e3


def energy_range_mev(dt_fs: float) -> float:
    """Largest representable |E| = h / (2 tau)."""
    return PLANCK_EV_S / (2.0 * dt_fs * 1e-15) * 1e3


def energy_roi_bins(seg_len: int, dt_fs: float, f_max_thz: float) -> np.ndarray:
    """Bins m whose |nu_m| <= f_max (inclusive), in FFT order."""
    nu = frequency_axis_thz(seg_len, dt_fs)
    step = 1.0 / (seg_len * dt_fs * 1e-15) / 1e12
    # inclusive comparison in units of the bin spacing, immune to last-digit noise
    return np.nonzero(np.abs(nu) / step <= f_max_thz / step + 1e-9)[0]


def quantum_factor(energy_mev: np.ndarray, temperature_k: float) -> np.ndarray:
    """beta E / (1 - exp(-beta E)) of Eq. 1 (limit 1 at E = 0; 1 for T = 0)."""
    e = np.asarray(energy_mev, dtype=np.float64)
    if temperature_k <= 0.0:
        return np.ones_like(e)
    kb_mev = 8.617333262e-2  # Boltzmann constant in meV/K
    x = e / (kb_mev * temperature_k)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = x[nz] / (-np.expm1(-x[nz]))
    return out


# --------------------------------------------------------------------------
# The reduction itself
# --------------------------------------------------------------------------

def dft_matrix(seg_len: int) -> np.ndarray:
    """F[m, t] = exp(-2 pi i m t / L), exponent reduced mod L for accuracy."""
    L = int(seg_len)
    mt = np.outer(np.arange(L), np.arange(L)) % L
    return np.exp(-2j * np.pi * mt / L)


def _as_series(psi: np.ndarray) -> np.ndarray:
    a = np.asarray(psi)
    if a.ndim < 2:
        raise ValueError("psi must be [n_frames, n_pixels, ...]")
    return a.reshape(a.shape[0], -1).astype(np.complex128)


def probe_mean(psi_p: np.ndarray, seg_len: int, hop: int, mean_mode: str) -> np.ndarray:
    """Elastic mean mu(k) of one probe's series [n_frames, n_k] (GLOBAL mode)."""
    z = _as_series(psi_p)
    if mean_mode == "none":
        return np.zeros(z.shape[1], dtype=np.complex128)
    if mean_mode != "global":
        raise ValueError("probe_mean covers the global mode only")
    nu = frames_used(z.shape[0], seg_len, hop)
    return z[:nu].sum(axis=0) / nu


def segment_spectra(psi_p, seg_len, hop, w, mean_mode="global", fft=False):
    """Per-chunk power P_s(m, k) = |X_s(m, k)|^2 / (L sum w^2), shape [N_s, L, n_k].

    X_s(m, k) = sum_t w(t) (psi(sH + t, k) - mu) exp(-2 pi i m t / L), computed
    as a dense DFT-matrix product (brute force) unless ``fft`` is set.
    """
    if mean_mode not in MEAN_MODES:
        raise ValueError(f"mean_mode must be one of {MEAN_MODES}")
    z = _as_series(psi_p)
    L, H = int(seg_len), int(hop)
    w = np.asarray(w, dtype=np.float64)
    if w.shape != (L,):
        raise ValueError("window length must equal the segment length")
    starts = segment_starts(z.shape[0], L, H)
    if not starts:
        return np.zeros((0, L, z.shape[1]))
    norm = 1.0 / (L * np.sum(w * w))
    if mean_mode == "global":
        mu = probe_mean(z, L, H, "global")
    F = None if fft else dft_matrix(L)
    out = np.empty((len(starts), L, z.shape[1]))
    for i, s0 in enumerate(starts):
        seg = z[s0:s0 + L]
        if mean_mode == "global":
            seg = seg - mu[None, :]
        elif mean_mode == "per_segment":
            seg = seg - seg.mean(axis=0, keepdims=True)
        y = w[:, None] * seg
        X = np.fft.fft(y, axis=0) if fft else F @ y
        out[i] = (X.real ** 2 + X.imag ** 2) * norm
    return out


def tacaw_spectra(psi, seg_len, hop, w, mean_mode="global", probe_reduce="mean", fft=False):
    """S(m, k) and per-probe S_p(m, k) for psi [P, n_frames, n_k...].

    S_p = (1/N_s) sum_s P_{p,s} (Eq. 2's chunk average); S = mean (or sum) of
    S_p over probes (the union over scan positions of Eq. 2).
    Returns (S [L, n_k], S_p [P, L, n_k]).
    """
    if probe_reduce not in PROBE_REDUCE:
        raise ValueError(f"probe_reduce must be one of {PROBE_REDUCE}")
    psi = np.asarray(psi)
    P = psi.shape[0]
    per_probe = []
    for p in range(P):
        segs = segment_spectra(psi[p], seg_len, hop, w, mean_mode, fft=fft)
        if segs.shape[0] == 0:
            raise ValueError("series shorter than one segment")
        per_probe.append(segs.mean(axis=0))
    Sp = np.stack(per_probe)
    S = Sp.sum(axis=0)
    if probe_reduce == "mean":
        S = S / P
    return S, Sp


def tacaw_spectra_fft(psi, seg_len, hop, w, mean_mode="global", probe_reduce="mean"):
    """Same as tacaw_spectra with numpy's FFT in place of the dense DFT."""
    return tacaw_spectra(psi, seg_len, hop, w, mean_mode, probe_reduce, fft=True)


def detector_spectra(S, masks):
    """D_j(m) = sum_k M_j(k) S(m, k); S [..., L, n_k], masks [n_det, n_k...]."""
    M = np.asarray(masks, dtype=np.float64).reshape(np.shape(masks)[0], -1)
    S = np.asarray(S, dtype=np.float64)
    return np.einsum("jk,...mk->...jm", M, S)


def detector_loss(psi, seg_len, hop, w, masks, a, mean_mode="global", probe_reduce="mean", b=None):
    """Scalar loss sum_j sum_m a_j(m) D_j(m) (+ sum_{j,p,m} b_{j,p}(m) D_{j,p}(m))."""
    S, Sp = tacaw_spectra(psi, seg_len, hop, w, mean_mode, probe_reduce)
    D = detector_spectra(S, masks)
    val = float(np.sum(np.asarray(a) * D))
    if b is not None:
        Dp = detector_spectra(Sp, masks)          # [P, n_det, L]
        val += float(np.sum(np.asarray(b) * np.transpose(Dp, (1, 0, 2))))
    return val


# --------------------------------------------------------------------------
# Adjoint (vector-Jacobian product) of the spectra
# --------------------------------------------------------------------------

def spectra_vjp(psi, seg_len, hop, w, gS, gSp=None, mean_mode="global",
                probe_reduce="mean", dw=None):
    """Gradient of  Lval = <gS, S> + sum_p <gSp_p, S_p>  with respect to psi (and r).

    The complex gradient follows the convention d/dRe + i d/dIm (twice the
    Wirtinger derivative with respect to conj(psi)). With
    X = sum_t w(t) z(t) e^{-2 pi i m t / L} and Lval = sum kappa G |X|^2:

      grad_y(t)  = 2 kappa sum_m G(m) X(m) e^{+2 pi i m t / L}
      grad_z(t)  = w(t) grad_y(t)
      grad_psi   = scatter of grad_z over the chunks, minus the mean term
      dLval/dw(t) = sum Re[conj(grad_y(t)) z(t)]

    and, when ``dw`` = dw/dr is given, dLval/dr = sum_t dLval/dw(t) dw(t)
    - 2 Lval sum_t w dw / sum_t w^2 (the normalisation depends on w too).
    Returns (grad_psi [P, n_frames, n_k] complex128, dLval/dr or None, Lval).
    """
    psi = np.asarray(psi)
    P, NT = psi.shape[0], psi.shape[1]
    L, H = int(seg_len), int(hop)
    w = np.asarray(w, dtype=np.float64)
    gS = np.asarray(gS, dtype=np.float64).reshape(L, -1)
    nk = gS.shape[1]
    Ns = segment_count(NT, L, H)
    Nu = frames_used(NT, L, H)
    if Ns == 0:
        raise ValueError("series shorter than one segment")
    base = 1.0 / (L * np.sum(w * w) * Ns)
    kappa_S = base / P if probe_reduce == "mean" else base
    F = dft_matrix(L)
    Finv = np.conj(F)          # e^{+2 pi i m t / L}
    grad = np.zeros((P, NT, nk), dtype=np.complex128)
    dLdw = np.zeros(L)
    lval = 0.0
    for p in range(P):
        z_all = psi[p].reshape(NT, -1).astype(np.complex128)
        if mean_mode == "global":
            mu = z_all[:Nu].sum(axis=0) / Nu
        G = kappa_S * gS
        if gSp is not None:
            G = G + base * np.asarray(gSp[p], dtype=np.float64).reshape(L, -1)
        mean_acc = np.zeros(nk, dtype=np.complex128)
        for s in range(Ns):
            s0 = s * H
            seg = z_all[s0:s0 + L]
            if mean_mode == "global":
                z = seg - mu[None, :]
            elif mean_mode == "per_segment":
                z = seg - seg.mean(axis=0, keepdims=True)
            else:
                z = seg
            X = F @ (w[:, None] * z)
            lval += float(np.sum(G * (X.real ** 2 + X.imag ** 2)))
            gy = 2.0 * (Finv @ (G * X))
            gz = w[:, None] * gy
            dLdw += np.sum(np.real(np.conj(gy) * z), axis=1)
            grad[p, s0:s0 + L] += gz
            if mean_mode == "global":
                mean_acc += gz.sum(axis=0)
            elif mean_mode == "per_segment":
                grad[p, s0:s0 + L] -= gz.sum(axis=0, keepdims=True) / L
        if mean_mode == "global":
            grad[p, :Nu] -= mean_acc[None, :] / Nu
    grad = grad.reshape(psi.shape)
    dr = None
    if dw is not None:
        dw = np.asarray(dw, dtype=np.float64)
        dr = float(np.sum(dLdw * dw) - 2.0 * lval * np.sum(w * dw) / np.sum(w * w))
    return grad, dr, lval


def detector_loss_vjp(psi, seg_len, hop, w, masks, a, mean_mode="global",
                      probe_reduce="mean", b=None, dw=None):
    """Gradient of detector_loss: gS(m,k) = sum_j a_j(m) M_j(k) (and the per-probe
    analogue from b); returns (grad_psi, dL/dr or None, loss)."""
    M = np.asarray(masks, dtype=np.float64).reshape(np.shape(masks)[0], -1)
    gS = np.einsum("jm,jk->mk", np.asarray(a, dtype=np.float64), M)
    gSp = None
    if b is not None:
        gSp = np.einsum("jpm,jk->pmk", np.asarray(b, dtype=np.float64), M)
    return spectra_vjp(psi, seg_len, hop, w, gS, gSp, mean_mode, probe_reduce, dw)
