"""Coordinates of the output bins (host helpers, no spectral arithmetic).

Bins are in FFT order: bin m has frequency m / (L dt) for m < L/2 and
(m - L) / (L dt) otherwise; energies E = h nu; the representable range is
+-h / (2 dt) (paper App. B, trajectory paragraph); the energy sampling is
h / (L dt) (Sec. III.A).
"""

import numpy as np

PLANCK_EV_S = 6.62607015e-34 / 1.602176634e-19


def frequency_thz(seg_len, dt_fs):
    m = np.arange(seg_len)
    signed = np.where(m < (seg_len + 1) // 2, m, m - seg_len)
    return signed / (seg_len * dt_fs * 1e-15) / 1e12


def energy_mev(seg_len, dt_fs):
    return frequency_thz(seg_len, dt_fs) * 1e12 * PLANCK_EV_S * 1e3


def energy_step_mev(seg_len, dt_fs):
    return PLANCK_EV_S / (seg_len * dt_fs * 1e-15) * 1e3


def centred_order(seg_len):
    """Permutation taking FFT-order bins to ascending frequency (fftshift)."""
    return np.fft.fftshift(np.arange(seg_len))


def roi_bins(seg_len, dt_fs, f_max_thz):
    """FFT-order bins with |nu| <= f_max_thz (inclusive)."""
    step = 1.0 / (seg_len * dt_fs * 1e-15) / 1e12
    m = np.arange(seg_len)
    signed = np.where(m < (seg_len + 1) // 2, m, m - seg_len)
    return np.nonzero(np.abs(signed) <= np.floor(f_max_thz / step + 1e-9))[0]
