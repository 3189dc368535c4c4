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


def omega_half_for(seg_len, dt_fs, f_max_thz=None, e_max_mev=None):
    """Energy-window half width M (bins) for |nu| <= f_max_thz or |E| <= e_max_mev:
    the largest M with M / (L dt) within the limit, capped at L/2 - 1."""
    step_thz = 1.0 / (seg_len * dt_fs * 1e-15) / 1e12
    if f_max_thz is None:
        f_max_thz = e_max_mev * 1e-3 / PLANCK_EV_S / 1e12
    return int(min(seg_len // 2 - 1, np.floor(f_max_thz / step_thz + 1e-9)))


def window_rows(seg_len, omega_half):
    """FFT-order bin of every output row: all bins (omega_half = 0) or the
    ascending bins -M..M of an energy window."""
    if omega_half == 0:
        return np.arange(seg_len)
    return np.mod(np.arange(-omega_half, omega_half + 1), seg_len)
