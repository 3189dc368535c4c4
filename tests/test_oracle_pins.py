"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each check uses a closed form, an
explicit brute-force sum written in loops, a library routine the method reduces
to (scipy.signal.welch), or a number the paper prints (tests/golden).
"""

import math

import numpy as np
import pytest
import scipy.signal

import oracle as O
from conftest import load_golden

RNG = np.random.default_rng(20260712)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- worked numbers

def test_worked_chunk_count_31():
    g = load_golden("worked_examples.txt")
    L = int(g["chunk_len"])
    H = O.hop_from_overlap(L, int(g["chunk_overlap_nu"]))
    assert H == 100
    assert O.segment_count(int(g["frames_after_skip"]), L, H) == int(g["chunk_count"])
    # frames_after_skip is itself 51 ps - 3 ps at 15 fs
    assert round((51_000 - 3_000) / g["timestep_fs"]) == int(g["frames_after_skip"])


def test_worked_energy_sampling_1p4_mev():
    g = load_golden("worked_examples.txt")
    de = O.energy_sampling_mev(int(g["chunk_len"]), g["timestep_fs"])
    digits = int(g["energy_sampling_digits"])
    assert float(f"{de:.{digits}g}") == g["energy_sampling_meV"]
    # the axis spacing equals the sampling
    ax = O.energy_axis_mev(int(g["chunk_len"]), g["timestep_fs"])
    assert ax[1] - ax[0] == pytest.approx(de, rel=1e-12)


def test_worked_energy_roi_181_bins():
    g = load_golden("worked_examples.txt")
    bins = O.energy_roi_bins(int(g["chunk_len"]), g["timestep_fs"], g["roi_THz"])
    assert len(bins) == int(g["roi_energy_bins"])
    nu = O.frequency_axis_thz(int(g["chunk_len"]), g["timestep_fs"])
    assert np.max(np.abs(nu[bins])) == pytest.approx(30.0, rel=1e-9)


def test_worked_energy_range_rule():
    g = load_golden("worked_examples.txt")
    # eps = h / (2 tau) with the paper's "~2000 meV / (tau/fs)" rule of thumb
    assert O.energy_range_mev(1.0) == pytest.approx(g["range_rule_meV_fs"], rel=0.05)
    assert O.energy_range_mev(5.0) == pytest.approx(413.567, rel=1e-5)
    # the largest FFT-order bin sits at -eps (even L): nu_{L/2} = -1/(2 dt)
    ax = O.energy_axis_mev(256, 5.0)
    assert ax[128] == pytest.approx(-O.energy_range_mev(5.0), rel=1e-12)


def test_segmentation_tail_and_frames_used():
    assert O.segment_count(2048, 512, 256) == 7
    assert O.frames_used(2048, 512, 256) == 2048
    assert O.segment_count(1000, 512, 256) == 2
    assert O.frames_used(1000, 512, 256) == 768
    assert O.segment_count(511, 512, 256) == 0
    assert O.segment_starts(1024, 512, 512) == [0, 512]
    with pytest.raises(ValueError):
        O.segment_count(100, 10, 0)


# ---------------------------------------------------------------- windows

@pytest.mark.parametrize("L", [8, 64, 200, 512])
def test_tukey_limits_and_scipy(L):
    # Sec. III.A: alpha = 1 is Hann, alpha = 0 is rectangular
    np.testing.assert_allclose(O.window("tukey", L, 1.0), O.window("hann", L), atol=1e-15)
    np.testing.assert_array_equal(O.window("tukey", L, 0.0), np.ones(L))
    for alpha in (0.1, 0.5, 0.9):
        np.testing.assert_allclose(O.window("tukey", L, alpha),
                                   scipy.signal.windows.tukey(L, alpha, sym=False), atol=1e-14)
    np.testing.assert_allclose(O.window("hann", L), scipy.signal.get_window("hann", L), atol=1e-15)


@pytest.mark.parametrize("L", [16, 512])
def test_hann_width_window_is_a_shorter_hann(L):
    # width r < 1: a periodic Hann of length r L centred on L/2, zero elsewhere
    # (scipy's periodic Hann is an independent definition of that shape)
    for r in (0.5, 0.25):
        M = int(r * L)
        want = np.zeros(L)
        want[L // 2 - M // 2:L // 2 + M // 2] = scipy.signal.get_window("hann", M)
        np.testing.assert_allclose(O.window("hann_width", L, r), want, atol=1e-15)


@pytest.mark.parametrize("L", [16, 512])
def test_hann_width_window(L):
    np.testing.assert_allclose(O.window("hann_width", L, 1.0), O.window("hann", L), atol=1e-15)
    for r in (0.7, 1.0, 1.3):
        h = 1e-6
        fd = (O.window("hann_width", L, r + h) - O.window("hann_width", L, r - h)) / (2 * h)
        # at r = 1 the support edge sits on t = 0 where w is C1 but not C2, so the
        # central difference there carries an O(h) error (about 1.2e-6 at h = 1e-6)
        np.testing.assert_allclose(O.window_width_derivative(L, r), fd, atol=5e-6)
        assert np.max(np.abs(O.window_width_derivative(L, r) - fd)[1:]) < 1e-7


# ---------------------------------------------------------------- transform core

def _raw_power(y):
    """|DFT|^2 of one column by explicit double loop (forward kernel e^{-i w t})."""
    L = len(y)
    out = np.zeros(L)
    for m in range(L):
        acc = 0j
        for t in range(L):
            acc += y[t] * complex(math.cos(-2 * math.pi * m * t / L), math.sin(-2 * math.pi * m * t / L))
        out[m] = abs(acc) ** 2
    return out


@pytest.mark.parametrize("kind", ["rect", "hann"])
def test_wiener_khinchin(kind):
    # |X(m)|^2 equals the DFT of the circular autocorrelation r(t) of y = w psi
    L = 12
    psi = crandn(L, 3)
    w = O.window(kind, L)
    P = O.segment_spectra(psi, L, L, w, mean_mode="none")[0]
    scale = L * np.sum(w * w)
    for k in range(3):
        y = w * psi[:, k]
        r = [sum(y[(u + t) % L] * np.conj(y[u]) for u in range(L)) for t in range(L)]
        wk = [sum(r[t] * complex(math.cos(2 * math.pi * m * t / L), -math.sin(2 * math.pi * m * t / L))
                  for t in range(L)) for m in range(L)]
        np.testing.assert_allclose(P[:, k] * scale, np.real(wk), rtol=1e-12, atol=1e-12)
        assert np.max(np.abs(np.imag(wk))) < 1e-10
        np.testing.assert_allclose(P[:, k] * scale, _raw_power(y), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", ["none", "global", "per_segment"])
def test_parseval_per_segment(mode):
    L, H, NT = 16, 8, 40
    psi = 1.0 + 0.1 * crandn(NT, 5)
    w = O.window("hann", L)
    P = O.segment_spectra(psi, L, H, w, mean_mode=mode)
    mu = psi[:O.frames_used(NT, L, H)].mean(axis=0)
    for s, s0 in enumerate(O.segment_starts(NT, L, H)):
        seg = psi[s0:s0 + L]
        if mode == "global":
            seg = seg - mu
        elif mode == "per_segment":
            seg = seg - seg.mean(axis=0)
        expect = np.sum(w[:, None] ** 2 * np.abs(seg) ** 2, axis=0) / np.sum(w * w)
        np.testing.assert_allclose(P[s].sum(axis=0), expect, rtol=1e-12)


@pytest.mark.parametrize("mode", ["none", "global"])
def test_on_bin_tone_rect_and_hann(mode):
    L, m0, A = 64, 5, 0.7 - 0.2j
    t = np.arange(L)
    psi = (A * np.exp(2j * np.pi * m0 * t / L))[:, None]
    rect = O.segment_spectra(psi, L, L, O.window("rect", L), mode)[0][:, 0]
    expect = np.zeros(L)
    expect[m0] = abs(A) ** 2
    np.testing.assert_allclose(rect, expect, atol=1e-14)
    hann = O.segment_spectra(psi, L, L, O.window("hann", L), mode)[0][:, 0]
    expect = np.zeros(L)
    expect[m0] = 2 / 3 * abs(A) ** 2
    expect[m0 - 1] = expect[m0 + 1] = abs(A) ** 2 / 6
    np.testing.assert_allclose(hann, expect, atol=1e-14)


def test_tone_sign_positive_frequency_lands_at_plus_m():
    # Sec. III.B forward kernel exp(-i omega t): exp(+i omega0 t) peaks at +omega0
    L = 32
    t = np.arange(L)
    psi = np.exp(2j * np.pi * 3 * t / L)[:, None]
    P = O.segment_spectra(psi, L, L, O.window("rect", L), "none")[0][:, 0]
    assert int(np.argmax(P)) == 3
    assert P[L - 3] < 1e-20


def test_off_bin_tone_hann_closed_form():
    L, nu0, A = 48, 7.37, 1.3
    t = np.arange(L)
    psi = (A * np.exp(2j * np.pi * nu0 * t / L))[:, None]
    P = O.segment_spectra(psi, L, L, O.window("hann", L), "none")[0][:, 0]

    def G(phi):  # sum_{t<L} e^{i phi t} as a geometric series
        return (1 - np.exp(1j * L * phi)) / (1 - np.exp(1j * phi))

    m = np.arange(L)
    phi = 2 * np.pi * (nu0 - m) / L
    X = A * (0.5 * G(phi) - 0.25 * G(phi + 2 * np.pi / L) - 0.25 * G(phi - 2 * np.pi / L))
    sum_w2 = 3 * L / 8  # periodic Hann
    np.testing.assert_allclose(P, np.abs(X) ** 2 / (L * sum_w2), rtol=1e-10, atol=1e-16)
    assert int(np.argmax(P)) == round(nu0)


def test_leakage_tails_hann_cubic_rect_linear():
    # Sec. III.A: the Hann window's leakage falls off as 1/omega^3 in amplitude, the
    # rectangular window's as 1/omega. A tone half-way between bins puts every other
    # bin in the tail; the log-log slope of |X| over 8.5 .. 32.5 bins away is -3 / -1.
    L, nu0 = 512, 100.5
    t = np.arange(L)
    psi = np.exp(2j * np.pi * nu0 * t / L)[:, None]
    d = np.array([8.5, 16.5, 32.5])
    m = (nu0 + d).astype(int)
    for kind, slope in (("hann", -3.0), ("rect", -1.0)):
        P = O.segment_spectra(psi, L, L, O.window(kind, L), "none")[0][:, 0]
        amp = np.sqrt(P[m])
        fit = np.polyfit(np.log(d), np.log(amp), 1)[0]
        assert abs(fit - slope) < 0.1, (kind, fit)
    # Hann: |X(delta)| ~ |sin(pi delta)| / (2 pi delta (delta^2 - 1)) for delta << L
    P = O.segment_spectra(psi, L, L, O.window("hann", L), "none")[0][:, 0]
    ref = (1.0 / (2 * np.pi * d * (d ** 2 - 1))) ** 2
    r = P[m] / ref
    assert np.ptp(r) / r.mean() < 0.03


def test_static_wave_gives_exact_zero():
    # mean subtraction must remove a time-independent wave exactly (S == 0)
    vals = (RNG.standard_normal(6) + 1j * RNG.standard_normal(6)).astype(np.complex64)
    psi = np.broadcast_to(vals, (3, 37, 6)).astype(np.complex64)
    S, Sp = O.tacaw_spectra(psi, 16, 8, O.window("hann", 16), "global")
    assert np.all(S == 0.0) and np.all(Sp == 0.0)
    S, _ = O.tacaw_spectra(psi, 16, 8, O.window("hann", 16), "per_segment")
    assert np.all(S == 0.0)


def test_zero_loss_peak_claims():
    # Sec. III.A: with a rectangular window the ZLP falls exactly in bin 0;
    # cosine-sum (Hann) windows keep it in bins 0 and +-1 only.
    L = 40
    c = 0.9 + 0.4j
    psi = np.full((L, 1), c)
    rect = O.segment_spectra(psi, L, L, O.window("rect", L), "none")[0][:, 0]
    assert rect[0] == pytest.approx(abs(c) ** 2, rel=1e-13)
    assert np.max(rect[1:]) < 1e-28
    hann = O.segment_spectra(psi, L, L, O.window("hann", L), "none")[0][:, 0]
    assert hann[0] == pytest.approx(2 / 3 * abs(c) ** 2, rel=1e-13)
    assert hann[1] == pytest.approx(abs(c) ** 2 / 6, rel=1e-13)
    assert hann[-1] == pytest.approx(abs(c) ** 2 / 6, rel=1e-13)
    assert np.max(hann[2:-1]) < 1e-28
    # a Tukey(0.1) window leaks the ZLP into far bins (the artefact Sec. III.A shows)
    tk = O.segment_spectra(psi, L, L, O.window("tukey", L, 0.1), "none")[0][:, 0]
    assert np.max(tk[3:-2]) > 1e-6


@pytest.mark.parametrize("mode,detrend", [("per_segment", "constant"), ("none", False)])
@pytest.mark.parametrize("L,H,NT", [(16, 8, 50), (32, 32, 96), (20, 10, 77)])
def test_scipy_welch_special_case(mode, detrend, L, H, NT):
    psi = 0.3 + crandn(NT, 4)
    w = O.window("hann", L)
    _, Sp = O.tacaw_spectra(psi[None], L, H, w, mean_mode=mode)
    fs = 1.0
    for k in range(4):
        f, pxx = scipy.signal.welch(psi[:, k], fs=fs, window="hann", nperseg=L, noverlap=L - H,
                                    detrend=detrend, return_onesided=False, scaling="density")
        np.testing.assert_allclose(Sp[0, :, k], pxx * fs / L, rtol=1e-11, atol=1e-15)


def test_modulation_theorem_shifts_bins():
    # Sec. III.B drift phase ramp: a linear phase exp(2 pi i m0 n / L) shifts S by m0
    L, H, NT, m0 = 16, 8, 48, 3
    psi = crandn(2, NT, 3)
    n = np.arange(NT)
    mod = psi * np.exp(2j * np.pi * m0 * n / L)[None, :, None]
    w = O.window("hann", L)
    S0, _ = O.tacaw_spectra(psi, L, H, w, "none")
    S1, _ = O.tacaw_spectra(mod, L, H, w, "none")
    np.testing.assert_allclose(S1, np.roll(S0, m0, axis=0), rtol=1e-11)


def test_detector_linearity_and_probe_union():
    L, H, NT = 16, 8, 40
    psi = 1 + 0.01 * crandn(4, NT, 3, 5)
    w = O.window("hann", L)
    S, Sp = O.tacaw_spectra(psi, L, H, w)
    parts = np.zeros((3, 3, 5))
    idx = RNG.integers(0, 3, size=(3, 5))
    for j in range(3):
        parts[j][idx == j] = 1.0
    D = O.detector_spectra(S, parts)
    np.testing.assert_allclose(D.sum(axis=0), S.sum(axis=1), rtol=1e-12)
    np.testing.assert_allclose(O.detector_spectra(S, np.ones((1, 15)))[0], S.sum(axis=1), rtol=1e-12)
    # Eq. 2: the union over scan batches equals the whole; SUM = P * MEAN
    Sa, _ = O.tacaw_spectra(psi[:1], L, H, w)
    Sb, _ = O.tacaw_spectra(psi[1:], L, H, w)
    np.testing.assert_allclose((Sa + 3 * Sb) / 4, S, rtol=1e-12)
    Ssum, _ = O.tacaw_spectra(psi, L, H, w, probe_reduce="sum")
    np.testing.assert_allclose(Ssum, 4 * S, rtol=1e-12)
    np.testing.assert_allclose(Sp.mean(axis=0), S, rtol=1e-12)


def test_global_mean_ignores_dropped_tail():
    L, H = 16, 8
    psi = 1 + 0.01 * crandn(1, 37, 2)
    assert O.frames_used(37, L, H) == 32
    tail = psi.copy()
    tail[0, 32:] = 1e6  # frames 32..36 belong to no full chunk
    w = O.window("hann", L)
    np.testing.assert_array_equal(O.tacaw_spectra(psi, L, H, w)[0], O.tacaw_spectra(tail, L, H, w)[0])


def test_fft_oracle_matches_brute_force():
    psi = 1 + 1e-3 * crandn(3, 300, 7)
    for L, H in [(64, 32), (128, 128), (100, 50)]:
        w = O.window("hann", L)
        Sb, Spb = O.tacaw_spectra(psi, L, H, w)
        Sf, Spf = O.tacaw_spectra_fft(psi, L, H, w)
        assert np.linalg.norm(Sf - Sb) / np.linalg.norm(Sb) < 1e-12
        assert np.linalg.norm(Spf - Spb) / np.linalg.norm(Spb) < 1e-12


def test_quantum_factor_limits_and_detailed_balance():
    e = np.array([-40.0, -3.0, 0.0, 3.0, 40.0])
    f = O.quantum_factor(e, 300.0)
    assert f[2] == 1.0
    beta = 1.0 / (8.617333262e-2 * 300.0)
    np.testing.assert_allclose(f[0] / f[4], np.exp(-beta * 40.0), rtol=1e-12)
    np.testing.assert_allclose(f[1] / f[3], np.exp(-beta * 3.0), rtol=1e-12)
    np.testing.assert_array_equal(O.quantum_factor(e, 0.0), np.ones(5))


# ---------------------------------------------------------------- gradient

def _fd_gradient(f, x, h):
    g = np.zeros_like(x)
    flat = x.reshape(-1)
    gflat = g.reshape(-1)
    for i in range(flat.size):
        for part, unit in ((0, 1.0), (1, 1j)):
            xp = flat.copy()
            xm = flat.copy()
            xp[i] += h * unit
            xm[i] -= h * unit
            d = (f(xp.reshape(x.shape)) - f(xm.reshape(x.shape))) / (2 * h)
            gflat[i] += d * unit
    return g


@pytest.mark.parametrize("mode", ["global", "per_segment", "none"])
@pytest.mark.parametrize("reduce_", ["mean", "sum"])
def test_gradient_matches_exhaustive_central_differences(mode, reduce_):
    # the loss is a quadratic form in psi, so central differences are exact up
    # to rounding for any step: every real component is checked
    L, H, NT, P = 8, 4, 14, 2
    psi = 1 + 0.1 * crandn(P, NT, 3)
    masks = RNG.random((2, 3))
    a = RNG.random((2, L))
    b = RNG.random((2, P, L))
    w = O.window("hann", L)

    def loss(x):
        return O.detector_loss(x, L, H, w, masks, a, mode, reduce_, b=b)

    g, _, val = O.detector_loss_vjp(psi, L, H, w, masks, a, mode, reduce_, b=b)
    assert val == pytest.approx(loss(psi), rel=1e-12)
    fd = _fd_gradient(loss, psi, 0.5)
    np.testing.assert_allclose(g, fd, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("r", [1.0, 0.85])
def test_window_width_gradient_matches_fd(r):
    L, H, NT, P = 16, 16, 32, 2
    psi = 1 + 0.1 * crandn(P, NT, 3)
    masks = RNG.random((2, 3))
    a = RNG.random((2, L))

    def loss(rr):
        return O.detector_loss(psi, L, H, O.window("hann_width", L, rr), masks, a)

    _, dr, _ = O.detector_loss_vjp(psi, L, H, O.window("hann_width", L, r), masks, a,
                                   dw=O.window_width_derivative(L, r))
    # at r = 1 the support edge is on t = 0 (w is C1, not C2 there): the central
    # difference has an O(h) error, so a smaller step is used at that point
    h = 1e-6 if r == 1.0 else 1e-4
    fd = (loss(r + h) - loss(r - h)) / (2 * h)
    assert dr == pytest.approx(fd, rel=1e-6)


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_planted_sign_error(monkeypatch):
    # a flipped transform sign must break the sign pin (a plausible mistake)
    real = O.tacaw_oracle.dft_matrix
    monkeypatch.setattr(O.tacaw_oracle, "dft_matrix", lambda L: np.conj(real(L)))
    with pytest.raises(AssertionError):
        test_tone_sign_positive_frequency_lands_at_plus_m()


def test_pins_catch_planted_normalisation_error(monkeypatch):
    real = O.tacaw_oracle.window

    def bad(kind, L, param=None):
        w = real(kind, L, param)
        return w * 1.0001 if kind == "hann" else w

    monkeypatch.setattr(O.tacaw_oracle, "window", bad)
    monkeypatch.setattr(O, "window", bad)
    with pytest.raises(AssertionError):
        test_hann_width_window(16)
