"""Named plan settings, the Python side of the plan descriptor.

Each ``Workload`` fixes the shape of a run: probes, frames, k-grid, frame
interval, chunking, transform, streaming ring and detector masks. It can
validate its descriptor on the host, build its masks and open a
``tacaw.Plan``. The presets are the benchmark workloads of this library and
the paper's own settings:

* ``PLAIN``, ``REALISTIC``, ``PRECISION``, ``GRADIENT``, ``STREAMING``: the
  five synthetic benchmark shapes (one probe at 64^2; 64 probes at 256^2;
  the DFT-GEMM precision form; the adjoint workload; the 256-probe 1024^2
  streaming run).
* ``PAPER_PLANE_WAVE``: Sec. III.A's window study, a plane wave (one probe)
  on a 383 x 383 k-space window of +-100 mrad, chunks of 200 snapshots at
  15 fs with nu = 2 (hop 100), 31 chunks, and the +-30 THz energy window
  (181 bins).
* ``PAPER_STEM``: Sec. IV's STEM-EELS scan, 16 x 16 probes, the same grid and
  chunking, 191 energy bins, batches of 4 x 8 probes in flight, and its four
  detectors (bright field 0-10 mrad, annuli 10-30, 30-60, 60-100 mrad) at the
  0.52 mrad pixel spacing of Sec. III.A.

Detector geometry is in pixels of the k-grid (``detectors`` builds the masks);
the benchmark shapes use the four detectors of the synthetic series (central
disk, annulus, two displaced disks) scaled with the grid.
"""

import dataclasses

import numpy as np

from . import axes, detectors

# k-space pixel spacing of the paper's 1680^2 multislice grid (Sec. III.A)
PAPER_MRAD_PER_PIXEL = 0.52


def _standard_four(ny):
    """Central disk r < 30, annulus 60..100, disks r < 30 displaced by +60 px
    along x and along y, in pixels of a 256-pixel grid scaled to ny."""
    s = ny / 256
    r, a0, a1, off = 30 * s, 60 * s, 100 * s, int(round(60 * s))
    return (("circular", 0.0, r, (0, 0)), ("annular", a0, a1, (0, 0)),
            ("circular", 0.0, r, (0, off)), ("circular", 0.0, r, (off, 0)))


def _mrad_rings(bounds_mrad, mrad_per_px=PAPER_MRAD_PER_PIXEL):
    """Centred detectors lo <= theta < hi for consecutive bounds, in pixels."""
    return tuple(("annular", lo / mrad_per_px, hi / mrad_per_px, (0, 0))
                 for lo, hi in zip(bounds_mrad[:-1], bounds_mrad[1:]))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_probe: int
    n_frames: int
    ny: int
    nx: int
    dt_fs: float
    seg_len: int
    hop: int
    in_dtype: str = "c64"
    window: str = "hann"
    window_param: float = 1.0
    mean_mode: str = "global"
    transform: str = "fft"
    omega_half: int = 0
    push_frames: int = 0          # frames per push (0: each probe's whole series at once)
    ring_frames: int = 0          # > seg_len: deferred streaming ring
    tiled_ring: bool = False
    max_probes_in_flight: int = 0  # 0: all probes
    # detectors: (kind, inner, outer, (dy, dx) offset of the centre from (ny//2, nx//2))
    detectors: tuple = ()

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    @property
    def n_segments(self) -> int:
        return (self.n_frames - self.seg_len) // self.hop + 1

    @property
    def frames_used(self) -> int:
        return (self.n_segments - 1) * self.hop + self.seg_len

    @property
    def n_omega(self) -> int:
        return 2 * self.omega_half + 1 if self.omega_half else self.seg_len

    @property
    def energy_step_mev(self) -> float:
        return axes.energy_step_mev(self.seg_len, self.dt_fs)

    @property
    def exit_wave_bytes(self) -> int:
        esz = 8 if self.in_dtype == "c64" else 16
        return self.n_probe * self.n_frames * self.ny * self.nx * esz

    def masks(self) -> np.ndarray:
        """[n_det, ny, nx] float64 masks (empty first axis without detectors)."""
        if not self.detectors:
            return np.zeros((0, self.ny, self.nx))
        cy, cx = self.ny // 2, self.nx // 2
        out = [detectors.annular(self.ny, self.nx, inner, outer, (cy + dy, cx + dx))
               for _, inner, outer, (dy, dx) in self.detectors]
        return np.stack(out)

    def _plan_kw(self) -> dict:
        return dict(window=self.window, window_param=self.window_param,
                    mean_mode=self.mean_mode, transform=self.transform, in_dtype=self.in_dtype,
                    dt_fs=self.dt_fs, max_probes_in_flight=self.max_probes_in_flight,
                    omega_half=self.omega_half, ring_frames=self.ring_frames)

    def check(self) -> None:
        """Host-only validation of the descriptor (detector masks aside); raises
        tacaw.TacawError."""
        from . import tacaw

        flags = tacaw.FLAG_TILED_RING if self.tiled_ring else 0
        tacaw.check_desc(n_probe=self.n_probe, ny=self.ny, nx=self.nx, n_frames=self.n_frames,
                         seg_len=self.seg_len, hop=self.hop, flags=flags, **self._plan_kw())

    def plan(self, masks=True, stream=None, **overrides):
        """Open a tacaw.Plan of this shape. masks: True = this workload's masks,
        None = no detectors, or a CUDA tensor [n_det, ny, nx]. Keyword overrides
        go to tacaw.Plan (e.g. probe_reduce, temperature_K, check_finite)."""
        import torch

        from . import tacaw

        if masks is True:
            m = self.masks()
            masks = torch.from_numpy(m).cuda() if m.shape[0] else None
        kw = self._plan_kw()
        kw.update(tiled_ring=self.tiled_ring, stream=stream)
        kw.update(overrides)
        return tacaw.Plan(self.n_probe, self.ny, self.nx, self.n_frames, self.seg_len, self.hop,
                          masks=masks, **kw)


PLAIN = Workload("plain", 1, 256, 64, 64, 5.0, 256, 256, in_dtype="c128",
                 detectors=(_standard_four(64)[1],))
REALISTIC = Workload("realistic", 64, 2048, 256, 256, 5.0, 512, 256,
                     detectors=_standard_four(256))
PRECISION = Workload("precision", 1, 512, 64, 64, 5.0, 512, 512, in_dtype="c128",
                     transform="gemm_bf16x3", detectors=(_standard_four(64)[1],))
GRADIENT = Workload("gradient", 16, 1024, 128, 128, 5.0, 512, 512, window="hann_width",
                    detectors=_standard_four(128))
STREAMING = Workload("streaming", 256, 4096, 1024, 1024, 5.0, 1024, 512, push_frames=256,
                     ring_frames=2048, tiled_ring=True, max_probes_in_flight=8,
                     detectors=_standard_four(1024))
PAPER_PLANE_WAVE = Workload("paper_plane_wave", 1, 30 * 100 + 200, 383, 383, 15.0, 200, 100,
                            omega_half=axes.omega_half_for(200, 15.0, f_max_thz=30.0))
PAPER_STEM = Workload("paper_stem", 16 * 16, 30 * 100 + 200, 383, 383, 15.0, 200, 100,
                      omega_half=95, push_frames=200, max_probes_in_flight=4 * 8,
                      detectors=_mrad_rings((0.0, 10.0, 30.0, 60.0, 100.0)))

PRESETS = {w.name: w for w in (PLAIN, REALISTIC, PRECISION, GRADIENT, STREAMING,
                               PAPER_PLANE_WAVE, PAPER_STEM)}


def mrad_radius_px(theta_mrad, mrad_per_px=PAPER_MRAD_PER_PIXEL) -> float:
    return theta_mrad / mrad_per_px


__all__ = ["Workload", "PRESETS", "PAPER_MRAD_PER_PIXEL", "mrad_radius_px"] + [
    n.upper() for n in PRESETS]
