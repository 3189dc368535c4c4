"""Thin ctypes binding of libtacaw.so (the C ABI in include/tacaw.h).

Argument marshalling only: every step of the spectral path runs in the HIP
library. torch supplies device memory and the HIP stream. There is no CPU
fallback: if the library is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
FLAG_TIME_KERNELS = 1  # TACAW_FLAG_TIME_KERNELS
FLAG_TILED_RING = 2  # TACAW_FLAG_TILED_RING
FLAG_CHECK_FINITE = 4  # TACAW_FLAG_CHECK_FINITE
LIB_PATH = os.environ.get("TACAW_LIB") or os.path.join(_HERE, "libtacaw.so")

OK = 0
ERR = {-1: "INVALID_ARG", -2: "SHAPE", -3: "STATE", -4: "OOM", -5: "HIP", -6: "UNSUPPORTED",
       -7: "NONFINITE"}
WINDOWS = {"hann": 0, "rect": 1, "hann_width": 2, "tukey": 3, "custom": 4}
MEANS = {"global": 0, "per_segment": 1, "none": 2}
TRANSFORMS = {"fft": 0, "gemm_bf16x3": 1, "gemm_f16x3": 2}
DTYPES = {"c64": 0, "c128": 1}
REDUCE = {"mean": 0, "sum": 1}


class TacawError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tacaw {ERR.get(code, code)}: {msg}")
        self.code = code
        self.kind = ERR.get(code, str(code))


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_probe", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
        ("n_frames", C.c_int64),
        ("seg_len", C.c_int32), ("hop", C.c_int32),
        ("window", C.c_int32), ("window_param", C.c_double),
        ("mean_mode", C.c_int32), ("transform", C.c_int32), ("in_dtype", C.c_int32),
        ("probe_reduce", C.c_int32), ("dt_fs", C.c_double),
        ("n_det", C.c_int32), ("d_masks", C.c_void_p),
        ("max_probes_in_flight", C.c_int32), ("flags", C.c_int32),
        ("temperature_K", C.c_double), ("h_window", C.c_void_p),
        ("ring_frames", C.c_int64), ("k_row_stride", C.c_int64), ("omega_half", C.c_int32),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n_segments", C.c_int32), ("n_omega", C.c_int32),
        ("frames_used", C.c_int64), ("frames_dropped", C.c_int64), ("device_bytes", C.c_int64),
        ("state", C.c_int32), ("probes_complete", C.c_int32),
        ("window_sum_sq", C.c_double), ("tile_pixels", C.c_int32), ("nonfinite", C.c_int32),
        ("last_chunk_kernel_ms", C.c_double),
    ]


class SynthDesc(C.Structure):
    _fields_ = [
        ("ny", C.c_int32), ("nx", C.c_int32), ("n_terms", C.c_int32), ("n_lines", C.c_int32),
        ("seed", C.c_uint32), ("reserved", C.c_int32),
        ("amplitude", C.c_double), ("noise_sigma", C.c_double),
        ("elastic_re", C.c_double), ("elastic_im", C.c_double),
        ("e_lo_mev", C.c_double), ("e_hi_mev", C.c_double),
        ("line_lo_mev", C.c_double), ("line_hi_mev", C.c_double),
        ("hwhm_lo_mev", C.c_double), ("hwhm_hi_mev", C.c_double), ("dt_fs", C.c_double),
        ("d_cos", C.c_void_p), ("d_sin", C.c_void_p), ("d_normal", C.c_void_p), ("d_tan", C.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2607_02236_amd.build")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "tacaw_plan": (C.c_int, [C.POINTER(PlanDesc), P, C.POINTER(P)]),
        "tacaw_plan_check": (C.c_int, [C.POINTER(PlanDesc)]),
        "tacaw_push_frames": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int64]),
        "tacaw_finalize": (C.c_int, [P, P]),
        "tacaw_detector_spectra": (C.c_int, [P, P, C.c_int32, P, P]),
        "tacaw_backward": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, P, P, P, P, P]),
        "tacaw_backward_static": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, P, P,
                                            P, P, P]),
        "tacaw_ingest_frames": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(P),
                                          C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "tacaw_commit_frames": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int64]),
        "tacaw_ingest_frames_tiled": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(P),
                                                C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                                C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
        "tacaw_synth_frames": (C.c_int, [C.POINTER(SynthDesc), P, C.c_int32, C.c_int32, C.c_int64,
                                         C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32, P]),
        "tacaw_reset": (C.c_int, [P]),
        "tacaw_plan_export": (C.c_int, [P, P, C.c_int64, C.POINTER(C.c_int64)]),
        "tacaw_plan_import": (C.c_int, [P, P, C.c_int64]),
        "tacaw_state_merge": (C.c_int, [P, P, P, C.c_int64]),
        "tacaw_set_stream": (C.c_int, [P, P]),
        "tacaw_plan_get_info": (C.c_int, [P, C.POINTER(PlanInfo)]),
        "tacaw_destroy": (None, [P]),
        "tacaw_last_error": (C.c_char_p, []),
        "tacaw_version": (C.c_char_p, []),
        "tacaw_read_probe": (C.c_int, [P, C.c_int64, P, P]),
        "tacaw_read_probe_columns": (C.c_int, [P, C.c_int64, C.c_int64, C.c_int32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()
EXPORTED = ("tacaw_plan", "tacaw_plan_check", "tacaw_push_frames", "tacaw_ingest_frames",
            "tacaw_commit_frames", "tacaw_ingest_frames_tiled", "tacaw_finalize",
            "tacaw_detector_spectra", "tacaw_backward", "tacaw_backward_static", "tacaw_reset",
            "tacaw_set_stream", "tacaw_plan_export", "tacaw_plan_import", "tacaw_state_merge",
            "tacaw_plan_get_info", "tacaw_destroy", "tacaw_last_error", "tacaw_version",
            "tacaw_read_probe", "tacaw_read_probe_columns", "tacaw_synth_frames")


def _check(rc):
    if rc != OK:
        raise TacawError(rc, lib.tacaw_last_error().decode())


def make_desc(n_probe, ny, nx, n_frames, seg_len, hop, window="hann", window_param=1.0,
              mean_mode="global", transform="fft", in_dtype="c64", probe_reduce="mean",
              dt_fs=5.0, n_det=0, masks_ptr=0, max_probes_in_flight=0, flags=0,
              temperature_K=0.0, window_values=None, omega_half=0, ring_frames=0,
              k_row_stride=0) -> PlanDesc:
    """window may be a name or an array of seg_len values (custom window).
    omega_half = M > 0 keeps only the 2M + 1 bins of signed index -M..M
    (ascending); axes.omega_half_for converts a frequency or energy limit.
    ring_frames > seg_len selects the deferred streaming mode (see include/tacaw.h);
    k_row_stride > nx reads a ny x nx k-space window of a wider grid in place."""
    wptr = None
    if not isinstance(window, str):
        import numpy as np

        vals = np.ascontiguousarray(np.asarray(window, dtype=np.float64))
        window, window_values = "custom", vals
    if window_values is not None:
        wptr = window_values.ctypes.data
    d = PlanDesc(int(n_probe), int(ny), int(nx), int(n_frames), int(seg_len), int(hop),
                 WINDOWS[window], float(window_param), MEANS[mean_mode],
                 TRANSFORMS[transform], DTYPES[in_dtype], REDUCE[probe_reduce],
                 float(dt_fs), int(n_det), C.c_void_p(masks_ptr or None),
                 int(max_probes_in_flight), int(flags), float(temperature_K), C.c_void_p(wptr),
                 int(ring_frames), int(k_row_stride), int(omega_half))
    d._window_values = window_values  # keep the host array alive with the descriptor
    return d


def merge_states(a: bytes, b: bytes) -> bytes:
    """Union of two exported plan states over disjoint probe sets (host only)."""
    if len(a) != len(b):
        raise TacawError(-2, "states of different sizes")
    out = C.create_string_buffer(len(a))
    _check(lib.tacaw_state_merge(a, b, out, len(a)))
    return out.raw


def check_desc(**kw) -> None:
    """Host-only validation of a plan descriptor (raises TacawError)."""
    d = make_desc(**kw)
    _check(lib.tacaw_plan_check(C.byref(d)))


class _DeviceView:
    """Device memory owned by the plan, exposed through the CUDA array interface."""

    def __init__(self, ptr, shape, strides, typestr):
        self.__cuda_array_interface__ = {"shape": shape, "strides": strides, "typestr": typestr,
                                         "data": (ptr, False), "version": 3}


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream, C.c_void_p(stream.cuda_stream)


class Plan:
    """One spectral reduction: push exit-wave frames, finalize, read spectra.

    masks: optional torch float64 CUDA tensor [n_det, ny, nx] (enables the fused
    per-probe detector spectra). ring_frames > seg_len: deferred streaming ring;
    tiled_ring: store that ring per pixel tile (hop = seg_len / 2; pushes, or a
    producer through ingest_tiled). check_finite: finalize counts NaN and Inf in S
    and D_p and raises TacawError (kind NONFINITE) if there are any; the plan is
    finalized all the same.
    """

    def __init__(self, n_probe, ny, nx, n_frames, seg_len, hop=None, window="hann",
                 window_param=1.0, mean_mode="global", transform="fft", in_dtype="c64",
                 probe_reduce="mean", dt_fs=5.0, masks=None, max_probes_in_flight=0,
                 stream=None, time_kernels=False, temperature_K=0.0, omega_half=0,
                 ring_frames=0, k_row_stride=0, tiled_ring=False, check_finite=False):
        self.handle = None
        hop = seg_len // 2 if hop is None else hop
        self.n_probe, self.ny, self.nx = int(n_probe), int(ny), int(nx)
        self.seg_len, self.hop, self.n_frames = int(seg_len), int(hop), int(n_frames)
        self.in_dtype = in_dtype
        self.tiled_ring = bool(tiled_ring)
        self.tdtype = torch.complex64 if in_dtype == "c64" else torch.complex128
        self.masks = None
        n_det, mptr = 0, 0
        if masks is not None:
            m = masks.detach().to(dtype=torch.float64).contiguous()
            if m.dim() == 2:
                m = m[None]
            if not m.is_cuda or tuple(m.shape[1:]) != (self.ny, self.nx):
                raise ValueError("masks must be a CUDA tensor [n_det, ny, nx]")
            self.masks = m
            n_det, mptr = m.shape[0], m.data_ptr()
        self.n_det = n_det
        self.stream, sptr = _stream_ptr(stream)
        self.desc = make_desc(n_probe, ny, nx, n_frames, seg_len, hop, window, window_param,
                              mean_mode, transform, in_dtype, probe_reduce, dt_fs, n_det, mptr,
                              max_probes_in_flight,
                              (FLAG_TIME_KERNELS if time_kernels else 0)
                              | (FLAG_TILED_RING if tiled_ring else 0)
                              | (FLAG_CHECK_FINITE if check_finite else 0), temperature_K,
                              omega_half=omega_half, ring_frames=ring_frames,
                              k_row_stride=k_row_stride)
        self.row_stride = int(k_row_stride) or self.nx
        h = C.c_void_p()
        _check(lib.tacaw_plan(C.byref(self.desc), sptr, C.byref(h)))
        self.handle = h
        self._keep = []
        self._n_omega = self.info()["n_omega"]

    # ------------------------------------------------------------------
    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib.tacaw_plan_get_info(self.handle, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    @property
    def n_omega(self):
        """Output bins: seg_len, or 2 omega_half + 1 with an energy window."""
        return self._n_omega

    def _frames_args(self, frames):
        if frames.dtype != self.tdtype:
            raise TypeError(f"frames must be {self.tdtype}")
        if not frames.is_cuda:
            raise ValueError("frames must be a CUDA tensor")
        if frames.dim() == 3:
            frames = frames[None]
        if frames.dim() != 4 or tuple(frames.shape[2:]) != (self.ny, self.nx):
            raise ValueError("frames must be [n_probes, n_frames, ny, nx]")
        if frames.stride(3) != 1 or frames.stride(2) != self.row_stride:
            raise ValueError("pixel rows must be contiguous and k_row_stride apart")
        return frames, frames.stride(0), frames.stride(1)

    def push(self, frames: torch.Tensor, probe0: int = 0):
        """Push frames [n_probes, n, ny, nx] for probes probe0.. (next n frames)."""
        frames, ps, fs = self._frames_args(frames)
        if frames.shape[1] == 0:
            return
        _check(lib.tacaw_push_frames(self.handle, C.c_void_p(frames.data_ptr()), int(probe0),
                                     int(frames.shape[0]), int(frames.shape[1]), int(ps), int(fs)))
        if self.stream != torch.cuda.current_stream():
            frames.record_stream(self.stream)

    def ingest(self, n_frames: int, probe0: int = 0, n_probes: int = 1) -> torch.Tensor:
        """Zero-copy ingest: a [n_probes, n_frames, ny, nx] CUDA tensor that aliases the
        plan's ring; write the next frames into it on the plan's stream, then commit()."""
        ptr, ps, fs = C.c_void_p(), C.c_int64(), C.c_int64()
        _check(lib.tacaw_ingest_frames(self.handle, int(probe0), int(n_probes), int(n_frames),
                                       C.byref(ptr), C.byref(ps), C.byref(fs)))
        esz = 8 if self.in_dtype == "c64" else 16
        view = _DeviceView(ptr.value, (int(n_probes), int(n_frames), self.ny, self.nx),
                           (ps.value * esz, fs.value * esz, self.nx * esz, esz),
                           "<c8" if self.in_dtype == "c64" else "<c16")
        self._ingest = (int(probe0), int(n_probes), int(n_frames))
        return torch.as_tensor(view, device="cuda")

    def ingest_tiled(self, n_frames: int, probe0: int = 0, n_probes: int = 1) -> dict:
        """Zero-copy ingest into a tiled ring: the layout (pointer and strides in
        elements) a producer writes the next frames to, then commit()."""
        ptr, ps, fs, ts, tp = C.c_void_p(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib.tacaw_ingest_frames_tiled(self.handle, int(probe0), int(n_probes), int(n_frames),
                                             C.byref(ptr), C.byref(ps), C.byref(fs), C.byref(ts),
                                             C.byref(tp)))
        self._ingest = (int(probe0), int(n_probes), int(n_frames))
        return {"ptr": ptr.value, "probe_stride": ps.value, "frame_stride": fs.value,
                "tile_stride": ts.value, "tile_pixels": tp.value}

    def commit(self):
        """Mark the frames of the last ingest() as written."""
        p0, n, nf = self._ingest
        _check(lib.tacaw_commit_frames(self.handle, p0, n, nf))
        self._ingest = None

    def finalize(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.n_omega, self.ny, self.nx), dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != self.n_omega * self.ny * self.nx:
            raise ValueError("out must be a contiguous float64 [n_omega, ny, nx] tensor")
        rc = lib.tacaw_finalize(self.handle, C.c_void_p(out.data_ptr()))
        if rc == -7:  # NONFINITE: finalized all the same; the spectrum rides on the error
            err = TacawError(rc, lib.tacaw_last_error().decode())
            err.result = out
            raise err
        _check(rc)
        return out

    def detector_spectra(self, masks=None, per_probe=False, out=None, out_p=None):
        """D [n_det, n_omega] (and per-probe [n_det, n_probe, n_omega] if per_probe)."""
        if masks is not None:
            m = masks.to(dtype=torch.float64).contiguous()
            if m.dim() == 2:
                m = m[None]
            n_det, mptr = m.shape[0], C.c_void_p(m.data_ptr())
            self._keep = [m]
        else:
            n_det, mptr = self.n_det, C.c_void_p(None)
        D = out if out is not None else torch.empty((n_det, self.n_omega), dtype=torch.float64, device="cuda")
        Dp = None
        if per_probe:
            Dp = out_p if out_p is not None else torch.empty((self.n_det, self.n_probe, self.n_omega),
                                                             dtype=torch.float64, device="cuda")
        _check(lib.tacaw_detector_spectra(self.handle, mptr, int(n_det), C.c_void_p(D.data_ptr()),
                                          C.c_void_p(Dp.data_ptr() if Dp is not None else None)))
        return (D, Dp) if per_probe else D

    def backward(self, frames, probe0=0, gS=None, gD=None, gDp=None, grad=None, grad_wparam=None,
                 static_scratch=False):
        """Adjoint: returns (grad_frames, dLoss/dwindow_param tensor of shape [1]).
        static_scratch: call tacaw_backward_static (the library's fixed scratch, no
        device allocation in the call)."""
        frames, ps, fs = self._frames_args(frames)
        if frames.shape[1] < self.info()["frames_used"]:
            raise ValueError("backward needs every frame that enters a chunk (frames_used)")
        if grad is None:
            # the adjoint writes every frame that enters a chunk; only the rest is zeroed
            grad = torch.empty_strided(frames.shape, frames.stride(), dtype=frames.dtype,
                                       device=frames.device)
            grad[:, self.info()["frames_used"]:].zero_()
        if grad.stride() != frames.stride():
            raise ValueError("grad must have the strides of frames")
        if grad_wparam is None:
            grad_wparam = torch.zeros(1, dtype=torch.float64, device="cuda")

        def ptr(t):
            return C.c_void_p(t.data_ptr() if t is not None else None)

        ins = [None if t is None else t.to(torch.float64).contiguous() for t in (gS, gD, gDp)]
        fn = lib.tacaw_backward_static if static_scratch else lib.tacaw_backward
        _check(fn(self.handle, C.c_void_p(frames.data_ptr()), int(probe0), int(frames.shape[0]),
                  int(ps), int(fs), ptr(ins[0]), ptr(ins[1]), ptr(ins[2]),
                  C.c_void_p(grad.data_ptr()), ptr(grad_wparam)))
        self._keep = ins
        return grad, grad_wparam

    def reset(self):
        _check(lib.tacaw_reset(self.handle))

    def export_state(self) -> bytes:
        """The accumulator state at a probe boundary (every probe untouched or
        complete), as bytes that import_state of a plan with the same descriptor
        and masks takes to continue the run."""
        n = C.c_int64(0)
        _check(lib.tacaw_plan_export(self.handle, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib.tacaw_plan_export(self.handle, buf, n.value, C.byref(n)))
        return buf.raw

    def import_state(self, state: bytes):
        """Load a state from export_state into this plan (no frames pushed since
        its creation or last reset)."""
        _check(lib.tacaw_plan_import(self.handle, state, len(state)))

    def set_stream(self, stream):
        self.stream, sptr = _stream_ptr(stream)
        _check(lib.tacaw_set_stream(self.handle, sptr))

    def close(self):
        if self.handle is not None:
            lib.tacaw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def spectra(frames, seg_len, hop=None, masks=None, per_probe=False, **kw):
    """One-shot: S [n_omega, ny, nx] and (if masks) D / per-probe D for a whole series."""
    if frames.dim() == 3:
        frames = frames[None]
    P, NT, ny, nx = frames.shape
    in_dtype = "c64" if frames.dtype == torch.complex64 else "c128"
    with Plan(P, ny, nx, NT, seg_len, hop, in_dtype=in_dtype, masks=masks, **kw) as plan:
        plan.push(frames)
        S = plan.finalize()
        if masks is None:
            return S
        D = plan.detector_spectra(per_probe=per_probe)
        torch.cuda.current_stream().synchronize()
        return (S, *D) if per_probe else (S, D)


def read_probe(buf: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Read every byte of a contiguous CUDA tensor once (the HBM read-ceiling probe);
    returns a 1-element int64 CUDA tensor with the wrapping sum of its 64-bit words."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("read_probe needs a contiguous CUDA tensor")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=buf.device)
    s, sptr = _stream_ptr(stream)
    _check(lib.tacaw_read_probe(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(), sptr,
                                C.c_void_p(out.data_ptr())))
    return out


def read_probe_columns(buf: torch.Tensor, rows: int, seg_bytes: int = 128,
                       out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Read a contiguous CUDA tensor, seen as `rows` equal rows (frames), once in the
    chunk transform's access pattern (columns seg_bytes wide across the rows);
    returns the wrapping 64-bit word sum."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("read_probe_columns needs a contiguous CUDA tensor")
    nbytes = buf.numel() * buf.element_size()
    if rows < 1 or nbytes % rows != 0:
        raise ValueError("rows must divide the tensor's bytes")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=buf.device)
    row_bytes = nbytes // rows
    s, sptr = _stream_ptr(stream)
    _check(lib.tacaw_read_probe_columns(C.c_void_p(buf.data_ptr()), rows, row_bytes, int(seg_bytes),
                                        sptr, C.c_void_p(out.data_ptr())))
    return out


class Producer:
    """The library's fused producer (tacaw_synth_frames): synthetic complex64 exit
    waves from Philox4x32-10 counters. spec carries the model parameters (a
    tacaw_synth.philox.ProducerSpec or anything with the same fields); tables are
    CUDA tensors cos, sin (2^20, float32), normal (2^16, float32), tan (2^16,
    float64)."""

    def __init__(self, spec, tables: dict, stream=None):
        self.spec = spec
        self.tables = {k: v.contiguous() for k, v in tables.items()}
        self.stream, self._sptr = _stream_ptr(stream)
        t = self.tables
        e = complex(spec.elastic)
        self.desc = SynthDesc(int(spec.ny), int(spec.nx), int(spec.n_terms), int(spec.n_lines),
                              int(spec.seed) & 0xFFFFFFFF, 0, float(spec.amplitude),
                              float(spec.noise_sigma), e.real, e.imag, float(spec.e_lo_mev),
                              float(spec.e_hi_mev), float(spec.line_lo_mev), float(spec.line_hi_mev),
                              float(spec.hwhm_lo_mev), float(spec.hwhm_hi_mev), float(spec.dt_fs),
                              t["cos"].data_ptr(), t["sin"].data_ptr(), t["normal"].data_ptr(),
                              t["tan"].data_ptr())

    def write(self, ptr: int, probe0: int, n_probes: int, frame0: int, n_frames: int,
              probe_stride: int, frame_stride: int, tile_stride: int = 0, tile_pixels: int = 0):
        """Frames [frame0, frame0 + n_frames) of probes probe0.. into device memory at ptr
        (strides in complex64 elements; tile_pixels 0 = plain frames)."""
        tp = int(tile_pixels) if tile_pixels else int(self.spec.ny * self.spec.nx)
        _check(lib.tacaw_synth_frames(C.byref(self.desc), C.c_void_p(ptr), int(probe0), int(n_probes),
                                      int(frame0), int(n_frames), int(probe_stride), int(frame_stride),
                                      int(tile_stride), tp, self._sptr))

    def into(self, dst: torch.Tensor, probe0: int = 0, frame0: int = 0):
        """Fill a complex64 CUDA tensor [n_probes, n_frames, ny, nx] (contiguous frames)."""
        if dst.dtype != torch.complex64 or not dst.is_cuda or dst.stride(3) != 1 \
                or dst.stride(2) != dst.shape[3]:
            raise ValueError("dst must be a complex64 CUDA tensor with contiguous frames")
        self.write(dst.data_ptr(), probe0, dst.shape[0], frame0, dst.shape[1], dst.stride(0),
                   dst.stride(1))
        return dst

    def into_ring(self, plan: "Plan", n_frames: int, probe0: int, n_probes: int, frame0: int):
        """Zero-copy: write the next n_frames frames straight into the plan's (tiled or
        per-frame) ring and commit them."""
        if plan.tiled_ring:
            lay = plan.ingest_tiled(n_frames, probe0, n_probes)
            self.write(lay["ptr"], probe0, n_probes, frame0, n_frames, lay["probe_stride"],
                       lay["frame_stride"], lay["tile_stride"], lay["tile_pixels"])
        else:
            view = plan.ingest(n_frames, probe0, n_probes)
            self.write(view.data_ptr(), probe0, n_probes, frame0, n_frames, view.stride(0),
                       view.stride(1))
        plan.commit()
