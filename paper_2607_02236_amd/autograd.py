"""torch.autograd.Function around the spectral reduction and its hand-written adjoint.

Forward: the HIP forward path (push, finalize, detector spectra). Backward: the
HIP adjoint (tacaw_backward), which recomputes every chunk transform instead of
storing spectra. Gradients follow torch's convention for complex inputs
(d/dRe + i d/dIm of a real loss).
"""

from __future__ import annotations

import torch

from . import tacaw


class TacawSpectra(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frames, window_param, masks, seg_len, hop, window, mean_mode, probe_reduce,
                omega_half, temperature_K, dt_fs):
        if frames.dim() == 3:
            frames = frames[None]
        P, NT, ny, nx = frames.shape
        in_dtype = "c64" if frames.dtype == torch.complex64 else "c128"
        plan = tacaw.Plan(P, ny, nx, NT, seg_len, hop, window=window,
                          window_param=float(window_param), mean_mode=mean_mode,
                          in_dtype=in_dtype, probe_reduce=probe_reduce, masks=masks,
                          omega_half=omega_half, temperature_K=temperature_K, dt_fs=dt_fs)
        plan.push(frames.detach())
        S = plan.finalize()
        if masks is not None:
            D, Dp = plan.detector_spectra(per_probe=True)
        else:
            D = Dp = torch.zeros(0, dtype=torch.float64, device=frames.device)
        ctx.plan = plan
        ctx.has_masks = masks is not None
        ctx.save_for_backward(frames)
        return S, D, Dp

    @staticmethod
    def backward(ctx, gS, gD, gDp):
        (frames,) = ctx.saved_tensors
        if frames.dim() == 3:
            frames = frames[None]
        # the plan stays open while the graph holds ctx (a second backward with
        # retain_graph=True reuses it); it is closed when ctx is freed
        grad, gw = ctx.plan.backward(frames.detach().contiguous(), gS=gS,
                                     gD=gD if ctx.has_masks else None,
                                     gDp=gDp if ctx.has_masks else None)
        return grad, gw.reshape(()), None, None, None, None, None, None, None, None, None


def spectra(frames, seg_len, hop=None, masks=None, window="hann", window_param=1.0,
            mean_mode="global", probe_reduce="mean", omega_half=0, temperature_K=0.0,
            dt_fs=5.0):
    """Differentiable (S, D, D_p); window_param may be a float64 tensor with requires_grad.
    omega_half and temperature_K as in tacaw.Plan (energy window, quantum factor)."""
    hop = seg_len // 2 if hop is None else hop
    if not torch.is_tensor(window_param):
        window_param = torch.tensor(float(window_param), dtype=torch.float64, device=frames.device)
    if masks is not None:
        masks = masks.to(device=frames.device, dtype=torch.float64)
    return TacawSpectra.apply(frames, window_param, masks, seg_len, hop, window, mean_mode,
                              probe_reduce, int(omega_half), float(temperature_K), float(dt_fs))
