"""Benchmark of the TACAW spectral hot path on one MI355X.

One step = one pass of the whole path over one batch: reset the plan, push the
whole exit-wave series (ingest, reference subtraction, Hann window, time FFT,
|X|^2, FP64 accumulation, per-probe detector partials), finalize (exact mean
correction, normalisation) and the detector spectra. The input series is
resident in HBM before timing starts (generated on the GPU by the seeded
generator; it is not part of the timed region).

Workload (default): 64 probes (8 x 8 scan) x 2048 frames at 5 fs x 256 x 256
pixels, complex64 (68.7 GB of exit waves); Welch chunks of L = 512 with 50 %
overlap, periodic Hann; 4 detector masks. Metric: exit-wave GB/s (unique
exit-wave bytes / step time).

Workload "gradient": 16 probes x 1024 frames x 128 x 128 complex64, L = H =
512, width-r Hann at r = 1, 4 masks; one step is the forward pass above plus
the adjoint (dL/dpsi and dL/dr for L = sum_j sum_m a_j(m) D_j(m)).

Prints ONE JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak for the instructions the kernels issue: non-packed FMA on 256 CUs x 64 lanes
# x 2 flops x 2.4 GHz (the chip's packed-FP32 figure, 157.3 TFLOP/s, needs packed instructions,
# which this build disables)
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3  # published FP32 vector peak of MI355X (packed)


def fft_flops_per_element(L, H):
    """Algorithmic flops per input element of the chunk kernel: each element is in L/H
    chunks; per chunk and point 5 log2 L for the complex FFT (the radix-2 count), 2 for
    the reference subtraction, 2 for the window, 3 for |X|^2 and 1 for the accumulation."""
    import math

    return (L / H) * (5.0 * math.log2(L) + 8.0)
# sources of the chunk kernel and of the adjoint (a counter summary is valid only for these bytes)
KERNEL_SOURCES = ["seg_fft_kernel.h", "regfft.h", "buffer_io.h", "tacaw_internal.h", "tacaw_fft.hip"]
ADJOINT_SOURCES = ["tacaw_adjoint.hip", "regfft.h", "buffer_io.h", "tacaw_internal.h"]
METRIC = "exit-wave GB/s -> S(k,omega) (frac. HBM peak); FFT vs MFMA DFT-GEMM at fixed err"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(paths):
    """sha256[:16] of the concatenated kernel sources (a path or a list of paths)."""
    h = hashlib.sha256()
    for path in [paths] if isinstance(paths, str) else paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_src, config, name="seg_fft_L512_64probes_counters.json"):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source and on this run's workload; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != source_sha(kernel_src) or d.get("config") != config:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(spec, L, H, n_pix, seed=0, gradient=False, mean_mode="global", twin=False):
    """The FP64 oracle (brute-force DFT) on all probes and frames of a seeded
    subset of pixels (with gradient: the forward and its vector-Jacobian product
    for the detector loss); returns exit-wave GB/s in the metric's unit. twin: the
    series comes from the fused producer's CPU twin (not part of the timing)."""
    import numpy as np
    import torch

    import oracle as O
    import tacaw_synth as T

    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(spec.n_k, size=n_pix, replace=False))
    if twin:
        psi = T.philox.generate(spec, pixels=pix)
    else:
        psi = T.generate(spec, pixels=pix).numpy()
    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    w = O.window("hann_width" if gradient else "hann", L, 1.0)
    t0 = time.perf_counter()
    O.tacaw_spectra(psi, L, H, w, mean_mode)
    if gradient:
        masks = T.standard_masks(spec.ny, spec.nx, scale=spec.ny / 256).reshape(4, -1)[:, pix]
        gS = np.einsum("jm,jk->mk", T.loss_weights(4, L, seed=4), masks)
        O.spectra_vjp(psi, L, H, w, gS, dw=O.window_width_derivative(L, 1.0))
    dt = time.perf_counter() - t0
    nbytes = psi.shape[0] * psi.shape[1] * n_pix * 8
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": int(cores), "kind": "oracle",
            "sample": ("forward + adjoint of the " if gradient else "")
                      + f"brute-force FP64 DFT oracle on all {psi.shape[0]} probes x "
                      f"{psi.shape[1]} frames of {n_pix} seeded pixels ({dt:.1f} s)"}


def compare_forms(psi, spec, L, H, masks, stream, e_max_mev=100.0, steps=3):
    """FFT vs DFT-GEMM on the same resident series at one energy window: each form's
    chunk-kernel time (HIP events, mean of `steps` after one warm-up) and the GEMM
    forms' executed MFMA rate, with the relative L2 difference of their S from the
    FFT form's S (whose own error against the FP64 oracle the parity tests bound at
    about 1e-7, so the difference is the GEMM form's error at that accuracy)."""
    import numpy as np
    import torch

    from paper_2607_02236_amd import axes, tacaw

    M = axes.omega_half_for(L, 5.0, e_max_mev=e_max_mev)
    res, S_ref = {}, None
    for form in ("fft", "gemm_bf16x3", "gemm_f16x3"):
        plan = tacaw.Plan(spec.n_probe, spec.ny, spec.nx, spec.n_frames, L, H, masks=masks,
                          transform=form, in_dtype=spec.dtype, time_kernels=True, stream=stream,
                          dt_fs=5.0, omega_half=M)
        S = torch.empty((plan.n_omega, spec.ny, spec.nx), dtype=torch.float64, device="cuda")
        k_ms = []
        for i in range(steps + 1):
            plan.reset()
            plan.push(psi)
            plan.finalize(S)
            if i:
                k_ms.append(plan.info()["last_chunk_kernel_ms"])
        torch.cuda.synchronize()
        t = float(np.mean(k_ms))
        r = {"kernel_ms": round(t, 4), "exit_wave_gbs": round(spec.nbytes / (t * 1e-3) / 1e9, 1)}
        if form == "fft":
            S_ref = S
        else:
            m_rows = (2 * plan.n_omega + 31) // 32 * 32
            flops = 3 * 2 * m_rows * 2 * L * plan.info()["n_segments"] * spec.n_probe * spec.n_k
            tf = flops / (t * 1e-3) / 1e12
            r.update(mfma_tflops=round(tf, 1), mfma_frac=round(tf / 2500.0, 4),
                     rel_diff_vs_fft=float(torch.linalg.vector_norm(S - S_ref)
                                           / torch.linalg.vector_norm(S_ref)))
            r["speed_vs_fft"] = round(res["fft"]["kernel_ms"] / t, 3)
        res[form] = r
        log(f"form comparison: {form} {t:.3f} ms")
        plan.close()
    res.update(energy_window_mev=e_max_mev, n_omega=2 * M + 1,
               note="same resident series, energy window |E| <= 100 meV (the DFT-GEMM forms "
                    "compute only its rows); chunk-kernel times by HIP events; MFMA flops are "
                    "the executed 3 split products")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--probes", type=int, default=64)
    ap.add_argument("--frames", type=int, default=2048)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--seg-len", type=int, default=512)
    ap.add_argument("--form", default="fft", choices=["fft", "gemm_bf16x3", "gemm_f16x3"])
    ap.add_argument("--workload", default="realistic",
                    choices=["realistic", "precision", "streaming", "gradient"],
                    help="realistic: 64 probes x 2048 frames x 256^2 c64 (default); precision: "
                         "1 probe x 512 frames x 64^2 c128, one chunk of 512; streaming: "
                         "--probes (default 16) x 4096 frames x 1024^2 c64, L=1024 H=512, "
                         "pushed in pieces of --push-frames frames through the plan's ring; "
                         "gradient: 16 probes x 1024 frames x 128^2 c64, L=H=512, forward + "
                         "adjoint")
    ap.add_argument("--hop", type=int, default=0,
                    help="chunk hop of the realistic workload (default seg_len / 2)")
    ap.add_argument("--mean-mode", default="global", choices=["global", "per_segment", "none"],
                    help="elastic-mean handling (per_segment: each chunk's own mean)")
    ap.add_argument("--push-frames", type=int, default=256)
    ap.add_argument("--ring-frames", type=int, default=0,
                    help="streaming: deferred ring depth per probe (0: chunks run in the push "
                         "that completes them)")
    ap.add_argument("--ring-layout", default="tiled", choices=["tiled", "frame"],
                    help="streaming with --ring-frames: store the ring per pixel tile (default) "
                         "or per frame")
    ap.add_argument("--resident-frames", type=int, default=512,
                    help="streaming: frames held in HBM per probe; pushes cycle through them "
                         "(4096 = the whole series)")
    ap.add_argument("--roi-mev", type=float, default=0.0,
                    help="keep only the energy window |E| <= this (0: all bins); the DFT-GEMM "
                         "form then computes only the window's rows")
    ap.add_argument("--producer", action="store_true",
                    help="streaming: the fused producer writes every frame straight into the "
                         "plan's tiled ring (zero-copy ingest) instead of pushes from resident "
                         "frames; probes default to 256 (the 16 x 16 scan)")
    ap.add_argument("--batch", type=int, default=8,
                    help="streaming with --producer: probes in flight (ring slots)")
    ap.add_argument("--cpu-pixels", type=int, default=0,
                    help="pixels of the oracle's sample (default 4096; 16 with --producer)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-form-compare", action="store_true",
                    help="skip the FFT vs DFT-GEMM comparison of the default workload")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of probes is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import tacaw_synth as T
    from paper_2607_02236_amd import tacaw

    torch.cuda.set_device(0)
    if args.workload == "precision":
        L, H = 512, 512
        spec = T.config_precision(n_frames=512)
    elif args.workload == "gradient":
        L, H = 512, 512
        spec = T.config_gradient()
    elif args.workload == "streaming" and args.producer:
        L, H = 1024, 512
        n_pr = args.probes if args.probes != 64 else 256
        spec = T.philox.ProducerSpec(n_pr, 4096, 1024, 1024, seed=5)
    elif args.workload == "streaming":
        L, H = 1024, 512
        n_pr = args.probes if args.probes != 64 else 16
        spec = T.config_streaming(n_probe=n_pr, n_frames=4096, ny=1024, nx=1024)
    else:
        L, H = args.seg_len, (args.hop or args.seg_len // 2)
        spec = T.config_realistic(n_probe=args.probes, n_frames=args.frames, ny=args.grid,
                                  nx=args.grid)
    streaming = args.workload == "streaming"
    producer = streaming and args.producer
    if producer:
        return bench_producer(args, spec, L, H)
    resident = spec
    if streaming:
        R = min(args.resident_frames, spec.n_frames)
        if R % args.push_frames or spec.n_frames % args.push_frames:
            sys.exit("--resident-frames and 4096 must be multiples of --push-frames")
        resident = T.config_streaming(n_probe=spec.n_probe, n_frames=R, ny=spec.ny, nx=spec.nx)
    log(f"allocating {resident.nbytes / 1e9:.1f} GB of exit waves on the GPU")
    psi = torch.empty((resident.n_probe, resident.n_frames, spec.ny, spec.nx),
                      dtype=spec.torch_dtype, device="cuda")
    spec_gen, spec = spec, resident  # generate the resident frames
    t0 = time.time()
    for p in range(spec.n_probe):
        T.generate_into(spec, psi[p:p + 1], probes=[p], frame_chunk=256)
        if p % 8 == 7:
            torch.cuda.synchronize()
            log(f"generated probe {p + 1}/{spec.n_probe} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    spec = spec_gen
    if args.copy_probe_gib > 0:
        n = int(args.copy_probe_gib * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read and written per copy")
        del src, dst
    gradient = args.workload == "gradient"
    masks = torch.from_numpy(T.standard_masks(spec.ny, spec.nx, scale=spec.ny / 256)).cuda()
    if args.workload == "precision":
        masks = torch.from_numpy(np.stack([T.disk_mask(64, 64, 24, inner=8),
                                           T.standard_masks(64, 64, 0.25)[0]])).cuda()
    stream = torch.cuda.current_stream()
    from paper_2607_02236_amd import axes

    dt_fs = 5.0
    M = axes.omega_half_for(L, dt_fs, e_max_mev=args.roi_mev) if args.roi_mev > 0 else 0
    win = dict(window="hann_width", window_param=1.0) if gradient else {}
    plan = tacaw.Plan(spec.n_probe, spec.ny, spec.nx, spec.n_frames, L, H, masks=masks,
                      transform=args.form, in_dtype=spec.dtype, time_kernels=True, stream=stream,
                      dt_fs=dt_fs, omega_half=M, ring_frames=args.ring_frames if streaming else 0,
                      tiled_ring=streaming and args.ring_frames > 0 and args.ring_layout == "tiled",
                      mean_mode=args.mean_mode, **win)
    R = psi.shape[1]
    pieces = [(f0, min(spec.n_frames, f0 + args.push_frames))
              for f0 in range(0, spec.n_frames, args.push_frames)] if streaming else [(0, spec.n_frames)]
    n_om = plan.n_omega
    S = torch.empty((n_om, spec.ny, spec.nx), dtype=torch.float64, device="cuda")
    D = torch.empty((masks.shape[0], n_om), dtype=torch.float64, device="cuda")
    Dp = torch.empty((masks.shape[0], spec.n_probe, n_om), dtype=torch.float64, device="cuda")
    if gradient:  # loss sum_j sum_m a_j(m) D_j(m): dLoss/dD = a
        gD = torch.from_numpy(T.loss_weights(masks.shape[0], n_om, seed=4)).cuda()
        grad = torch.empty_like(psi)
        gw = torch.zeros(1, dtype=torch.float64, device="cuda")
    bwd_ms = []
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)

    def step(measure=False):
        plan.reset()
        k_ms = 0.0
        for f0, f1 in pieces:
            plan.push(psi[:, f0 % R:f0 % R + (f1 - f0)])
            if streaming and measure:  # sum the chunk-kernel durations of the pushes
                t = plan.info()["last_chunk_kernel_ms"]
                k_ms += t if t > 0 else 0.0  # -1: this push completed no chunk
        plan.finalize(S)
        plan.detector_spectra(per_probe=True, out=D, out_p=Dp)
        if gradient:
            gw.zero_()
            b0.record(stream)
            plan.backward(psi, gD=gD, grad=grad, grad_wparam=gw)
            b1.record(stream)
        return k_ms

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")
    kernel_ms = []
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step()
        if not streaming:  # waits for this step's chunk kernel
            kernel_ms.append(plan.info()["last_chunk_kernel_ms"])
        if gradient:  # the adjoint's kernels (the plan's stream is this stream)
            b1.synchronize()
            bwd_ms.append(b0.elapsed_time(b1))
    e1.record(stream)
    torch.cuda.synchronize()
    if streaming:  # one more (untimed) step that reads the kernel time after every push
        kernel_ms.append(step(measure=True))
        torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step; chunk kernel {np.mean(kernel_ms):.3f} ms")

    # measured HBM read ceiling: the read probe over the resident input (untimed region)
    ceil_ms = []
    for _ in range(5):
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        tacaw.read_probe(psi, stream=stream)
        c1.record(stream)
        c1.synchronize()
        ceil_ms.append(c0.elapsed_time(c1))
    read_ceiling = psi.numel() * psi.element_size() / (float(np.median(ceil_ms)) * 1e-3) / 1e9
    log(f"read probe over {psi.numel() * psi.element_size() / 1e9:.1f} GB: {read_ceiling:.0f} GB/s")
    # the same bytes in the chunk transform's pattern: tile-wide columns across frames
    seg = plan.info()["tile_pixels"] * psi.element_size()
    col_ms = []
    row_bytes = spec.n_k * psi.element_size()
    if seg in (64, 128, 256, 512) and row_bytes % seg == 0 and row_bytes // seg <= 65535:
        for _ in range(3):
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            tacaw.read_probe_columns(psi, psi.shape[0] * psi.shape[1], seg, stream=stream)
            c1.record(stream)
            c1.synchronize()
            col_ms.append(c0.elapsed_time(c1))
    col_ceiling = (psi.numel() * psi.element_size() / (float(np.median(col_ms)) * 1e-3) / 1e9
                   if col_ms else None)
    if col_ceiling:
        log(f"column read probe ({seg}-byte tiles): {col_ceiling:.0f} GB/s")

    b_alg = spec.nbytes  # each unique exit-wave value once
    value = b_alg / (ms * 1e-3) / 1e9
    k_ms = float(np.mean(kernel_ms))
    achieved = b_alg / (k_ms * 1e-3) / 1e9
    n_elem = spec.n_probe * spec.n_frames * spec.n_k
    alu_tf = n_elem * fft_flops_per_element(L, H) / (k_ms * 1e-3) / 1e12
    n_seg = plan.info()["n_segments"]
    m_rows = (2 * n_om + 31) // 32 * 32  # GEMM rows computed (window rows, padded to 32)
    gemm_flops = 3 * 2 * m_rows * 2 * L * n_seg * spec.n_probe * spec.n_k  # executed, 3 products
    csrc = os.path.join(ROOT, "paper_2607_02236_amd", "csrc")
    # what the committed counter summaries must have measured for their traffic to apply
    run_cfg = dict(probes=spec.n_probe, frames=spec.n_frames, ny=spec.ny, nx=spec.nx, seg_len=L,
                   hop=H, dtype=spec.dtype, form=args.form, mean_mode=args.mean_mode,
                   streaming=bool(streaming), gradient=bool(gradient), omega_half=int(M))
    ksrc = [os.path.join(csrc, f) for f in KERNEL_SOURCES] \
        if args.form == "fft" else [os.path.join(csrc, "tacaw_gemm.hip")]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator: elastic 1 + 8 Lorentzian-line tones of 1e-3/sqrt(8) per pixel + 1e-5 noise)"
                + (f"; frames repeat with period {R} (resident block)" if R < spec.n_frames else ""),
        "config": {
            "workload": f"{spec.n_probe} probes x {spec.n_frames} frames x {spec.ny}x{spec.nx} {spec.dtype}, "
                        f"Welch L={L} H={H} " + ("width-r Hann r=1" if gradient else "periodic Hann")
                        + f", {args.mean_mode.replace('_', '-')} mean, {masks.shape[0]} detector masks, "
                          f"transform {args.form}"
                        + (", forward + adjoint (dL/dpsi and dL/dr of sum_j a_j . D_j)" if gradient else "")
                        + (f", pushed in pieces of {args.push_frames} frames" if streaming else "")
                        + (f", deferred ring of {args.ring_frames} frames ({args.ring_layout} layout)"
                           if streaming and args.ring_frames else "")
                        + (f", energy window |E| <= {args.roi_mev:g} meV ({n_om} bins)" if M else ""),
            "probes": spec.n_probe, "frames": spec.n_frames, "ny": spec.ny, "nx": spec.nx,
            "seg_len": L, "hop": H, "n_omega": n_om, "exit_wave_bytes": b_alg,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "seg_fft_kernel",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(ksrc, run_cfg),
            "kernel_ms": round(k_ms, 4),
            "algorithmic_bytes_per_launch": b_alg,
            "note": "achieved = algorithmic bytes of one launch (every exit-wave value once: "
                    "probes x frames x pixels x 8 B) / the chunk kernel's average launch time "
                    "(HIP events on the plan's stream); traffic = HBM bytes per launch from "
                    "rocprofv3 FETCH_SIZE/WRITE_SIZE (null unless taken on these kernel sources "
                    "and this workload)",
            "flops": {
                "per_element": round(fft_flops_per_element(L, H), 2),
                "achieved_tflops": round(alu_tf, 2),
                "frac_of_fp32_157_3": round(alu_tf / FP32_PEAK_TFLOPS, 4),
                "frac_of_fp32_nonpacked_78_6": round(alu_tf / VALU_PEAK_TFLOPS, 4),
                "note": "algorithmic flops (per_element x elements) / kernel time, against the "
                        "published 157.3 TFLOP/s FP32 peak (packed instructions) and the "
                        "78.6 TFLOP/s the non-packed FMAs this build issues can reach "
                        "(256 CU x 64 lanes x 2 flops x 2.4 GHz)",
            },
        },
    }
    if gradient:
        t_b = float(np.mean(bwd_ms))
        ach_b = 2 * b_alg / (t_b * 1e-3) / 1e9
        out["roofline"] = {
            "bound": "hbm", "kernel": "bwd_kernel", "achieved": round(ach_b, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach_b / HBM_PEAK_GBS, 4),
            "kernel_ms": round(t_b, 4),
            "traffic": traffic_from_profiles([os.path.join(csrc, f) for f in ADJOINT_SOURCES], run_cfg,
                                             "bwd_kernel_L512_16probes_counters.json"),
            "forward_chunk_kernel_ms": round(k_ms, 4),
            "note": "adjoint launch (bwd_kernel and the window-parameter reduction): reads "
                    "psi once and writes dL/dpsi once (2 x exit-wave bytes). HBM is its nearest "
                    "roofline; it recomputes each chunk's transform and runs a second one, whose "
                    "VALU issue and latency keep it below",
        }
    if args.form != "fft":
        tf = gemm_flops / (k_ms * 1e-3) / 1e12
        out["dtype"] = "f16x3" if args.form == "gemm_f16x3" else "bf16x3"
        out["roofline"] = {
            "bound": "mfma", "kernel": "seg_gemm_kernel", "achieved": round(tf, 2),
            "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4),
            "kernel_ms": round(k_ms, 4), "traffic": None,
            "note": "executed MFMA flops (3 split products of the real GEMM with "
                    f"{m_rows} rows x {2 * L} per chunk); useful flops are one third",
        }
    out["roofline"]["read_ceiling_gbs"] = round(read_ceiling, 1)
    out["roofline"]["value_frac_of_read_ceiling"] = round(value / read_ceiling, 4)
    if col_ceiling and args.form == "fft" and not gradient:
        # the chunk kernel's loads alone, in its own tile pattern: its HBM rate against that
        out["roofline"]["tile_pattern_read_ceiling_gbs"] = round(col_ceiling, 1)
        out["roofline"]["kernel_frac_of_tile_pattern_ceiling"] = round(achieved / col_ceiling, 4)
    if (args.form == "fft" and not streaming and not gradient and args.mean_mode == "global"
            and args.workload == "realistic" and not args.no_form_compare):
        plan.close()
        out["form_comparison"] = compare_forms(psi, spec, L, H, masks, stream)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        del psi
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(spec, L, H,
                                           (args.cpu_pixels or 4096) if not gradient else 8192,
                                           gradient=gradient, mean_mode=args.mean_mode)
    plan.close()
    print(json.dumps(out), flush=True)


def bench_producer(args, spec, L, H):
    """The large streaming workload fed by the fused producer: every frame is written
    by tacaw_synth_frames straight into the plan's tiled ring (zero-copy ingest) and
    reduced from there; the series never exists whole. One step = reset, all probes
    in batches of args.batch through 256-frame ingests, finalize, detector spectra."""
    import numpy as np
    import torch

    import tacaw_synth as T
    from paper_2607_02236_amd import tacaw

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    P, NT, piece, batch = spec.n_probe, spec.n_frames, args.push_frames, args.batch
    if P % batch or NT % piece:
        sys.exit("--probes must be a multiple of --batch and 4096 of --push-frames")
    ring = args.ring_frames or 2048
    masks = torch.from_numpy(T.standard_masks(spec.ny, spec.nx, scale=spec.ny / 256)).cuda()
    tabs = {k: torch.from_numpy(v).cuda() for k, v in T.philox.tables().items()}
    prod = tacaw.Producer(spec, tabs, stream=stream)
    from paper_2607_02236_amd import axes

    M = axes.omega_half_for(L, spec.dt_fs, e_max_mev=args.roi_mev) if args.roi_mev > 0 else 0
    plan = tacaw.Plan(P, spec.ny, spec.nx, NT, L, H, masks=masks, time_kernels=True, stream=stream,
                      ring_frames=ring, tiled_ring=args.ring_layout == "tiled",
                      max_probes_in_flight=batch, mean_mode=args.mean_mode, transform=args.form,
                      dt_fs=spec.dt_fs, omega_half=M)
    log(f"plan: {P} probes x {NT} frames x {spec.ny}x{spec.nx}, ring of {ring} frames for "
        f"{batch} probes ({plan.info()['device_bytes'] / 1e9:.1f} GB on the device)")
    n_om = plan.n_omega
    S = torch.empty((n_om, spec.ny, spec.nx), dtype=torch.float64, device="cuda")
    D = torch.empty((masks.shape[0], n_om), dtype=torch.float64, device="cuda")
    Dp = torch.empty((masks.shape[0], P, n_om), dtype=torch.float64, device="cuda")

    def step(measure=False):
        plan.reset()
        k_ms = 0.0
        for p0 in range(0, P, batch):
            for f0 in range(0, NT, piece):
                prod.into_ring(plan, piece, p0, batch, f0)
                if measure:
                    t = plan.info()["last_chunk_kernel_ms"]
                    k_ms += t if t > 0 else 0.0
            log(f"  probes {p0}..{p0 + batch - 1} done")
        plan.finalize(S)
        plan.detector_spectra(per_probe=True, out=D, out_p=Dp)
        return k_ms

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step()
        log(f"step {i + 1}/{args.steps} enqueued")
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.1f} ms/step")
    k_ms = step(measure=True)
    torch.cuda.synchronize()
    # the producer alone, into a scratch buffer of one batch's piece (same writes)
    scratch = torch.empty((batch, piece, spec.ny, spec.nx), dtype=torch.complex64, device="cuda")
    p_0 = torch.cuda.Event(enable_timing=True)
    p_1 = torch.cuda.Event(enable_timing=True)
    p_0.record(stream)
    for p0 in range(0, P, batch):
        for f0 in range(0, NT, piece):
            prod.into(scratch, probe0=p0, frame0=f0)
    p_1.record(stream)
    torch.cuda.synchronize()
    prod_ms = p_0.elapsed_time(p_1)
    del scratch
    log(f"chunk kernels {k_ms:.1f} ms, producer alone {prod_ms:.1f} ms per step")
    b_alg = spec.nbytes
    value = b_alg / (ms * 1e-3) / 1e9
    achieved = b_alg / (k_ms * 1e-3) / 1e9
    csrc = os.path.join(ROOT, "paper_2607_02236_amd", "csrc")
    run_cfg = dict(probes=P, frames=NT, ny=spec.ny, nx=spec.nx, seg_len=L, hop=H, dtype="c64",
                   form=args.form, mean_mode=args.mean_mode, streaming=True, gradient=False,
                   omega_half=int(M), producer=True)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (fused producer: Philox4x32-10, elastic 1 + 8 Lorentzian-line tones "
                "of 1e-3/sqrt(8) per pixel + 1e-5 noise), written on the GPU into the ring",
        "config": {
            "workload": f"{P} probes x {NT} frames x {spec.ny}x{spec.nx} c64, Welch L={L} H={H} "
                        f"periodic Hann, {args.mean_mode.replace('_', '-')} mean, "
                        f"{masks.shape[0]} detector masks, transform {args.form}"
                        + (f", energy window |E| <= {args.roi_mev:g} meV ({n_om} bins)" if M else "")
                        + ", frames written by the "
                        f"fused producer in pieces of {piece} straight into a {args.ring_layout} "
                        f"ring of {ring} frames ({batch} probes in flight); the step includes "
                        "the producer",
            "probes": P, "frames": NT, "ny": spec.ny, "nx": spec.nx, "seg_len": L, "hop": H,
            "n_omega": n_om, "exit_wave_bytes": b_alg,
        },
        "producer_ms": round(prod_ms, 1),
        "reduction_gbs": round(b_alg / ((ms - prod_ms) * 1e-3) / 1e9, 2) if ms > prod_ms else None,
        "roofline": {
            "bound": "hbm", "kernel": "seg_fft_kernel (tiled ring)", "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles([os.path.join(csrc, f) for f in KERNEL_SOURCES], run_cfg),
            "kernel_ms": round(k_ms, 2), "algorithmic_bytes_per_launch": None,
            "note": "achieved = exit-wave bytes of the step / the summed chunk-kernel time of "
                    "all its launches (HIP events on the plan's stream)",
        },
    }
    if args.form != "fft":
        n_seg = (NT - L) // H + 1
        m_rows = (2 * n_om + 31) // 32 * 32  # GEMM rows computed (window rows, padded to 32)
        flops = 3 * 2 * m_rows * 2 * L * n_seg * P * spec.n_k  # executed, 3 products
        tf = flops / (k_ms * 1e-3) / 1e12
        out["dtype"] = "f16x3" if args.form == "gemm_f16x3" else "bf16x3"
        out["roofline"] = {
            "bound": "mfma", "kernel": "seg_gemm_kernel (tiled ring)", "achieved": round(tf, 2),
            "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4),
            "kernel_ms": round(k_ms, 2), "traffic": None,
            "note": "executed MFMA flops (3 split products of the real GEMM with "
                    f"{m_rows} rows x {2 * L} per chunk) / the summed chunk-kernel time of "
                    "all launches of the step; useful flops are one third",
        }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(spec, L, H, args.cpu_pixels or 16,
                                           mean_mode=args.mean_mode, twin=True)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
