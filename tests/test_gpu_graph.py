"""One whole reduction (reset, pushes, finalize, detector spectra) captured once in
a HIP graph and replayed on new exit waves written into the same input buffer:
every launch the plan makes is stream-ordered, allocation-free once the plan has
run, and clears its accumulators with fill kernels, so each replay must equal an
eager run on the same data (S bit for bit; the detector spectra to FP64 rounding,
their partials are added atomically). Replays are interleaved with eager work and
synchronisations, and every replay is checked."""

import numpy as np
import pytest
import torch

import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("pieces,kw", [
    (None, {}),                                             # one whole-series push
    ([200, 300, 140], {}),                                  # chunks straddle pushes (ring)
    ([128] * 5, {"ring_frames": 256, "tiled_ring": True}),  # deferred tiled ring
    ([333, 307], {"mean_mode": "per_segment"}),             # per-chunk mean sums
])
def test_captured_reduction_replays_match_eager(pieces, kw):
    from paper_2607_02236_amd import tacaw

    P, NT, ny, nx, L, H = 3, 640, 12, 10, 128, 64
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=0.08)).cuda()
    series = [T.generate(T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=s, model="lines",
                                      n_terms=8)).cuda() for s in (11, 12, 13)]
    pieces = pieces or [NT]
    cuts = np.concatenate([[0], np.cumsum(pieces)])
    side = torch.cuda.Stream()
    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks, stream=side, **kw)
    n_om = plan.n_omega
    x = torch.empty_like(series[0])
    S = torch.empty((n_om, ny, nx), dtype=torch.float64, device="cuda")
    D = torch.empty((4, n_om), dtype=torch.float64, device="cuda")
    Dp = torch.empty((4, P, n_om), dtype=torch.float64, device="cuda")

    def reduce():
        plan.reset()
        for i in range(len(pieces)):
            plan.push(x[:, cuts[i]:cuts[i + 1]])
        plan.finalize(out=S)
        plan.detector_spectra(per_probe=True, out=D, out_p=Dp)

    def eager(data):
        x.copy_(data)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            reduce()
        torch.cuda.synchronize()
        return S.clone(), D.clone(), Dp.clone()

    ref = [eager(d) for d in series]  # the first run also allocates lazy plan buffers
    assert not torch.equal(ref[0][0], ref[1][0])
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        reduce()
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(2):
        for k in (2, 0, 1):
            x.copy_(series[k])
            S.fill_(-1.0)
            D.fill_(-1.0)
            Dp.fill_(-1.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            # S has one owner thread per value; detector sums add per-tile
            # partials with FP64 atomics, whose order may vary between runs
            eD, eDp = rel(D, ref[k][1]), rel(Dp, ref[k][2])
            print(f"replay {rep}.{k}: S equal {torch.equal(S, ref[k][0])}, D {eD:.1e}, "
                  f"Dp {eDp:.1e}", flush=True)
            assert torch.equal(S, ref[k][0]) and eD <= 1e-13 and eDp <= 1e-13
            junk.add_(x.real.sum())  # eager work between replays
            torch.cuda.synchronize()
    del g
    plan.close()
