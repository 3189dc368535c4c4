"""Discarding a thermalisation period and keeping every s-th snapshot (the
trajectories of Sec. IV drop their first picoseconds and store a snapshot every
few MD steps): a push takes any frame stride, so the kept frames are a strided
view of the stored series, with no copy. The result must equal pushing a
contiguous copy of the same frames bit for bit (same arithmetic, other
addresses) and the FP64 oracle on those frames."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    # relative L2 error; absolute where the reference is exactly zero (a mask
    # that misses a tiny grid gives D_j = 0 on both sides)
    a = np.asarray(a)
    b = np.asarray(b)
    nb = float(np.linalg.norm(b.ravel()))
    d = float(np.linalg.norm((a - b).ravel()))
    return d / nb if nb > 0 else d


def spectra(plan, views):
    for v in views:
        plan.push(v)
    S = plan.finalize()
    _, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    out = S.cpu().numpy().reshape(plan.n_omega, -1), Dp.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("skip,stride,pieces,kw", [
    (100, 3, None, {}),
    (37, 2, [150, 1, 200, 249], {}),
    (64, 4, [128, 128, 44], {"ring_frames": 256, "tiled_ring": True}),
    (10, 5, [90, 150], {"mean_mode": "per_segment"}),
])
def test_strided_view_equals_contiguous_copy_and_oracle(skip, stride, pieces, kw):
    from paper_2607_02236_amd import tacaw

    P, ny, nx, L, H = 2, 9, 10, 128, 64
    spec = T.SeriesSpec(P, skip + 1200, ny, nx, dtype="c64", seed=skip + stride, model="lines",
                        n_terms=8, amplitude=1e-3 / np.sqrt(8))
    full = T.generate(spec)
    kept = full[:, skip::stride]
    NT = kept.shape[1]
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=0.08)).cuda()
    xf = full.cuda()
    view = xf[:, skip::stride]
    assert view.stride(1) == stride * ny * nx
    copy = view.contiguous()
    pieces = pieces or [NT]
    assert sum(pieces) == NT
    cuts = np.concatenate([[0], np.cumsum(pieces)])

    def run(x):
        plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks, **kw)
        return spectra(plan, [x[:, cuts[i]:cuts[i + 1]] for i in range(len(pieces))])

    S_v, Dp_v = run(view)
    S_c, Dp_c = run(copy)
    assert np.array_equal(S_v, S_c) and np.array_equal(Dp_v, Dp_c)
    So, _ = O.tacaw_spectra(kept.numpy(), L, H, O.window("hann", L),
                            kw.get("mean_mode", "global"))
    e = rel(S_v, So)
    print(f"skip {skip} stride {stride}: S {e:.2e}", flush=True)
    assert e <= 1e-5
