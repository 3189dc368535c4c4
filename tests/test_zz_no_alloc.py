"""tacaw_backward_static (the allocation-free adjoint, fixed library scratch)
against tacaw_backward on the same plans, through the C ABI: two calls in a row,
the second with a smaller input, for the mean term taken from the forward sums
(Hann, r = 1) and for the separate mean-term pass that reads the scratch
(width-r Hann at r != 1); and a call beyond the fixed scratch is refused."""

import numpy as np
import pytest
import torch

import tacaw_synth as T

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return t


def forward_plan(tacaw, psi, L, H, r):
    P, NT, ny, nx = psi.shape
    masks = torch.from_numpy(T.standard_masks(ny, nx, scale=min(ny, nx) / 64)).cuda()
    plan = tacaw.Plan(P, ny, nx, NT, L, H, masks=masks, window="hann_width", window_param=r)
    plan.push(psi)
    plan.finalize()
    return plan


def both(plan, x, probe0, gD):
    print(f"backward probes {probe0}..{probe0 + x.shape[0] - 1} shape {tuple(x.shape)}", flush=True)
    g0, w0 = plan.backward(x, probe0=probe0, gD=gD)
    g1, w1 = plan.backward(x, probe0=probe0, gD=gD, static_scratch=True)
    torch.cuda.synchronize()
    return (g0.cpu().numpy(), float(w0)), (g1.cpu().numpy(), float(w1))


@pytest.mark.parametrize("r", [1.0, 1.1])
def test_static_scratch_matches_backward_twice(tacaw, r):
    L, H, NT, ny, nx, P = 256, 128, 600, 9, 13, 3
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=91, model="lines", n_terms=8)
    psi = T.generate(spec).cuda()
    plan = forward_plan(tacaw, psi, L, H, r)
    gD = torch.from_numpy(T.loss_weights(4, plan.n_omega, seed=4)).cuda()
    # first call: every probe; second call: one probe (a smaller input)
    for probe0, n in [(0, P), (1, 1)]:
        (g0, w0), (g1, w1) = both(plan, psi[probe0:probe0 + n], probe0, gD)
        e = rel(g1, g0)
        print(f"  r={r}: grad rel diff {e:.2e} (bit-equal {np.array_equal(g0, g1)}), "
              f"dL/dr {w0:.9e} vs {w1:.9e}", flush=True)
        assert e <= 1e-12
        assert w1 == pytest.approx(w0, rel=1e-12, abs=1e-30)
    plan.close()


def test_static_scratch_limit_is_refused(tacaw):
    # 16 probes x 256^2 pixels need 16 MiB + tile partials: more than the fixed scratch
    L, H, NT, ny, nx, P = 64, 64, 64, 256, 256, 16
    spec = T.SeriesSpec(P, NT, ny, nx, dtype="c64", seed=92, model="lines", n_terms=2)
    psi = torch.empty((P, NT, ny, nx), dtype=torch.complex64, device="cuda")
    T.generate_into(spec, psi)
    plan = forward_plan(tacaw, psi, L, H, 1.0)
    gD = torch.from_numpy(T.loss_weights(4, plan.n_omega, seed=4)).cuda()
    with pytest.raises(tacaw.TacawError) as err:
        plan.backward(psi, gD=gD, static_scratch=True)
    assert err.value.kind == "SHAPE"
    # half the probes fit and match the allocating adjoint
    (g0, w0), (g1, w1) = both(plan, psi[:8], 0, gD)
    assert rel(g1, g0) <= 1e-12
    plan.close()
