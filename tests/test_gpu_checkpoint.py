"""Checkpoint and resume (tacaw_plan_export / tacaw_plan_import).

A run that stops at a probe boundary and continues in a new plan from the
exported state must give the results of the same pushes made in one
uninterrupted plan: the state holds every accumulator as stored, so the
remaining chunk launches add the same values in the same order and S is bitwise
equal. The detector sums D and D_p are FP64 atomic sums over pixel tiles, whose
order varies from run to run even without a checkpoint: they agree to a few
FP64 roundings (relative 1e-12). Covered for the
FFT and both GEMM forms, the per-chunk mean, the deferred ring (per frame and per
pixel tile), complex128 input
with an energy window and probe sums, a state taken before any push, and probes
completed out of order; the uninterrupted run itself is checked against the FP64
oracle once. The refusals (mid-probe export, import into a used plan or one with
another descriptor or masks, truncated or foreign bytes) are checked too, and the
union of states exported by plans that each reduced one shard of the probes."""

import numpy as np
import pytest
import torch

import oracle as O
import tacaw_synth as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return t


P, NT, NY, NX, L, H = 4, 1000, 24, 20, 256, 128


def series(dtype="c64", seed=5):
    spec = T.SeriesSpec(P, NT, NY, NX, dtype=dtype, seed=seed, model="lines", n_terms=8,
                        amplitude=1e-3 / np.sqrt(8))
    return T.generate(spec)


def masks(seed=3):
    m = T.standard_masks(NY, NX, scale=min(NY, NX) / 128)
    m[3] = np.random.default_rng(seed).random((NY, NX))
    return torch.from_numpy(m).cuda()


def push_group(plan, x, p0, n, piece):
    for f0 in range(0, NT, piece):
        plan.push(x[p0:p0 + n, f0:f0 + piece], probe0=p0)


def same(got, want, label):
    assert np.array_equal(got["S"], want["S"]), f"{label}: S differs"
    for k in ("D", "Dp"):
        e = np.linalg.norm((got[k] - want[k]).ravel()) / np.linalg.norm(want[k].ravel())
        assert e <= 1e-12, f"{label}: {k} differs by {e:.2e}"


def results(plan):
    S = plan.finalize()
    D, Dp = plan.detector_spectra(per_probe=True)
    torch.cuda.synchronize()
    out = {"S": S.cpu().numpy(), "D": D.cpu().numpy(), "Dp": Dp.cpu().numpy(),
           "info": plan.info()}
    plan.close()
    return out


CASES = {
    "fft": dict(kw={}, piece=300),
    "per_chunk_mean": dict(kw={"mean_mode": "per_segment"}, piece=300),
    "deferred_ring": dict(kw={"ring_frames": 512}, piece=200),
    "tiled_ring": dict(kw={"ring_frames": 512, "tiled_ring": True}, piece=200),
    "gemm_bf16x3": dict(kw={"transform": "gemm_bf16x3"}, piece=300),
    "gemm_f16x3": dict(kw={"transform": "gemm_f16x3"}, piece=NT),
    "c128_window_sum": dict(kw={"in_dtype": "c128", "omega_half": 40, "probe_reduce": "sum"},
                            piece=250),
}


@pytest.mark.parametrize("order", [((0, 2), (2, 2)), ((2, 2), (0, 2))], ids=["in_order", "reversed"])
@pytest.mark.parametrize("case", list(CASES))
def test_resume_is_bitwise_equal_to_one_run(tacaw, case, order):
    kw, piece = CASES[case]["kw"], CASES[case]["piece"]
    dtype = kw.get("in_dtype", "c64")
    x = series(dtype).cuda()
    m = masks()
    print(f"checkpoint case {case}, order {order}", flush=True)

    ref = tacaw.Plan(P, NY, NX, NT, L, H, masks=m, **kw)
    for p0, n in order:
        push_group(ref, x, p0, n, piece)
    want = results(ref)

    first = tacaw.Plan(P, NY, NX, NT, L, H, masks=m, **kw)
    push_group(first, x, *order[0], piece)
    state = first.export_state()
    first.close()
    # a new plan with its own copy of the masks continues the run
    resumed = tacaw.Plan(P, NY, NX, NT, L, H, masks=m.clone(), **kw)
    resumed.import_state(state)
    assert resumed.info()["probes_complete"] == 2
    push_group(resumed, x, *order[1], piece)
    got = results(resumed)

    same(got, want, case)
    for k in ("frames_dropped", "probes_complete"):
        assert got["info"][k] == want["info"][k]
    assert want["info"]["frames_dropped"] == P * (NT - ((NT - L) // H * H + L))

    if case == "fft" and order[0] == (0, 2):
        So, Sp = O.tacaw_spectra(x.cpu().numpy(), L, H, O.window("hann", L), "global")
        e = np.linalg.norm(got["S"].reshape(L, -1) - So) / np.linalg.norm(So)
        print(f"resumed run vs FP64 oracle: rel L2 {e:.2e}")
        assert e <= 1e-5


def test_state_before_any_push_and_repeated_resume(tacaw):
    # a state taken from an untouched plan, and a run resumed twice (one probe at a time)
    x = series(seed=9).cuda()
    m = masks()
    ref = tacaw.Plan(P, NY, NX, NT, L, H, masks=m)
    for p in range(P):
        push_group(ref, x, p, 1, 400)
    want = results(ref)

    plan = tacaw.Plan(P, NY, NX, NT, L, H, masks=m)
    state = plan.export_state()
    plan.close()
    for p in range(P):
        plan = tacaw.Plan(P, NY, NX, NT, L, H, masks=m)
        plan.import_state(state)
        push_group(plan, x, p, 1, 400)
        state = plan.export_state()
        if p < P - 1:
            plan.close()
    got = results(plan)
    same(got, want, "repeated resume")


def test_export_and_import_refusals(tacaw):
    x = series(seed=11).cuda()
    m = masks()
    plan = tacaw.Plan(P, NY, NX, NT, L, H, masks=m)
    push_group(plan, x, 0, 1, NT)
    good = plan.export_state()
    n0 = len(good)

    # mid-probe: probe 1 partially pushed
    plan.push(x[1:2, :300], probe0=1)
    with pytest.raises(tacaw.TacawError) as e:
        plan.export_state()
    assert e.value.kind == "STATE"
    # import into a plan that has frames pushed
    with pytest.raises(tacaw.TacawError) as e:
        plan.import_state(good)
    assert e.value.kind == "STATE"
    # finalized
    plan.push(x[1:2, 300:], probe0=1)
    push_group(plan, x, 2, 2, NT)
    plan.finalize()
    with pytest.raises(tacaw.TacawError) as e:
        plan.export_state()
    assert e.value.kind == "STATE"
    plan.close()

    other = tacaw.Plan(P, NY, NX, NT, L, H + 64, masks=m)
    with pytest.raises(tacaw.TacawError) as e:
        other.import_state(good)
    assert e.value.kind == "SHAPE"
    other.close()
    other = tacaw.Plan(P, NY, NX, NT, L, H, masks=m * 2.0)
    with pytest.raises(tacaw.TacawError) as e:
        other.import_state(good)
    assert e.value.kind == "SHAPE"
    other.close()

    fresh = tacaw.Plan(P, NY, NX, NT, L, H, masks=m)
    with pytest.raises(tacaw.TacawError) as e:
        fresh.import_state(good[: n0 - 8])
    assert e.value.kind == "SHAPE"
    with pytest.raises(tacaw.TacawError) as e:
        fresh.import_state(b"\x00" * n0)
    assert e.value.kind == "INVALID_ARG"
    # a refused import leaves the plan usable; the good state still loads
    fresh.import_state(good)
    assert fresh.info()["probes_complete"] == 1
    fresh.close()


@pytest.mark.parametrize("case", ["fft", "per_chunk_mean", "gemm_bf16x3", "c128_window_sum"])
def test_union_of_probe_shards(tacaw, case):
    # two shards of the probes reduced by separate plans (as separate processes or
    # GPUs would), their states merged on the host, imported and finalized: the
    # spectra of one run over all probes, up to the FP64 order of the shard sums
    kw, piece = CASES[case]["kw"], CASES[case]["piece"]
    x = series(kw.get("in_dtype", "c64"), seed=21).cuda()
    m = masks()
    print(f"probe shards, case {case}", flush=True)
    ref = tacaw.Plan(P, NY, NX, NT, L, H, masks=m, **kw)
    push_group(ref, x, 0, 2, piece)
    push_group(ref, x, 2, 2, piece)
    want = results(ref)

    states = []
    for p0 in (0, 2):
        shard = tacaw.Plan(P, NY, NX, NT, L, H, masks=m, **kw)
        push_group(shard, x, p0, 2, piece)
        states.append(shard.export_state())
        shard.close()
    merged = tacaw.merge_states(*states)
    final = tacaw.Plan(P, NY, NX, NT, L, H, masks=m, **kw)
    final.import_state(merged)
    got = results(final)
    for k in ("S", "D", "Dp"):
        e = np.linalg.norm((got[k] - want[k]).ravel()) / np.linalg.norm(want[k].ravel())
        assert e <= 1e-12, f"{case}: {k} differs by {e:.2e}"
    for k in ("frames_dropped", "probes_complete"):
        assert got["info"][k] == want["info"][k]


def test_resume_and_merge_without_masks(tacaw):
    # a plan with no detector masks has no per-probe detector spectra in its state
    x = series(seed=31).cuda()
    ref = tacaw.Plan(P, NY, NX, NT, L, H)
    push_group(ref, x, 0, 2, 300)
    push_group(ref, x, 2, 2, 300)
    want = ref.finalize().cpu().numpy()
    ref.close()
    shards = []
    for p0 in (0, 2):
        sh = tacaw.Plan(P, NY, NX, NT, L, H)
        push_group(sh, x, p0, 2, 300)
        shards.append(sh.export_state())
        sh.close()
    for state, label in ((shards[0], "resume"), (tacaw.merge_states(*shards), "merge")):
        plan = tacaw.Plan(P, NY, NX, NT, L, H)
        plan.import_state(state)
        if label == "resume":
            push_group(plan, x, 2, 2, 300)
            assert np.array_equal(plan.finalize().cpu().numpy(), want)
        else:
            got = plan.finalize().cpu().numpy()
            assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-12
        plan.close()
    # a state with masks does not load into a plan without them
    with_masks = tacaw.Plan(P, NY, NX, NT, L, H, masks=masks())
    other = with_masks.export_state()
    with_masks.close()
    plan = tacaw.Plan(P, NY, NX, NT, L, H)
    with pytest.raises(tacaw.TacawError) as e:
        plan.import_state(other)
    assert e.value.kind == "SHAPE"
    plan.close()
