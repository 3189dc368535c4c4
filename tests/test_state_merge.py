"""tacaw_state_merge, the union of two exported plan states over disjoint probe
sets (host code, no device): forged states with the exported layout (header,
per-probe frame cursors, FP64 accumulators) check the element-wise sum, the
cursor and counter bookkeeping, in-place output, and every refusal."""

import ctypes
import struct

import numpy as np
import pytest

MAGIC = 0x31305354574154
HEADER = "<QQqiiiiiiq"  # magic, fingerprint, total bytes, n_probe, n_k, n_om, n_det,
#                         per-chunk flag, S defined, frames dropped


def state(cursors, body, fingerprint=7, dropped=0, s_defined=1, n_k=6, n_om=5, n_det=2,
          magic=MAGIC, total=None):
    n_probe = len(cursors)
    size = struct.calcsize(HEADER) + 8 * n_probe + 8 * body.size
    head = struct.pack(HEADER, magic, fingerprint, size if total is None else total, n_probe,
                       n_k, n_om, n_det, 0, s_defined, dropped)
    return head + np.asarray(cursors, dtype=np.int64).tobytes() + body.astype(np.float64).tobytes()


def parse(buf, n_probe):
    h = struct.unpack_from(HEADER, buf)
    off = struct.calcsize(HEADER)
    cur = np.frombuffer(buf, dtype=np.int64, count=n_probe, offset=off)
    body = np.frombuffer(buf, dtype=np.float64, offset=off + 8 * n_probe)
    return h, cur, body


@pytest.fixture(scope="module")
def tacaw():
    from paper_2607_02236_amd import tacaw as t

    return t


def test_merge_adds_accumulators_and_keeps_cursors(tacaw):
    rng = np.random.default_rng(3)
    ba, bb = rng.standard_normal(97), rng.standard_normal(97)
    a = state([896, 896, 0, 0], ba, dropped=208, s_defined=1)
    b = state([0, 0, 1000, 896], bb, dropped=104, s_defined=0)
    out = tacaw.merge_states(a, b)
    h, cur, body = parse(out, 4)
    assert h[0] == MAGIC and h[1] == 7 and h[2] == len(a)
    assert h[8] == 1 and h[9] == 312  # S defined in either; dropped frames added
    assert cur.tolist() == [896, 896, 1000, 896]
    assert np.array_equal(body, ba + bb)  # the same IEEE sums, bit for bit
    # the merge is symmetric, and an untouched state is its identity
    assert tacaw.merge_states(b, a) == out
    empty = state([0, 0, 0, 0], np.zeros(97), s_defined=0)
    assert tacaw.merge_states(a, empty) == a


def test_merge_in_place(tacaw):
    rng = np.random.default_rng(4)
    ba, bb = rng.standard_normal(40), rng.standard_normal(40)
    a = ctypes.create_string_buffer(state([5, 0], ba), len(state([5, 0], ba)))
    b = state([0, 9], bb)
    assert tacaw.lib.tacaw_state_merge(a, b, a, len(b)) == 0
    _, cur, body = parse(a.raw, 2)
    assert cur.tolist() == [5, 9] and np.array_equal(body, ba + bb)


def test_merge_refusals(tacaw):
    z = np.zeros(30)
    a = state([5, 0, 0], z)
    with pytest.raises(tacaw.TacawError) as e:  # probe 0 pushed in both
        tacaw.merge_states(a, state([5, 0, 7], z))
    assert e.value.kind == "INVALID_ARG"
    with pytest.raises(tacaw.TacawError) as e:  # another descriptor
        tacaw.merge_states(a, state([0, 5, 0], z, fingerprint=8))
    assert e.value.kind == "SHAPE"
    with pytest.raises(tacaw.TacawError) as e:  # another grid
        tacaw.merge_states(a, state([0, 5, 0], z, n_k=7))
    assert e.value.kind == "SHAPE"
    with pytest.raises(tacaw.TacawError) as e:  # not a state
        tacaw.merge_states(a, state([0, 5, 0], z, magic=1))
    assert e.value.kind == "INVALID_ARG"
    with pytest.raises(tacaw.TacawError) as e:  # header size disagrees with the buffer
        tacaw.merge_states(state([5, 0, 0], z, total=64), state([0, 5, 0], z, total=64))
    assert e.value.kind == "SHAPE"
    with pytest.raises(tacaw.TacawError) as e:  # different lengths
        tacaw.merge_states(a, state([0, 5, 0], np.zeros(31)))
    assert e.value.kind == "SHAPE"
    assert tacaw.lib.tacaw_state_merge(None, a, None, len(a)) == -1
