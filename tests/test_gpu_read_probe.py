"""The HBM read-ceiling probe reads every byte once: its 64-bit wrapping sum must
equal numpy's over the same bytes (small, ragged-grid and multi-gigabyte
buffers), and sizes that are not whole 16-byte words are refused."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_bytes", [16, 4096 + 16, (1 << 20) * 37 + 48, 3 << 30])
def test_sum_matches_numpy(n_bytes):
    from paper_2607_02236_amd import tacaw

    g = torch.Generator(device="cuda").manual_seed(n_bytes % 1000)
    buf = torch.randint(-(1 << 62), 1 << 62, (n_bytes // 8,), dtype=torch.int64, device="cuda",
                        generator=g)
    s = int(tacaw.read_probe(buf).item()) & ((1 << 64) - 1)
    host = buf.cpu().numpy().view(np.uint64)
    want = int(np.sum(host, dtype=np.uint64))  # numpy wraps modulo 2^64
    print(f"{n_bytes} B: sum {s:#x}", flush=True)
    assert s == want


def test_refuses_partial_words():
    from paper_2607_02236_amd import tacaw

    buf = torch.zeros(6, dtype=torch.int32, device="cuda")  # 24 bytes
    with pytest.raises(tacaw.TacawError) as e:
        tacaw.read_probe(buf)
    assert e.value.kind == "INVALID_ARG"


@pytest.mark.parametrize("rows,row_bytes,seg", [(2048, 4096, 128), (37, 1024, 64), (5, 512, 512),
                                                (1000, 256 * 256 * 8, 128)])
def test_column_probe_reads_every_byte_once(rows, row_bytes, seg):
    from paper_2607_02236_amd import tacaw

    g = torch.Generator(device="cuda").manual_seed(rows)
    buf = torch.randint(-(1 << 62), 1 << 62, (rows * row_bytes // 8,), dtype=torch.int64,
                        device="cuda", generator=g)
    s = int(tacaw.read_probe_columns(buf, rows, seg).item()) & ((1 << 64) - 1)
    whole = int(tacaw.read_probe(buf).item()) & ((1 << 64) - 1)
    want = int(np.sum(buf.cpu().numpy().view(np.uint64), dtype=np.uint64))
    assert s == want and whole == want


def test_column_probe_refusals():
    from paper_2607_02236_amd import tacaw

    buf = torch.zeros(1024, dtype=torch.int64, device="cuda")
    for rows, seg in ((4, 96), (3, 128), (16, 1024)):  # bad width; rows not dividing; too wide
        with pytest.raises((tacaw.TacawError, ValueError)):
            tacaw.read_probe_columns(buf, rows, seg)
