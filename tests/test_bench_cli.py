"""bench.py contract checks that need no GPU."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a refused run


def test_counter_summaries_name_their_sources_and_commands():
    # the committed counter summaries carry the hash of the kernel sources they were
    # taken on; bench.py reports their traffic only while that hash matches
    sys.path.insert(0, ROOT)
    import bench

    for name, srcs in [("seg_fft_L512_64probes_counters.json", bench.KERNEL_SOURCES),
                       ("bwd_kernel_L512_16probes_counters.json", bench.ADJOINT_SOURCES)]:
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert len(d["source_sha"]) == 16 and d["commands"]
        assert d["hbm_bytes_per_launch"] > d["algorithmic_bytes_per_launch"] * 0.99
        for f in srcs:
            assert os.path.exists(os.path.join(ROOT, "paper_2607_02236_amd", "csrc", f))


def test_counter_traffic_applies_only_to_the_measured_workload():
    # the default lines resolve to the committed counters while they were taken on
    # the current kernel sources (null otherwise); another workload (here a streamed
    # run of the same sizes) or another kernel source always gives null traffic
    sys.path.insert(0, ROOT)
    import bench

    csrc = os.path.join(ROOT, "paper_2607_02236_amd", "csrc")
    fwd = [os.path.join(csrc, f) for f in bench.KERNEL_SOURCES]
    bwd = [os.path.join(csrc, f) for f in bench.ADJOINT_SOURCES]

    def current(name, srcs):
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        return d["source_sha"] == bench.source_sha(srcs)

    cfg = dict(probes=64, frames=2048, ny=256, nx=256, seg_len=512, hop=256, dtype="c64",
               form="fft", mean_mode="global", streaming=False, gradient=False, omega_half=0)
    t = bench.traffic_from_profiles(fwd, cfg)
    if current("seg_fft_L512_64probes_counters.json", fwd):
        assert t > 6.8e10
    else:
        assert t is None
    assert bench.traffic_from_profiles(fwd, dict(cfg, streaming=True)) is None
    assert bench.traffic_from_profiles(bwd, cfg) is None  # other sources
    gcfg = dict(cfg, probes=16, frames=1024, ny=128, nx=128, hop=512, gradient=True)
    tb = bench.traffic_from_profiles(bwd, gcfg, "bwd_kernel_L512_16probes_counters.json")
    if current("bwd_kernel_L512_16probes_counters.json", bwd):
        assert tb > 4e9
    else:
        assert tb is None
