"""CPU tests of bench.py's host logic: the key under which measured HBM traffic is kept
(a digest of a kernel's code regions), the arrival times of the rate sweep and the refusal of
more than one GPU."""
from __future__ import annotations

import importlib.util
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent


def _bench(tmp_path=None):
    spec = importlib.util.spec_from_file_location("bench_under_test", ROOT / "bench.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if tmp_path is not None:
        mod.ROOT = tmp_path
    return mod


def test_kernel_digest_ignores_comments_only(tmp_path):
    b = _bench(tmp_path)
    src = tmp_path / "k.hip"
    base = "// header\n__global__ void k(int* a) {\n  a[0] = 1;  // store\n}\n// end\n"
    regions = [["k.hip", "", "// end"]]
    src.write_text(base)
    d0 = b.kernel_source_digest(regions)
    assert d0 is not None
    # comments, trailing blanks and empty lines do not change the kernel
    src.write_text("// other header\n\n__global__ void k(int* a) {   \n  a[0] = 1;\n}\n// end\n")
    assert b.kernel_source_digest(regions) == d0
    # a change of code does
    src.write_text(base.replace("a[0] = 1", "a[0] = 2"))
    assert b.kernel_source_digest(regions) != d0
    # a region that cannot be found gives no digest (the traffic is then not reported)
    assert b.kernel_source_digest([["k.hip", "no such text", "// end"]]) is None
    assert b.kernel_source_digest([["missing.hip", "", "x"]]) is None


def test_committed_traffic_entries_are_well_formed():
    entries = json.loads((ROOT / "profiles" / "traffic.json").read_text())
    for name, e in entries.items():
        for key in ("kernel", "source_regions", "source_sha256", "workload", "fetch_kib_per_dispatch",
                    "write_kib_per_dispatch", "fetch_scale", "write_scale", "hbm_bytes_per_launch"):
            assert key in e, (name, key)
        # bytes per launch = (fetch x scale + write x scale) KiB
        kib = e["fetch_kib_per_dispatch"] * e["fetch_scale"] + e["write_kib_per_dispatch"] * e["write_scale"]
        assert abs(kib * 1024 - e["hbm_bytes_per_launch"]) < 1e-3 * e["hbm_bytes_per_launch"], name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_rescaled_arrivals_keep_the_requests_and_scale_the_rate():
    """The sweep's streams: the same requests in the same order, the warm-up ones (before t0)
    kept ahead, the gaps after the first timed arrival scaled so that the mean rate is the new
    one (Poisson draws of mean gap 1/2 s at 2 requests/s become mean gap 1/0.5 s at 0.5)."""
    import numpy as np

    b = _bench()
    rng = np.random.default_rng(1)
    times = np.cumsum(rng.exponential(0.5, 2000))
    stream = [(float(t), i) for i, t in enumerate(times)]
    t0 = stream[4][0]
    out = b.rescale_arrivals(stream, t0, 2.0, 0.5)
    assert [w for _, w in out] == list(range(2000))
    assert out[4][0] == t0
    assert all(out[i][0] <= t0 for i in range(4))
    gaps = np.diff([t for t, _ in out[4:]])
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 2.0) < 0.1
    assert np.allclose(gaps, 4.0 * np.diff(times[4:]))
