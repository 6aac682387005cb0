"""CPU test of the benchmark's counter summary: rocprof counter rows of the
kernel section's pass loops (synthetic here) are grouped into loops by
their clearing and finishing kernels, each loop is attributed to the kernel
shape whose launch sequence it is (a change-tracking loop starts with two
dense launches), and byte counters are scaled by the calibration copies."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PK = "void phg::pass_kernel<2, 1, %d, %d, %d, false>(phg::PassArgs)"
DENSE = PK % (8, 4, 0)


def loop(kernels):
    return (["void phg::zero2_u64_kernel(unsigned long long*, long long, unsigned long long*, long long)"]
            + kernels + ["void phg::finish_kernel(phg::FinishArgs)"])


def write_dir(path, counter, dispatches):
    os.makedirs(path)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(dispatches):
            w.writerow([i + 1, name, counter, value])


@pytest.fixture(scope="module")
def lib():
    from paper_1306_5390_amd import _api
    if not os.path.exists(_api.LIB_PATH):
        from paper_1306_5390_amd import build
        build.build()
    return _api.load_library()


def test_loops_are_attributed_to_their_shapes(lib, tmp_path):
    import bench
    seqs = {
        "3": loop([DENSE] * 32),
        "7": loop([DENSE] * 2 + [PK % (8, 4, 1)] * 30),
        "12": loop([DENSE] * 2 + [PK % (8, 2, 2)] + [PK % (8, 2, 3)] * 29),
    }
    # per-dispatch KiB: distinct per shape so that a misattribution shows
    kib = {"3": (1000.0, 3000.0), "7": (500.0, 1500.0), "12": (100.0, 300.0)}
    fetch, write = [], []
    for s in ("3", "7", "12"):
        for name in seqs[s]:
            is_pass = "pass_kernel" in name
            fetch.append((name, kib[s][0] if is_pass else 1.0))
            write.append((name, kib[s][1] if is_pass else 1.0))
    for _ in range(3):   # the calibration copies: 64 MiB read and written
        fetch.append(("__amd_rocclr_copyBuffer", 32768.0))
        write.append(("__amd_rocclr_copyBuffer", 65536.0))
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    write_dir(fd, "FETCH_SIZE", fetch)
    write_dir(wd, "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    bench.summarize_counters("large8192", [fd, wd], out_path=out)
    d = json.load(open(out))
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert set(d["shapes"]) == {"3", "7", "12"}
    for s, (f, w) in kib.items():
        row = d["shapes"][s]
        assert row["launches"] == 32
        assert row["bytes_per_launch"] == pytest.approx((2.0 * f + w) * 1024.0)
        assert row["algorithmic_bytes_per_launch"] == 2.0 * 8192 * 8192
