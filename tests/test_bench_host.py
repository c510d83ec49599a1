"""Host logic of the benchmark (no GPU): the HBM-traffic figure and the
single-GPU guard.

The traffic of a kernel site comes from two rocprofv3 counter runs
(FETCH_SIZE, WRITE_SIZE): the mean KiB per dispatch of the site's kernel,
each scaled by what the same counter reads for a copy kernel of known size
(2^25 doubles each way), and is withdrawn (None) once the kernel sources no
longer hash to the value recorded with the counters.
"""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY = ("void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<double, "
        "double, double, at::native::MulFunctor<double> > >(int, ...)")
TRIDIAG = ("void fkf::(anonymous namespace)::k_tridiag<8, 1>(double const*, long, int, int, "
           "double*, double*, double*, double*, unsigned long long*, int*)")


def _csv(path, ctr, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for name, grid, v in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": ctr,
                        "Counter_Value": v})


def test_traffic_scaling_and_source_hash(tmp_path):
    true_kib = (8 << 25) / 1024.0
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # the copy reads half its true bytes on FETCH_SIZE (factor 2) and all of
    # them on WRITE_SIZE (factor 1); a copy of another size is not the
    # calibration; two dispatches of the round kernel average
    _csv(fetch, "FETCH_SIZE", [(COPY, 1 << 23, true_kib / 2), (COPY, 1 << 20, 1.0),
                               (TRIDIAG, 119040, 100.0), (TRIDIAG, 119040, 300.0),
                               ("fkf::k_unlisted(int)", 256, 5.0)])
    _csv(write, "WRITE_SIZE", [(COPY, 1 << 23, true_kib), (TRIDIAG, 119040, 50.0)])
    out = tmp_path / "traffic.json"
    bench.write_traffic(str(fetch), str(write), out=str(out))
    rec = json.load(open(out))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["sites"] == {"eig_tridiag": {"fetch_kib": 200.0, "write_kib": 50.0}}
    assert bench.traffic_for("eig_tridiag", path=str(out)) == (200.0 * 2 + 50.0) * 1024.0
    assert bench.traffic_for("filter_gemv", path=str(out)) is None
    assert bench.traffic_for("eig_tridiag", path=str(tmp_path / "absent.json")) is None
    rec["sources_sha256"] = "0" * 64     # counters taken on other kernel sources
    json.dump(rec, open(out, "w"))
    assert bench.traffic_for("eig_tridiag", path=str(out)) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
