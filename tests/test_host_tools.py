"""Host-side measurement code on the CPU: the rocprofv3 summaries
(profsummary: per-kernel statistics, HBM-counter scaling by the copy kernel,
multi-kernel steps, the source digest that marks a summary stale) and the
parts of bench.py that need no GPU (its refusal of --gpus > 1, the
algorithmic bytes per site, the coarsening length of a known field)."""

import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1405_6162_amd import profsummary  # noqa: E402

COUNTER_FIELDS = ["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


COPY = "lbk::k_stream_copy(unsigned int const*, unsigned int*, unsigned long)"


def _counter_csv(path, name, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=COUNTER_FIELDS)
        w.writeheader()
        for k, (kernel, value) in enumerate(rows):
            w.writerow({"Correlation_Id": k, "Dispatch_Id": k, "Grid_Size": 256, "Kernel_Name": kernel,
                        "Counter_Name": name, "Counter_Value": value})


def test_pmc_scaling_and_multi_kernel_step(tmp_path, capsys):
    """a copy whose FETCH_SIZE reads half its bytes gets scale 2, one whose
    WRITE_SIZE reads all of them scale 1; a step of two kernels sums their per-dispatch
    traffic, taking the most-dispatched match of each substring."""
    kib = 1024.0
    copy = COPY
    fetch = [(copy, 1048576.0), (copy, 10.0), ("void k_a<1, true>(x)", 100.0), ("void k_a<1, true>(x)", 102.0),
             ("void k_a<1, false>(x)", 500.0), ("void k_b<2>(y)", 40.0)]
    write = [(copy, 2097152.0), (copy, 10.0), ("void k_a<1, true>(x)", 200.0), ("void k_a<1, true>(x)", 200.0),
             ("void k_a<1, false>(x)", 900.0), ("void k_b<2>(y)", 60.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fp, "FETCH_SIZE", fetch)
    _counter_csv(wp, "WRITE_SIZE", write)
    profsummary.main(["pmc", str(fp), str(wp), "--kernel", "k_a<,k_b<"])
    out = capsys.readouterr().out
    (tmp_path / "s.txt").write_text(out)
    info = profsummary.read_traffic(str(tmp_path / "s.txt"))
    assert info["kernel"] == "void k_a<1, true>(x) + void k_b<2>(y)"
    assert float(info["fetch_scale"]) == pytest.approx(2.0)
    assert float(info["write_scale"]) == pytest.approx(1.0)
    want = ((101.0 + 40.0) * 2.0 + (200.0 + 60.0) * 1.0) * kib
    assert float(info["traffic_bytes_per_launch"]) == pytest.approx(want, rel=1e-6)
    assert info["source_digest"] == profsummary.kernel_source_digest()


def test_pmc_missing_kernel_and_missing_copy(tmp_path):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fp, "FETCH_SIZE", [(COPY, 1.0), ("k_a", 1.0)])
    _counter_csv(wp, "WRITE_SIZE", [(COPY, 1.0), ("k_a", 1.0)])
    with pytest.raises(SystemExit):
        profsummary.main(["pmc", str(fp), str(wp), "--kernel", "k_missing"])
    _counter_csv(fp, "FETCH_SIZE", [("k_a", 1.0)])
    with pytest.raises(SystemExit):
        profsummary.main(["pmc", str(fp), str(wp), "--kernel", "k_a"])


def test_stats_summary(tmp_path, capsys):
    p = tmp_path / "stats.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void lbk::k_x<1>(int)", 4, 4000, 1000.0, 80.0, 900, 1100, 1.0])
    profsummary.main(["stats", str(p), "--title", "t", "--command", "a ;; b"])
    out = capsys.readouterr().out.splitlines()
    assert out[0] == "# t" and out[1] == "# command: a" and out[2] == "# command: b"
    assert "void lbk::k_x<1>(int)" in out[4] and "1.00" in out[4]


def test_committed_profiles_match_the_sources():
    """bench.py reports traffic only from a summary whose digest equals the
    current kernel sources (else null); reported here as a skip when the
    kernels changed after the counters were taken."""
    pdir = os.path.join(ROOT, "profiles")
    stale = []
    for name in sorted(os.listdir(pdir)):
        if name.startswith("pmc_"):
            info = profsummary.read_traffic(os.path.join(pdir, name))
            assert float(info["traffic_bytes_per_launch"]) > 0
            if info["source_digest"] != profsummary.kernel_source_digest():
                stale.append(name)
    if stale:
        pytest.skip("counter summaries older than the kernel sources: %s" % ", ".join(stale))


def test_bench_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_bench_host_helpers():
    import bench
    assert bench.algorithmic_bytes("binary", "f64") == {"collide": 608}
    assert bench.algorithmic_bytes("single", "f32") == {"collide": 152}
    assert bench.algorithmic_bytes("binary", "f16") == {"collide": 152}
    assert bench.algorithmic_bytes("adjoint", "f64")["adjoint"] == 456
    assert bench.algorithmic_bytes("adjoint_binary", "f64")["adjoint"] == 912
    import torch
    # the two per-moment error metrics: max norm and L2, a vector moment as one array
    ref = torch.tensor([[1.0, 2.5], [-2.0, 0.0]], dtype=torch.float64)
    got = ref + torch.tensor([[0.0, -0.5], [0.0, 0.0]], dtype=torch.float64)
    e = bench.relative_errors("u", got, ref)
    assert e["u"] == pytest.approx(0.5 / 2.5, rel=1e-15)
    assert e["u_l2"] == pytest.approx(0.5 / np.sqrt(1 + 6.25 + 4), rel=1e-15)
    # one Fourier mode of wavenumber k: L = 2 pi / k
    n = 32
    x = torch.arange(n, dtype=torch.float64)
    phi = torch.cos(2 * np.pi * 4 * x / n).view(1, 1, n).expand(n, n, n).contiguous()
    assert bench.coarsening_length(phi) == pytest.approx(n / 4, rel=1e-12)
    # cos(2 pi 4 x / n) changes sign 8 times along x and never along y, z
    phi = phi + 0.123                     # avoid exact zeros at the nodes
    assert bench.interface_density(phi) == pytest.approx(8 / n / 3, rel=1e-12)


def test_source_digest_ignores_comments_not_code():
    """A counter summary goes stale when the kernels' code changes, not when
    a comment or the spacing does."""
    code = 'int a = 1; // one\n/* two\n   lines */ const char* s = "x // y /* z */";\n'
    same = 'int a = 1;   // another comment\nconst char* s = "x // y /* z */";  /* trailing */\n'
    other = 'int a = 2; // one\n/* two\n   lines */ const char* s = "x // y /* z */";\n'
    assert profsummary._code_only(code) == profsummary._code_only(same)
    assert profsummary._code_only(code) != profsummary._code_only(other)
    assert "// y /* z */" in profsummary._code_only(code)          # inside a string literal: kept
