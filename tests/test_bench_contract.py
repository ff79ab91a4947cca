"""Host-side checks of bench.py's contract with the committed rocprofv3
summaries and its command line (no GPU: nothing here launches a kernel)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summaries():
    d = os.path.join(ROOT, "profiles")
    out = []
    for name in sorted(os.listdir(d)):
        m = re.match(r"sweepk(\d+)_f64_(\d+)_traffic\.md$", name)
        if m:
            out.append((int(m.group(1)), int(m.group(2)), os.path.join(d, name)))
    return out


def test_traffic_summaries_exist_for_the_benchmark_stencils():
    have = {(st, n) for st, n, _ in _summaries()}
    assert (9, 8192) in have and (17, 8192) in have


@pytest.mark.parametrize("st,n,path", _summaries())
def test_bench_reads_every_height_a_summary_lists(monkeypatch, st, n, path):
    """measured_traffic returns the summary's figure for its workload line and for
    each other tile height it lists, and None for heights or geometries it does
    not list, when the summary's kernel hash is the source's."""
    text = open(path).read()
    h = re.search(r"kernels\.hip sha256\[:16\][^:\n]*:\s*([0-9a-f]{16})", text).group(1)
    monkeypatch.setattr(bench, "kernel_hash", lambda: h)
    w = re.search(r"workload:\s*n=(\d+)\s+stencil=(\d+)\s+K=(\d+)\s+rows=(\d+)", text)
    wn, wst, wk, wrows = (int(v) for v in w.groups())
    assert (wn, wst) == (n, st)
    main = float(re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text).group(1))
    assert bench.measured_traffic(n, st, wk, wrows) == main
    # counted bytes lie between the compulsory 24 B per point and 1.3 times that
    assert 24.0 * n * n <= main <= 1.3 * 24.0 * n * n
    others = re.findall(r"^traffic rows=(\d+)\b[^:\n]*:\s*([0-9.eE+]+)", text, re.M)
    assert others
    for r, b in others:
        assert bench.measured_traffic(n, st, wk, int(r)) == float(b)
    assert bench.measured_traffic(n, st, wk, 7) is None
    assert bench.measured_traffic(n, st, wk + 1, wrows) is None
    # a changed kernel source voids the figure
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.measured_traffic(n, st, wk, wrows) is None


def test_no_summary_means_no_traffic():
    assert bench.measured_traffic(1234, 9, 10, 283) is None


def test_kernel_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("// leading comment\nint f(int x)   {\n  /* block\n comment */ return x + 1;  // trailing\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    hashes = []
    for p in (a, b, c):
        monkeypatch.setattr(bench, "KERNEL_SRC", str(p))
        hashes.append(bench.kernel_hash())
    assert hashes[0] == hashes[1] != hashes[2]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
