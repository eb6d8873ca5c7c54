"""Host-side checks of bench.py that need no GPU: the multi-GPU refusal and
the parsing of the committed traffic summaries the bench line cites."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _fields(path):
    out = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.strip().lstrip("-* ").partition(":")
            if sep:
                out[k.strip()] = v.strip().strip("`")
    return out


def test_traffic_summaries_parse():
    """Each committed compositing traffic summary names its kernel, tile and
    source digest and gives positive byte counts; bench.measured_traffic
    reads the same fields (and drops the figure when the digest or the tile
    setting differs)."""
    import bench
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "raster_*.*.md")))
    paths = [p for p in paths if not os.path.basename(p).startswith("raster_sq")]
    assert paths
    for p in paths:
        f = _fields(p)
        assert len(f["sources_sha256"]) == 16, p
        w, _, h_b = f["tile"].partition("x")
        h, _, b = h_b.partition("/")
        assert int(w) > 0 and int(h) > 0 and int(b) > 0, p
        assert float(f["traffic_bytes_per_launch"]) > 0, p
        assert float(f["average duration (kernel trace)"].split()[0]) > 0, p
    assert len(bench.sources_digest()) == 16
