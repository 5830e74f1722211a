"""Host logic of bench.py (no GPU): the measured-traffic gate and the
committed counter summaries it reads."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary(sha, traffic=1234.0):
    return ("# a counter summary\nkernel: k_query_grad\nsource_sha256: %s\n"
            "traffic_bytes_per_launch: %.0f\n" % (sha, traffic))


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    path = tmp_path / "k_query_grad_room20m_traffic.txt"
    sha = bench._source_sha("k_query_grad")
    assert sha is not None and len(sha) == 64
    path.write_text(_summary(sha))
    assert bench.measured_traffic("k_query_grad", 5) == 1234.0
    # another digest (the kernel or the header it inlines changed): no number
    path.write_text(_summary("0" * 64))
    assert bench.measured_traffic("k_query_grad", 5) is None
    # no summary, or a kernel without sources: no number
    assert bench.measured_traffic("k_query_grad", 2) is None
    assert bench._source_sha("no_such_kernel") is None


def test_the_digest_covers_the_shared_header(tmp_path, monkeypatch):
    """The digest is that of the kernel's file followed by gp_internal.h, so a
    change to the header alone invalidates the counters."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2308_13175_amd", "csrc")
    h = hashlib.sha256()
    for name in ("pull.hip", "gp_internal.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    assert bench._source_sha("k_query_grad") == h.hexdigest()
    with open(os.path.join(csrc, "pull.hip"), "rb") as f:
        assert bench._source_sha("k_query_grad") != hashlib.sha256(f.read()).hexdigest()

