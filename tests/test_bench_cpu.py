"""Host logic of bench.py: the measured-traffic lookup and the comment-
insensitive hash of the kernel sources it is keyed on."""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _args(**kw):
    a = dict(workload="swiss_roll_100k", precision="mixed", cheb_iterates="fp32",
             cheb_degree=128, eps_tol=None)
    a.update(kw)
    return argparse.Namespace(**a)


def _recorded_hash(name):
    with open(os.path.join(bench.ROOT, "profiles", name)) as fh:
        for line in fh:
            if line.startswith("kernel_sources_sha256:"):
                return line.split(":", 1)[1].strip()
    return None


def test_traffic_only_from_the_matching_summary(monkeypatch):
    """Each committed summary serves only its own workload and configuration
    while the kernel sources still hash to the value it records; any other
    run reports no traffic."""
    for (wl, prec, it), name in bench.TRAFFIC_FILES.items():
        assert os.path.exists(os.path.join(bench.ROOT, "profiles", name)), name
        rec = _recorded_hash(name)
        assert rec
        monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None, rec=rec: rec)
        t = bench.measured_traffic(_args(workload=wl, precision=prec, cheb_iterates=it))
        assert t is not None and t > 0, (wl, prec, it)
        monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "0" * 64)
        assert bench.measured_traffic(_args(workload=wl, precision=prec, cheb_iterates=it)) is None
    monkeypatch.undo()
    assert bench.measured_traffic(_args(workload="square_2k")) is None
    assert bench.measured_traffic(_args(precision="fp64")) is None
    assert bench.measured_traffic(_args(cheb_degree=96)) is None
    assert bench.measured_traffic(_args(eps_tol=1e-8)) is None
    assert bench.measured_traffic(_args(workload="batch")) is None


def test_traffic_void_after_a_code_change():
    base = bench.kernel_source_hash()
    texts = []
    for f in bench.KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            texts.append(fh.read())
    assert bench.kernel_source_hash(texts) == base
    # comments do not count, code does
    assert bench.kernel_source_hash([t + "\n// note\n" for t in texts]) == base
    assert bench.kernel_source_hash([texts[0] + "\nint x;\n"] + texts[1:]) != base
