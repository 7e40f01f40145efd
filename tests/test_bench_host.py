"""CPU checks of bench.py's host logic: the staleness hash behind roofline.traffic
ignores comments but not code, committed counter readings are used only while
their kernels' code is unchanged, and every timed stage maps to kernel names."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_drops_comments_and_blank_lines_only():
    a = "int x = 1;  // one\n\n// a whole comment line\nint y = 2;\n"
    b = "int x = 1;\nint y = 2;  // two, reworded\n"
    c = "int x = 1;\nint y = 3;\n"
    assert bench.code_text(a) == bench.code_text(b) == "int x = 1;\nint y = 2;"
    assert bench.code_text(c) != bench.code_text(a)


def test_committed_traffic_is_current_or_reported_stale(tmp_path, monkeypatch):
    # every committed stage either matches the current code (used) or is reported
    # as None; a reading under a changed hash must come back as None
    for form in ("f32", "f64"):
        path = bench.traffic_path(form)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            t = json.load(fh)
        for stage, st in t["stages"].items():
            v = bench.stage_traffic(form, stage)
            if st["sha"] == bench.source_hash(st["source"]):
                assert v is not None and v > 0
            else:
                assert v is None
        stale = dict(t)
        stale["stages"] = {k: dict(v, sha="0" * 16) for k, v in t["stages"].items()}
        p = tmp_path / ("traffic_%s.json" % form)
        p.write_text(json.dumps(stale))
        monkeypatch.setattr(bench, "traffic_path", lambda f, p=p: str(p))
        for stage in stale["stages"]:
            assert bench.stage_traffic(form, stage) is None
        monkeypatch.undo()


def test_every_stage_has_kernels_in_its_source():
    # the name patterns must name kernels that the stated source defines
    for stage, (pats, src) in bench.STAGE_KERNELS.items():
        text = open(os.path.join(bench.CSRC, src)).read()
        kernels = [p.split("<")[0] for p in pats]
        assert any(("void %s(" % k) in text for k in kernels), stage
