"""The off-line tuner on the GPU, over a small size range: the full sweep and
adaptive sampling both time every selectable variant, write plans the runtime
accepts, and the adaptive run samples no more sizes than the sweep."""
import json

import pytest

from paper_1405_2915_amd import autotune as at

pytestmark = pytest.mark.gpu


def test_full_and_adaptive_plans_load(skel, tmp_path):
    logs = []
    try:
        table, report = at.tune(10, 12, reps=1, log=logs.append)
        assert report["mode"] == "full" and len(logs) == 6 * 3
        for name, per_k in report["results"].items():
            assert sorted(per_k, key=int) == ["10", "11", "12"], name
            assert all(v > 0 for r in per_k.values() for v in r.values())
        atable, areport = at.tune(10, 12, reps=1, log=logs.append, adaptive=True)
        assert areport["mode"] == "adaptive"
        for name, ks in areport["sampled"].items():
            assert ks[0] == 10 and ks[-1] == 12 and len(ks) <= 3, (name, ks)
        summary, _ = at.compare_with_full(atable, report)
        assert set(summary) == set(report["results"])
        assert all(v["worst"] >= 1.0 for v in summary.values())
        json.dumps(areport)  # the report is plain data
        for t, nm in ((table, "full.plan"), (atable, "adaptive.plan")):
            path = tmp_path / nm
            at.write_plan(t, str(path), ["test"])
            skel.skel_load_plan(str(path))  # raises if the runtime rejects it
    finally:
        # the tuner cleared the plan: the default one is back for the tests
        # that follow
        skel.skel_init(0, "torch")
