"""Bulk selection over a chain of calls (paper_1405_2915_amd.compose), on the
CPU with a synthetic cost: the chain's time depends on pairs of neighbouring
choices, so the best assignment for the chain differs from each call's own
best, and an unselectable variant must be skipped."""
from paper_1405_2915_amd import compose


def test_bulk_select_finds_the_chain_optimum():
    # call b's variant 1 is slower alone but makes call c's variant 1 cheap
    alone = {("a", 0): 1.0, ("a", 1): 1.2, ("b", 0): 1.0, ("b", 1): 1.1,
             ("c", 0): 2.0, ("c", 1): 1.9}
    calls = []

    def time_chain(asg):
        calls.append(dict(asg))
        if asg["a"] == 2:
            raise RuntimeError("not selectable")
        t = sum(alone[(k, v)] for k, v in asg.items())
        if asg["b"] == 1 and asg["c"] == 1:
            t -= 1.0  # the pair helps each other
        return t
    sites = {"a": [0, 1, 2], "b": [0, 1], "c": [0, 1]}
    start = {"a": 0, "b": 0, "c": 0}  # each call's own best
    best, rep = compose.bulk_select(time_chain, sites, start, passes=3)
    assert best == {"a": 0, "b": 1, "c": 1}
    assert rep["start_ms"] == 4.0 and abs(rep["final_ms"] - 3.0) < 1e-12
    assert all(t[1] != 2 for t in rep["trials"])  # the refused variant is skipped


def test_bulk_select_keeps_start_within_noise():
    def time_chain(asg):
        return 1.0 - (0.001 if asg["x"] == 1 else 0.0)  # 0.1 %: below min_gain
    best, _ = compose.bulk_select(time_chain, {"x": [0, 1]}, {"x": 0}, min_gain=0.003)
    assert best == {"x": 0}
