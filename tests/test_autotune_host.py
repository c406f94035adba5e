"""Host logic of the off-line tuner (no GPU): adaptive sampling of sizes,
the plan built from sampled sizes, and the comparison with a full sweep.

Adaptive sampling is the method Section II cites for spending fewer off-line
sample executions on a dispatch structure at a small loss of precision.  The
synthetic cost models below have known crossover sizes, so the tests can
check that the sampled plan switches exactly where the full sweep's does."""
import pytest

from paper_1405_2915_amd import autotune as at


def model(k):
    """Three variants with crossovers at log2 n = 15 (A -> B) and 23 (B -> C)."""
    n = 2.0 ** k
    return {"A": 1.0 + n / 2 ** 14,          # cheap start, steep
            "B": 2.5 + n / 2 ** 17,          # middle
            "C": 40.0 + n / 2 ** 20}         # expensive start, flattest


def run_bisection(measure, lo, hi, tol=0.05):
    b = at.Bisection(lo, hi, tol)
    while True:
        want = b.wanted()
        if not want:
            break
        for k in want:
            b.add(k, measure(k))
        if not b.step():
            break
    return b


def full_report(measure, lo, hi):
    return {"results": {"X": {str(k): measure(k) for k in range(lo, hi + 1)}},
            "dtypes": {"X": "f32"}}


def test_bisection_finds_the_crossovers_with_fewer_samples():
    b = run_bisection(model, 10, 28)
    assert len(b.res) < 19
    table = at.plan_from_report({"results": {"X": {str(k): r for k, r in b.res.items()}},
                                 "dtypes": {"X": "f32"}})
    full = at.plan_from_report(full_report(model, 10, 28))
    for k in range(10, 29):
        assert at.plan_choice(table, "X", k) == at.plan_choice(full, "X", k), k
    # the switch sizes themselves were sampled
    for k in range(11, 29):
        if at.plan_choice(full, "X", k) != at.plan_choice(full, "X", k - 1):
            assert k in b.res


def test_one_variant_everywhere_needs_only_the_ends():
    b = run_bisection(lambda k: {"A": 1.0 * k, "B": 2.0 * k}, 10, 28)
    assert sorted(b.res) == [10, 28]


def test_choice_within_tolerance_is_kept_across_the_interval():
    # B is 3% faster than A at the top end only: within 5%, so [10, 28] is
    # settled on A and nothing in between is sampled
    b = run_bisection(lambda k: {"A": 1.0, "B": 1.0 - 0.03 * (k - 10) / 18}, 10, 28)
    assert sorted(b.res) == [10, 28]


def test_excluded_variant_never_chosen():
    b = at.Bisection(10, 12, 0.05, exclude={"R3_atomic"})
    b.add(10, {"R3_atomic": 0.5, "R1": 1.0})
    b.add(12, {"R3_atomic": 0.5, "R1": 1.0})
    assert b.settled(10, 12)
    assert b.step() is False


def test_unsupported_variant_at_the_upper_end_splits():
    # the choice at the lower end is not selectable at the upper end (e.g. a
    # flat look-back limited in tiles): the interval is split down to unit width
    meas = lambda k: {"S5": 1.0, "S2": 2.0} if k <= 22 else {"S2": 2.0, "S3": 1.9}
    b = run_bisection(meas, 10, 28)
    assert 22 in b.res and 23 in b.res
    table = at.plan_from_report({"results": {"X": {str(k): r for k, r in b.res.items()}},
                                 "dtypes": {"X": "f32"}})
    assert at.plan_choice(table, "X", 22) == "S5"
    assert at.plan_choice(table, "X", 23) == "S3"


def test_compare_with_full_reports_the_slowdown():
    full = full_report(model, 10, 28)
    table = [("X", "f32", 10, "A", None)]  # A everywhere: slower past 2^15
    summary, ratios = at.compare_with_full(table, full)
    assert summary["X"]["sizes"] == 19
    assert ratios[("X", 10)] == pytest.approx(1.0)
    assert summary["X"]["worst"] > 10
    assert summary["X"]["over_tol"] == sum(
        1 for k in range(10, 29) if model(k)["A"] > 1.05 * min(model(k).values()))


def test_plan_choice_below_the_first_entry_is_none():
    assert at.plan_choice([("X", "f32", 12, "A", None)], "X", 11) is None
    assert at.plan_choice([("X", "f32", 12, "A", None)], "X", 12) == "A"
