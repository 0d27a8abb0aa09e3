"""Selection rule of the autotuner (host logic only, no GPU)."""
from paper_1408_1605_amd import autotune


def _row(ms, parity=True, **knobs):
    return dict(knobs, parity=parity, ms=ms if parity else None)


def test_pick_fastest_when_start_is_clearly_slower():
    table = [_row(5.0, ept=4), _row(4.0, ept=2), _row(3.0, ept=8, parity=False)]
    assert autotune._pick(table, {"ept": 4})["ept"] == 2


def test_pick_keeps_start_within_tie():
    table = [_row(5.05, ept=4), _row(5.0, ept=2)]
    assert autotune._pick(table, {"ept": 4}, tie=0.02)["ept"] == 4
    assert autotune._pick(table, {"ept": 4}, tie=0.005)["ept"] == 2


def test_pick_ignores_start_that_failed_parity():
    table = [_row(1.0, ept=4, parity=False), _row(5.0, ept=2)]
    assert autotune._pick(table, {"ept": 4})["ept"] == 2


def test_pick_none_without_passing_rows():
    assert autotune._pick([_row(1.0, ept=4, parity=False)], {"ept": 4}) is None
    assert autotune._pick([], {"ept": 4}) is None
