"""Host-side checks of the autotuner's candidate schedules and of the shipped
gfx950 table (no GPU)."""
import json
import math
import os

import pytest

from paper_1408_4675_amd import autotune as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [16, 32, 48, 64, 80, 96, 128, 160, 192, 256, 512, 1024])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_candidates_factor_the_length(axis, n):
    cands = T.candidates(axis, n)
    assert cands
    for sched, tile in cands:
        assert math.prod(sched) == n, (sched, n)
        assert all(r in (2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20, 24, 25, 30, 32) for r in sched)
        assert tile in ((0, 4, 8, 16, 32) if axis == 0 else (0, 8, 16, 32))


@pytest.mark.parametrize("n", [16, 64, 128, 256, 1024])
def test_power_of_two_lengths_offer_every_fixed_width(n):
    """Each fixed engine (largest radix 4, 8 or 16) is among the candidates."""
    widths = {max(s) for s, _ in T.candidates(0, n) if max(s) <= 16}
    assert {4, 8, 16} <= widths


@pytest.mark.parametrize("n", [32, 64, 512, 1024])
def test_radix32_candidates_are_fixed_engine_plans(n):
    """Candidates with a radix-32 pass are radix-32 passes only (the schedules
    the 32-wide fixed engine runs): 32 and 1024 have one, 64 and 512 none."""
    s32 = [s for s, _ in T.candidates(1, n) if 32 in s]
    assert all(set(s) == {32} for s in s32)
    assert bool(s32) == (n in (32, 1024))


def test_shipped_table_is_well_formed():
    with open(os.path.join(ROOT, "paper_1408_4675_amd", "tuning", "gfx950.json")) as fh:
        tab = json.load(fh)
    assert tab
    for key, e in tab.items():
        arch, axis, n = key.split("|")
        assert arch == "gfx950" and axis in ("x", "y", "z")
        assert math.prod(e["radices"]) == int(n), key
        assert e["tile"] in (0, 4, 8, 16, 32)
