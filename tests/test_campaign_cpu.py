"""Host logic of staged campaigns (no GPU): the stage ranges."""

import math

import pytest

campaign = pytest.importorskip("paper_1705_08210_amd.campaign")


@pytest.mark.parametrize("n_v,n_stages", [(3, 1), (3, 5), (10, 3), (100, 7), (1024, 16),
                                          (1024, 1), (50, 48), (50, 200)])
def test_stage_bounds_cover_and_balance(n_v, n_stages):
    b = campaign.stage_bounds(n_v, n_stages)
    assert b[0][0] == 1 and b[-1][1] == n_v - 1
    assert all(a < e for a, e in b)
    assert all(b[k][1] == b[k + 1][0] for k in range(len(b) - 1))
    assert len(b) <= min(n_stages, n_v - 2)
    sizes = [sum(j * (n_v - 1 - j) for j in range(a, e)) for a, e in b]
    assert sum(sizes) == math.comb(n_v, 3)
    if len(b) > 1 and n_v >= 100:
        # no stage much larger than an equal share plus one slab
        share = math.comb(n_v, 3) / len(b)
        biggest_slab = max(j * (n_v - 1 - j) for j in range(1, n_v - 1))
        assert max(sizes) <= share + biggest_slab


def test_stage_bounds_degenerate():
    assert campaign.stage_bounds(2, 4) == []
    assert campaign.stage_bounds(0, 1) == []
