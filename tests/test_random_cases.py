"""The randomized parity sweep's cases are valid problems: the oracle
accepts every one and runs it, or stops at a non-finite mass."""
import pytest

from oracle import core as ora
from tests._random_cases import random_case

N_CASES = 24
STEPS = 60


@pytest.mark.parametrize("k", range(N_CASES))
def test_oracle_accepts_random_case(k):
    p, tile_w, tile_h = random_case(k)
    assert tile_w in (64, 128, 256) and 1 <= tile_h <= 20
    o = ora.Oracle(p)
    try:
        o.step(STEPS)
    except ora.OracleError:
        assert 0 < o.t <= STEPS


N_OPEN = 12
OPEN_STEPS = 100


@pytest.mark.parametrize("k", range(N_OPEN))
def test_oracle_accepts_random_open_case(k):
    from tests._random_cases import random_open_case
    p, tile_w, tile_h = random_open_case(k)
    assert p.open_x and tile_w in (64, 128, 256) and 1 <= tile_h <= 20
    o = ora.Oracle(p)
    o.step(OPEN_STEPS)
    assert o.wall_force()[0] != 0.0
