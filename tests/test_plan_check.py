"""Host-only checks of the projector plans (no GPU): the forward projector's
fixed-point walk is replayed over every strip and staged row, and every LDS
read must fall inside its staged window, every skipped row must be empty."""
import numpy as np
import pytest

ct = pytest.importorskip("paper_1810_03275_amd")

GEOMS = [
    (64, 90, 96), (54, 37, 81), (48, 61, 50, 1.0, 1.3), (40, 33, 64, 1.0, 0.8), (96, 1, 140),
    (2, 3, 4), (128, 180, 192, 0.7, 0.7), (100, 45, 150), (48, 60, 72), (100, 4, 150),
    (64, 8, 96), (90, 180, 128, 1.0, 1.4), (90, 180, 128, 1.0, 0.75), (33, 720, 50),
    (512, 720, 768),
]


@pytest.mark.parametrize("geom", GEOMS, ids=[str(g) for g in GEOMS])
def test_plan_walk_in_bounds(geom):
    assert ct.plan_check(*geom) > 0


@pytest.mark.parametrize("shape", [(256, 358, 384), (384, 538, 576), (1024, 1440, 1536)])
def test_plan_walk_batched_shapes(shape):
    assert ct.plan_check(*shape) > 0


@pytest.mark.parametrize("seed,N", [(0, 17), (1, 90), (2, 200)])
def test_plan_walk_arbitrary_angles(seed, N):
    a = np.random.default_rng(seed).uniform(-np.pi, 2 * np.pi, N)
    assert ct.plan_check(64, N, 96, angles=a) > 0


def test_plan_check_rejects_bad_geometry():
    with pytest.raises(ct.CtpdError):
        ct.plan_check(1, 4, 8)


def test_plan_walk_largest_geometry():
    """2048^2, 2880 angles, 3072 bins: every (strip, row) step of the plan
    (5.7e9 steps, about 40 s on one core)."""
    assert ct.plan_check(2048, 2880, 3072) > 1e9
