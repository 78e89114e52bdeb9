"""Host-side schedules that the solves are driven by (no GPU): the eps
schedule of Sec. 4.2 and the stage-to-level lists of the multilevel starts
(Sec. 5.3, with the reading that runs the schedule on the coarsest level)."""
import math

import pytest

from paper_2507_23602_amd import warmstart
from paper_2507_23602_amd import workloads as W


@pytest.mark.parametrize("eps", [1e-3, 2.5e-3, 1e-2, 0.07, 0.1, 0.3])
def test_eps_schedule_halves_down_from_at_most_eps0(eps):
    """eps * 2^K, ..., 2 eps, eps with the largest K such that eps * 2^K <= 0.1."""
    s = warmstart.eps_schedule(eps)
    assert s[-1] == eps
    assert all(a == 2.0 * b for a, b in zip(s, s[1:]))
    assert s[0] <= 0.1 * (1 + 1e-12) or len(s) == 1
    assert len(s) == 1 or 2.0 * s[0] > 0.1
    if eps >= 0.1:
        assert s == [eps]


def test_eps_schedule_of_the_3d_benchmark():
    assert warmstart.eps_schedule(1e-3) == pytest.approx(
        [0.064, 0.032, 0.016, 0.008, 0.004, 0.002, 0.001], rel=0, abs=1e-15)


def test_blob_family_multilevel_stages():
    """The whole schedule on the coarsest level, then the final eps alone on
    the two finer levels."""
    for eps in (1e-3, 4e-3, 0.05):
        E, lev = warmstart._ml_stages(eps)
        sched = warmstart.eps_schedule(eps)
        assert E == sched + [eps, eps]
        assert lev == [0] * len(sched) + [1, 2]


def test_disk_workload_stage_lists():
    """Stage lists of the disk workload: default (schedule on level 0, the
    final eps on levels 1-3) and the spread reading (stages over all four
    levels); levels never decrease and every level is visited."""
    c = W.config3(rings=6, n_targets=64, target_levels=(8, 16, 32, 64))
    sched = [0.1 * 2.0 ** (-k) for k in range(10)] + [1e-4]
    assert c["eps"] == sched + [1e-4] * 3
    assert c["level"] == [0] * len(sched) + [1, 2, 3]
    assert c["eps_spread"] == sched
    lv = c["level_spread"]
    assert len(lv) == len(sched)
    assert lv == sorted(lv) and set(lv) == {0, 1, 2, 3}
    assert lv[-1] == 3 and lv[-2] == 3          # final eps first reached on the finest level
    assert all(math.isclose(a, 2 * b) for a, b in zip(sched[:9], sched[1:10]))
