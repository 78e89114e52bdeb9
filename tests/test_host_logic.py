"""Host-side schedules that the solves are driven by (no GPU): the eps
schedule of Sec. 4.2 and the stage-to-level lists of the multilevel starts
(Sec. 5.3, with the reading that runs the schedule on the coarsest level)."""
import math
import os

import pytest

from paper_2507_23602_amd import warmstart
from paper_2507_23602_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def test_join_halves_widening(tmp_path):
    """The 64-bit join used to make descriptor pointers wave-uniform widens
    each signed 32-bit half through uint32_t: values whose low word has bit 31
    set (where a sign-extending cast corrupts the high word) come back intact.
    Compiled host-only with hipcc from the library's own device header."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    src = tmp_path / "join.cpp"
    src.write_text(r'''
#include "rsot_device.h"
#include <cstdio>
int main() {
    const uint64_t vals[] = {0x0ull, 0x80000000ull, 0x00007f12c0000010ull,
                             0xffffffff00000000ull, 0x00000000ffffffffull,
                             0x7fffffff80000001ull, 0xdeadbeefcafef00dull};
    int bad = 0;
    for (uint64_t v : vals) {
        const uint64_t r = join_halves((int)(uint32_t)v, (int)(uint32_t)(v >> 32));
        if (r != v) { std::printf("%llx -> %llx\n", (unsigned long long)v,
                                  (unsigned long long)r); ++bad; }
    }
    return bad;
}
''')
    exe = tmp_path / "join"
    csrc = os.path.join(ROOT, "paper_2507_23602_amd", "csrc")
    subprocess.run([hipcc, "--offload-host-only", "-x", "hip", "-I", csrc, str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
