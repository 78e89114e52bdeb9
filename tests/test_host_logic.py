"""Host-side logic (no GPU): the eps schedule of Sec. 4.2, the stage-to-level
lists of the multilevel starts (Sec. 5.3, with the reading that runs the
schedule on the coarsest level), the 64-bit widening of wave-uniform halves,
and the shapes of the seeded workloads."""
import math
import os

import numpy as np
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


@pytest.mark.parametrize("refinement,order", [(2, 1), (2, 2), (2, 3), (3, 3)])
def test_gpu_size_workload_shapes_and_rule(refinement, order):
    """The App. C workload: (2^(r+1))^3 cubes of [-1, 1]^3 with order^3 points
    each and the ball target counts of its Table of problem sizes; the tensor
    Gauss rule integrates x^(2 order - 1) and lower exactly (moments of the
    uniform density on [-1, 1]: 1/3 for x^2, 1/5 for x^4), and the targets lie
    in the unit ball."""
    p = W.gpu_size(refinement, order)
    table = {(2, 1): 512, (2, 2): 4096, (2, 3): 13824, (3, 3): 110592}
    assert p.nq == table[(refinement, order)]
    assert p.n == {2: 507, 3: 3817}[refinement]
    assert abs(p.mu.sum() - 1.0) < 1e-14
    assert np.all(np.abs(p.x) < 1.0)
    assert np.all(np.linalg.norm(p.y, axis=1) <= 1.0)
    for k in range(3):
        assert abs((p.mu * p.x[:, k]).sum()) < 1e-14
        if 2 * order - 1 >= 2:
            assert abs((p.mu * p.x[:, k] ** 2).sum() - 1.0 / 3.0) < 1e-14
        if 2 * order - 1 >= 4:
            assert abs((p.mu * p.x[:, k] ** 4).sum() - 1.0 / 5.0) < 1e-14


def test_truncation_study_inputs():
    """The two densities of the truncation study share mesh, points and
    targets; only the source masses differ (uniform: equal cell volumes, so
    equal masses)."""
    c, u = W.trunc_study("custom"), W.trunc_study("uniform")
    assert c.nq == u.nq == 375000 and c.n == u.n == 14761
    assert np.array_equal(c.x, u.x) and np.array_equal(c.y, u.y)
    assert np.allclose(u.mu, 1.0 / u.nq, rtol=1e-12)
    assert not np.allclose(c.mu, u.mu)


def test_drivers_continue_from_a_stalled_solve():
    """The Lloyd and barycentre drivers take the best iterate of a solve
    that ends on RSOT_ERR_LINESEARCH (the noise floor) and re-raise any
    other error."""
    import numpy as np
    import pytest
    from paper_2507_23602_amd import barycenter, rsot, sphere

    class Fake:
        def __init__(self, code):
            self.code = code

        def solve(self, eps, psi0=None, tol=None):
            raise rsot.RsotError(self.code, "rsot_solve", psi=np.ones(3), info={"J": -1.0})

    for mod in (sphere, barycenter):
        psi, info = mod._solve(Fake(rsot.ERR_LINESEARCH), 1e-2, np.zeros(3), 1e-8)
        assert np.all(psi == 1.0) and info["J"] == -1.0
        with pytest.raises(rsot.RsotError):
            mod._solve(Fake(rsot.ERR_NONFINITE), 1e-2, np.zeros(3), 1e-8)
