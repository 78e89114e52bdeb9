"""rsot_dual_eval_noalloc (the dense evaluation with its partials in a static
device array) against rsot_dual_eval, through the C ABI: bit for bit where the
default segmentation fits the array, within the mixed-precision bounds
(objective 1e-9 relative, gradient e_g <= 1e-6) where the coarser one is
used, and on calls in a row whose inputs shrink, so contents left in the
array by an earlier call cannot leak into a later one."""
import sys

import numpy as np
import pytest

from paper_2507_23602_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_matches_dual_eval_on_shrinking_calls():
    import torch
    from paper_2507_23602_amd import rsot
    cases = [("cube 48^3 x 24, 65,536 targets (coarse split)", W.cube_mixture(48, 65536, 1e-3),
              False),
             ("cube 12^3 x 24, 2,048 targets", W.cube_mixture(12, 2048, 1e-3), True),
             ("square 32 x 32 x 6, 256 targets", W.config1(), True)]
    for name, p, exact in cases:
        _say(f"noalloc: {name}: nq={p.nq} n={p.n}")
        prob = rsot.Problem(torch.as_tensor(p.x, device="cuda"),
                            torch.as_tensor(p.mu, device="cuda"),
                            torch.as_tensor(p.y, device="cuda"),
                            torch.as_tensor(p.nu, device="cuda"))
        psi = torch.as_tensor(W.random_psi(5, p.n, p.eps), device="cuda")
        a = prob.dual_eval(psi, p.eps)
        ga = a.grad.clone()
        b = prob.dual_eval_noalloc(psi, p.eps)
        gb = b.grad.cpu().numpy()
        g = ga.cpu().numpy()
        eg = float(np.max(np.abs(gb - g) / (p.nu + g + p.nu)))
        ej = abs(b.J - a.J) / abs(a.J)
        _say(f"  J {a.J:.15e} vs {b.J:.15e} (rel {ej:.1e}), e_g {eg:.1e}")
        assert b.info["kept_pairs"] == a.info["kept_pairs"] == p.nq * p.n
        if exact:
            assert b.J == a.J and np.array_equal(gb, g)
        else:
            assert ej <= 1e-9 and eg <= 1e-6
        c = prob.dual_eval_noalloc(psi, p.eps, want_grad=False)
        assert c.J == b.J and c.grad is None
        prob.close()


def test_noalloc_rejections():
    import torch
    from paper_2507_23602_amd import rsot
    # partials beyond the static array even at the coarsest split
    p = W.cube_mixture(64, 64, 1e-3)
    prob = rsot.Problem(p.x, p.mu, p.y, p.nu)
    psi = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    with pytest.raises(rsot.RsotError) as e:
        prob.dual_eval_noalloc(psi, p.eps)
    assert e.value.code == rsot.ERR_OOM
    prob.close()
    # truncated rules need run-time-sized lists: rejected
    q = W.config1()
    prob = rsot.Problem(q.x, q.mu, q.y, q.nu, truncation="tile")
    with pytest.raises(rsot.RsotError) as e:
        prob.dual_eval_noalloc(torch.zeros(q.n, dtype=torch.float64, device="cuda"), q.eps)
    assert e.value.code == rsot.ERR_INVALID_ARG
    prob.close()
