"""Status codes of the solve forced from the host (no kernel is made to fail): non-convergence within
the iteration limit keeps the last iterate; a non-finite right-hand side is reported as such."""
import numpy as np
import pytest
import torch

from paper_2403_11636_amd import inputs

pytestmark = pytest.mark.gpu


def fcg():
    from paper_2403_11636_amd import fcgmg
    return fcgmg


@pytest.mark.parametrize("dim", [2, 3])
def test_iteration_limit_reports_noconv_and_keeps_the_iterate(dim):
    f = fcg()
    p = inputs.small_problem(2, 16, 3, seed=0) if dim == 2 else inputs.small_problem(3, 8, 2, seed=0)
    h = f.Hierarchy(p, f.CACHE_INVERSE)
    b = h.rhs()
    x, iters, rel, hist, rc = h.solve(b, rtol=1e-30, max_iter=1, raise_on_noconv=False)
    assert rc == f.E_NOCONV
    assert iters == 1 and 0 < rel < 1 and len(hist) == 2
    # the iterate left in x is one V-cycle from zero
    xv = h.zeros()
    h.vcycle(xv, b)
    torch.cuda.synchronize()
    assert torch.equal(x, xv)
    with pytest.raises(f.FcgmgError) as ei:
        h.solve(b, rtol=1e-30, max_iter=1)
    assert ei.value.code == f.E_NOCONV
    h.close()


@pytest.mark.parametrize("solver", ["gmg", "fgmres"])
def test_non_finite_right_hand_side_is_reported(solver):
    f = fcg()
    p = inputs.small_problem(2, 16, 3, seed=0)
    h = f.Hierarchy(p, f.CACHE_INVERSE, solver=f.SOLVER_GMG if solver == "gmg" else f.SOLVER_FGMRES)
    b = h.rhs()
    b[5] = float("nan")
    with pytest.raises(f.FcgmgError) as ei:
        h.solve(b, rtol=1e-8, max_iter=10)
    assert ei.value.code == f.E_NAN
    # the handle stays usable: a finite right-hand side solves afterwards
    b2 = h.rhs()
    x, iters, rel, _, rc = h.solve(b2, rtol=1e-8, max_iter=100)
    assert rc == f.OK and rel <= 1e-8 and np.isfinite(rel)
    h.close()
