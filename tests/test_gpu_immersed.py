"""Immersed Nitsche (cache_inverse; 2D also cache_matrix and cache_none): the obstacle surfaces as
no-slip Dirichlet boundaries of Eq. 5, imposed by the wall forms on the obstacle arcs (2D) or sphere
pieces (3D) of the cut cells; the HIP path against the oracle with the same option.

Both sides take the surface quadrature from the same reading and factorise the local blocks, which
may be indefinite here, by LU with partial pivoting (3D: 402 x 402 blocks at set-up). Tolerances follow test_gpu_parity: residual
componentwise 1e-13 (|b| + |L||x|); one or two sweeps relative 2-norm 1e-12 (measured up to 3.7e-13);
V-cycles 1e-9, bounded by the condition of the coarse solve (measured up to 1e-11); solves by the
oracle's residual of the GPU iterate.
"""
import dataclasses

import numpy as np
import pytest

from oracle.oracle import MODE_INVERSE, Oracle
from paper_2403_11636_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "2d_16_l3_s0": lambda: inputs.small_problem(2, 16, 3, seed=0),
    "2d_32_l3_s2": lambda: inputs.small_problem(2, 32, 3, seed=2, n_balls=3),
    "c1_32_l3": lambda: inputs.config1(32, 3),
    "2d_64_l4_discs": lambda: inputs.config2(0, n_cells=64, n_levels=4),
    "3d_8_l2_s0": lambda: inputs.small_problem(3, 8, 2, seed=0, n_balls=1, rmin=0.15, rmax=0.2),
    "3d_12_l2_s3": lambda: inputs.small_problem(3, 12, 2, seed=3, n_balls=2, rmin=0.08, rmax=0.14),
    # a sphere through the inflow face (its surface clipped by the box), and two spheres whose gap
    # lies inside one cell (that cell's surface terms come from both)
    "2d_16_edge_inflow": lambda: inputs.edge_problem(2, 16, 3, "inflow_wall"),
    "3d_8_edge_inflow": lambda: inputs.edge_problem(3, 8, 2, "inflow_wall"),
    "3d_8_edge_two": lambda: inputs.edge_problem(3, 8, 2, "two_in_cell"),
}

_cache = {}


def setup_case(name):
    if name not in _cache:
        from paper_2403_11636_amd import fcgmg
        p = dataclasses.replace(CASES[name](), immersed_nitsche=1)
        _cache[name] = (p, Oracle(p), fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE))
    return _cache[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_immersed_residual_parity(name):
    p, o, h = setup_case(name)
    plain = Oracle(dataclasses.replace(p, immersed_nitsche=0))
    for lev in range(h.n_levels):
        n = o.ndofs(lev)
        x = inputs.random_vector(n, 30 + lev)
        b = inputs.random_vector(n, 40 + lev)
        r_gpu = host(h.residual(dev(x), dev(b), lev))
        r_orc = o.residual(lev, x, b)
        bound = 1e-13 * (np.abs(b) + o.abs_matvec(lev, np.abs(x))) + 1e-300
        assert np.all(np.abs(r_gpu - r_orc) <= bound), (lev, np.max(np.abs(r_gpu - r_orc) / bound))
        # the immersed terms are present (the operator differs from the one without them)
        assert rel(r_orc, plain.residual(lev, x, b)) > 1e-6


@pytest.mark.parametrize("name", list(CASES))
def test_immersed_sweep_parity(name):
    p, o, h = setup_case(name)
    for lev, sweeps in ((h.fine, 1), (h.fine, 2), (max(h.fine - 1, 0), 2)):
        n = o.ndofs(lev)
        x = inputs.random_vector(n, 50 + sweeps)
        b = inputs.random_vector(n, 60 + sweeps)
        xg = dev(x)
        h.smooth(xg, dev(b), sweeps, lev)
        x_orc = o.smooth(lev, x, b, sweeps, p.omega)
        err = rel(host(xg), x_orc)
        print(f"{name} level {lev} sweeps {sweeps}: {err:.2e}")
        assert err <= 1e-12, err


@pytest.mark.parametrize("name", list(CASES))
def test_immersed_vcycle_and_solve(name):
    p, o, h = setup_case(name)
    b = o.rhs()
    xg = h.zeros()
    h.vcycle(xg, dev(b))
    x_orc = o.vcycle(np.zeros_like(b), b, mode=MODE_INVERSE)
    err = rel(host(xg), x_orc)
    print(f"{name} V-cycle: {err:.2e}")
    assert err <= 1e-9, err
    from paper_2403_11636_amd import fcgmg
    hk = fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE, solver=fcgmg.SOLVER_FGMRES, krylov_restart=30)
    x, it, relk, _, rc = hk.solve(dev(b), rtol=1e-8, max_iter=200)
    assert rc == 0 and relk <= 1e-8
    r = o.residual(o.fine, host(x), b)
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
    print(f"{name}: FGMRES {it} cycles")
    hk.close()


def test_immersed_mixed_precision_fgmres():
    # FP32 V-cycles (rounded from the FP64 LU rows) inside FP64 FGMRES: the oracle's FP64 residual of
    # the iterate meets the stopping test.
    from paper_2403_11636_amd import fcgmg
    p, o, _ = setup_case("2d_32_l3_s2")
    h = fcgmg.Hierarchy(p, fcgmg.CACHE_INVERSE, precision=fcgmg.PREC_MIXED, solver=fcgmg.SOLVER_FGMRES,
                        krylov_restart=30)
    b = o.rhs()
    x, it, relk, _, rc = h.solve(dev(b), rtol=1e-8, max_iter=200)
    assert rc == 0 and relk <= 1e-8
    r = o.residual(o.fine, host(x), b)
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
    h.close()


@pytest.mark.parametrize("policy", [1, 2])
@pytest.mark.parametrize("name", ["2d_16_l3_s0", "c1_32_l3"])
def test_immersed_matrix_and_none_policies(name, policy):
    # cache_matrix (stored blocks) and cache_none (blocks assembled on the fly, arcs included) with the
    # dense LU at every application: one and two sweeps against the oracle and the cache_inverse sweep.
    from paper_2403_11636_amd import fcgmg
    p, o, hi = setup_case(name)
    h = fcgmg.Hierarchy(p, policy)
    n = o.ndofs(o.fine)
    x = inputs.random_vector(n, 70)
    b = inputs.random_vector(n, 71)
    for sweeps in (1, 2):
        xg, xi = dev(x), dev(x)
        h.smooth(xg, dev(b), sweeps)
        hi.smooth(xi, dev(b), sweeps)
        x_orc = o.smooth(o.fine, x, b, sweeps, p.omega)
        err, err_inv = rel(host(xg), x_orc), rel(host(xg), host(xi))
        print(f"{name} policy {policy} sweeps {sweeps}: vs oracle {err:.2e}, vs cache_inverse {err_inv:.2e}")
        assert err <= 1e-12 and err_inv <= 1e-12, (err, err_inv)
    h.close()


@pytest.mark.parametrize("policy", [1, 2])
def test_immersed_3d_needs_cache_inverse(policy):
    from paper_2403_11636_amd import fcgmg
    p = dataclasses.replace(inputs.small_problem(3, 8, 2, seed=0, n_balls=1, rmin=0.15, rmax=0.2), immersed_nitsche=1)
    with pytest.raises(fcgmg.FcgmgError):
        fcgmg.Hierarchy(p, policy)
