"""Pin of the oracle's V-cycle and standalone solve (Sec. 3 and the solver settings of Sec. 4).

The oracle's cycle is compared with a dense numpy composition of parts that are pinned on their own:
  * the smoother operator S = sum_i Rt_i^T omega L_i^{-1} R_i of Eq. (15), built densely from the
    structural pattern of each level operator (the brute-force sweep pin);
  * the Q1 interpolation P written as Kronecker products of the 1D two-grid interpolation (it
    reproduces linear fields), and the restriction R = P^T of Eq. (13) with the transfer T the
    identity on one process;
  * the coarsest solve by numpy's dense solver, bordered with sum(p) = 0 when the operator has the
    constant-pressure null space.
The level operators themselves come from the oracle's assembly, which the element, invariant and
manufactured-solution pins cover. The cycle is: nu1 sweeps of Eq. (14), restriction of the residual
taken after them, the coarse correction from a zero initial guess (one recursive call), its
prolongation, nu2 sweeps. nu1 != nu2 and a non-zero initial iterate make swapped sweep counts, a
residual taken before pre-smoothing, a non-zero coarse guess or an extra sweep visible: the test
checks that each of those variants of the numpy cycle differs from the oracle's.
"""
import numpy as np
import pytest

from oracle.oracle import MODE_INVERSE, MODE_LU, Oracle
from paper_2403_11636_amd import inputs


def interp_1d(nc):
    """Two-grid linear interpolation on [0, 1]: nc coarse cells -> 2 nc fine cells."""
    P = np.zeros((2 * nc + 1, nc + 1))
    for i in range(2 * nc + 1):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, (i - 1) // 2] = 0.5
            P[i, (i + 1) // 2] = 0.5
    return P


def prolongation(d, nc):
    """Q1 interpolation of all d+1 fields, nodes lexicographic with x fastest."""
    P1 = interp_1d(nc)
    Pn = P1
    for _ in range(1, d):
        Pn = np.kron(P1, Pn)  # the new (slower) axis goes to the left factor
    return np.kron(np.eye(d + 1), Pn)


def dense_smoother(o, level, omega):
    """S of Eq. (15) from the structural pattern of L (all in-grid couplings, numerical zeros too)."""
    rows, cols, _ = o.coo(level)
    n = o.ndofs(level)
    N = o.nnodes(level)
    d = o.d
    A = o.matrix(level).toarray()
    pat = np.zeros((n, n), bool)
    pat[rows, cols] = True
    S = np.zeros((n, n))
    for i in range(N):
        pi = d * N + i
        pp = np.nonzero(pat[pi, d * N:])[0] + d * N
        vel = np.nonzero(pat[pp, :d * N].any(axis=0))[0]
        Si = np.r_[vel, pp]
        Inv = np.linalg.inv(A[np.ix_(Si, Si)])
        for f in range(d + 1):
            k = int(np.nonzero(Si == f * N + i)[0][0])
            S[f * N + i, Si] += omega * Inv[k, :]
    return A, S


class DenseGMG:
    def __init__(self, o, omega):
        self.o = o
        self.d = o.d
        self.A, self.S = [], []
        for lev in range(o.nlev):
            A, S = dense_smoother(o, lev, omega)
            self.A.append(A)
            self.S.append(S)
        self.P = [None] + [prolongation(o.d, o.prob.level_cells(lev - 1)) for lev in range(1, o.nlev)]
        A0 = self.A[0]
        self.bordered = o.bordered()
        if self.bordered:
            N0 = o.nnodes(0)
            e = np.zeros(A0.shape[0])
            e[self.d * N0:] = 1.0
            A0 = np.block([[A0, e[:, None]], [e[None, :], np.zeros((1, 1))]])
        self.A0 = A0

    def coarse(self, b):
        if self.bordered:
            return np.linalg.solve(self.A0, np.r_[b, 0.0])[:-1]
        return np.linalg.solve(self.A0, b)

    def sweep(self, lev, x, b):
        return x + self.S[lev] @ (b - self.A[lev] @ x)

    def vcycle(self, lev, x, b, nu1, nu2, variant=None):
        if lev == 0:
            return self.coarse(b)
        x = x.copy()
        r_before = b - self.A[lev] @ x
        for _ in range(nu1 + (1 if variant == "extra_sweep" else 0)):
            x = self.sweep(lev, x, b)
        r = r_before if variant == "residual_before" else b - self.A[lev] @ x
        bc = self.P[lev].T @ r
        xc0 = np.zeros_like(bc)
        if variant == "nonzero_coarse_guess":
            xc0 = self.P[lev].T @ x
        xc = self.vcycle(lev - 1, xc0, bc, nu1, nu2, variant)
        x = x + self.P[lev] @ xc
        for _ in range(nu2):
            x = self.sweep(lev, x, b)
        return x

    def solve(self, b, rtol, max_iter, nu1, nu2):
        lev = len(self.A) - 1
        x = np.zeros_like(b)
        hist = [np.linalg.norm(b - self.A[lev] @ x)]
        it = 0
        while it < max_iter:
            x = self.vcycle(lev, x, b, nu1, nu2)
            it += 1
            hist.append(np.linalg.norm(b - self.A[lev] @ x))
            if hist[-1] <= rtol * hist[0]:
                break
        return x, it, np.array(hist)


CASES = {
    # 2D, three levels (8 / 4 / 2 cells), a disc crossing cells of every level, inflow and outflow
    "2d_8_l3": lambda: inputs.Problem(dim=2, n_cells=8, n_levels=3, balls=np.array([[0.41, 0.56, 0.0, 0.21]]),
                                      bcs=(1, 2, 0, 0, 0, 0), alpha_fict=1e-3, force=1),
    # 2D, three levels, all walls Dirichlet and no obstacle: the coarsest solve is bordered
    "2d_8_l3_bordered": lambda: inputs.Problem(dim=2, n_cells=8, n_levels=3, balls=np.zeros((0, 4)),
                                               bcs=(0,) * 6, force=1),
    # 2D, four levels (16 / 8 / 4 / 2 cells), two discs with the workloads' alpha_f = 1e-8
    "2d_16_l4": lambda: inputs.small_problem(2, 16, 4, seed=0),
    # 3D, two levels (4 / 2 cells), one sphere
    "3d_4_l2": lambda: inputs.Problem(dim=3, n_cells=4, n_levels=2, balls=np.array([[0.45, 0.52, 0.48, 0.27]]),
                                      bcs=(1, 2, 0, 0, 0, 0), alpha_fict=1e-3, force=1),
}

_dense = {}


def setup(name):
    if name not in _dense:
        p = CASES[name]()
        o = Oracle(p)
        _dense[name] = (p, o, DenseGMG(o, p.omega))
    return _dense[name]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("nu1,nu2", [(1, 2), (2, 1), (2, 2)])
@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_equals_dense_composition(name, nu1, nu2):
    p, o, g = setup(name)
    n = o.ndofs(o.fine)
    x0 = inputs.random_vector(n, 3)
    b = inputs.random_vector(n, 4) if not o.bordered() else o.rhs()
    ref = g.vcycle(o.fine, x0, b, nu1, nu2)
    for mode in (MODE_LU, MODE_INVERSE):
        got = o.vcycle(x0, b, nu1=nu1, nu2=nu2, mode=mode)
        assert rel(got, ref) <= 1e-12, (mode, rel(got, ref))


@pytest.mark.parametrize("name", ["2d_8_l3", "2d_16_l4", "3d_4_l2"])
def test_vcycle_pin_rejects_plausible_mistakes(name):
    # each wrong composition must be far (1000x the tolerance) from the oracle's cycle, so the 1e-12 pin
    # above detects it
    p, o, g = setup(name)
    n = o.ndofs(o.fine)
    x0 = inputs.random_vector(n, 3)
    b = inputs.random_vector(n, 4)
    got = o.vcycle(x0, b, nu1=1, nu2=2, mode=MODE_LU)
    wrong = {
        "swapped_nu": g.vcycle(o.fine, x0, b, 2, 1),
        "residual_before": g.vcycle(o.fine, x0, b, 1, 2, "residual_before"),
        "nonzero_coarse_guess": g.vcycle(o.fine, x0, b, 1, 2, "nonzero_coarse_guess"),
        "extra_sweep": g.vcycle(o.fine, x0, b, 1, 2, "extra_sweep"),
    }
    if o.nlev == 2:
        del wrong["nonzero_coarse_guess"]  # the direct coarsest solve ignores its initial guess
    for what, w in wrong.items():
        assert rel(got, w) > 1e-9, what


@pytest.mark.parametrize("name", list(CASES))
def test_solve_equals_dense_loop(name):
    # standalone GMG (Sec. 4): same iteration count and the same residual history, cycle by cycle
    p, o, g = setup(name)
    b = o.rhs()
    for nu1, nu2 in ((2, 2), (1, 2)):
        x_ref, it_ref, hist_ref = g.solve(b, 1e-8, 60, nu1, nu2)
        x, it, relres, hist, rc = o.solve(b, rtol=1e-8, max_iter=60, mode=MODE_INVERSE, nu1=nu1, nu2=nu2)
        assert rc == 0 and it == it_ref, (it, it_ref)
        assert np.all(np.abs(hist - hist_ref) <= 1e-11 * hist_ref[0]), np.max(np.abs(hist - hist_ref)) / hist_ref[0]
        assert abs(relres - hist_ref[-1] / hist_ref[0]) <= 1e-11
        assert rel(x, x_ref) <= 1e-10
