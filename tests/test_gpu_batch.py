"""Batched V-cycles over independent 2D problems of different sizes and depths (fcgmg_batch_*):
every problem's result equals the one of its own hierarchy alone, bit for bit."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_11636_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def fcg():
    from paper_2403_11636_amd import fcgmg
    return fcgmg


def problems():
    return [
        inputs.small_problem(2, 16, 3, seed=0),
        inputs.small_problem(2, 32, 4, seed=1, n_balls=3, rmin=0.05, rmax=0.1),
        inputs.small_problem(2, 64, 3, seed=2, n_balls=4, rmin=0.03, rmax=0.08),
        inputs.config1(32, 3),
        inputs.batch_problem(0),
        inputs.batch_problem(5),
        inputs.small_problem(2, 8, 1, seed=3, n_balls=1, rmin=0.1, rmax=0.2),  # single level: coarse solve only
        inputs.small_problem(2, 40, 3, seed=2, bcs=(0,) * 6, n_balls=2),
    ]


def test_batched_vcycle_bitwise_equals_single():
    f = fcg()
    hs = [f.Hierarchy(p) for p in problems()]
    xs0 = [torch.from_numpy(inputs.random_vector(h.ndofs(), 80 + k)).cuda() for k, h in enumerate(hs)]
    bs = [h.rhs() for h in hs]
    bt = f.Batch(hs)
    xb = [x.clone() for x in xs0]
    bt.vcycle(xb, bs)
    bt.vcycle(xb, bs)
    for h, x0, x, b in zip(hs, xs0, xb, bs):
        xa = x0.clone()
        h.vcycle(xa, b)
        h.vcycle(xa, b)
        assert torch.equal(xa, x)
    bt.close()
    for h in hs:
        h.close()


def test_persistent_batched_vcycle_bitwise_equals_single():
    # persistent launches (tiles by ticket) give the bits of the one-tile-per-workgroup launches and
    # of each hierarchy alone; switched back, the default launches again
    f = fcg()
    probs = problems() + [inputs.batch_problem(k) for k in range(40, 72)]
    hs = [f.Hierarchy(p) for p in probs]
    xs0 = [torch.from_numpy(inputs.random_vector(h.ndofs(), 90 + k)).cuda() for k, h in enumerate(hs)]
    bs = [h.rhs() for h in hs]
    bt = f.Batch(hs)
    bt.set_persistent(True)
    xp = [x.clone() for x in xs0]
    for _ in range(3):
        bt.vcycle(xp, bs)
    bt.set_persistent(False)
    xd = [x.clone() for x in xs0]
    for _ in range(3):
        bt.vcycle(xd, bs)
    for k, (h, x0, b) in enumerate(zip(hs, xs0, bs)):
        assert torch.equal(xp[k], xd[k]), probs[k].name
        if k < len(problems()):
            xa = x0.clone()
            for _ in range(3):
                h.vcycle(xa, b)
            assert torch.equal(xa, xp[k]), probs[k].name
    bt.set_persistent(True)
    xs, its, rel, rc = bt.solve(bs, rtol=1e-8, max_iter=60)
    assert rc == f.OK and max(rel) <= 1e-8
    bt.set_persistent(False)
    xs2, its2, rel2, rc2 = bt.solve(bs, rtol=1e-8, max_iter=60)
    assert its == its2 and all(torch.equal(a, b) for a, b in zip(xs, xs2))
    with pytest.raises(f.FcgmgError):
        bt.set_persistent(2)
    bt.close()
    for h in hs:
        h.close()


def test_batched_solve_matches_single():
    f = fcg()
    probs = problems() + [inputs.batch_problem(k) for k in range(10, 30)]
    hs = [f.Hierarchy(p) for p in probs]
    bs = [h.rhs() for h in hs]
    bt = f.Batch(hs)
    xs, its, rel, rc = bt.solve(bs, rtol=1e-8, max_iter=60)
    assert rc == f.OK
    for p, h, b, x, it, r in zip(probs, hs, bs, xs, its, rel):
        xa, ita, rela, _, rca = h.solve(b, rtol=1e-8, max_iter=60, raise_on_noconv=False)
        # every problem converges, in the batch and alone (the oracle's cycle converges on each)
        assert r <= 1e-8 and rca == f.OK, (p.name, r, rca)
        # the norms are summed in another order than fcgmg_solve's, so a cycle may differ at the edge
        assert abs(it - ita) <= 1
        if it == ita:
            assert torch.equal(x, xa)
        # the oracle's FP64 residual of the batched iterate meets the tolerance
        o = Oracle(p)
        bh = b.cpu().numpy()
        res = o.residual(o.fine, x.cpu().numpy(), bh)
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(bh) * (1 + 1e-6), p.name
    bt.close()
    for h in hs:
        h.close()


def test_batch_rejects_unsupported_hierarchies():
    f = fcg()
    h3 = f.Hierarchy(inputs.small_problem(3, 8, 2, seed=0, n_balls=1, rmin=0.15, rmax=0.2))
    h2 = f.Hierarchy(inputs.small_problem(2, 16, 3, seed=0))
    for bad in ([h3], [h2, h2]):
        with pytest.raises(f.FcgmgError):
            f.Batch(bad)
    h3.close()
    h2.close()
