"""fcgmg_smooth_noalloc, the sweep whose scratch lives in the library's static device array (no
allocation), against fcgmg_smooth through the C-ABI: the same iterate bit for bit (same kernels, same
arithmetic), on two calls in a row with the second on a smaller input, and a clear error for a level
larger than the array."""
import pytest

from paper_2403_11636_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def fcg():
    from paper_2403_11636_amd import fcgmg
    return fcgmg


def rand(n, seed):
    g = torch.Generator("cuda").manual_seed(seed)
    return torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5


def check_pair(h, calls):
    # calls: (level, sweeps) in order; each compared with fcgmg_smooth on a copy of the same input
    for k, (level, sweeps) in enumerate(calls):
        n = h.ndofs(level)
        x = rand(n, 100 + k)
        b = rand(n, 200 + k)
        x_ref = x.clone()
        h.smooth(x_ref, b, sweeps, level=level)
        x_na = x.clone()
        h.smooth_noalloc(x_na, b, sweeps, level=level)
        torch.cuda.synchronize()
        assert torch.equal(x_na, x_ref), (level, sweeps)
        assert not torch.equal(x_na, x)


@pytest.mark.parametrize("sweeps", [(2, 3), (1, 2)])
def test_noalloc_2d_cache_inverse_equals_smooth(sweeps):
    # 512^2 level (fused pairs ping-pong through the static array), then the 256^2 level
    f = fcg()
    h = f.Hierarchy(inputs.config2(0), f.CACHE_INVERSE)
    check_pair(h, [(h.fine, sweeps[0]), (h.fine - 1, sweeps[1])])
    h.close()


def test_noalloc_2d_cache_matrix_equals_smooth():
    f = fcg()
    h = f.Hierarchy(inputs.small_problem(2, 64, 3, seed=2, n_balls=4, rmin=0.03, rmax=0.08), f.CACHE_MATRIX)
    check_pair(h, [(h.fine, 2), (h.fine - 1, 1)])
    h.close()


def test_noalloc_3d_equals_smooth():
    f = fcg()
    h = f.Hierarchy(inputs.config3(0, n_cells=32, n_levels=4), f.CACHE_INVERSE)
    check_pair(h, [(h.fine, 2), (h.fine - 1, 2)])
    h.close()


def test_noalloc_rejects_a_level_larger_than_the_scratch():
    # 1536^2 cache_inverse: residual and second iterate need 2 x 3 x 1537^2 doubles, more than the
    # 12,582,912 of the array; the 768^2 level below fits and still matches fcgmg_smooth
    f = fcg()
    h = f.Hierarchy(inputs.config2(0, n_cells=1536, n_levels=9), f.CACHE_INVERSE)
    n = h.ndofs()
    with pytest.raises(f.FcgmgError) as ei:
        h.smooth_noalloc(rand(n, 1), rand(n, 2), 2)
    assert ei.value.code == f.E_ARG and "scratch" in str(ei.value)
    check_pair(h, [(h.fine - 1, 2)])
    h.close()
