"""The allocation-free entry point lbm_macros_noalloc through the C ABI: the
same p and u as lbm_macros, bit for bit, on two calls in a row (the second
on a smaller lattice and range, so the shared static scratch holds the
first call's values when it starts), and sizes beyond its maximum or
outside the lattice rejected before any device work."""
import numpy as np
import pytest

from paper_1503_03337_amd import inputs, lbm, params

pytestmark = pytest.mark.gpu


def _lattice(q, dims, storage, seed):
    cfg = params.cavity(q, dims[0], 400.0, lid=0.1)
    lat = lbm.Lattice(q, *dims, cfg["s_vec"], faces=cfg["faces"], wall_u=cfg["wall_u"],
                      storage=storage, pattern="aa", F0=(1e-5, 0.0, 0.0))
    lat.set_f(inputs.random_populations(q, *dims, seed=seed))
    lat.step(3)  # odd parity: the swapped AA layout is read
    return lat


@pytest.mark.parametrize("storage", ("f32", "f64"))
def test_noalloc_macros_equal_lbm_macros_on_two_calls(storage):
    cap = lbm.NOALLOC_MAX_NODES
    big = _lattice(18, (80, 70, 50), storage, seed=71)      # 280,000 nodes
    small = _lattice(26, (37, 19, 11), storage, seed=72)    # 7,733 nodes
    assert big.N > cap
    # first call: a full-size range (the maximum) not starting at node 0
    n0 = big.N - cap - 1000
    p, u = big.macros_noalloc(n0, cap)
    pr, ur = big.macros()
    assert np.array_equal(p, pr.reshape(-1)[n0:n0 + cap])
    assert np.array_equal(u, ur.reshape(3, -1)[:, n0:n0 + cap])
    # second call: a smaller lattice and range, read whole
    p2, u2 = small.macros_noalloc(0, small.N)
    pr2, ur2 = small.macros()
    assert np.array_equal(p2, pr2.reshape(-1))
    assert np.array_equal(u2, ur2.reshape(3, -1))
    # a ragged tail of the big lattice again, after the small call
    p3, u3 = big.macros_noalloc(big.N - 77, 77)
    assert np.array_equal(p3, pr.reshape(-1)[-77:])
    assert np.array_equal(u3, ur.reshape(3, -1)[:, -77:])
    big.close()
    small.close()


def test_noalloc_macros_rejects_sizes_beyond_its_maximum():
    lat = _lattice(14, (80, 70, 50), "f32", seed=73)
    cap = lbm.NOALLOC_MAX_NODES
    for n0, count in ((0, cap + 1), (lat.N - 10, 11), (-1, 5), (0, -1)):
        with pytest.raises(lbm.LbmError) as e:
            lat.macros_noalloc(n0, count)
        assert e.value.code == lbm.EINVAL
    assert "exceeds" in str(pytest.raises(lbm.LbmError, lat.macros_noalloc, 0, cap + 1).value)
    p, u = lat.macros_noalloc(lat.N, 0)  # an empty range is fine
    assert p.size == 0 and u.shape == (3, 0)
    lat.close()
