"""Both addressings of the odd AA step agree.  The odd step of FP16 and
26-velocity lattices addresses populations through 32-bit buffer offsets
while the population buffer spans less than 4 GiB and through 64-bit
addresses beyond.  A lattice periodic in z whose state does not depend on z
gives every z-plane the same values whatever its depth, so a lattice more
than 4 GiB deep must equal a 4-plane one, plane for plane: the interior
planes exercise the two inner paths against each other, the periodic end
planes the general path of both."""
import numpy as np
import pytest

from paper_1503_03337_amd import lbm, params

pytestmark = pytest.mark.gpu

NX = NY = 128
FACES = ("wall", "wall", "wall", "wall", "periodic", "periodic")
WALL_U = {"+y": (0.05, 0.0, 0.0)}  # a lid on +y moving along x


def lattice(q, storage, nz):
    # nearest rounding: the stochastic dither draws per node index and would
    # make planes differ
    return lbm.Lattice(q, NX, NY, nz, params.s_vec(q, 0.02), faces=FACES, wall_u=WALL_U,
                       storage=storage, pattern="aa", f16_rounding="nearest")


def plane(lat, z):
    return lat.macros_noalloc(z * NX * NY, NX * NY)


@pytest.mark.parametrize("q,storage,deep", [(18, "f16dev", 7400), (26, "f32", 2600)])
def test_odd_step_beyond_4gib_equals_a_shallow_lattice(q, storage, deep):
    kw = dict(faces=FACES, wall_u=WALL_U, storage=storage, pattern="aa")
    assert lbm.footprint_bytes(q, NX, NY, deep, **kw) > 1 << 32
    assert lbm.footprint_bytes(q, NX, NY, 4, **kw) < 1 << 32
    small, big = lattice(q, storage, 4), lattice(q, storage, deep)
    for lat in (small, big):
        lat.step(201)  # ends after an odd step
        lat.sync()
    ref = [plane(small, z) for z in range(4)]
    assert np.max(np.abs(ref[1][1])) > 1e-3  # the lid has driven a flow
    for zb, zs in ((1, 1), (deep // 2, 2), (deep - 2, 2), (0, 0), (deep - 1, 3)):
        p, u = plane(big, zb)
        assert np.array_equal(p, ref[zs][0]), (zb, zs)
        assert np.array_equal(u, ref[zs][1]), (zb, zs)
    small.close()
    big.close()
