"""Geometry of the seeded lattice generator (inputs shared by the oracle and
the library): the neighbour shells every crystal must have, for cubic and
orthorhombic supercells and for hcp in its orthorhombic cell."""
import numpy as np
import pytest

from paper_2201_04622_amd import inputs as I


def _shells(x, L, i, k):
    d = x - x[i]
    d -= L * np.rint(d / L)
    r = np.sort(np.sqrt((d ** 2).sum(1)))[1:]
    return r[:k]


@pytest.mark.parametrize("kind,cells,first,count,second", [
    ("bcc", (3, 4, 5), np.sqrt(3) / 2, 8, 1.0),
    ("fcc", (3, 3, 4), 1 / np.sqrt(2), 12, 1.0),
    ("hcp", (4, 3, 3), 1.0, 12, np.sqrt(2.0)),
])
def test_every_site_has_its_neighbour_shells(kind, cells, first, count, second):
    """Each site's nearest-neighbour distances (minimum image in the
    orthorhombic box) in units of a: bcc 8 at sqrt(3)/2 then 1; fcc 12 at
    1/sqrt(2) then 1; ideal hcp 12 at 1 then sqrt(2)."""
    a = 2.0
    r = I.Replica(kind, 0, a, 300.0, 5.0, 1, cells=cells)
    x, L = r.sites(), r.box
    assert x.shape == (len(I.BASIS[kind]) * int(np.prod(cells)), 3) == (r.natoms, 3)
    assert np.allclose(L, np.array(cells) * I.CELL[kind] * a)
    assert (x >= -1e-12).all() and (x < L + 1e-12).all()
    for i in range(0, len(x), max(1, len(x) // 17)):
        s = _shells(x, L, i, count + 1)
        assert np.allclose(s[:count], first * a, atol=1e-9), (kind, i, s)
        assert s[count] == pytest.approx(second * a, abs=1e-9)


def test_cubic_cells_keep_the_site_order():
    """A cube given as n or as (n, n, n) gives the same sites, in the order
    id = ((ix ny + iy) nz + iz) nb + b."""
    x = I.lattice_sites("fcc", 3, 3.0)
    assert np.array_equal(x, I.lattice_sites("fcc", (3, 3, 3), 3.0))
    assert np.allclose(x[4 * 5 + 2], (np.array([0, 1, 2]) + I.BASIS["fcc"][2]) * 3.0)
    r = I.Replica("bcc", 5, 2.5, 300.0, 5.0, 1)
    assert r.dims == (5, 5, 5) and r.natoms == 250 and np.allclose(r.box, 12.5)
