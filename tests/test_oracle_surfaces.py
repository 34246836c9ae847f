"""Slabs with free surfaces (the defect extension of the summary section:
gamma = (F_surf - F_bulk) / A): geometry of the seeded slab input, and the
oracle's static surface energies pinned by what locality and symmetry fix.

The crystal is bcc at the synthetic potential's zero-pressure lattice
parameter; its (001) slab keeps x and y periodic and has empty space along z.
"""
import numpy as np
import pytest

from paper_2201_04622_amd import inputs as I
from paper_2201_04622_amd import surfaces as S

A0_BCC = 1.9646   # zero-pressure lattice parameter of the synthetic potential (0 K)
R_CUT = 5.3


def _pair(cells=(6, 6, 8), vacuum=8.0):
    bulk = I.Replica("bcc", 0, A0_BCC, 10.0, 50.0, 0, cells=cells)
    return bulk, S.slab(bulk, vacuum)


def test_slab_geometry():
    """A slab is the bulk supercell's sites in a box lengthened along z by the
    vacuum; both faces count in the area."""
    bulk, slab = _pair()
    assert np.array_equal(slab.sites(), bulk.sites())
    assert slab.natoms == bulk.natoms
    assert np.allclose(slab.box, bulk.box + np.array([0.0, 0.0, 8.0]))
    assert S.surface_area(slab) == pytest.approx(2.0 * bulk.box[0] * bulk.box[1])
    with pytest.raises(ValueError):
        S.slab(bulk, 0.0)
    arr = I.batch_arrays([bulk, slab])
    assert np.allclose(arr["box"][1], slab.box)


def test_interior_atoms_keep_the_bulk_energy(opot):
    """Atoms farther than the cutoff from both faces see a bulk environment,
    so their energies equal the bulk per-atom energy to rounding; atoms of the
    outer layers lose neighbours and each carries a positive excess."""
    bulk, slab = _pair()
    x = bulk.sites()
    eb = opot.eam(x, bulk.box)["e_atom"]
    es = opot.eam(x, slab.box)["e_atom"]
    assert np.allclose(eb, eb[0], rtol=0, atol=1e-11)   # a perfect crystal: every atom alike
    z = x[:, 2]
    top = (bulk.dims[2] - 0.5) * A0_BCC                # the last layer sits at nz a - a/2
    depth = np.minimum(z - 0.0, top - z)
    inner = depth > R_CUT + 1e-9
    assert inner.sum() > 0
    assert np.allclose(es[inner], eb[0], rtol=0, atol=1e-10)
    outer = depth < 0.25 * A0_BCC
    assert (es[outer] - eb[0] > 0.1).all()
    # the excess sits within the cutoff of a face
    assert np.allclose(es[depth > R_CUT + 1e-9], eb[0], atol=1e-10)


def test_vacuum_beyond_the_cutoff_changes_nothing(opot):
    """Once the empty space is wider than the cutoff no pair reaches across
    it: energies and forces do not depend on how much wider."""
    bulk, s1 = _pair(vacuum=R_CUT + 0.7)
    _, s2 = _pair(vacuum=2.0 * R_CUT + 1.0)
    x = bulk.sites()
    r1, r2 = opot.eam(x, s1.box), opot.eam(x, s2.box)
    assert r1["U"] == pytest.approx(r2["U"], rel=1e-13)
    assert np.allclose(r1["f"], r2["f"], atol=1e-11)
    # a vacuum inside the cutoff lets the faces interact through the boundary
    _, s3 = _pair(vacuum=0.5 * R_CUT)
    assert abs(opot.eam(x, s3.box)["U"] - r1["U"]) > 1.0


def test_relaxed_surface_energy(opot):
    """FIRE relaxation of the slab: the forces vanish, the relaxed excess is
    positive and below the unrelaxed one, the slab keeps its mirror symmetry
    about the middle plane (layer by layer), and x and y stay untouched (every layer is a
    square net of equivalent atoms, so lateral forces cancel)."""
    from oracle.minimize import fire

    bulk, slab = _pair(cells=(6, 6, 6))
    x = bulk.sites()
    A = S.surface_area(slab)
    Ub = opot.eam(x, bulk.box)["U"]
    g_unrelaxed = (opot.eam(x, slab.box)["U"] - Ub) / A
    xr, U, steps = fire(opot, x, slab.box, fmax=1e-6)
    g = (U - Ub) / A
    assert np.abs(opot.eam(xr, slab.box)["f"]).max() < 1e-6
    assert 0.0 < g < g_unrelaxed
    assert np.allclose(xr[:, :2], x[:, :2], atol=1e-9)
    # (001) layers l = 0 .. 2 nz - 1 at z = l a / 2; layer l mirrors layer 2 nz - 1 - l
    layer = np.rint(x[:, 2] / (0.5 * A0_BCC)).astype(int)
    nl = 2 * bulk.dims[2]
    dz = xr[:, 2] - x[:, 2]
    per_layer = np.array([dz[layer == l].mean() for l in range(nl)])
    assert np.allclose(dz, per_layer[layer], atol=1e-8)       # every atom of a layer alike
    assert np.allclose(per_layer, -per_layer[::-1], atol=1e-7)
    assert abs(per_layer[0]) > 1e-3   # the outer layers moved (outwards, for this potential)
