"""The protein-like input generator: closed oriented manifold, charges inside, seeded."""
import numpy as np

from oracle import operator as O
from paper_1301_5914_amd import inputs


def test_molecule_surface_is_a_valid_closed_surface():
    p = inputs.molecule(20, seed=11)
    assert p.nf > 1000
    st = O.setup(p.xyz, p.nrm, p.tri)           # raises on a bad mesh
    amin, comps, euler = inputs.mesh_quality(p.xyz, p.tri)
    assert euler <= 2 * comps                       # chi = 2 - 2 g per component
    assert p.nv - p.nf // 2 == euler               # closed triangulation: 2E = 3F
    assert amin > 0.0
    # every charge (atom centre) is enclosed: solid-angle fraction 1
    np.testing.assert_allclose(O.solid_angle_fraction(st, p.qpos), 1.0, atol=2e-3)
    # integer net charge, normals unit and outward (on average along the position from the centre)
    assert abs(p.q.sum() - round(p.q.sum())) < 1e-12
    np.testing.assert_allclose(np.linalg.norm(p.nrm, axis=1), 1.0, atol=1e-12)


def test_molecule_is_seeded():
    a = inputs.molecule(10, seed=5)
    b = inputs.molecule(10, seed=5)
    np.testing.assert_array_equal(a.xyz, b.xyz)
    np.testing.assert_array_equal(a.tri, b.tri)
    np.testing.assert_array_equal(a.q, b.q)


def test_vertices_lie_on_the_density_isosurface():
    c, r, q = inputs.pack_atoms(12, inputs.protein_ball_radius(12), 3)
    xyz, nrm, tri = inputs.molecule_surface(c, r)
    ag = inputs._AtomGrid(c, r)
    rho, g = ag.eval(xyz, grad=True)
    np.testing.assert_allclose(rho, 1.0, atol=1e-8)
    np.testing.assert_allclose(nrm, -g / np.linalg.norm(g, axis=1, keepdims=True), atol=1e-12)


def test_atom_packing_respects_spacing():
    c, r, q = inputs.pack_atoms(200, 8.0, 9)
    d = np.linalg.norm(c[:, None] - c[None], axis=-1) + np.eye(200) * 10
    assert d.min() >= 1.4
    assert np.all(np.linalg.norm(c, axis=1) <= 8.0)
    assert np.all((r >= 1.2) & (r <= 2.0))
