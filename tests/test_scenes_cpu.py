"""Stand-in scenes and the protocol's host helpers (no GPU)."""
import numpy as np

from paper_2302_14344_amd import scenes as S
from paper_2302_14344_amd.protocol import accuracy_index, linear_fit


def test_beam_stand_in_shape():
    fs = S.beam_scene()
    # 20 pieces of 3 x 5 x 5 nodes: 0.5 x 0.05 x 0.05 m, 4500 DOF
    assert fs.n_sub == 20 and int(fs.sub_ndof.sum()) == 4500
    ext = fs.rest.max(0) - fs.rest.min(0)
    np.testing.assert_allclose(ext, [0.5, 0.05, 0.05], rtol=1e-12)
    # 19 shared faces of 25 node pairs, 20 pieces x 15 bottom nodes in contact
    kinds = np.bincount(fs.if_kind, minlength=2)
    assert kinds[0] == 19 * 25 and kinds[1] == 20 * 15
    np.testing.assert_array_equal(np.unique(fs.young), [1e7])
    np.testing.assert_array_equal(np.unique(fs.poisson), [0.45])
    # every tetrahedron positively oriented, six per lattice cube
    X = fs.rest[fs.tets]
    vol = np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])) / 6
    assert np.all(vol > 0) and len(vol) == 20 * 2 * 4 * 4 * 6
    np.testing.assert_allclose(vol.sum(), 0.5 * 0.05 * 0.05, rtol=1e-12)


def test_anisotropic_block_nodes_match_cubic_case():
    a = S.fem_scene(seed=5, blocks=(2, 2, 1), nodes_per_block=4)
    b = S.fem_scene(seed=5, blocks=(2, 2, 1), nodes_per_block=(4, 4, 4))
    np.testing.assert_array_equal(a.tets, b.tets)
    np.testing.assert_array_equal(a.rest, b.rest)
    np.testing.assert_array_equal(a.if_node, b.if_node)


def test_linear_fit_and_index():
    x = np.array([1.0, 2.0, 4.0, 8.0])
    f = linear_fit(x, 3.0 + 0.5 * x)
    assert abs(f["slope"] - 0.5) < 1e-12 and abs(f["intercept"] - 3.0) < 1e-12 and abs(f["r2"] - 1.0) < 1e-12
    g = linear_fit([0.0, 1.0, 2.0], [0.0, 1.0, 0.0])
    assert abs(g["r2"]) < 1e-12
    assert accuracy_index([1e-3, 1e-5]) == 4.0


def test_mixed_scene_shape_and_gaps():
    import oracle as O
    sc = S.mixed_scenes()
    # 64 scenes of 64 boxes (4096) and one seven-link arm each
    assert sc.n_scenes == 64 and sc.n_bodies == 64 * (64 + 7) and sc.n_sub == 64 * 65
    assert int(sc.sub_ndof.max()) == 42 and np.all(np.sort(np.unique(sc.sub_ndof)) == [6, 42])
    sizes = 2 * sc.half[sc.sub_ndof[sc.body_sub] == 6]
    assert sizes.min() >= 0.05 and sizes.max() <= 0.3
    # every contact starts open (gap >= 0), none further than the tallest box
    A, b, J, e = O.rigid_assemble(sc)
    eoff = np.concatenate([[0], np.cumsum(sc.if_dim)])
    gaps = np.array([e[eoff[j]] * sc.dt for j in range(sc.n_if) if sc.if_kind[j] == S.KIND_CONTACT])
    assert gaps.min() >= 0.0 and gaps.max() < 0.3
    two = np.sum((np.asarray(sc.if_kind) == S.KIND_CONTACT) & (np.asarray(sc.if_nsub) == 2))
    assert two == 64 * (32 * 4 + (7 * 4 + 8 * 3) + 1)
    # the arm's joint controllers are folded into the arm subsystem
    assert np.sum(sc.link_if < 0) == 64 * 6


def test_stir_stand_in_shape_and_gaps():
    import oracle as O
    sc = S.stir_scene()
    # 216 spheres of 1 cm and 4 g, each a subsystem, and the arm with its stirrer: 217
    assert sc.n_sub == 217 and int(sc.sub_ndof.sum()) == 216 * 6 + 8 * 6
    sph = np.nonzero(np.isclose(sc.mass, 0.004))[0]
    assert len(sph) == 216
    np.testing.assert_allclose(sc.inertia[sph], 0.4 * 0.004 * 1e-4, rtol=1e-12)
    assert np.all(sc.link_type[np.asarray(sc.link_if) >= 0][:10] == S.LINK_SPHERE)
    A, b, J, e = O.rigid_assemble(sc)
    eoff = np.concatenate([[0], np.cumsum(sc.if_dim)])
    gaps = np.array([e[eoff[j]] * sc.dt for j in range(sc.n_if) if sc.if_kind[j] == S.KIND_CONTACT])
    assert gaps.min() >= 0.0
    # every joint and ball joint closed at the start
    eq = [np.abs(e[eoff[j]:eoff[j + 1]]).max() for j in range(sc.n_if) if sc.if_kind[j] == S.KIND_EQUALITY]
    assert max(eq) < 1e-12
