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
