"""Surrogate trees for generic meshes (Algorithm 7 with k-means splits and
the surrogate functional of Appendix A), built on the host by the library.

Pins: the tree is a proper partition with contiguous children and bounded
fanout; the library's epsilons equal the oracle's smallest conservative
epsilons; the oracle's exact descent over the tree finds exactly the flat
contact set (Lemma 1) while testing far fewer pairs."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from generic_mesh import two_tori_scene
from paper_2105_12415_amd import _abi, api


@pytest.fixture(scope="module")
def tori():
    return two_tori_scene()


def test_tree_structure(tori):
    scene, trees = tori
    for v, t, tree in trees:
        n_fine = len(t)
        sizes = tree["level_sizes"]
        n_sur = int(sizes[:-1].sum())
        assert sizes[-1] == n_fine and len(tree["tris"]) == n_sur + n_fine
        assert sorted(tree["fine_order"].tolist()) == list(range(n_fine))
        # fine triangles are the input triangles, in fine_order
        assert np.array_equal(tree["tris"][n_sur:], t[tree["fine_order"]])
        par = tree["parent"]
        offs = np.cumsum([0] + list(sizes))
        assert par[0] == -1 and sizes[0] == 1
        for l in range(1, len(sizes)):
            p = par[offs[l]:offs[l + 1]]
            lo = 0 if l == len(sizes) - 1 else offs[l - 1]
            assert np.all((p >= lo) & (p < offs[l])) and np.all(np.diff(p) >= 0)  # grouped by parent
        cnt = np.bincount(par[1:], minlength=n_sur)
        assert np.all((cnt >= 1) & (cnt <= 8))  # default fanout
        # a surrogate's children are all surrogates or all fine
        for s in range(n_sur):
            kids = np.nonzero(par == s)[0]
            assert np.all(kids >= n_sur) or np.all(kids < n_sur)
        # surrogate triangles are not degenerate
        V = tree["verts"][tree["tris"][:n_sur]]
        assert np.all(np.linalg.norm(np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]), axis=1) > 0)
        assert len(sizes) - 1 <= int(np.ceil(np.log(n_fine) / np.log(8))) + 3


def test_tree_eps_are_the_oracles_conservative_eps(tori):
    scene, trees = tori
    for v, t, tree in trees:
        h = api.build_hierarchy(tree["verts"], tree["tris"], tree["parent"], tree["level_sizes"], 0.05,
                                rel_slack=0.0, coord_scale=0.0)
        n_sur = int(tree["level_sizes"][:-1].sum())
        is_fine = np.arange(len(tree["tris"])) >= n_sur
        ref = oracle.surrogate_eps(tree["verts"], tree["tris"], tree["parent"], is_fine, 0.05)
        assert np.allclose(h["eps"], ref, rtol=0, atol=1e-12)


def test_lemma1_on_generic_mesh_trees(tori):
    scene, _ = tori
    r = oracle.descent(oracle.tree(scene))
    fs = oracle.fine_scene(scene)
    ref = oracle.find_contacts(fs)
    P = np.asarray(scene.pairs)
    key = lambda c, tb: {(int(a), int(b)) for a, b in zip(c["ti"], c["tj"])}
    # descent ids are global over all levels; map to fine-local ids
    T = oracle.tree(scene)
    got = {(int(a) - int(T.fine_begin[0]), int(b) - int(T.fine_begin[1])) for a, b in zip(r["ti"], r["tj"])}
    want = {(int(a), int(b)) for a, b in zip(ref["ti"], ref["tj"])}
    assert got == want and len(want) > 100
    assert r["tests_per_depth"].sum() < 0.01 * len(fs.tris) ** 2 / 4


def test_builder_validates_arguments():
    v, t, _, _ = sg.two_tori()[0]
    for bad in ({"fanout": 1}, {"fanout": 17}, {"alpha_area": 0.0}, {"beta_size": 1.0}):
        with pytest.raises(_abi.DemError):
            api.build_surrogate_tree(v, t, **bad)
    with pytest.raises(_abi.DemError):
        api.build_surrogate_tree(v, np.array([[0, 1, len(v)]], np.int32))
    small = api.build_surrogate_tree(v, t[:5])  # fewer triangles than the fanout: one surrogate
    assert list(small["level_sizes"]) == [1, 5]
