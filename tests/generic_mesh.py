"""Scenes of generic meshes whose surrogate trees come from the library's
builder (dem_build_surrogate_tree): the trees are inputs of the tests; the
oracle checks them (surrogate epsilons, Lemma 1) and decides the contacts
from the fine meshes alone."""
import numpy as np

import scenegen as sg
from paper_2105_12415_amd import api


def particle_from_tree(tree, rot, centre, radius):
    L = tree["levels"]
    offs = np.cumsum([0] + [len(l) for l in L])
    parents = [None] + [tree["parent"][offs[l]:offs[l + 1]] for l in range(1, len(L))]
    return sg.Particle(body=tree["verts"], rot=rot, centre=centre, levels=L, parents=parents,
                       radius=radius, subdiv=[], parents_absolute=True)


def two_tori_scene(dtype="f32", **opts):
    parts, trees = [], []
    for v, t, rot, c in sg.two_tori():
        tree = api.build_surrogate_tree(v, t, **opts)
        trees.append((v, t, tree))
        parts.append(particle_from_tree(tree, rot, c, 1.35))
    return sg.Scene("two_tori", parts, np.array([[0, 1]], np.int32), dtype), trees
