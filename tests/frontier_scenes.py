"""Small hand-built hierarchies for the active-set (frontier) tests.

Particle A lies in the plane z = 0 with a surrogate tree given level by level;
particle B is one fine triangle that the tests move above A.  The triangle
numbering of every scene is the global one (particle by particle, coarsest
level first): listed in each builder's docstring so that the expected active
sets in the tests can be written out by hand.
"""
from __future__ import annotations

import numpy as np

import scenegen as sg

B_TRI = np.array([[0.2, 0.2, 0.0], [0.4, 0.2, 0.0], [0.2, 0.4, 0.0]])
NEAR = (0.0, 0.0, 0.05)   # B hovers 0.05 above A's first fine triangle: delta = 0.1
FAR = (0.0, 0.0, 10.0)


def _particle(tris_by_level, parents):
    verts = np.concatenate([np.asarray(t, np.float64).reshape(-1, 3) for lev in tris_by_level for t in lev])
    levels, k = [], 0
    for lev in tris_by_level:
        levels.append(np.arange(k, k + 3 * len(lev), dtype=np.int32).reshape(-1, 3))
        k += 3 * len(lev)
    return sg.Particle(body=verts, rot=np.eye(3), centre=np.zeros(3), levels=levels, parents=parents,
                       radius=1.0, subdiv=list(range(len(levels))))


def _scene(a: sg.Particle, dtype: str, where) -> sg.Scene:
    b = sg.Particle(body=B_TRI.copy(), rot=np.eye(3), centre=np.asarray(where, np.float64),
                    levels=[np.array([[0, 1, 2]], np.int32)], parents=[None], radius=1.0, subdiv=[0])
    return sg.Scene("frontier_tiny", [a, b], np.array([[0, 1]], np.int32), dtype)


def two_level(dtype: str = "f64", where=NEAR) -> sg.Scene:
    """A: S (0) with fine children a0 (1), a1 (2); B: b (3).  a0 lies under B,
    a1 two units away."""
    S = [[(-0.5, -0.5, 0), (4, -0.5, 0), (-0.5, 2, 0)]]
    kids = [[(0, 0, 0), (1, 0, 0), (0, 1, 0)], [(2, 0, 0), (3, 0, 0), (2, 1, 0)]]
    return _scene(_particle([S, kids], [None, np.array([0, 0], np.int32)]), dtype, where)


def three_level(dtype: str = "f64", where=NEAR) -> sg.Scene:
    """A: S (0); S0 (1), S1 (2); a00 (3), a01 (4) below S0 and a10 (5), a11 (6)
    below S1; B: b (7).  a00 lies under B; S1's subtree is four units away."""
    S = [[(0, 0, 0), (8, 0, 0), (0, 1, 0)]]
    mid = [[(0, 0, 0), (2.5, 0, 0), (0, 1, 0)], [(5, 0, 0), (8, 0, 0), (5, 1, 0)]]
    fine = [[(0, 0, 0), (1, 0, 0), (0, 1, 0)], [(1.5, 0, 0), (2.5, 0, 0), (1.5, 1, 0)],
            [(5, 0, 0), (6, 0, 0), (5, 1, 0)], [(7, 0, 0), (8, 0, 0), (7, 1, 0)]]
    return _scene(_particle([S, mid, fine], [None, np.array([0, 0], np.int32),
                                             np.array([0, 0, 1, 1], np.int32)]), dtype, where)


def move_b(scene: sg.Scene, where) -> None:
    scene.particles[1].centre = np.asarray(where, np.float64)
