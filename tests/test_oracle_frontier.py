"""Pins of the oracle's persistent active sets (Section 5.3, Algorithm 6 in
the pairwise reading, with the memory set of its implementation note).

The expected active sets of the two hand-built hierarchies are worked out
from the rules alone (which pairs are in range follows from the geometry in
``frontier_scenes``); the sphere tests check properties any correct
implementation has: the active pairs partition the fine pairs at every step,
at most one level is unfolded per step, a fixed point reports exactly the
all-pairs contact set (Lemma 1), separation narrows one level per step, and
the memory set keeps pairs that came back from being removed again.
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle.frontier import Frontier
import frontier_scenes as fsc


def leaves_abf(f: Frontier):
    return [tuple(int(v) for v in r[:3]) for r in f.leaves()]


def contacts_ab(r):
    return sorted(zip(r["a"].tolist(), r["b"].tolist()))


def test_two_level_hand_sequence():
    sc = fsc.two_level()
    f = Frontier(oracle.tree(sc))
    assert leaves_abf(f) == [(0, 3, 0)]
    # (position of B, contacts of the step, active set after it, unfolded, narrowed)
    script = [
        (fsc.NEAR, [], [(1, 3, 0), (2, 3, 0)], 1, 0),   # S in range: widen one level
        (fsc.NEAR, [(1, 3)], [(1, 3, 0), (2, 3, 0)], 0, 0),
        (fsc.FAR, [], [(0, 3, 1)], 0, 1),               # both children out of range: narrow
        (fsc.FAR, [], [(0, 3, 1)], 0, 0),               # roots stay
        (fsc.NEAR, [], [(1, 3, 2), (2, 3, 2)], 1, 0),   # back: widen, children now vetoed
        (fsc.FAR, [], [(1, 3, 2), (2, 3, 2)], 0, 0),    # memory set: no second narrowing
        (fsc.NEAR, [(1, 3)], [(1, 3, 2), (2, 3, 2)], 0, 0),
    ]
    for where, con, after, nu, nc in script:
        fsc.move_b(sc, where)
        r = f.step(oracle.tree(sc))
        assert contacts_ab(r) == con
        assert leaves_abf(f) == after
        assert (r["unfolded"], r["collapsed"]) == (nu, nc)


def test_three_level_hand_sequence():
    sc = fsc.three_level()
    f = Frontier(oracle.tree(sc))
    script = [
        (fsc.NEAR, [], [(1, 7, 0), (2, 7, 0)], 1, 0),
        (fsc.NEAR, [], [(3, 7, 0), (4, 7, 0), (2, 7, 0)], 1, 0),   # S0 widens, S1 is out of range
        (fsc.NEAR, [(3, 7)], [(3, 7, 0), (4, 7, 0), (2, 7, 0)], 0, 0),
        (fsc.FAR, [], [(1, 7, 1), (2, 7, 0)], 0, 1),               # one level per step ...
        (fsc.FAR, [], [(0, 7, 1)], 0, 1),                          # ... and the next
        (fsc.NEAR, [], [(1, 7, 3), (2, 7, 2)], 1, 0),              # (1, 7) and (0, 7) remembered
        (fsc.NEAR, [], [(3, 7, 6), (4, 7, 6), (2, 7, 2)], 1, 0),
        (fsc.FAR, [], [(3, 7, 6), (4, 7, 6), (2, 7, 2)], 0, 0),    # both groups vetoed
        (fsc.NEAR, [(3, 7)], [(3, 7, 6), (4, 7, 6), (2, 7, 2)], 0, 0),
    ]
    for where, con, after, nu, nc in script:
        fsc.move_b(sc, where)
        r = f.step(oracle.tree(sc))
        assert contacts_ab(r) == con
        assert leaves_abf(f) == after
        assert (r["unfolded"], r["collapsed"]) == (nu, nc)


def test_hand_geometry_is_as_the_scripts_assume():
    """The distances behind the scripts' decisions (so a change of the scene
    builders cannot silently change what the scripts test)."""
    sc = fsc.three_level()
    t = oracle.tree(sc)
    d = lambda a, b: oracle.tri_tri(t.verts[t.tris[a]], t.verts[t.tris[b]])["d"]
    assert abs(d(3, 7) - 0.05) < 1e-12 and d(3, 7) <= t.eps[3] + t.eps[7]
    assert d(0, 7) <= t.eps[0] + t.eps[7] and d(1, 7) <= t.eps[1] + t.eps[7]
    for s in (2, 4):
        assert d(s, 7) > t.eps[s] + t.eps[7] + 0.5


def fine_desc(t, x):
    c = int(t.child_count[x])
    if c == 0:
        return [x]
    out = []
    for k in range(int(t.child_begin[x]), int(t.child_begin[x]) + c):
        out += fine_desc(t, k)
    return out


def assert_cover(t, f: Frontier):
    """Every fine pair of the candidate pair lies below exactly one active pair."""
    lv = f.leaves()
    got = []
    for a, b, _, _ in lv:
        fa, fb = np.array(fine_desc(t, a)), np.array(fine_desc(t, b))
        got.append((fa[:, None] * 1_000_000 + fb[None, :]).ravel())
    got = np.sort(np.concatenate(got))
    pi, pj = t.pairs[0]
    Fi = np.arange(t.fine_begin[pi], t.root_begin[pi] + np.sum(t.tri_count_all[pi]))
    Fj = np.arange(t.fine_begin[pj], t.root_begin[pj] + np.sum(t.tri_count_all[pj]))
    want = np.sort((Fi[:, None] * 1_000_000 + Fj[None, :]).ravel())
    assert np.array_equal(got, want)


def _spheres(sep):
    return sg.two_spheres(3, [1, 2, 3], "f64", sep, 11, "two_spheres_s3_levels123")


def _with_counts(t, sc):
    # total triangles per particle (all levels), for the cover check
    t.tri_count_all = [sum(len(l) for l in p.levels) for p in sc.particles]
    return t


def test_spheres_cover_depth_and_fixed_point():
    sc = _spheres(2.02)
    t = _with_counts(oracle.tree(sc), sc)
    f = Frontier(t)
    assert_cover(t, f)
    hist = []
    for s in range(1, 12):
        r = f.step(t)
        hist.append(r)
        assert_cover(t, f)
        assert f.leaves()[:, 3].max() <= s  # at most one level per step
        if r["unfolded"] == 0 and r["collapsed"] == 0:
            break
    else:
        pytest.fail("no fixed point")
    # three levels (depths 0..2): two widening steps reach the fine pairs; a
    # group narrowed under a parent still in range comes back once (vetoed)
    assert hist[0]["unfolded"] > 0 and hist[1]["unfolded"] > 0 and len(hist) <= 6
    fs = oracle.fine_scene(sc)
    flat = oracle.find_contacts(fs)
    last = hist[-1]
    got = sorted(zip((last["a"] - t.fine_begin[0]).tolist(), (last["b"] - t.fine_begin[1]).tolist()))
    want = sorted(zip(flat["ti"].tolist(), flat["tj"].tolist()))
    assert len(want) > 20 and got == want
    # every earlier step reported a subset of the contacts
    for h in hist[:-1]:
        sub = set(zip((h["a"] - t.fine_begin[0]).tolist(), (h["b"] - t.fine_begin[1]).tolist()))
        assert sub <= set(want)


def test_spheres_narrow_one_level_per_step_then_memory_holds():
    sc = _spheres(2.02)
    t = _with_counts(oracle.tree(sc), sc)
    f = Frontier(t)
    f.run_until_fixed(t)
    depth0 = f.leaves()[:, 3].max()
    assert depth0 == 2
    n_contact = len(f.leaves())
    roots = int(t.root_count[0] * t.root_count[1])
    # separate: groups narrow one level per step until only vetoed ones are left
    far = _spheres(6.0)
    tf = _with_counts(oracle.tree(far), far)
    n_prev = len(f.leaves())
    for k in range(6):
        r = f.step(tf)
        assert_cover(tf, f)
        assert len(r["a"]) == 0 and r["unfolded"] == 0
        n = len(f.leaves())
        assert (n < n_prev) == (r["collapsed"] > 0)
        n_prev = n
        if r["collapsed"] == 0:
            break
    assert k <= depth0 + 1
    lv = f.leaves()
    assert len(lv) < n_contact
    # pairs kept below the roots: vetoed groups, and siblings of vetoed subtrees
    deep = lv[lv[:, 3] > 0]
    assert len(deep) and np.any((deep[:, 2] >> deep[:, 3]) & 1)
    # back into contact and apart again: the pairs that came back stay
    f.run_until_fixed(t)
    n_back = len(f.leaves())
    for _ in range(4):
        f.step(tf)
        assert_cover(tf, f)
    lv = f.leaves()
    assert len(lv) == n_back > roots
