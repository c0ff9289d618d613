"""CPU checks of the product's triangle geometry (dem_geom.hpp compiled for
the host) against the FP64 oracle: exact distances and the conservativeness
of the iteration's lower bound, in FP64 and FP32."""
import numpy as np
import pytest

import host_geom
import oracle
import scenegen as sg


def _h(P):
    e = lambda X: np.linalg.norm(X - np.roll(X, 1, 1), axis=2).max(1)
    return np.maximum(e(P[:, 0]), e(P[:, 1]))


def _cases():
    P = sg.random_triangle_pairs(60000, seed=21)
    rng = np.random.default_rng(22)
    A = rng.uniform(-1, 1, (20000, 3, 3))
    B = A + rng.normal(0, 1e-3, A.shape) + rng.normal(0, 0.05, (20000, 1, 3))  # near parallel
    C = sg.random_triangle_pairs(20000, seed=23, scale=0.05, spread=0.2) + 20.0  # far from origin
    from test_oracle_geometry import degenerate_pairs
    D = degenerate_pairs(4000, seed=24)  # segments, points, slivers
    return np.concatenate([P, np.stack([A, B], 1), C.astype(np.float32).astype(np.float64), D])


@pytest.mark.parametrize("double,r,a", [(True, 1e-12, 1e-13), (False, 1e-5, 1e-6)])
def test_exact_distance_matches_oracle(double, r, a):
    P = _cases()
    ref = oracle.tri_tri_batch(P)
    got = host_geom.exact(P, double)
    err = np.abs(got["d"] - ref["d"]) - (r * ref["d"] + a * _h(P))
    assert np.all(err <= 0), np.max(err)
    # returned points realise the returned distance and sit on their triangles
    assert np.allclose(np.linalg.norm(got["p2"] - got["p1"], axis=1), got["d"],
                       atol=(1e-12 if double else 1e-5) * (1 + _h(P)))
    assert np.all(got["w1"] >= -1e-6) and np.allclose(got["w1"].sum(1), 1, atol=1e-5)
    assert np.all(got["w2"] >= -1e-6) and np.allclose(got["w2"].sum(1), 1, atol=1e-5)
    # the weights reproduce the points (the adjoint scatters with them)
    h = _h(P)[:, None]
    tol = (1e-12 if double else 1e-5) * (1 + h)
    sep = got["d"] > 0
    assert np.all(np.abs(np.einsum("nk,nki->ni", got["w1"], P[:, 0]) - got["p1"])[sep] <= tol[sep])
    assert np.all(np.abs(np.einsum("nk,nki->ni", got["w2"], P[:, 1]) - got["p2"])[sep] <= tol[sep])
    # closest points are unique for separated pairs without a near tie
    # between features (FP32: no other candidate within 1e-5 of the edge
    # scale, the criterion the GPU gradient tests use): compare them, and the
    # unit direction the adjoint uses, with the oracle's.  Rounding moves
    # the points by ulps of h times the conditioning of the feature (nearly
    # parallel edges), and the direction by that over d.
    oracle.set_ambiguity_tol(1e-9 if double else 1e-5)
    try:
        amb = oracle.tri_tri_batch(P)["ambiguous"]
    finally:
        oracle.set_ambiguity_tol(1e-9)
    uniq = sep & ~amb & (ref["d"] > 1e-3 * h[:, 0])
    assert uniq.sum() > len(P) // 4
    c = 1e-10 if double else 2e-5
    ptol = c * h[uniq]
    assert np.all(np.abs(got["p1"] - ref["p1"])[uniq] <= ptol)
    assert np.all(np.abs(got["p2"] - ref["p2"])[uniq] <= ptol)
    u_g = (got["p2"] - got["p1"])[uniq] / got["d"][uniq, None]
    u_r = (ref["p2"] - ref["p1"])[uniq] / ref["d"][uniq, None]
    assert np.all(np.abs(u_g - u_r) <= c * h[uniq] / ref["d"][uniq, None])


@pytest.mark.parametrize("double,r,a", [(True, 1e-12, 1e-13), (False, 1e-5, 1e-6)])
def test_exact_distance_degenerate_triangles(double, r, a):
    """Segments, points and slivers: the product's exact distance against the
    oracle (pinned to brute force on the same cases)."""
    from test_oracle_geometry import degenerate_pairs
    P = degenerate_pairs(4000, seed=9)
    ref = oracle.tri_tri_batch(P)
    got = host_geom.exact(P, double)
    err = np.abs(got["d"] - ref["d"]) - (r * ref["d"] + a * _h(P))
    assert np.all(err <= 0), (np.max(err), int(np.argmax(err)))


@pytest.mark.parametrize("double", [True, False])
@pytest.mark.parametrize("n_iter,omega,centroid", [(4, 1.0, 0), (4, 0.5, 1), (0, 1.0, 0), (8, 0.7, 0)])
def test_lower_bound_never_exceeds_distance(double, n_iter, omega, centroid):
    """The pruning test L > delta + slack is safe: L - slack <= d always."""
    P = _cases()
    ref = oracle.tri_tri_batch(P)
    b = host_geom.bound(P, double, n_iter=n_iter, omega=omega, centroid=centroid)
    assert np.all(b["L"] - b["slack"] <= ref["d"])
    # the bound is informative for well separated pairs
    far = ref["d"] > _h(P)
    assert np.mean(b["L"][far] > 0.5 * ref["d"][far]) > 0.9


def _contact_like_pairs(n, seed):
    """Nearby pairs of bumped-sphere-like triangles: small triangles a short
    gap apart with random orientations (the pairs the descent hands on)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(n, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    A = rng.uniform(-0.05, 0.05, (n, 3, 3))
    B = rng.uniform(-0.05, 0.05, (n, 3, 3)) + (c * rng.uniform(0.0, 0.12, (n, 1)))[:, None, :]
    return np.stack([A, B], 1) + rng.uniform(-20, 20, (n, 1, 1, 3))


@pytest.mark.parametrize("double,r,a", [(True, 1e-12, 1e-13), (False, 1e-5, 1e-6)])
def test_certified_distances_are_exact(double, r, a):
    """Whenever the certificate accepts, the distance meets the parity bar."""
    for P in (_contact_like_pairs(40000, 31).astype(np.float32).astype(np.float64), _cases()):
        ref = oracle.tri_tri_batch(P)
        c = host_geom.certify(P, double)
        ok = c["ok"]
        err = np.abs(c["d"][ok] - ref["d"][ok]) - (r * ref["d"][ok] + a * _h(P)[ok])
        assert np.all(err <= 0), np.max(err)
        assert ok.mean() > 0.3  # it settles a good share of pairs


@pytest.mark.parametrize("n_iter,omega", [(4, 1.0), (4, 0.5), (8, 0.7)])
def test_reduced_precision_iteration_bound_is_safe(n_iter, omega):
    """The reduced-precision iteration (Newton steps in FP16, bound in FP32)
    keeps the pruning test safe on every case, including edges and offsets
    beyond the half-precision range, and prunes nearly as well as the FP32
    iteration on separated pairs."""
    P = _cases()
    big = sg.random_triangle_pairs(2000, seed=25, scale=3e3, spread=2e4)  # offsets beyond 65504
    tiny = sg.random_triangle_pairs(2000, seed=26, scale=1e-4, spread=3e-4)  # diagonals beyond the range
    P = np.concatenate([P, big, tiny])
    ref = oracle.tri_tri_batch(P)
    b = host_geom.bound(P, False, n_iter=n_iter, omega=omega, half=True)
    assert np.all(b["L"] - b["slack"] <= ref["d"])
    f = host_geom.bound(P, False, n_iter=n_iter, omega=omega)
    far = ref["d"] > _h(P)
    assert np.mean(b["L"][far] > 0.5 * ref["d"][far]) > 0.9
    # at the descent's thresholds (delta = 0.1 on unit-size pairs) it keeps few more pairs than FP32
    sel = ref["d"] < 3.0
    delta = 0.1 * _h(P)[sel]
    pruned32 = f["L"][sel] > delta + f["slack"][sel]
    pruned16 = b["L"][sel] > delta + b["slack"][sel]
    assert pruned16.sum() >= 0.97 * pruned32.sum()
