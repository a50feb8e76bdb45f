"""Pins of the Barnes-Hut monopole gravity oracle (section 3.3, eq. gravitational_force;
the tree of section 3.5.1): theta = 0 against the direct sum written out here, the
inner nodes against a brute-force enumeration of the cubes holding two or more
particles and their masses and centres of mass, a distant cluster acting as one
pseudo-particle, momentum conservation of the direct sum, the error's decay with
theta, the smoothing closed form, and the degenerate trees."""
import numpy as np
import pytest

from oracle import native


def direct(pos, m, G, eps=0.0):
    """a_a = sum over b with r_ab > 0 of G m_b (x_b - x_a) / (r_ab + eps)^3."""
    d = pos[:, None, :] - pos[:, :, None]  # d[:, a, b] = x_b - x_a
    r = np.sqrt((d ** 2).sum(0))
    w = np.zeros_like(r)
    nz = r > 0
    w[nz] = G * np.broadcast_to(m[None, :], r.shape)[nz] / (r[nz] + eps) ** 3
    return (d * w[None]).sum(2)


def cloud(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(3, n)), rng.uniform(1.0, 2.0, n)


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_theta_zero_is_the_direct_sum(eps):
    pos, m = cloud(1500, 1)
    g = native.gravity(pos, m, 6.674e-11, 0.0, eps)
    ref = direct(pos, m, 6.674e-11, eps)
    assert np.abs(g["acc"] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.all(g["count"] == 1499)


def quantise(pos):
    lo = pos.min(axis=1)
    s0 = (pos.max(axis=1) - lo).max()
    q = np.floor((pos - lo[:, None]) / s0 * 2.0 ** 21)
    return np.minimum(q, 2 ** 21 - 1).astype(np.int64)


def test_inner_nodes_are_the_cubes_holding_two_or_more_particles():
    pos, m = cloud(3000, 2)
    # a few close pairs force deep chains of one-child nodes
    pos[:, 10] = pos[:, 11] + 1e-9
    pos[:, 20] = pos[:, 21]  # coincident: shares a depth-21 cube
    tr = native.gravity_tree(pos, m)
    q = quantise(pos)
    want = {}
    for d in range(22):
        key = q >> (21 - d)
        k, inv, cnt = np.unique(key.T, axis=0, return_inverse=True, return_counts=True)
        inv = inv.ravel()
        for j in np.nonzero(cnt >= 2)[0]:
            sel = inv == j
            M = m[sel].sum()
            want[(d, *k[j])] = (M, (pos[:, sel] * m[sel]).sum(1) / M)
    got = {(int(d), *map(int, c)): (M, x) for d, c, M, x in
           zip(tr["depth"], tr["corner"], tr["mass"], tr["com"])}
    assert set(got) == set(want)
    assert max(got)[0] == 21
    for key, (M, x) in want.items():
        gM, gx = got[key]
        assert abs(gM - M) <= 1e-13 * M
        assert np.abs(gx - x).max() <= 1e-12 * (np.abs(x).max() + 1.0)


def test_a_distant_cluster_acts_as_one_pseudo_particle():
    rng = np.random.default_rng(3)
    k = 200
    B = np.array([[10.0], [10.0], [10.0]]) + rng.uniform(-0.1, 0.1, (3, k))
    pos = np.concatenate([np.zeros((3, 1)), B], axis=1)
    m = np.concatenate([[1.0], rng.uniform(1.0, 2.0, k)])
    g = native.gravity(pos, m, 1.0, 0.5)
    M = m[1:].sum()
    c = (B * m[1:]).sum(1) / M
    r = np.linalg.norm(c)
    assert g["count"][0] == 1
    assert np.abs(g["acc"][:, 0] - M * c / r ** 3).max() <= 1e-13 * M / r ** 2


def test_direct_sum_conserves_momentum():
    pos, m = cloud(1200, 4)
    a = native.gravity(pos, m, 1.0, 0.0)["acc"]
    p = (a * m).sum(1)
    assert np.abs(p).max() <= 1e-13 * np.abs(a * m).sum()


def test_error_decays_with_theta():
    pos, m = cloud(2000, 5)
    ref = direct(pos, m, 1.0)
    err = {}
    for th in (0.125, 0.25, 0.5):
        a = native.gravity(pos, m, 1.0, th)["acc"]
        e = np.sqrt(((a - ref) ** 2).sum(0) / (ref ** 2).sum(0))
        err[th] = np.sqrt((e ** 2).mean())
    assert err[0.125] < err[0.25] < err[0.5] < 1e-2
    assert 3.0 < err[0.5] / err[0.25] < 16.0


def test_smoothing_of_two_particles():
    pos = np.array([[0.0, 3.0], [0.0, 0.0], [0.0, 4.0]])
    m = np.array([2.0, 5.0])
    g = native.gravity(pos, m, 0.5, 0.4, eps=0.25)
    d = 5.25 ** 3
    assert np.allclose(g["acc"][:, 0], 0.5 * 5.0 * np.array([3.0, 0.0, 4.0]) / d, rtol=1e-15)
    assert np.allclose(g["acc"][:, 1], -0.5 * 2.0 * np.array([3.0, 0.0, 4.0]) / d, rtol=1e-15)


def test_degenerate_trees():
    g = native.gravity(np.zeros((3, 1)), np.ones(1), 1.0, 0.5)
    assert np.all(g["acc"] == 0.0) and g["count"][0] == 0 and g["nodes"] == 1
    # all particles at one point: a chain down to depth 21 holding them all; no force
    g = native.gravity(np.ones((3, 5)), np.ones(5), 1.0, 0.5)
    assert np.all(g["acc"] == 0.0) and g["nodes"] == 22 and np.all(g["count"] == 4)
    # two coincident particles and a third: the pair adds nothing to each other
    pos = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    g = native.gravity(pos, np.array([1.0, 2.0, 3.0]), 1.0, 0.0)
    assert np.allclose(g["acc"][:, 0], [3.0, 0.0, 0.0], rtol=1e-15)
    assert np.allclose(g["acc"][:, 2], [-3.0, 0.0, 0.0], rtol=1e-15)


def test_opening_criterion_is_strict_on_the_node_edge_over_the_com_distance():
    # section 3.3: a node acts as one pseudo-particle when s / r < theta, s its edge
    # and r the distance to its centre of mass.  Root cube [0, 8]^3 (s0 = 8, set by
    # the target at the origin and a body at (8, 8, 8)); the octant z >= 4, x, y < 4
    # (edge 4) holds two unit masses in different sub-octants, centre of mass
    # (2, 2, 6) exactly, at r = sqrt(44) from the target.  The root (s / r = 8 /
    # sqrt(43) > 1) is always opened.
    pos = np.array([[0.0, 8.0, 1.0, 3.0], [0.0, 8.0, 1.0, 3.0], [0.0, 8.0, 5.0, 7.0]])
    m = np.ones(4)
    tie = 4.0 / np.sqrt(44.0)
    above = native.gravity(pos, m, 1.0, np.nextafter(tie, 1.0), targets=[0])
    at = native.gravity(pos, m, 1.0, tie, targets=[0])
    below = native.gravity(pos, m, 1.0, np.nextafter(tie, 0.0), targets=[0])
    assert above["count"][0] == 2  # the body at (8, 8, 8) and the node as one
    assert at["count"][0] == 3 and below["count"][0] == 3  # the node opened: both bodies
    # as one pseudo-particle of mass 2 at (2, 2, 6) (G = 1, no smoothing)
    c = np.array([2.0, 2.0, 6.0])
    b = np.array([8.0, 8.0, 8.0])
    want = 2.0 * c / 44.0 ** 1.5 + b / np.linalg.norm(b) ** 3
    assert np.abs(above["acc"][:, 0] - want).max() <= 1e-15 * np.abs(want).max()
    p1, p2 = pos[:, 2], pos[:, 3]
    want3 = p1 / np.linalg.norm(p1) ** 3 + p2 / np.linalg.norm(p2) ** 3 + b / np.linalg.norm(b) ** 3
    assert np.abs(at["acc"][:, 0] - want3).max() <= 1e-15 * np.abs(want3).max()
