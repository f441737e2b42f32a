"""Pins of the FP64 oracle's ligand-receptor bonds in 3D (sites on a
membrane's triangles, anchors on the tube wall, Sec. 2.5 carried to 3D):
the spring force of a bond stretched by a known length, the formation and
rupture counts against their binomial laws, the anchors on the wall and the
capture distance."""
import numpy as np
import pytest

from oracle import tube3d as otube
from paper_2210_06043_amd import inputs

NX, N, R = 40, 24, 11.0
C0 = 0.5 * (N - 1)


def _particle(ns=300, seed=5, center=(20.3, C0 + 4.6, C0 - 0.4), **bond):
    """A 642-vertex sphere of radius 3 near the wall, with ns sites at random
    triangles and barycentric coordinates; only the bond force acts."""
    xyz, tri = inputs.icosphere(3, 3.0, center)
    t = otube.Tube(NX, N, N, 0.9, 0.0, radius=R)
    t.add_membrane(xyz, tri, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0)
    rng = np.random.default_rng(seed)
    st = rng.integers(0, len(tri), ns).astype(np.int32)
    u = rng.random((ns, 2))
    u[u.sum(axis=1) > 1] = 1 - u[u.sum(axis=1) > 1]
    p = dict(sigma=1e-3, yeq=0.5, ycr=1.0, kf=0.3, kr0=0.0, lb=1.0, seed=77)
    p.update(bond)
    t.add_bonds(0, st, u, p["sigma"], p["yeq"], p["ycr"], p["kf"], p["kr0"], p["lb"], p["seed"])
    return t, xyz, tri, st, u


def _site(xyz, tri, st, u, q):
    a, b, c = xyz[tri[st[q]]]
    n = np.cross(b - a, c - a)
    return a + u[q, 0] * (b - a) + u[q, 1] * (c - a), n / np.linalg.norm(n)


def test_a_bond_stretched_by_a_known_length():
    """One bound site at a triangle's centroid, its anchor L along the
    triangle's outward normal: each corner feels sigma (L - y_eq) / 3 along
    the normal, nothing else moves."""
    t, xyz, tri, st, u = _particle(ns=1, sigma=2e-3, yeq=0.4)
    st = np.array([17])
    t2 = otube.Tube(NX, N, N, 0.9, 0.0, radius=R)
    t2.add_membrane(xyz, tri, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0)
    t2.add_bonds(0, st.astype(np.int32), np.array([[1 / 3, 1 / 3]]), 2e-3, 0.4, 1.0, 0.3, 0.0, 1.0, 1)
    p, n = _site(xyz, tri, st, np.array([[1 / 3, 1 / 3]]), 0)
    L = 1.3
    t2.set_bonds([1], (p + L * n)[None, :])
    F = t2.membrane_forces(0)
    expect = np.zeros_like(F)
    expect[tri[17]] = 2e-3 * (L - 0.4) / 3 * n
    assert np.abs(F - expect).max() < 1e-15
    assert F.sum(axis=0) == pytest.approx(2e-3 * (L - 0.4) * n, rel=1e-12)


def test_formation_follows_the_binomial_law_and_anchors_lie_on_the_wall():
    """k_r0 = 0 and a capture distance that every site meets: after n steps a
    site is bound with probability 1 - (1 - P_f)^n, P_f = 1 - exp(-k_f); each
    anchor lies on the wall radius, straight out from its site."""
    ns, kf = 300, 0.3
    t, xyz, tri, st, u = _particle(ns=ns, ycr=100.0, kf=kf)
    pf = 1 - np.exp(-kf)
    t.step(1)
    b, a, nb = t.bonds()
    assert abs(nb - ns * pf) < 4 * np.sqrt(ns * pf * (1 - pf)), (nb, ns * pf)
    # the anchors formed at x^1 (the positions now): on the wall radius,
    # straight out from the site
    X = t.membrane_vertices()
    for q in np.nonzero(b)[0]:
        s, _ = _site(X, tri, st, u, q)
        rho = np.hypot(s[1] - C0, s[2] - C0)
        expect = np.array([s[0], C0 + R * (s[1] - C0) / rho, C0 + R * (s[2] - C0) / rho])
        assert np.abs(a[q] - expect).max() < 1e-12
    t.step(3)
    nb = t.bonds()[2]
    p = 1 - (1 - pf) ** 4
    assert abs(nb - ns * p) < 4 * np.sqrt(ns * p * (1 - p)), (nb, ns * p)


def test_no_capture_beyond_y_cr():
    t, *_ = _particle(ns=100, ycr=-1.0, kf=5.0)
    t.step(3)
    assert t.bonds()[2] == 0


def test_rupture_follows_the_binomial_law():
    """Every site bound at the start, k_f = 0 and l_B so large that the rate
    is k_r0 at any stretch: one step breaks each bond with probability
    P_r = 1 - exp(-k_r0)."""
    ns, kr0 = 300, 0.2
    t, xyz, tri, st, u = _particle(ns=ns, kf=0.0, kr0=kr0, lb=1e12)
    anc = np.array([_site(xyz, tri, st, u, q)[0] for q in range(ns)])
    anc[:, 2] += 0.7
    t.set_bonds(np.ones(ns, dtype=np.int32), anc)
    t.step(1)
    nb = t.bonds()[2]
    pr = 1 - np.exp(-kr0)
    assert abs((ns - nb) - ns * pr) < 4 * np.sqrt(ns * pr * (1 - pr)), (ns - nb, ns * pr)
    assert t.bond_margins()[2] == ns - nb
