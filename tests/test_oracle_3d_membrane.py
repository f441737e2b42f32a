"""Pins of the FP64 oracle's deformable membranes in 3D (Skalak elements,
dihedral bending, area and volume penalties, the 2D path's vertex update
carried to 3D),
each against something other than the oracle's own formulas: invariants
written from edge lengths and areas, the closed form of a uniform
dilation, the icosahedron's dihedral angle, a hinge folded by a known angle,
central finite differences of the energies, the conservation of force and
torque, and one step in a uniform flow."""
import numpy as np
import pytest

from oracle import tube3d as otube
from paper_2210_06043_amd import inputs

GS, CS, KA, KV, MASS, KB = 2e-3, 2.0, 0.05, 0.03, 1.0, 4e-3


def _box_with(xyz, tri, n=20, **kw):
    t = otube.Tube(n, n, n, 1.0, 0.0, geom=otube.BOX)
    p = dict(gs=GS, c=CS, ka=KA, kv=KV, mass=MASS, kb=KB)
    p.update(kw)
    t.add_membrane(xyz, tri, p["gs"], p["c"], p["ka"], p["kv"], p["mass"], p["kb"])
    return t


def _skalak_from_edges(X0, X, tri, gs, c):
    """Skalak's energy with the invariants taken from the triangles' edge
    lengths and areas: tr C = sum over edges of cot(rest opposite angle)
    times the deformed squared length, over twice the rest area (the linear
    map's Dirichlet identity); det C = (area / rest area)^2."""
    E = 0.0
    for t in tri:
        P, Q = X0[t], X[t]
        A0 = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        A = 0.5 * np.linalg.norm(np.cross(Q[1] - Q[0], Q[2] - Q[0]))
        trC = 0.0
        for k in range(3):
            i, j, o = t[k], t[(k + 1) % 3], t[(k + 2) % 3]   # edge (i, j) opposite vertex o
            a, b = X0[i] - X0[o], X0[j] - X0[o]
            cot = np.dot(a, b) / np.linalg.norm(np.cross(a, b))
            trC += cot * np.sum((X[i] - X[j]) ** 2)
        trC /= 2.0 * A0
        I1, I2 = trC - 2.0, (A / A0) ** 2 - 1.0
        E += A0 * gs / 4.0 * (I1 * I1 + 2 * I1 - 2 * I2 + c * I2 * I2)
    return E


def test_rest_shape_is_force_free():
    xyz, tri = inputs.icosphere(2, 3.0, (10.2, 9.9, 10.1))
    t = _box_with(xyz, tri)
    assert np.all(np.abs(t.membrane_energy(0)) < 1e-16)
    assert np.abs(t.membrane_forces(0)).max() < 1e-15


def test_rest_totals_are_the_sphere_within_the_triangulation_error():
    xyz, tri = inputs.icosphere(3, 4.0, (10.0, 10.0, 10.0))
    A, V, A0, V0 = _box_with(xyz, tri).membrane_totals(0)
    assert A == A0 and V == V0
    assert abs(A / (4 * np.pi * 16) - 1) < 0.01 and abs(V / (4 / 3 * np.pi * 64) - 1) < 0.015
    assert V > 0   # counter-clockwise seen from outside


@pytest.mark.parametrize("lam", [0.97, 1.0, 1.04])
def test_uniform_dilation_energies_in_closed_form(lam):
    """Every triangle stretched by lam in both directions: I1 = 2 lam^2 - 2,
    I2 = lam^4 - 1, so the Skalak energy is the rest area times
    G_s/4 (I1^2 + 2 I1 - 2 I2 + C I2^2); the penalties follow from A = lam^2 A0
    and V = lam^3 V0; the forces' work along the dilation is dE/dlam."""
    c0 = np.array([10.3, 9.8, 10.1])
    xyz, tri = inputs.icosphere(2, 3.0, tuple(c0))
    t = _box_with(xyz, tri)
    _, _, A0, V0 = t.membrane_totals(0)
    t.set_membrane_vertices(c0 + lam * (xyz - c0))
    I1, I2 = 2 * lam ** 2 - 2, lam ** 4 - 1
    ws = A0 * GS / 4 * (I1 * I1 + 2 * I1 - 2 * I2 + CS * I2 * I2)
    ea = KA * (lam ** 2 * A0 - A0) ** 2 / (2 * A0)
    ev = KV * (lam ** 3 * V0 - V0) ** 2 / (2 * V0)
    E = t.membrane_energy(0)
    assert E == pytest.approx([ws, ea, ev, 0.0], rel=1e-9, abs=1e-15)   # dilation keeps every angle
    # along the dilation mode the forces do the closed form's work: with r_v
    # the rest radius vector, dE/dlam = -sum_v f_v . r_v
    F = t.membrane_forces(0)
    dws = A0 * GS / 4 * (2 * I1 * 4 * lam + 2 * 4 * lam - 2 * 4 * lam ** 3 + 2 * CS * I2 * 4 * lam ** 3)
    dea = KA * (lam ** 2 - 1) * A0 * 2 * lam
    dev = KV * (lam ** 3 - 1) * V0 * 3 * lam ** 2
    assert -np.sum(F * (xyz - c0)) == pytest.approx(dws + dea + dev, rel=1e-9, abs=1e-14)


def test_skalak_energy_matches_edge_length_invariants_under_a_general_deformation():
    rng = np.random.default_rng(4)
    xyz, tri = inputs.icosphere(2, 3.0, (10.0, 10.0, 10.0))
    t = _box_with(xyz, tri)
    M = np.eye(3) + 0.08 * rng.standard_normal((3, 3))
    X = 10.0 + (xyz - 10.0) @ M.T + 0.03 * rng.standard_normal(xyz.shape)
    t.set_membrane_vertices(X)
    assert t.membrane_energy(0)[0] == pytest.approx(_skalak_from_edges(xyz, X, tri, GS, CS), rel=1e-10)


def test_forces_are_minus_the_energy_gradient():
    """Central differences of the total energy (Skalak + area + volume) at a
    randomly deformed sphere, every component of a sample of vertices."""
    rng = np.random.default_rng(7)
    xyz, tri = inputs.icosphere(2, 3.0, (10.0, 10.0, 10.0))
    t = _box_with(xyz, tri)
    X = xyz * (1.0 + 0.03 * rng.standard_normal((len(xyz), 1))) + 0.02 * rng.standard_normal(xyz.shape)
    X += 10.0 - X.mean(axis=0)
    t.set_membrane_vertices(X)
    F = t.membrane_forces(0)
    h = 1e-5
    for v in rng.choice(len(X), 12, replace=False):
        for q in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[v, q] += h
            Xm[v, q] -= h
            t.set_membrane_vertices(Xp)
            ep = t.membrane_energy(0).sum()
            t.set_membrane_vertices(Xm)
            em = t.membrane_energy(0).sum()
            fd = -(ep - em) / (2 * h)
            assert F[v, q] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(F).max())
    t.set_membrane_vertices(X)


def test_internal_forces_carry_no_net_force_or_torque():
    rng = np.random.default_rng(9)
    xyz, tri = inputs.icosphere(2, 3.0, (10.0, 10.0, 10.0))
    t = _box_with(xyz, tri)
    X = xyz + 0.05 * rng.standard_normal(xyz.shape)
    t.set_membrane_vertices(X)
    F = t.membrane_forces(0)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale
    assert np.abs(np.cross(X - X.mean(axis=0), F).sum(axis=0)).max() < 1e-11 * scale


def test_one_step_in_a_uniform_flow():
    """In a periodic box moving uniformly at U0 the interpolated velocity is
    U0 exactly (the delta sums to one) and the rest shape carries no elastic
    force, so every vertex moves by U0, its velocity for the forcing is
    3/2 U0 (no previous displacement), the spread force is (3/2 U0 - U0) dV
    with dV a third of the adjacent triangles' area, and the force field
    spread into the fluid totals their sum."""
    U0 = np.array([2e-3, -1e-3, 5e-4])
    xyz, tri = inputs.icosphere(2, 3.0, (10.2, 9.7, 10.4))
    t = otube.Tube(20, 20, 20, 1.0, 0.0, geom=otube.BOX)
    A = np.zeros((19, 20, 20, 20))
    A[:] = otube.heq(0.0, *U0)[:, None, None, None]
    t.set_populations(A)
    t.add_membrane(xyz, tri, GS, CS, KA, KV, MASS)
    t.step(1)
    assert np.abs(t.membrane_vertices() - (xyz + U0)).max() < 1e-15
    dV = np.zeros(len(xyz))
    for tr in tri:
        a = 0.5 * np.linalg.norm(np.cross(xyz[tr[1]] - xyz[tr[0]], xyz[tr[2]] - xyz[tr[0]]))
        dV[tr] += a / 3
    F = t.membrane_spread_forces()
    assert np.abs(F - 0.5 * U0[None, :] * dV[:, None]).max() < 1e-15
    tot = t.ib_force().reshape(3, -1).sum(axis=1)
    assert tot == pytest.approx(F.sum(axis=0), rel=1e-11)


def test_a_stretched_membrane_relaxes_in_a_quiescent_box():
    """A sphere dilated by 3 % in fluid at rest shrinks back: its Skalak,
    area and volume energies all fall over 300 coupled steps, and the fluid's
    momentum stays zero to rounding (the spread forces sum to zero)."""
    c0 = np.array([12.0, 12.0, 12.0])
    xyz, tri = inputs.icosphere(2, 3.0, tuple(c0))
    t = otube.Tube(24, 24, 24, 1.0, 0.0, geom=otube.BOX)
    t.add_membrane(xyz, tri, 5e-3, 1.0, 0.05, 0.05, 1.0)
    t.set_membrane_vertices(c0 + 1.03 * (xyz - c0))
    e0 = t.membrane_energy(0)[:3]
    t.step(300)
    e1 = t.membrane_energy(0)[:3]
    assert np.all(e1 < e0)
    mom = t.totals()[1:]
    assert np.abs(mom).max() < 1e-13


def test_icosahedron_dihedral_angles():
    """Every edge of the regular icosahedron has the same angle between its
    faces' outward normals, pi minus the interior dihedral angle
    arccos(-sqrt(5)/3); the rest angles are the current ones."""
    xyz, tri = inputs.icosphere(0, 2.0, (10.0, 10.0, 10.0))
    t = _box_with(xyz, tri)
    th, th0 = t.membrane_dihedrals(0)
    assert len(th) == 30 and np.array_equal(th, th0)
    assert np.abs(np.abs(th) - (np.pi - np.arccos(-np.sqrt(5) / 3))).max() < 1e-12
    assert np.all(np.sign(th) == np.sign(th[0]))


@pytest.mark.parametrize("delta", [0.05, -0.3, 1.2])
def test_a_hinge_folded_by_a_known_angle(delta):
    """Two triangles sharing an edge (an open surface: one interior edge);
    turning the far vertex about the edge by delta changes the dihedral angle
    by delta, so the bending energy is k_b (1 - cos delta), and the forces are
    minus its gradient."""
    x = np.array([[10.0, 10.0, 10.0], [11.5, 10.2, 10.1], [10.6, 11.3, 10.0], [10.9, 9.1, 10.4]])
    tri = np.array([[0, 1, 2], [1, 0, 3]])
    t = otube.Tube(20, 20, 20, 1.0, 0.0, geom=otube.BOX)
    t.add_membrane(x, tri, 0.0, 0.0, 0.0, 0.0, 1.0, KB)
    e = (x[1] - x[0]) / np.linalg.norm(x[1] - x[0])
    r = x[3] - x[0]
    # Rodrigues' rotation of x3 about the edge axis through x0
    rr = r * np.cos(delta) + np.cross(e, r) * np.sin(delta) + e * np.dot(e, r) * (1 - np.cos(delta))
    X = x.copy()
    X[3] = x[0] + rr
    t.set_membrane_vertices(X)
    th, th0 = t.membrane_dihedrals(0)
    assert len(th) == 1 and abs(abs(th[0] - th0[0]) - abs(delta)) < 1e-12
    assert t.membrane_energy(0)[3] == pytest.approx(KB * (1 - np.cos(delta)), rel=1e-12)
    F = t.membrane_forces(0)
    h = 1e-6
    for v in range(4):
        for q in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[v, q] += h
            Xm[v, q] -= h
            t.set_membrane_vertices(Xp)
            ep = t.membrane_energy(0)[3]
            t.set_membrane_vertices(Xm)
            em = t.membrane_energy(0)[3]
            assert F[v, q] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-9 * KB)
