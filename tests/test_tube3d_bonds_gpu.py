"""Ligand-receptor bonds in the 3D extension's tube on the GPU (sites on a
membrane's triangles, anchors on the tube wall, Sec. 2.5 and Eq. 13 carried
to 3D) against the FP64 oracle through the C-ABI: every bond state and
anchor exactly as the oracle's over 200 coupled steps with some 20 state
changes (the seed is chosen so that no decision lies near its threshold,
and the test checks that), and the host's refusals."""
import numpy as np
import pytest

from helpers import rel_max, say
from oracle import tube3d as otube
from paper_2210_06043_amd import capib, inputs, tube3d

pytestmark = pytest.mark.gpu
NX, N, R, TAU, GX = 48, 24, 11.0, 0.9, 3e-6
C0 = 0.5 * (N - 1)
MEM = dict(gs=5e-2, c=1.0, ka=0.5, kv=0.5, mass=1.0, kb=2e-2)
BONDS = dict(sigma=1e-3, yeq=1.0, ycr=2.2, kf=0.05, kr0=0.005, lb=1.0, seed=2)


def _sites(ntri, ns=300, seed=3):
    rng = np.random.default_rng(seed)
    st = rng.integers(0, ntri, ns).astype(np.int32)
    u = rng.random((ns, 2))
    u[u.sum(axis=1) > 1] = 1 - u[u.sum(axis=1) > 1]
    return st, u


def _pair(ns=300):
    xyz, tri = inputs.icosphere(3, 3.0, (24.3, C0 + 5.9, C0 - 0.3))
    st, u = _sites(len(tri), ns)
    prof = tube3d.hagen_poiseuille(N, N, R, TAU, GX)
    g = tube3d.Tube3D(NX, N, N, TAU, GX, radius=R, max_membranes=1, max_membrane_vertices=len(xyz),
                      max_membrane_triangles=len(tri), max_sites=ns)
    o = otube.Tube(NX, N, N, TAU, GX, radius=R)
    g.init_flow(prof)
    o.init_flow(prof)
    o.set_populations(g.populations())
    g.add_membrane(xyz, tri, **MEM)
    o.add_membrane(xyz, tri, *(MEM[k] for k in ("gs", "c", "ka", "kv", "mass", "kb")))
    g.add_bonds(0, st, u, **BONDS)
    o.add_bonds(0, st, u, *(BONDS[k] for k in ("sigma", "yeq", "ycr", "kf", "kr0", "lb", "seed")))
    return g, o


def test_bond_states_follow_the_oracle_exactly():
    g, o = _pair()
    changes = []
    for k in range(4):
        g.step(50)
        o.step(50)
        bg, ag, ng = g.bonds()
        bo, ao, no = o.bonds()
        m = o.bond_margins()
        say(f"3d bonds, step {50 * (k + 1)}: {ng} bound (oracle {no}), {int(m[2])} changes, margins {m[0]:.2e} "
            f"{m[1]:.2e}")
        assert m[0] > 1e-7 and m[1] > 1e-7
        assert np.array_equal(bg, bo)
        if no:
            assert np.abs(ag[bo == 1] - ao[bo == 1]).max() < 1e-8
        changes.append(m[2])
    assert changes[-1] >= 15 and no > 0
    _, uxg, uyg, uzg = g.macro()
    _, uxo, uyo, uzo = o.macro()
    eu = rel_max(np.stack([uxg, uyg, uzg]), np.stack([uxo, uyo, uzo]))
    X0 = inputs.icosphere(3, 3.0, (24.3, C0 + 5.9, C0 - 0.3))[0]
    ex = np.abs(g.membrane_vertices() - o.membrane_vertices()).max() / np.abs(o.membrane_vertices() - X0).max()
    say(f"3d bonds: velocity rel err {eu:.2e}, vertex err {ex:.2e} of the displacement")
    assert eu < 1e-5 and ex < 1e-5


def test_bond_refusals():
    g, _ = _pair(ns=10)
    with pytest.raises(capib.CapibError) as e:
        g.add_bonds(0, np.zeros(2, dtype=np.int32), np.array([[0.2, 0.2], [0.3, 0.3]]), **BONDS)
    assert e.value.status == capib.CAPIB_E_STATE
    xyz, tri = inputs.icosphere(2, 3.0, (20.0, C0, C0))
    h = tube3d.Tube3D(40, N, N, TAU, GX, radius=R, max_membranes=1, max_membrane_vertices=len(xyz),
                      max_membrane_triangles=len(tri), max_sites=4)
    h.init_flow()
    h.add_membrane(xyz, tri, **MEM)
    for st, bary, status in ((np.array([0, 1, 2, 3, 4]), np.full((5, 2), 0.2), capib.CAPIB_E_CAPACITY),
                             (np.array([len(tri)]), np.array([[0.2, 0.2]]), capib.CAPIB_E_ARG),
                             (np.array([0]), np.array([[0.7, 0.6]]), capib.CAPIB_E_ARG)):
        with pytest.raises(capib.CapibError) as e:
            h.add_bonds(0, st.astype(np.int32), bary, **BONDS)
        assert e.value.status == status
    h.add_bonds(0, np.array([0], dtype=np.int32), np.array([[0.2, 0.2]]), **BONDS)
    h.step(2)
    assert h.bonds()[2] == 0
