"""Deformable membranes in the 3D extension's tube on the GPU (Skalak
elements, dihedral bending, area and volume penalties, the 2D membranes' vertex update in 3D,
fixed-point spreading) against the FP64 oracle through the C-ABI: every
node's velocity, every vertex's position and direct force, and the FP64
area and volume sums, on small tubes (a membrane across the periodic end,
two membranes, a membrane moved from the host mid-run, one added after
steps, FP16 storage), the 256 x 64 x 64 tube with four 2562-vertex
cells and a 642-vertex sphere (FP32 and FP16 storage); bitwise repeatability; the host's refusals
and the wall flag."""
import numpy as np
import pytest

from helpers import rel_max, say
from oracle import tube3d as otube
from paper_2210_06043_amd import capib, inputs, tube3d

pytestmark = pytest.mark.gpu
TOL = 1e-5
FP16_TOL = 1e-3
PAR = dict(gs=5e-3, c=1.0, ka=0.05, kv=0.05, mass=1.0, kb=2e-3)


def _pair(nx, ny, nz, tau, gx, radius, membranes, dilate=1.02, fp16=False, par=PAR):
    prof = tube3d.hagen_poiseuille(ny, nz, radius, tau, gx)
    nv = sum(len(m[0]) for m in membranes)
    nt = sum(len(m[1]) for m in membranes)
    kw = dict(storage=capib.FP16_SHIFTED, fp16_scale=tube3d.fp16_scale_for(max(prof.max(), 1e-4))) if fp16 else {}
    g = tube3d.Tube3D(nx, ny, nz, tau, gx, radius=radius, max_membranes=len(membranes), max_membrane_vertices=nv,
                      max_membrane_triangles=nt, **kw)
    o = otube.Tube(nx, ny, nz, tau, gx, radius=radius)
    g.init_flow(prof)
    o.init_flow(prof)
    o.set_populations(g.populations())
    for xyz, tri in membranes:
        v0 = g.add_membrane(xyz, tri, **par)
        assert o.add_membrane(xyz, tri, par["gs"], par["c"], par["ka"], par["kv"], par["mass"], par["kb"]) == v0
    # start from a dilated shape so that the elastic forces act from the first step
    X = o.membrane_vertices()
    for v0, n in o.mranges:
        c = X[v0:v0 + n].mean(axis=0)
        X[v0:v0 + n] = c + dilate * (X[v0:v0 + n] - c)
    g.set_membrane_vertices(X)
    o.set_membrane_vertices(X)
    return g, o


def _compare(g, o, steps, label, tol=TOL):
    X0 = o.membrane_vertices()
    g.step(steps - 1)
    o.step(steps - 1)
    before = [o.membrane_totals(m) for m in range(len(o.mranges))]
    g.step(1)
    o.step(1)
    _, uxg, uyg, uzg = g.macro()
    _, uxo, uyo, uzo = o.macro()
    eu = rel_max(np.stack([uxg, uyg, uzg]), np.stack([uxo, uyo, uzo]))
    Xg, Xo = g.membrane_vertices(), o.membrane_vertices()
    Fg, Fo = g.membrane_spread_forces(), o.membrane_spread_forces()
    ex = np.abs(Xg - Xo).max() / np.abs(Xo - X0).max()
    ef = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    et = max(max(abs(g.membrane_totals(m)[k] - before[m][k]) / before[m][k] for k in (0, 1))
             for m in range(len(before)))
    say(f"{label}: velocity rel err {eu:.3e}, vertex err {ex:.3e} of the largest displacement, direct force "
        f"rel err {ef:.3e}, area/volume rel err {et:.2e}, flags {g.error_flags()}")
    assert eu < tol and ex < tol and ef < tol and et < tol * 1e-3 and g.error_flags() == 0
    return eu


def test_membrane_across_the_periodic_end():
    """A 642-vertex membrane of radius 4 centred at x = 45.5 of a 48-node
    tube (its stencils wrap around the periodic end), dilated 2 %, in
    Poiseuille flow: 200 steps."""
    m = inputs.icosphere(3, 4.0, (45.5, 11.8, 11.3))
    g, o = _pair(48, 24, 24, 0.9, 3e-6, 11.0, [m])
    _compare(g, o, 200, "3d membrane at the periodic end")


def test_two_membranes_of_different_sizes():
    """A 162-vertex sphere and a 642-vertex oblate membrane (axes 1, 1, 0.5)
    in one tube: 150 steps; the vertex numbering follows the order of
    addition."""
    m1 = inputs.icosphere(2, 3.0, (20.3, 12.4, 12.1))
    m2 = inputs.icosphere(3, 4.5, (58.1, 11.7, 12.9), axes=(1.0, 1.0, 0.5))
    g, o = _pair(80, 25, 25, 1.0, 4e-6, 12.0, [m1, m2])
    assert g.membranes == 2 and g.membrane_vertex_count == len(m1[0]) + len(m2[0])
    _compare(g, o, 150, "3d two membranes")


def test_membrane_moved_from_the_host_mid_run():
    """40 steps, then the membrane moved from the host by (40, 2.5, -1.5)
    nodes on both sides (the work items under its stencils change: other
    columns and another 64-node segment of x; those of the old position keep
    their flags from the last step), then 60 more steps against the
    oracle."""
    m = inputs.icosphere(3, 4.0, (30.2, 11.8, 11.3))
    g, o = _pair(96, 24, 24, 0.9, 3e-6, 11.0, [m])
    g.step(40)
    o.step(40)
    X = o.membrane_vertices() + np.array([40.0, 2.5, -1.5])
    g.set_membrane_vertices(X)
    o.set_membrane_vertices(X)
    _compare(g, o, 60, "3d membrane moved from the host")


def test_membrane_added_after_steps():
    """One membrane for 30 steps, then a second added on both sides (its
    vertices numbered after the first's), then 80 more steps against the
    oracle."""
    m1 = inputs.icosphere(3, 4.0, (20.2, 11.8, 11.3))
    m2 = inputs.icosphere(2, 3.0, (60.7, 12.3, 10.9))
    prof = tube3d.hagen_poiseuille(24, 24, 11.0, 0.9, 3e-6)
    g = tube3d.Tube3D(96, 24, 24, 0.9, 3e-6, radius=11.0, max_membranes=2,
                      max_membrane_vertices=len(m1[0]) + len(m2[0]), max_membrane_triangles=len(m1[1]) + len(m2[1]))
    o = otube.Tube(96, 24, 24, 0.9, 3e-6, radius=11.0)
    g.init_flow(prof)
    o.init_flow(prof)
    o.set_populations(g.populations())
    for mm in (m1,):
        assert g.add_membrane(*mm, **PAR) == o.add_membrane(*mm, PAR["gs"], PAR["c"], PAR["ka"], PAR["kv"],
                                                            PAR["mass"], PAR["kb"])
    g.step(30)
    o.step(30)
    assert g.add_membrane(*m2, **PAR) == o.add_membrane(*m2, PAR["gs"], PAR["c"], PAR["ka"], PAR["kv"], PAR["mass"],
                                                       PAR["kb"]) == len(m1[0])
    _compare(g, o, 80, "3d membrane added after steps")


def test_fp16_storage_with_a_membrane():
    m = inputs.icosphere(3, 4.0, (30.2, 11.8, 11.3))
    g, o = _pair(64, 24, 24, 0.9, 3e-6, 11.0, [m], fp16=True)
    _compare(g, o, 200, "3d membrane fp16", tol=FP16_TOL)


def _full_tube(fp16):
    """The 3D workload (inputs.tube3d_workload): the 256 x 64 x 64 tube at
    Re = 0.01 with four 2562-vertex oblate cells and a 642-vertex oblate
    particle 2.5 nodes from the wall carrying 300 ligand sites: 50 steps,
    every node and vertex, and every bond state and anchor exactly as the
    oracle's (its smallest decision margins are checked first, against the
    run's own position error)."""
    p = inputs.tube3d_params()
    w = inputs.tube3d_workload(p)
    prof = tube3d.hagen_poiseuille(p["ny"], p["nz"], p["radius"], p["tau"], p["gx"])
    mem = w["cells"] + [w["particle"]]
    pars = [w["cell"]] * 4 + [w["part"]]
    kw = dict(storage=capib.FP16_SHIFTED, fp16_scale=tube3d.fp16_scale_for(max(prof.max(), 1e-4))) if fp16 else {}
    g = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"], max_membranes=5,
                      max_membrane_vertices=sum(len(m[0]) for m in mem),
                      max_membrane_triangles=sum(len(m[1]) for m in mem), max_sites=len(w["sites"][0]), **kw)
    o = otube.Tube(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"])
    g.init_flow(prof)
    o.init_flow(prof)
    o.set_populations(g.populations())
    for (xyz, tri), q in zip(mem, pars):
        g.add_membrane(xyz, tri, **q)
        o.add_membrane(xyz, tri, q["gs"], q["c"], q["ka"], q["kv"], q["mass"], q["kb"])
    b = w["bonds"]
    g.add_bonds(4, *w["sites"], **b)
    o.add_bonds(4, *w["sites"], b["sigma"], b["yeq"], b["ycr"], b["kf"], b["kr0"], b["lb"], b["seed"])
    label = "3d full tube, 4 cells + bonded particle" + (", fp16" if fp16 else "")
    _compare(g, o, 50, label, tol=FP16_TOL if fp16 else TOL)
    bg, ag, ng = g.bonds()
    bo, ao, no = o.bonds()
    margins = o.bond_margins()
    dx = np.abs(g.membrane_vertices() - o.membrane_vertices()).max()
    say(f"{label}: {ng} bound after 50 steps (oracle {no}), {int(margins[2])} state changes, smallest margins "
        f"{margins[0]:.2e} (draw) {margins[1]:.2e} (gap), largest vertex error {dx:.2e}")
    # a site's gap and stretch move by at most the vertex error, and the
    # decision probabilities by less than that (their slopes are below 1 here)
    assert margins[0] > 100 * dx and margins[1] > 100 * dx and margins[2] > 20
    assert np.array_equal(bg, bo) and ng == no
    assert np.abs(ag[bo == 1] - ao[bo == 1]).max() < (1e-5 if fp16 else 1e-7)


def test_full_tube_with_four_cells_and_a_bonded_particle():
    _full_tube(fp16=False)


def test_full_tube_with_fp16_storage():
    """The same workload with FP16 storage (the configuration the FP16
    membrane timing runs), against the same FP64 oracle run."""
    _full_tube(fp16=True)


def test_repeated_runs_are_bit_identical():
    """The fixed-point spreading sums the same integers in any order, so two
    runs of the same set-up give the same populations and vertices, bit for
    bit."""
    m = inputs.icosphere(3, 4.0, (30.2, 11.8, 11.3))
    out = []
    for _ in range(2):
        g, _ = _pair(64, 24, 24, 0.9, 3e-6, 11.0, [m])
        g.step(60)
        out.append((g.populations(), g.membrane_vertices()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_refusals_and_the_wall_flag():
    """Capacity, a stencil reaching the wall, a degenerate triangle and a
    context that already holds fixed bodies are refused on the host; a
    membrane moved against the wall from the host raises flag 1 on the next
    step and the run goes on."""
    xyz, tri = inputs.icosphere(2, 3.0, (16.0, 11.5, 11.5))
    g = tube3d.Tube3D(32, 24, 24, 0.9, 0.0, radius=11.0, max_membranes=1, max_membrane_vertices=len(xyz),
                      max_membrane_triangles=len(tri), max_vertices=len(xyz))
    g.init_flow()
    with pytest.raises(capib.CapibError) as e:
        g.add_membrane(xyz + np.array([0.0, 8.0, 0.0]), tri, **PAR)
    assert e.value.status == capib.CAPIB_E_ARG
    flat = xyz.copy()
    flat[tri[0, 1]] = flat[tri[0, 0]]
    with pytest.raises(capib.CapibError) as e:
        g.add_membrane(flat, tri, **PAR)
    assert e.value.status == capib.CAPIB_E_ARG
    with pytest.raises(capib.CapibError) as e:
        g.add_membrane(xyz[:, [0, 2, 1]], tri, **PAR)   # mirrored: clockwise from outside
    assert e.value.status == capib.CAPIB_E_ARG
    assert g.add_membrane(xyz, tri, **PAR) == 0
    with pytest.raises(capib.CapibError) as e:
        g.add_membrane(xyz, tri, **PAR)
    assert e.value.status == capib.CAPIB_E_CAPACITY
    with pytest.raises(capib.CapibError) as e:
        g.add_fixed_body(xyz, tri)
    assert e.value.status == capib.CAPIB_E_STATE
    g.step(3)
    assert g.error_flags() == 0
    g.set_membrane_vertices(g.membrane_vertices() + np.array([0.0, 7.5, 0.0]))
    g.step(2)
    assert g.error_flags() & 1
    assert np.isfinite(g.membrane_vertices()).all()
