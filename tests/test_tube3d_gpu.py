"""The 3D extension's lattice on the GPU (D3Q19 BGK with the Guo term in a
capillary tube, FP32 deviation storage, FP64 collision) against the FP64
oracle, element by element, through the C-ABI: small lattices with ragged x
segments in all three geometries from a perturbed state, and the full
256 x 64 x 64 tube at Re = 0.01."""
import numpy as np
import pytest

from helpers import rel_max, say
from oracle import tube3d as otube
from paper_2210_06043_amd import capib, inputs, tube3d

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _pair(nx, ny, nz, tau, gx, geom, radius, profile=None, perturb=0.0, seed=0, fp16_umax=0.0):
    if fp16_umax:
        g = tube3d.Tube3D(nx, ny, nz, tau, gx, geometry=geom, radius=radius, storage=capib.FP16_SHIFTED,
                          fp16_scale=tube3d.fp16_scale_for(fp16_umax))
    else:
        g = tube3d.Tube3D(nx, ny, nz, tau, gx, geometry=geom, radius=radius)
    o = otube.Tube(nx, ny, nz, tau, gx, geom=geom, radius=radius)
    g.init_flow(profile)
    o.init_flow(profile)
    if perturb:
        A = o.populations()
        fl = o.fluid()
        rng = np.random.default_rng(seed)
        A += perturb * rng.standard_normal(A.shape) * fl[None, :, :, None]
        g.set_populations(A)
    # the oracle starts from exactly what the GPU stores (FP32 deviations)
    o.set_populations(g.populations())
    return g, o


def _compare(g, o, steps, label, tol=TOL):
    g.step(steps)
    o.step(steps)
    dg, uxg, uyg, uzg = g.macro()
    do, uxo, uyo, uzo = o.macro()
    eu = rel_max(np.stack([uxg, uyg, uzg]), np.stack([uxo, uyo, uzo]))
    scale = max(np.abs(do).max(), np.abs(np.stack([uxo, uyo, uzo])).max())
    ed = np.abs(dg - do).max() / scale
    dgn, tot = g.diagnostics(), o.totals()
    say(f"{label}: velocity rel err {eu:.3e}, drho err {ed:.3e}; mass {dgn['mass']:.6e} vs {tot[0]:.6e}, "
        f"momentum x {dgn['mom_x']:.9e} vs {tot[1]:.9e}")
    assert eu < tol and ed < tol
    n = g.fluid_nodes
    # FP16 stores deviations to 2^-11 of the flow scale per node, so the sums
    # are compared at that resolution; FP32 to rounding
    r = 1.0 if tol > TOL else 1e-4
    assert abs(dgn["mass"] - tot[0]) < 1e-5 * r * n
    assert abs(dgn["mom_x"] - tot[1]) < tol * abs(tot[1]) + 1e-12 * n
    assert abs(dgn["mom_y"] - tot[2]) < 1e-5 * r * n and abs(dgn["mom_z"] - tot[3]) < 1e-5 * r * n
    return eu


@pytest.mark.parametrize("geom,nx,ny,nz,tau,radius", [(tube3d.TUBE, 40, 14, 14, 0.8, 6.3),
                                                      (tube3d.SLAB, 70, 6, 9, 1.3, 0.0),
                                                      (tube3d.BOX, 33, 5, 7, 0.6, 0.0)])
def test_small_lattices_from_a_perturbed_state(geom, nx, ny, nz, tau, radius):
    """200 steps from the Hagen-Poiseuille (tube) or rest state plus a
    random perturbation of 2e-4: x segments of 64 with a ragged last one,
    bounce-back on every kind of link, periodic wrap in every direction the
    geometry has."""
    gx = 2e-6
    prof = tube3d.hagen_poiseuille(ny, nz, radius, tau, gx) if geom == tube3d.TUBE else None
    g, o = _pair(nx, ny, nz, tau, gx, geom, radius, prof, perturb=2e-4, seed=geom)
    _compare(g, o, 200, f"3d geom {geom} {nx}x{ny}x{nz} tau {tau}")


def test_full_tube_at_re_0_01():
    """The 256 x 64 x 64 tube (R = 32, 822k fluid nodes) at Re = 0.01 from
    the Hagen-Poiseuille profile with a perturbation of 1e-3 u_mean: 100
    steps, every node."""
    p = inputs.tube3d_params()
    prof = tube3d.hagen_poiseuille(p["ny"], p["nz"], p["radius"], p["tau"], p["gx"])
    g, o = _pair(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], tube3d.TUBE, p["radius"], prof,
                 perturb=1e-3 * p["u_mean"], seed=5)
    assert g.fluid_nodes == 256 * 3228
    _compare(g, o, 100, "3d tube 256x64x64")


def test_tube_keeps_its_mass_and_gains_momentum_from_the_drive():
    """Over 400 steps the FP64 device sums keep the mass to rounding and
    the momentum grows by the body force per fluid node and step."""
    p = inputs.tube3d_params(nx=64, diameter=24)
    g = tube3d.Tube3D(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], radius=p["radius"])
    g.init_flow()
    d0 = g.diagnostics()
    g.step(1)
    d1 = g.diagnostics()
    n = g.fluid_nodes
    say(f"3d: mass {d0['mass']:.3e} -> {d1['mass']:.3e}; momentum gain {d1['mom_x'] - d0['mom_x']:.9e} vs "
        f"{n * p['gx']:.9e}")
    assert abs(d1["mass"] - d0["mass"]) < 1e-9 * n
    # from rest one step adds exactly g per node (walls act from the second)
    assert d1["mom_x"] - d0["mom_x"] == pytest.approx(n * p["gx"], rel=1e-5)
    g.step(399)
    d2 = g.diagnostics()
    assert abs(d2["mass"] - d0["mass"]) < 1e-9 * n and d2["step"] == 400


FP16_TOL = 1e-3


def test_fp16_storage_small_tube():
    """FP16 deviation storage (FP32 arithmetic), 300 steps of a small tube
    from the Hagen-Poiseuille profile plus a perturbation of 1e-2 of the
    flow speed: within 1e-3 of the FP64 oracle."""
    nx, n, R, tau, gx = 40, 14, 6.3, 0.8, 2e-6
    prof = tube3d.hagen_poiseuille(n, n, R, tau, gx)
    g, o = _pair(nx, n, n, tau, gx, tube3d.TUBE, R, prof, perturb=1e-2 * prof.max(), seed=9,
                 fp16_umax=prof.max())
    _compare(g, o, 300, "3d fp16 tube 40x14x14", tol=FP16_TOL)


def test_fp16_storage_full_tube():
    """The 256 x 64 x 64 tube at Re = 0.01 with FP16 storage, 100 steps."""
    p = inputs.tube3d_params()
    prof = tube3d.hagen_poiseuille(p["ny"], p["nz"], p["radius"], p["tau"], p["gx"])
    g, o = _pair(p["nx"], p["ny"], p["nz"], p["tau"], p["gx"], tube3d.TUBE, p["radius"], prof,
                 perturb=1e-3 * p["u_mean"], seed=6, fp16_umax=prof.max())
    _compare(g, o, 100, "3d fp16 tube 256x64x64", tol=FP16_TOL)
