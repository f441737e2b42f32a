"""The synthetic batched-ensemble recipe (256 capillaries of uneven length,
1-4 cells, one adhered particle each) has the sizes and value ranges it
states, and its members are valid inputs (bodies inside the channel, apart
from each other, bonds engaged at t = 0)."""
import numpy as np
import pytest

from paper_2210_06043_amd import inputs


@pytest.fixture(scope="module")
def c3():
    return inputs.config_c3(seed=0)


def test_c3_sizes_and_ranges(c3):
    assert len(c3) == 256
    for k, c in enumerate(c3):
        assert c.ny == 64 and 256 <= c.nx <= 2048 and c.tau == 1.0
        assert 1 <= c.meta["ncell"] <= 4 and len(c.bodies) == c.meta["ncell"] + 1
        for b in c.bodies[:-1]:
            assert b.kind == inputs.DEFORMABLE and 128 <= len(b.xy) <= 256
        part = c.bodies[-1]
        assert len(part.xy) == 64 and part.tag == inputs.TAG_PARTICLE
        assert 0.25 <= c.meta["ar"] <= 1.0
        ca = c.meta["ca"]
        assert (ca == 0.0 and part.kind == inputs.RIGID) or (1e-5 <= ca <= 1e-3 and part.kind == inputs.DEFORMABLE)
        assert c.bonds[0].seed == 0 * (1 << 20) + k
    # all members share the drive and profile, so they can share one ensemble
    assert len({(c.gx, c.tau) for c in c3}) == 1
    assert all(np.array_equal(c.ux_init, c3[0].ux_init) for c in c3)
    # the rigid class: about a quarter (binomial, 3 sigma)
    nr = sum(c.meta["ca"] == 0.0 for c in c3)
    assert abs(nr - 64) < 3 * np.sqrt(256 * 0.25 * 0.75)
    lengths = np.array([c.nx for c in c3])
    assert 900 < lengths.mean() < 1400      # U{256..2048} has mean 1152


def test_c3_members_are_valid_inputs(c3):
    for c in c3[:64]:
        ys = np.concatenate([b.xy[:, 1] for b in c.bodies])
        assert ys.min() > -0.5 and ys.max() < c.ny - 0.5
        for a in range(len(c.bodies)):
            for b in range(a + 1, len(c.bodies)):
                A, B = c.bodies[a].xy, c.bodies[b].xy
                dx = A[:, None, 0] - B[None, :, 0]
                dx -= c.nx * np.round(dx / c.nx)
                assert np.sqrt(dx ** 2 + (A[:, None, 1] - B[None, :, 1]) ** 2).min() > 5.0
        # the particle's engaged sites sit within y_cr of the wall
        bd = c.bonds[0]
        xy = c.bodies[bd.body].xy
        e = bd.host
        nxt = xy[(e + 1) % len(xy)]
        ys = xy[e, 1] + bd.frac * (nxt[:, 1] - xy[e, 1])
        assert np.sum(ys + 0.5 < bd.ycr) == 20


def test_small_ensemble_shares_its_profile():
    m = inputs.config_ensemble_small()
    assert [c.nx for c in m] == [37, 64, 100, 131] and all(c.ny == 24 for c in m)
    assert all(np.array_equal(c.ux_init, m[0].ux_init) for c in m)
    assert [len(c.bodies) for c in m] == [2, 1, 2, 0]
