"""Launch configurations and the autotuner: the schedules of the step (far
tiles in their own launch or in the sweep, the membrane launch's far share,
the marking layout) compute the same results bit for bit, a larger
membrane class (other thread counts, so other orders of the FP64 membrane
sums) the same to rounding, and capib_autotune leaves the run's state as it
found it, applies a valid configuration and reuses its cache.  All calls
go through the C-ABI."""
import numpy as np
import pytest

from helpers import gpu_sim, say
from paper_2210_06043_amd import capib, inputs

pytestmark = pytest.mark.gpu

CONFIGS = [dict(), dict(split=1), dict(split=0, far_share_pct=20), dict(split=0, far_share_pct=95),
           dict(mark_pairs=0), dict(mark_pairs=1), dict(membrane_class=512), dict(membrane_class=1024)]
ROUNDING_ONLY = ("membrane_class",)


def _state(g, cfg):
    return [g.read_populations()] + [g.vertices(k) for k in range(len(cfg.bodies))] + \
        [g.bonds(bd.body)[0] for bd in cfg.bonds]


@pytest.mark.parametrize("name", ["tiny", "c1", "ensemble"])
def test_every_configuration_gives_the_same_bits(name):
    if name == "ensemble":
        cfgs = inputs.config_ensemble_small()
        make = lambda: capib.from_ensemble(cfgs, graph=True)[0]
        cfg = inputs.Config("ens", 0, 0, 1.0, 0.0)
    else:
        cfg = inputs.config_tiny() if name == "tiny" else inputs.config_c1()
        make = lambda: gpu_sim(cfg, graph=True)
    ref = None
    for t in CONFIGS:
        g = make()
        g.set_tuning(**t)
        g.step(60)
        st = [g.read_populations()] if name == "ensemble" else _state(g, cfg)
        say(f"{name} {t}: resolved {g.tuning()}")
        if ref is None:
            ref = st
        elif any(k in t for k in ROUNDING_ONLY):
            for a, b in zip(ref, st):
                np.testing.assert_allclose(b, a, rtol=0, atol=1e-6 * max(np.abs(a).max(), 1e-30))
        else:
            for a, b in zip(ref, st):
                assert np.array_equal(a, b), (name, t)
        assert g.diagnostics()["error_flags"] == 0


def test_autotune_keeps_the_state_and_uses_its_cache(tmp_path):
    cfg = inputs.config_c1()
    a = gpu_sim(cfg, graph=True)
    b = gpu_sim(cfg, graph=True)
    a.step(50)
    b.step(50)
    cache = tmp_path / "tune.txt"
    t1 = b.autotune(steps_per_trial=64, cache_path=str(cache))
    say(f"c1 autotune: {t1}")
    assert t1["split"] in (0, 1) and t1["mark_pairs"] in (0, 1) and 0 <= t1["far_share_pct"] <= 100
    assert t1["membrane_class"] in (256, 512, 1024) and t1["ms_per_step"] > 0
    assert b.tuning() == {k: t1[k] for k in ("split", "far_share_pct", "mark_pairs", "membrane_class")}
    assert b.diagnostics()["step"] == 50
    a.step(50)
    b.step(50)
    for x, y in zip(_state(a, cfg), _state(b, cfg)):
        assert np.array_equal(x, y)
    assert cache.read_text().count("\t") == 1
    c = gpu_sim(cfg, graph=True)
    t2 = c.autotune(steps_per_trial=64, cache_path=str(cache))
    assert {k: t2[k] for k in t2 if k != "ms_per_step"} == {k: t1[k] for k in t1 if k != "ms_per_step"}
    assert abs(t2["ms_per_step"] - t1["ms_per_step"]) < 1e-6         # read back from the cache
    assert cache.read_text().count("\t") == 1


def test_tuning_is_validated():
    g = gpu_sim(inputs.config_tiny())
    for bad in (dict(split=2), dict(far_share_pct=101), dict(mark_pairs=-2), dict(membrane_class=300)):
        with pytest.raises(capib.CapibError):
            g.set_tuning(**bad)
