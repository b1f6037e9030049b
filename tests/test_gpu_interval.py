"""A new solution interval through calib_set_data: the same context, new visibilities and
coherencies (same array, frequencies and flags).  The repacked inputs and coherency statistics
must give exactly what a context built on the new interval gives, and non-finite inputs must mark
their subbands."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


@pytest.mark.parametrize("precision,solver", [(0, 0), (1, 3)])
def test_set_data_equals_a_fresh_context(cal, synth_mod, precision, solver):
    cfg = synth_mod.SynthConfig("iv", N=9, P=5, Q=2, K=3, T=3, n_chan=[1, 3, 2, 4, 2],
                                n_dirs=[3, 2, 3, 3, 2], flag_frac_max=0.25, lm_iters=4,
                                config_index=21)
    a = synth_mod.episode_interval(cfg, 0, 1, 4)
    b = synth_mod.episode_interval(cfg, 0, 2, 4)
    np.testing.assert_array_equal(a["flags"], b["flags"])
    kw = dict(precision=precision, lm_iters=4, options=0, lm_tol=1e-7, solver=solver)
    va, ca, fa = cal.device_inputs(a, precision)
    vb, cb, fb = cal.device_inputs(b, precision)
    reused = cal.Calib(a, va, ca, fa, **kw)
    reused.solve(2)                       # a solve on interval a, then the next interval
    J = reused.get(cal.FIELD_J)
    reused.set_data(vb, cb)
    fresh = cal.Calib(b, vb, cb, fb, **kw)
    reused.set_state(J)
    fresh.set_state(J)
    np.testing.assert_array_equal(reused.get(cal.FIELD_COST).cpu().numpy(),
                                  fresh.get(cal.FIELD_COST).cpu().numpy())
    ta, tb = reused.solve(3), fresh.solve(3)
    np.testing.assert_array_equal(ta, tb)
    np.testing.assert_array_equal(reused.get(cal.FIELD_J).cpu().numpy(),
                                  fresh.get(cal.FIELD_J).cpu().numpy())


def test_set_data_reports_non_finite_inputs(cal, synth_mod):
    cfg = synth_mod.SynthConfig("iv", N=7, P=4, Q=2, K=2, T=3, n_chan=2, lm_iters=3, config_index=22)
    a = synth_mod.episode_interval(cfg, 0, 0, 3)
    b = dict(synth_mod.episode_interval(cfg, 0, 1, 3))
    b["vis"] = b["vis"].copy()
    b["vis"][b["vis_off"][3] + 5, 1, 0] = np.nan   # a sample of subband 3
    va, ca, fa = cal.device_inputs(a, 0)
    vb, cb, _ = cal.device_inputs(b, 0)
    c = cal.Calib(a, va, ca, fa, lm_iters=3, options=0)
    c.set_data(vb, cb)
    np.testing.assert_array_equal(c.get(cal.FIELD_STATUS).cpu().numpy(), [0, 0, 0, 5])
    with pytest.raises(cal.CalibError) as e:
        c.solve(1)
    assert e.value.status == 5
