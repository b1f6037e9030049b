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


@pytest.mark.parametrize("precision", [0, 1])
def test_statistics_only_context(cal, synth_mod, oracle_mod, precision):
    """CALIB_OPT_STATS_ONLY keeps no packed copy of the samples: the matrix-free solve, which
    reads only the coherency statistics, gives bitwise what a context with the copy gives, over a
    new interval too; the data cost comes from the statistics, formed in FP64 also from FP32
    inputs (within 1e-12 of the oracle's per-sample sum on the same, FP32-rounded, inputs); the
    model visibilities are refused, and so is any other solver."""
    cfg = synth_mod.SynthConfig("so", N=9, P=5, Q=2, K=3, T=3, n_chan=[1, 3, 2, 4, 2],
                                n_dirs=[3, 2, 3, 3, 2], flag_frac_max=0.25, lm_iters=4,
                                config_index=23)
    a = synth_mod.episode_interval(cfg, 0, 1, 4)
    b = synth_mod.episode_interval(cfg, 0, 2, 4)
    kw = dict(precision=precision, lm_iters=4, lm_tol=1e-7, solver=3, cg_tol=1e-10)
    va, ca, fa = cal.device_inputs(a, precision)
    vb, cb, _ = cal.device_inputs(b, precision)
    full = cal.Calib(a, va, ca, fa, options=0, **kw)
    only = cal.Calib(a, va, ca, fa, options=cal.OPT_STATS_ONLY, **kw)
    for c in (full, only):
        c.solve(2)
        c.set_data(vb, cb)
    ta, tb = full.solve(3), only.solve(3)
    np.testing.assert_array_equal(ta, tb)
    J = only.get(cal.FIELD_J).cpu().numpy()
    np.testing.assert_array_equal(full.get(cal.FIELD_J).cpu().numpy(), J)
    g_full = full.get(cal.FIELD_COST).cpu().numpy()
    g_only = only.get(cal.FIELD_COST).cpu().numpy()
    # the full context's cost is a pass over the samples, in FP32 per sample on the FP32 path
    np.testing.assert_allclose(g_only, g_full, rtol=1e-12 if precision == 0 else 1e-6)
    inputs = b if precision == 0 else synth_mod.as_fp32_inputs(b)
    want = oracle_mod.Problem(inputs).subband_cost(J)
    np.testing.assert_allclose(g_only, want, rtol=1e-12)
    with pytest.raises(cal.CalibError) as e:
        only.get(cal.FIELD_MODEL_VIS)
    assert e.value.status == 6
    full.close()
    only.close()
    with pytest.raises(cal.CalibError) as e:
        cal.Calib(a, va, ca, fa, options=cal.OPT_STATS_ONLY, precision=precision, solver=1)
    assert e.value.status == 1
