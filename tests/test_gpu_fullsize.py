"""Parity at the benchmark's full sizes and launch configuration, and the tile-shape tuner.

At full size the oracle checks what it can compute one subband at a time: the first local step
(Y = Z = 0, so subbands are independent) of sampled subbands of c2 (62 stations, 5 directions,
32 subbands x 4 channels) and of the batched c3 (256 subbands, 1-16 channels, 3-10 directions,
0-30% flagged baselines), and whole C-ADMM iterations of c2, with the Cholesky solvers and with
the benchmark's solver settings.  FP32 streaming against the FP64
oracle on the FP32-rounded inputs: 1e-5 relative on data costs.
"""
import numpy as np
import pytest

from conftest import subset

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


_DATA = {}


def _data(synth_mod, name):
    """Full-size inputs, generated once per module (c3 takes ~30 s to simulate)."""
    if name not in _DATA:
        print(f"{name}: generating full-size inputs", flush=True)
        d = synth_mod.generate(synth_mod.named_config(name))
        _DATA[name] = (d, synth_mod.as_fp32_inputs(d))
    return _DATA[name]


def _first_local_step_sampled(cal, oracle_mod, synth_mod, name, sample, oracle_kw=None, **shape):
    cfg = synth_mod.named_config(name)
    d, d32 = _data(synth_mod, name)
    print(f"{name}: P={cfg.P} sampled subbands {sample} "
          f"n_chan={list(np.asarray(d['n_chan'])[sample])} K_f={list(np.asarray(d['n_dirs'])[sample])}",
          flush=True)
    vis, coh, flags = cal.device_inputs(d, cal.CALIB_FP32_MIXED)
    c = cal.Calib(d, vis, coh, flags, precision=cal.CALIB_FP32_MIXED, **shape)
    c.local_step(0)
    g = c.get(cal.FIELD_COST).cpu().numpy()
    c.close()
    sub = subset(d32, sample)
    pb = oracle_mod.Problem(sub, **(oracle_kw or {}))
    J0 = synth_mod.identity_jones(len(sample), cfg.K, cfg.N)
    z = np.zeros_like(J0)
    want = pb.subband_cost(pb.local_step(J0, z, z))
    np.testing.assert_allclose(g[sample], want, rtol=1e-5)


def test_c2_first_local_step_sampled_subbands(cal, oracle_mod, synth_mod):
    _first_local_step_sampled(cal, oracle_mod, synth_mod, "c2", [0, 13, 31])


def test_c3_first_local_step_sampled_subbands(cal, oracle_mod, synth_mod):
    _first_local_step_sampled(cal, oracle_mod, synth_mod, "c3", [0, 77, 200, 255])


def test_c3_persistent_grid_sampled_subbands(cal, oracle_mod, synth_mod):
    _first_local_step_sampled(cal, oracle_mod, synth_mod, "c3", [5, 128], tile_group=16,
                              stream_grid=512)


def test_c2_whole_iteration(cal, oracle_mod, synth_mod):
    cfg = synth_mod.named_config("c2")
    d, d32 = _data(synth_mod, "c2")
    vis, coh, flags = cal.device_inputs(d, cal.CALIB_FP32_MIXED)
    c = cal.Calib(d, vis, coh, flags, precision=cal.CALIB_FP32_MIXED)
    trg = c.solve(1)
    c.close()
    print("c2: one C-ADMM iteration, oracle on all 32 subbands", flush=True)
    pb = oracle_mod.Problem(d32)
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 1)["trace"]
    np.testing.assert_allclose(trg[0, :2], tro[0, :2], rtol=1e-5)
    # residuals are norms of differences J - B_f Z of size ~1e-2: FP32 rounding of J (1e-7
    # relative) is amplified by ~1e2
    np.testing.assert_allclose(trg[0, 2:], tro[0, 2:], rtol=1e-3)


def test_c2_stopping_rule_solve(cal, oracle_mod, synth_mod):
    """The benchmark's launch configuration on the full c2 problem: FP32 streaming, the LM stopping
    rule at lm_tol 1e-7 (each subband moving through its own directions, the host reading the
    device's stop flag), three C-ADMM iterations from identity; the oracle runs the same rule on
    the FP32-rounded inputs of all 32 subbands.  Data cost and Lagrangian within 1e-5 (a stop
    decision that the FP32 energies flip changes the cost by about lm_tol)."""
    cfg = synth_mod.named_config("c2")
    d, d32 = _data(synth_mod, "c2")
    vis, coh, flags = cal.device_inputs(d, cal.CALIB_FP32_MIXED)
    c = cal.Calib(d, vis, coh, flags, precision=cal.CALIB_FP32_MIXED, lm_tol=1e-7)
    trg = c.solve(3)
    c.close()
    print("c2: three C-ADMM iterations under the stopping rule, oracle on all 32 subbands", flush=True)
    pb = oracle_mod.Problem(d32, lm_tol=1e-7)
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 3)["trace"]
    np.testing.assert_allclose(trg[:, :2], tro[:, :2], rtol=1e-5)


# the benchmark's solver settings: matrix-free CG at cg_tol 1e-2 in the one-launch local step, LM
# stopping rule at lm_tol 1e-7, no packed sample copy (CALIB_OPT_STATS_ONLY, data costs from the
# coherency statistics); the oracle takes the same reading (block-Jacobi CG to the same
# relative residual, same rule)
BENCH_GPU = dict(solver=3, cg_tol=1e-2, lm_tol=1e-7, options=1 | 4)   # GPA first, statistics only


def _bench_oracle(oracle_mod):
    return dict(solver=oracle_mod.SOLVE_PCG, cg_tol=1e-2, lm_tol=1e-7)


def test_c3_first_local_step_benchmark_solver(cal, oracle_mod, synth_mod):
    _first_local_step_sampled(cal, oracle_mod, synth_mod, "c3", [0, 77, 200, 255],
                              oracle_kw=_bench_oracle(oracle_mod), **BENCH_GPU)


def test_c2_benchmark_configuration(cal, oracle_mod, synth_mod):
    """The timed configuration on the full c2 problem: FP32 streaming, the one-launch local step
    with CG at cg_tol 1e-2 and the stopping rule at lm_tol 1e-7, three C-ADMM iterations from
    identity replayed from the captured graph; the oracle runs the same reading on the
    FP32-rounded inputs of all 32 subbands.  Data cost and Lagrangian within 1e-5: a CG run that
    stops one iteration apart on the two sides (a residual within rounding of the tolerance)
    moves that LM step by about cg_tol relative, and a flipped stop decision the cost by about
    lm_tol."""
    cfg = synth_mod.named_config("c2")
    d, d32 = _data(synth_mod, "c2")
    vis, coh, flags = cal.device_inputs(d, cal.CALIB_FP32_MIXED)
    c = cal.Calib(d, vis, coh, flags, precision=cal.CALIB_FP32_MIXED, **BENCH_GPU)
    trg = c.solve(3)
    c.close()
    print("c2: three C-ADMM iterations in the benchmark's configuration, oracle on all 32 subbands",
          flush=True)
    pb = oracle_mod.Problem(d32, **_bench_oracle(oracle_mod))
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 3)["trace"]
    print(f"  data cost {np.max(np.abs(trg[:, 0] / tro[:, 0] - 1)):.2e}, Lagrangian "
          f"{np.max(np.abs(trg[:, 1] / tro[:, 1] - 1)):.2e} relative", flush=True)
    np.testing.assert_allclose(trg[:, :2], tro[:, :2], rtol=1e-5)


def test_autotune_measures_and_caches(cal, synth_mod, tmp_path, monkeypatch):
    from paper_1502_00858_amd import autotune
    cfg = synth_mod.SynthConfig("tune", N=12, P=6, Q=2, K=3, T=4, n_chan=[1, 9, 3, 16, 2, 5],
                                n_dirs=[3, 2, 3, 3, 1, 2], flag_frac_max=0.3, config_index=9)
    d = synth_mod.generate(cfg)
    vis, coh, flags = cal.device_inputs(d, cal.CALIB_FP32_MIXED)
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(d, vis, coh, flags, cal.CALIB_FP32_MIXED, grids=[0, 4], cache=cache)
    assert best["tile_group"] in autotune.GROUPS and best["stream_grid"] in (0, 4)
    assert len(best["candidates"]) == 2 * len(autotune.GROUPS)
    assert best["ms"] == min(r["ms"] for r in best["candidates"])
    # the solver: every candidate timed, the fastest chosen
    assert sorted(best["solver_ms"]) == ["1", "2", "3"]
    assert best["solver_ms"][str(best["solver"])] == min(best["solver_ms"].values())

    def no_measure(*a, **k):
        raise AssertionError("cached shape measured again")
    monkeypatch.setattr(autotune, "measure", no_measure)
    monkeypatch.setattr(autotune, "measure_solver", no_measure)
    again = autotune.tune(d, vis, coh, flags, cal.CALIB_FP32_MIXED, grids=[0, 4], cache=cache)
    assert again == best
