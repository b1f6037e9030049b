"""The basis of the GPU parity tolerances (tests/parity_tol.py): how far the oracle's own results
move when its inputs are perturbed by 1e-15 relative.

One local step from identical state does not amplify rounding (the visibilities move by ~1e-15),
so the GPU is held to FP64_VIS_TOL = 1e-10 there.  Over several C-ADMM iterations an LM accept
decision can be taken at a gain ratio of rounding size; a perturbation then flips it and the
trajectory moves by the effect of one LM step (7.5e-9 on the smoke problem after 4 iterations,
~4e-10 on c1 after 20).  The trajectory tests use traj_vis_tol, which measures this per case.
"""
import numpy as np

from conftest import tiny_cfg
from parity_tol import (FLIP_MARGIN, FP64_VIS_TOL, AdmmRun, LocalStepRun, oracle_sensitivity,
                        traj_vis_tol)


def test_single_local_steps_do_not_amplify_rounding(oracle_mod, synth_mod):
    cases = [  # the single-local-step cases of tests/test_gpu_parity.py
        (dict(N=6, P=3, K=2, T=3, n_chan=2, lm_iters=6), 1),
        (dict(N=5, P=2, Q=1, K=16, T=3, n_chan=2, n_dirs=[16, 11], lm_iters=3), 1),
        (dict(N=6, P=3, K=3, T=3, n_chan=2, lm_iters=4), 2),
    ]
    for kw, sweeps in cases:
        cfg = tiny_cfg(synth_mod, **kw)
        d = synth_mod.generate(cfg)
        run = LocalStepRun(cfg.P, cfg.K, cfg.N, lm_iters=cfg.lm_iters, sage_sweeps=sweeps)
        sens = oracle_sensitivity(oracle_mod, d, run)
        print(f"one local step {kw}: oracle sensitivity {sens:.2e}")
        assert sens < 1e-13 < FP64_VIS_TOL


def test_trajectory_sensitivity_comes_from_flipped_decisions(oracle_mod, synth_mod):
    cfg = synth_mod.SynthConfig("smoke", N=8, P=5, Q=3, K=2, T=4, n_chan=2, rho=5.0, lm_iters=6,
                                config_index=11)
    d = synth_mod.generate(cfg)
    run = AdmmRun(cfg.P, cfg.K, cfg.N, 4, lm_iters=6)
    sens = oracle_sensitivity(oracle_mod, d, run)
    print(f"smoke problem, 4 C-ADMM iterations: oracle sensitivity {sens:.2e}")
    # far above the perturbation: a decision flipped; far below the size of a step
    assert 1e-10 < sens < 1e-6
    tol = traj_vis_tol(oracle_mod, d, run)
    assert tol == max(FP64_VIS_TOL, FLIP_MARGIN * sens)
    # the same problem over one local step: no flip
    one = oracle_sensitivity(oracle_mod, d, LocalStepRun(cfg.P, cfg.K, cfg.N, lm_iters=6))
    assert one < 1e-13
    # and the data cost, which the trace tests compare, is far less sensitive than the J the flip moved
    pa, pb = oracle_mod.Problem(d, lm_iters=6), oracle_mod.Problem(
        dict(d, vis=d["vis"] * (1 + 1e-15 * np.random.default_rng(1000).standard_normal(d["vis"].shape))),
        lm_iters=6)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    ta, tb = pa.admm_solve(J0, 4)["trace"], pb.admm_solve(J0, 4)["trace"]
    assert np.max(np.abs(ta[:, 0] - tb[:, 0]) / ta[:, 0]) < 1e-10
