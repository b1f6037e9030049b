"""GPU library against the FP64 CPU oracle on identical seeded inputs.

Tolerances (tests/parity_tol.py): FP64 path 1e-10 relative on predicted visibilities and
per-iteration cost; over multi-iteration trajectories the visibility bound is derived per case
from the oracle's own sensitivity (a flipped LM decision moves the trajectory by one step); the
FP32-streaming path 1e-5 relative, compared with the oracle run on the FP32-rounded inputs.
"""
import numpy as np
import pytest

from conftest import rand_jones, tiny_cfg
from parity_tol import FP64_VIS_TOL, AdmmRun, traj_vis_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


def _ctx(cal, d, precision=0, jones0=None, **kw):
    vis, coh, flags = cal.device_inputs(d, precision)
    J0 = None if jones0 is None else torch.from_numpy(np.ascontiguousarray(jones0)).cuda()
    return cal.Calib(d, vis, coh, flags, J0, precision=precision, **kw)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_model_vis_and_cost_fp64(cal, oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=7, P=3, K=3, T=4, n_chan=3)
    d = synth_mod.generate(cfg)
    J = rand_jones(np.random.default_rng(11), cfg.P, cfg.K, cfg.N)
    c = _ctx(cal, d, 0, jones0=J)
    pb = oracle_mod.Problem(d)
    model = c.get(cal.FIELD_MODEL_VIS).cpu().numpy()
    assert _rel(model, pb.predict(J)) < 1e-12
    cost = c.get(cal.FIELD_COST).cpu().numpy()
    np.testing.assert_allclose(cost, pb.subband_cost(J), rtol=1e-11)


def test_local_step_lm_trace_fp64(cal, oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=3, K=2, T=3, n_chan=2, lm_iters=6)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    c = _ctx(cal, d, 0, lm_iters=6)
    c.local_step(0)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    trg = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
    pb = oracle_mod.Problem(d, lm_iters=6)
    z = np.zeros_like(J0)
    Jo, tro = pb.local_step(J0, z, z, trace=True)
    # per LM iteration: objective, damping, accept decision
    np.testing.assert_array_equal(trg[..., 2], tro[:, 0, :, :, 2])
    np.testing.assert_allclose(trg[..., 0], tro[:, 0, :, :, 0], rtol=1e-10)
    # lambda is scaled by a function of the gain ratio (F - F_new)/ell, a quotient of the difference
    # of two nearly equal objectives: its rounding is amplified by F/(F - F_new) (up to ~1e6 here)
    np.testing.assert_allclose(trg[..., 1], tro[:, 0, :, :, 1], rtol=1e-5)
    err = _rel(pb.predict(Jg), pb.predict(Jo))
    print(f"visibilities after one local step: {err:.2e}")
    assert err < FP64_VIS_TOL


def test_max_directions_fp64(cal, oracle_mod, synth_mod):
    """The largest direction count (16 per subband, the size of the per-sample direction arrays of
    the streaming and coherency-statistics kernels), subbands carrying 16 and 11 of them: the local
    step's LM trace and J agree with the oracle."""
    cfg = tiny_cfg(synth_mod, N=5, P=2, Q=1, K=16, T=3, n_chan=2, n_dirs=[16, 11], lm_iters=3)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    c = _ctx(cal, d, 0, lm_iters=3)
    c.local_step(0)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    trg = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
    pb = oracle_mod.Problem(d, lm_iters=3)
    z = np.zeros_like(J0)
    Jo, tro = pb.local_step(J0, z, z, trace=True)
    np.testing.assert_array_equal(trg[..., 2], tro[:, 0, :, :, 2])
    np.testing.assert_allclose(trg[..., 0], tro[:, 0, :, :, 0], rtol=1e-10)
    err = _rel(pb.predict(Jg), pb.predict(Jo))
    print(f"visibilities after one local step: {err:.2e}")
    assert err < FP64_VIS_TOL


@pytest.mark.parametrize("solver", [0, 3])
def test_two_sage_sweeps_fp64(cal, oracle_mod, synth_mod, solver):
    """Two SAGE sweeps per local step: each commit then updates every direction's statistics (the
    second sweep starts again from direction 0).  The last sweep's LM trace, the local step's J and
    a short C-ADMM trajectory agree with the oracle, for the Cholesky and the matrix-free solver
    (CG at cg_tol 1e-10 on both sides)."""
    cfg = tiny_cfg(synth_mod, N=6, P=3, K=3, T=3, n_chan=2, lm_iters=4)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    gkw = dict(solver=3, cg_tol=1e-10) if solver == 3 else {}
    okw = dict(solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10) if solver == 3 else {}
    c = _ctx(cal, d, 0, lm_iters=4, sage_sweeps=2, **gkw)
    c.local_step(0)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    trg = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
    pb = oracle_mod.Problem(d, lm_iters=4, sage_sweeps=2, **okw)
    z = np.zeros_like(J0)
    Jo, tro = pb.local_step(J0, z, z, trace=True)
    np.testing.assert_array_equal(trg[..., 2], tro[:, 1, :, :, 2])
    np.testing.assert_allclose(trg[..., 0], tro[:, 1, :, :, 0], rtol=1e-10)
    err = _rel(pb.predict(Jg), pb.predict(Jo))
    print(f"visibilities after one local step: {err:.2e}")
    assert err < FP64_VIS_TOL
    trg = _ctx(cal, d, 0, lm_iters=4, sage_sweeps=2, **gkw).solve(3)
    tro = pb.admm_solve(J0, 3)["trace"]
    np.testing.assert_allclose(trg[:, 0], tro[:, 0], rtol=1e-10)


def test_consensus_step_fp64(cal, oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=5, P=6, Q=3, K=2, rho=2.0)
    d = synth_mod.generate(cfg)
    J = rand_jones(np.random.default_rng(12), cfg.P, cfg.K, cfg.N)
    c = _ctx(cal, d, 0, jones0=J)
    c.consensus_update(1)     # not the first iteration: no alignment
    pb = oracle_mod.Problem(d)
    Y, Z, BZ, pr, du = pb.consensus(J, np.zeros_like(J), np.zeros(pb.zshape(), np.complex128))
    assert _rel(c.get(cal.FIELD_BZ).cpu().numpy(), BZ) < 1e-12
    assert _rel(c.get(cal.FIELD_Y).cpu().numpy(), Y) < 1e-11
    assert _rel(c.get(cal.FIELD_Z).cpu().numpy(), Z) < 1e-9
    tr = c.get(cal.FIELD_TRACE)
    assert abs(tr[1, 2] - pr) < 1e-12 * max(pr, 1) and abs(tr[1, 3] - du) < 1e-12 * max(du, 1)


def test_gpa_first_iteration_fp64(cal, oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=5, P=5, Q=2, K=2)
    d = synth_mod.generate(cfg)
    J = rand_jones(np.random.default_rng(13), cfg.P, cfg.K, cfg.N, scale=0.5)
    c = _ctx(cal, d, 0, jones0=J)
    c.consensus_update(0)
    pb = oracle_mod.Problem(d)
    Ja = pb.gpa(J, rounds=3)
    assert _rel(c.get(cal.FIELD_J).cpu().numpy(), Ja) < 1e-11


def test_admm_c1_fp64(cal, oracle_mod, synth_mod):
    cfg = synth_mod.named_config("c1")
    d = synth_mod.generate(cfg)
    c = _ctx(cal, d, 0, lm_iters=cfg.lm_iters)
    trg = c.solve(cfg.admm_iters)
    pb = oracle_mod.Problem(d, lm_iters=cfg.lm_iters)
    out = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), cfg.admm_iters)
    tro = out["trace"]
    np.testing.assert_allclose(trg[:, 0], tro[:, 0], rtol=1e-10)
    np.testing.assert_allclose(trg[:, 1], tro[:, 1], rtol=1e-10)
    model_g = c.get(cal.FIELD_MODEL_VIS).cpu().numpy()
    err = _rel(model_g, pb.predict(out["J"]))
    tol = traj_vis_tol(oracle_mod, d, AdmmRun(cfg.P, cfg.K, cfg.N, cfg.admm_iters, lm_iters=cfg.lm_iters))
    print(f"visibilities after {cfg.admm_iters} iterations: {err:.2e} (bound {tol:.2e})")
    assert err < tol


def test_admm_fp32_mixed(cal, oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=10, P=6, Q=3, K=3, T=5, n_chan=4, lm_iters=8)
    d = synth_mod.generate(cfg)
    c = _ctx(cal, d, 1, lm_iters=8)
    trg = c.solve(6)
    pb = oracle_mod.Problem(synth_mod.as_fp32_inputs(d), lm_iters=8)
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 6)["trace"]
    np.testing.assert_allclose(trg[:, 0], tro[:, 0], rtol=1e-5)
    np.testing.assert_allclose(trg[:, 1], tro[:, 1], rtol=1e-5)


def test_ragged_flags_fp64(cal, oracle_mod, synth_mod):
    cfg = synth_mod.SynthConfig("rag", N=9, P=7, Q=3, K=4, T=3, n_chan=[1, 3, 2, 5, 1, 4, 2],
                                n_dirs=[4, 3, 4, 2, 4, 3, 4], flag_frac_max=0.3, lm_iters=5,
                                config_index=8)
    d = synth_mod.generate(cfg)
    assert d["flags"].sum() > 0
    c = _ctx(cal, d, 0, lm_iters=5)
    trg = c.solve(4)
    pb = oracle_mod.Problem(d, lm_iters=5)
    out = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 4)
    # data cost and augmented Lagrangian (whose penalty covers only the directions a subband
    # carries)
    np.testing.assert_allclose(trg[:, :2], out["trace"][:, :2], rtol=1e-10)
    model_g = c.get(cal.FIELD_MODEL_VIS).cpu().numpy()
    err = _rel(model_g, pb.predict(out["J"]))
    tol = traj_vis_tol(oracle_mod, d, AdmmRun(cfg.P, cfg.K, cfg.N, 4, lm_iters=5))
    print(f"visibilities after 4 iterations: {err:.2e} (bound {tol:.2e})")
    assert err < tol


def test_rank_and_numeric_errors(cal, synth_mod):
    cfg = tiny_cfg(synth_mod, N=4, P=2, Q=3, K=1)
    d = synth_mod.generate(cfg)
    with pytest.raises(cal.CalibError) as e:
        _ctx(cal, d, 0)
    assert e.value.status == 4
    cfg = tiny_cfg(synth_mod, N=4, P=3, Q=2, K=1)
    d = synth_mod.generate(cfg)
    d["vis"] = d["vis"].copy()
    d["vis"][5, 0, 1] = np.nan
    with pytest.raises(cal.CalibError) as e:
        _ctx(cal, d, 0)
    assert e.value.status == 5


def test_flagged_samples_never_read(cal, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=3, Q=2, K=2, flag_frac_max=0.4)
    d = synth_mod.generate(cfg)
    B, spb = cfg.B, cfg.T * 2
    vis = d["vis"].copy()
    for f in range(cfg.P):
        for b in np.nonzero(d["flags"][f * B:(f + 1) * B])[0]:
            s0 = d["vis_off"][f] + b * spb
            vis[s0:s0 + spb] = np.nan
    d2 = dict(d, vis=vis)
    tr1 = _ctx(cal, d, 0).solve(2)
    tr2 = _ctx(cal, d2, 0).solve(2)
    np.testing.assert_array_equal(tr1, tr2)


def test_run_to_run_bitwise(cal, synth_mod):
    cfg = tiny_cfg(synth_mod, N=8, P=4, Q=2, K=2, T=3, n_chan=3)
    d = synth_mod.generate(cfg)
    a = _ctx(cal, d, 1)
    b = _ctx(cal, d, 1)
    np.testing.assert_array_equal(a.solve(3), b.solve(3))
    np.testing.assert_array_equal(a.get(cal.FIELD_J).cpu().numpy(), b.get(cal.FIELD_J).cpu().numpy())


@pytest.mark.parametrize("solver", [1, 2, 3])
def test_normal_equation_solve_fp64(cal, oracle_mod, synth_mod, solver):
    """One LM iteration from a random state: the GPU step solves (H_GN + (rho+lambda) I) delta = -G
    with the oracle's Gauss-Newton matrix, for both Cholesky solvers (one workgroup per matrix;
    64-column panels over many workgroups) and the matrix-free conjugate gradients (16 stations
    per wavefront up to N = 64, 32 above), and station counts that give padded factors and
    partial last panels (8N = 48, 72, 136, 264 columns), 8N = 528 (past the 512 columns of the
    panel solver's register-ring back substitution: its 1024-thread back substitution) and the
    largest array, N = 128 (8N = 1024: two columns per thread in the one-workgroup solver, one in
    the 1024-thread back substitution, 16 panels); the smallest, N = 2 (one baseline, one tile)."""
    for N in (2, 6, 9, 17, 33, 66, 128):
        print(f"solver {solver} N {N}", flush=True)
        cfg = tiny_cfg(synth_mod, N=N, P=2, Q=1, K=1, T=3, n_chan=2, rho=3.0, lm_iters=1)
        d = synth_mod.generate(cfg)
        J = rand_jones(np.random.default_rng(14), cfg.P, 1, N)
        # solver 3 (conjugate gradients) at a tolerance below rounding: it runs to 8N iterations
        # or an exact zero residual, the dense solve's accuracy
        c = _ctx(cal, d, 0, jones0=J, lm_iters=1, options=0, solver=solver, cg_tol=1e-15)
        c.local_step(1)
        step = c.get(cal.FIELD_LM_STEP).cpu().numpy()
        pb = oracle_mod.Problem(d, lm_iters=1)
        z = np.zeros_like(J)
        for f in range(cfg.P):
            _, G = pb.dir_objective(J, z, z, f, 0)
            g = np.stack([G.reshape(-1).real, G.reshape(-1).imag], 1).reshape(-1)
            np.testing.assert_allclose(step[f, 0], g, rtol=1e-10, atol=1e-10 * np.abs(g).max())
            H = pb.dir_gn_hessian(f, 0, J[f, 0]) + 3.0 * np.eye(8 * N)
            lam = 1e-3 * np.max(np.diag(H))
            delta = np.linalg.solve(H + lam * np.eye(8 * N), -g)
            np.testing.assert_allclose(step[f, 1], delta, rtol=1e-9, atol=1e-9 * np.abs(delta).max())


def test_graph_replay_equals_eager(cal, synth_mod):
    """Iterations >= 1 replay a captured graph; with kernel timing on every launch is eager."""
    cfg = synth_mod.SynthConfig("g", N=9, P=6, Q=3, K=3, T=3, n_chan=[2, 1, 3, 2, 4, 1],
                                n_dirs=[3, 2, 3, 3, 1, 3], flag_frac_max=0.2, lm_iters=4,
                                config_index=9)
    d = synth_mod.generate(cfg)
    for prec in (0, 1):
        a = _ctx(cal, d, prec, lm_iters=4)
        b = _ctx(cal, d, prec, lm_iters=4)
        b.set_kernel_timing(True)
        ta, tb = a.solve(5), b.solve(5)
        np.testing.assert_array_equal(ta, tb)
        np.testing.assert_array_equal(a.get(cal.FIELD_J).cpu().numpy(), b.get(cal.FIELD_J).cpu().numpy())
        # a second solve on the same context replays the same graph from a reset state
        J0 = torch.from_numpy(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)).cuda()
        a.set_jones(J0)
        np.testing.assert_array_equal(a.solve(5), ta)


def test_tile_shapes_and_persistent_grid(cal, synth_mod):
    """Every lanes-per-baseline choice and a persistent streaming grid give the same numbers
    (the per-tile reduction order does not depend on the grid)."""
    cfg = tiny_cfg(synth_mod, N=8, P=4, Q=2, K=2, T=5, n_chan=3)
    d = synth_mod.generate(cfg)
    ref = _ctx(cal, d, 1).solve(3)
    np.testing.assert_array_equal(_ctx(cal, d, 1, stream_grid=3).solve(3), ref)
    for g in (4, 8, 16, 32, 64):
        tr = _ctx(cal, d, 1, tile_group=g).solve(3)
        np.testing.assert_allclose(tr, ref, rtol=1e-6)


def test_lm_stopping_rule_fp64(cal, oracle_mod, synth_mod):
    """With the LM stopping rule on, the GPU stops each (subband, direction) at the same iteration
    as the oracle and the whole C-ADMM trajectory still agrees."""
    cfg = tiny_cfg(synth_mod, N=7, P=4, Q=2, K=2, T=3, n_chan=2, lm_iters=10)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    z = np.zeros_like(J0)
    c = _ctx(cal, d, 0, lm_iters=10, lm_tol=1e-7)
    c.local_step(0)
    trg = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
    pb = oracle_mod.Problem(d, lm_iters=10, lm_tol=1e-7)
    _, tro = pb.local_step(J0, z, z, trace=True)
    np.testing.assert_array_equal(trg[..., 2], tro[:, 0, :, :, 2])
    np.testing.assert_allclose(trg[..., 0], tro[:, 0, :, :, 0], rtol=1e-10)
    assert np.sum(trg[..., 2] == 0) > 0
    c2 = _ctx(cal, d, 0, lm_iters=10, lm_tol=1e-7)
    tr = c2.solve(5)
    ref = pb.admm_solve(J0, 5)["trace"]
    np.testing.assert_allclose(tr[:, 0], ref[:, 0], rtol=1e-10)
    np.testing.assert_allclose(tr[:, 1], ref[:, 1], rtol=1e-10)


@pytest.mark.parametrize("solver", [1, 2, 3])
def test_stopping_rule_skip_is_exact(cal, synth_mod, solver):
    """Under the LM stopping rule, solve() launches one LM iteration per step for every subband
    still working, each on its own direction, and ends the local step once every subband has
    finished (stopped runs write their remaining trace rows); stepping the same problem with
    local_step / consensus_update launches every direction's every iteration.  Both give identical
    states, objective traces and LM traces, in both precisions."""
    cfg = tiny_cfg(synth_mod, N=9, P=5, Q=2, K=3, T=3, n_chan=2, lm_iters=7, flag_frac_max=0.2)
    d = synth_mod.generate(cfg)
    for prec in (0, 1):
        print(f"solver {solver} precision {prec}", flush=True)
        a = _ctx(cal, d, prec, lm_iters=7, lm_tol=1e-6, solver=solver)
        b = _ctx(cal, d, prec, lm_iters=7, lm_tol=1e-6, solver=solver)
        ta = a.solve(6)
        for n in range(6):
            b.local_step(n)
            b.consensus_update(n)
        np.testing.assert_array_equal(a.get(cal.FIELD_J).cpu().numpy(), b.get(cal.FIELD_J).cpu().numpy())
        np.testing.assert_array_equal(a.get(cal.FIELD_Y).cpu().numpy(), b.get(cal.FIELD_Y).cpu().numpy())
        lm = b.get(cal.FIELD_LM_TRACE).cpu().numpy()
        np.testing.assert_array_equal(a.get(cal.FIELD_LM_TRACE).cpu().numpy(), lm)
        np.testing.assert_array_equal(ta, b.get(cal.FIELD_TRACE)[:6])
        # runs stopped before the last iteration (the skip was taken)
        assert np.sum(lm[..., -1, 2] == 0) > 0


@pytest.mark.parametrize("sweeps", [1, 2])
def test_own_direction_progression_ragged(cal, synth_mod, sweeps):
    """Under the stopping rule each subband moves through its directions on its own (a subband
    whose run stopped commits it and starts the next direction while others still iterate, and
    wraps to the next SAGE sweep on its own).  With subbands of 1 to 4 directions (one finishing its
    local step long before the rest) the states and LM traces equal those of the lockstep local
    step, which launches every direction's every LM iteration for all subbands."""
    cfg = tiny_cfg(synth_mod, N=8, P=6, Q=2, K=4, T=3, n_chan=2, n_dirs=[4, 1, 3, 4, 2, 4],
                   flag_frac_max=0.2, lm_iters=6)
    d = synth_mod.generate(cfg)
    for prec in (0, 1):
        print(f"sweeps {sweeps} precision {prec}", flush=True)
        a = _ctx(cal, d, prec, lm_iters=6, lm_tol=1e-5, sage_sweeps=sweeps)
        b = _ctx(cal, d, prec, lm_iters=6, lm_tol=1e-5, sage_sweeps=sweeps)
        ta = a.solve(4)
        for n in range(4):
            b.local_step(n)
            b.consensus_update(n)
        np.testing.assert_array_equal(a.get(cal.FIELD_J).cpu().numpy(), b.get(cal.FIELD_J).cpu().numpy())
        np.testing.assert_array_equal(a.get(cal.FIELD_BZ).cpu().numpy(), b.get(cal.FIELD_BZ).cpu().numpy())
        lm = b.get(cal.FIELD_LM_TRACE).cpu().numpy()
        np.testing.assert_array_equal(a.get(cal.FIELD_LM_TRACE).cpu().numpy(), lm)
        np.testing.assert_array_equal(ta, b.get(cal.FIELD_TRACE)[:4])
        # runs stopped before their last LM iteration (so the subbands moved on unevenly)
        assert np.sum(lm[..., -1, 2] == 0) > 0


def test_solvers_agree_on_a_local_step(cal, synth_mod):
    """The two Cholesky solvers sum in different orders: whole local steps agree to rounding."""
    cfg = tiny_cfg(synth_mod, N=20, P=5, Q=2, K=3, T=3, n_chan=2, lm_iters=6, flag_frac_max=0.2)
    d = synth_mod.generate(cfg)
    tr = []
    for solver in (1, 2):
        c = _ctx(cal, d, 0, lm_iters=6, solver=solver)
        c.local_step(0)
        tr.append(c.get(cal.FIELD_LM_TRACE).cpu().numpy())
    np.testing.assert_array_equal(tr[0][..., 2], tr[1][..., 2])
    np.testing.assert_allclose(tr[0][..., 0], tr[1][..., 0], rtol=1e-11)


def test_pcg_local_step_matches_oracle_pcg(cal, oracle_mod, synth_mod):
    """The matrix-free solver (conjugate gradients at cg_tol 1e-10) against the oracle's reading of
    the same iteration: per-LM-iteration objective within 1e-10, accept decisions equal wherever
    the step moves the objective by more than rounding, visibilities after the local step within
    1e-10; then a short C-ADMM trajectory with the stopping rule, station counts on both sides of
    the 64-station switch of the work layout."""
    for N, K in ((7, 3), (70, 2)):
        print(f"pcg local step N={N} K={K}", flush=True)
        cfg = tiny_cfg(synth_mod, N=N, P=3, K=K, T=3, n_chan=2, lm_iters=6, flag_frac_max=0.2)
        d = synth_mod.generate(cfg)
        J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
        z = np.zeros_like(J0)
        c = _ctx(cal, d, 0, lm_iters=6, solver=3, cg_tol=1e-10)
        c.local_step(0)
        Jg = c.get(cal.FIELD_J).cpu().numpy()
        trg = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
        pb = oracle_mod.Problem(d, lm_iters=6, solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10)
        Jo, tro = pb.local_step(J0, z, z, trace=True)
        tro = tro[:, 0]
        prev = np.concatenate([np.full(tro.shape[:-2] + (1,), np.inf), tro[..., :-1, 0]], axis=-1)
        decisive = np.abs(tro[..., 0] - prev) > 1e-12 * np.abs(tro[..., 0])
        np.testing.assert_array_equal(trg[..., 2][decisive], tro[..., 2][decisive])
        np.testing.assert_allclose(trg[..., 0], tro[..., 0], rtol=1e-10)
        err = _rel(pb.predict(Jg), pb.predict(Jo))
        same = np.array_equal(trg[..., 2], tro[..., 2])
        print(f"  visibilities after the local step: {err:.2e} (accept sequences equal: {same})",
              flush=True)
        # a step taken or refused at a rounding tie near the optimum (where the objective is
        # quadratic) has size ~sqrt(eps) relative; without such a tie the bound is FP64_VIS_TOL
        assert err < (FP64_VIS_TOL if same else 1e-7)
        tr = _ctx(cal, d, 0, lm_iters=6, solver=3, cg_tol=1e-10, lm_tol=1e-7).solve(4)
        ref = oracle_mod.Problem(d, lm_iters=6, solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10,
                                 lm_tol=1e-7).admm_solve(J0, 4)["trace"]
        np.testing.assert_allclose(tr[:, :2], ref[:, :2], rtol=1e-10)
