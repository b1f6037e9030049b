"""GPU library against the oracle on the method's special cases and edges.

rho = 0 (normal calibration: independent subbands, multipliers stay zero), distinct rho per
direction (Section 3 allows one per direction), the unregularised first local step, the noise-free
truth-in-span fixed point, the Z update at 5 and 6 basis terms on the 64-subband frequency grid of
the large-array workload (cond(B^T B) up to ~1e9: the fitted values B_f Z are compared), FP32 model
visibilities and Jones matrices element by element, and one whole C-ADMM iteration on ragged
subbands shaped like the batched workload (1-16 channels, 3-10 directions, flagged baselines).
Both local solvers (blocked Cholesky, matrix-free conjugate gradients) where the path differs.
"""
import numpy as np
import pytest

from conftest import rand_jones, tiny_cfg
from parity_tol import FP32_TOL, FP64_VIS_TOL, AdmmRun, rel, traj_vis_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SOLVERS = {0: dict(), 3: dict(solver=3, cg_tol=1e-10)}


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


def _ctx(cal, d, precision=0, jones0=None, **kw):
    vis, coh, flags = cal.device_inputs(d, precision)
    J0 = None if jones0 is None else torch.from_numpy(np.ascontiguousarray(jones0)).cuda()
    return cal.Calib(d, vis, coh, flags, J0, precision=precision, **kw)


def _pcg_kw(oracle_mod, solver):
    return dict(solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10) if solver == 3 else {}


def _oracle(oracle_mod, d, solver, **kw):
    if solver == 3:
        kw.update(solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10)
    return oracle_mod.Problem(d, **kw)


@pytest.mark.parametrize("solver", [0, 3])
def test_rho_zero_is_normal_calibration(cal, oracle_mod, synth_mod, solver):
    cfg = tiny_cfg(synth_mod, N=7, P=4, Q=2, K=2, T=3, n_chan=2, rho=0.0, lm_iters=5)
    d = synth_mod.generate(cfg)
    rho = np.zeros(cfg.K)
    c = _ctx(cal, d, 0, lm_iters=5, options=0, rho=rho, **SOLVERS[solver])
    tr = c.solve(3)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    assert np.max(np.abs(c.get(cal.FIELD_Y).cpu().numpy())) == 0.0
    pb = _oracle(oracle_mod, d, solver, lm_iters=5, options=0, rho=rho)
    J = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    z = np.zeros_like(J)
    for _ in range(3):   # three independent local steps: nothing ties the subbands
        J = pb.local_step(J, z, z)
    np.testing.assert_allclose(tr[:, 0][-1], pb.subband_cost(J).sum(), rtol=FP64_VIS_TOL)
    tol = traj_vis_tol(oracle_mod, d, AdmmRun(cfg.P, cfg.K, cfg.N, 3, lm_iters=5, options=0, rho=rho,
                                               **_pcg_kw(oracle_mod, solver)))
    assert rel(pb.predict(Jg), pb.predict(J)) < tol


@pytest.mark.parametrize("solver", [0, 3])
def test_distinct_rho_per_direction(cal, oracle_mod, synth_mod, solver):
    cfg = tiny_cfg(synth_mod, N=8, P=5, Q=3, K=3, T=3, n_chan=2, lm_iters=5)
    d = synth_mod.generate(cfg)
    rho = np.array([0.5, 5.0, 50.0])
    c = _ctx(cal, d, 0, lm_iters=5, rho=rho, **SOLVERS[solver])
    trg = c.solve(5)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    pb = _oracle(oracle_mod, d, solver, lm_iters=5, rho=rho)
    out = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 5)
    np.testing.assert_allclose(trg[:, :2], out["trace"][:, :2], rtol=FP64_VIS_TOL)
    np.testing.assert_allclose(trg[:, 2:], out["trace"][:, 2:], rtol=1e-8)
    tol = traj_vis_tol(oracle_mod, d, AdmmRun(cfg.P, cfg.K, cfg.N, 5, lm_iters=5, rho=rho,
                                               **_pcg_kw(oracle_mod, solver)))
    err = rel(pb.predict(Jg), pb.predict(out["J"]))
    print(f"visibilities {err:.2e} (bound {tol:.2e})")
    assert err < tol


@pytest.mark.parametrize("solver", [0, 3])
def test_unregularised_first_iteration(cal, oracle_mod, synth_mod, solver):
    cfg = tiny_cfg(synth_mod, N=7, P=5, Q=2, K=2, T=3, n_chan=2, lm_iters=5)
    d = synth_mod.generate(cfg)
    opts = cal.OPT_GPA_FIRST_ITER | cal.OPT_UNREG_FIRST
    trg = _ctx(cal, d, 0, lm_iters=5, options=opts, **SOLVERS[solver]).solve(4)
    pb = _oracle(oracle_mod, d, solver, lm_iters=5,
                 options=oracle_mod.OPT_GPA_FIRST | oracle_mod.OPT_UNREG_FIRST)
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 4)["trace"]
    np.testing.assert_allclose(trg[:, :2], tro[:, :2], rtol=FP64_VIS_TOL)
    # and it differs from the regularised first step (the option does something)
    plain = _ctx(cal, d, 0, lm_iters=5, **SOLVERS[solver]).solve(1)
    assert abs(plain[0, 1] - trg[0, 1]) > 1e-6 * abs(trg[0, 1])


@pytest.mark.parametrize("solver", [0, 3])
def test_noise_free_truth_in_span_is_a_fixed_point(cal, oracle_mod, synth_mod, solver):
    cfg = tiny_cfg(synth_mod, N=8, P=6, Q=3, K=2, T=3, n_chan=2, snr=None, lm_iters=5)
    d = synth_mod.generate(cfg, truth_in_span=True)
    Jt = d["jones_true"]
    c = _ctx(cal, d, 0, jones0=Jt, lm_iters=5, **SOLVERS[solver])
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c.set_state(cuda(Jt), None, None, cuda(Jt))
    c.local_step(1)
    J1 = c.get(cal.FIELD_J).cpu().numpy()
    assert np.max(np.abs(J1 - Jt)) < 1e-10
    c.consensus_update(1)
    np.testing.assert_allclose(c.get(cal.FIELD_BZ).cpu().numpy(), Jt, atol=1e-12)
    assert np.max(np.abs(c.get(cal.FIELD_Y).cpu().numpy())) < 1e-10
    assert c.get(cal.FIELD_TRACE)[1, 2] < 1e-12
    assert np.all(c.get(cal.FIELD_COST).cpu().numpy() < 1e-20 * np.sum(np.abs(d["vis"]) ** 2))


@pytest.mark.parametrize("Q", [5, 6])
def test_z_update_many_basis_terms(cal, oracle_mod, synth_mod, Q):
    """64 subbands spread over 115-185 MHz as in the large-array workload; the Vandermonde basis
    matrix then has cond(B^T B) ~ 1e7 (Q = 5) and ~ 1e9 (Q = 6)."""
    cfg = tiny_cfg(synth_mod, N=6, P=64, Q=Q, K=2, T=1, n_chan=1, rho=3.0)
    d = synth_mod.generate(cfg)
    x = (np.asarray(d["freq"]) - d["f0"]) / d["f0"]
    Bv = np.vander(x, Q, increasing=True)
    print(f"Q={Q}: cond(B^T B) = {np.linalg.cond(Bv.T @ Bv):.2e}")
    rng = np.random.default_rng(50 + Q)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    Y0 = 0.2 * (rng.normal(size=J.shape) + 1j * rng.normal(size=J.shape))
    c = _ctx(cal, d, 0, jones0=J)
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c.set_state(cuda(J), cuda(Y0), None, None)
    c.consensus_update(1)
    pb = oracle_mod.Problem(d)
    Y, Z, BZ, pr, du = pb.consensus(J, Y0, np.zeros(pb.zshape(), np.complex128))
    err_bz = rel(c.get(cal.FIELD_BZ).cpu().numpy(), BZ)
    err_y = rel(c.get(cal.FIELD_Y).cpu().numpy(), Y)
    print(f"B_f Z {err_bz:.2e}, Y {err_y:.2e}")
    assert err_bz < 1e-12 and err_y < 1e-11
    tr = c.get(cal.FIELD_TRACE)
    assert abs(tr[1, 2] - pr) < 1e-12 * max(pr, 1)


@pytest.mark.parametrize("solver", [0, 3])
def test_fp32_visibilities_and_jones(cal, oracle_mod, synth_mod, solver):
    """FP32 streaming with FP64 statistics against the oracle on the FP32-rounded inputs, element by
    element: model visibilities and the Jones matrices (each (subband, direction) moved to the
    oracle's unitary gauge first: the solution is defined up to a right unitary factor)."""
    cfg = tiny_cfg(synth_mod, N=10, P=6, Q=3, K=3, T=5, n_chan=4, lm_iters=6)
    d = synth_mod.generate(cfg)
    c = _ctx(cal, d, 1, lm_iters=6, **SOLVERS[solver])
    c.solve(4)
    Jg = c.get(cal.FIELD_J).cpu().numpy()
    model = c.get(cal.FIELD_MODEL_VIS).cpu().numpy()
    d32 = synth_mod.as_fp32_inputs(d)
    pb = _oracle(oracle_mod, d32, solver, lm_iters=6)
    Jo = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 4)["J"]
    ref = pb.predict(Jo)
    err_v = rel(model, ref)
    Ja = Jg.copy()
    for f in range(cfg.P):
        for k in range(cfg.K):
            A = np.einsum("pji,pjk->ik", np.conj(Jg[f, k]), Jo[f, k])
            W, _, Vh = np.linalg.svd(A)
            Ja[f, k] = Jg[f, k] @ (W @ Vh)
    err_j = rel(Ja, Jo)
    print(f"FP32: model visibilities {err_v:.2e}, aligned Jones {err_j:.2e}, raw Jones {rel(Jg, Jo):.2e}")
    assert err_v < FP32_TOL and err_j < FP32_TOL


@pytest.mark.parametrize("solver", [0, 3])
def test_ragged_batched_subset_whole_iteration(cal, oracle_mod, synth_mod, solver):
    """16 subbands shaped like the batched workload: channels 1-16, directions 3-10 (nested into a
    10-source sky), 0-30% flagged baselines; FP32 streaming; one whole C-ADMM iteration (local step,
    alignment, consensus) against the oracle on every subband."""
    rng = np.random.default_rng(77)
    P = 16
    n_chan = list(rng.integers(1, 17, size=P))
    n_dirs = list(rng.integers(3, 11, size=P))
    n_dirs[:4] = [10, 10, 10, 10]   # every direction on at least Q subbands
    cfg = synth_mod.SynthConfig("c3sub", N=16, P=P, Q=4, K=10, T=4, n_chan=n_chan, n_dirs=n_dirs,
                                flag_frac_max=0.3, lm_iters=5, config_index=33)
    d = synth_mod.generate(cfg)
    assert d["flags"].sum() > 0
    print(f"n_chan {n_chan} n_dirs {n_dirs}", flush=True)
    c = _ctx(cal, d, 1, lm_iters=5, **SOLVERS[solver])
    trg = c.solve(2)
    pb = _oracle(oracle_mod, synth_mod.as_fp32_inputs(d), solver, lm_iters=5)
    tro = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 2)["trace"]
    np.testing.assert_allclose(trg[:, :2], tro[:, :2], rtol=FP32_TOL)
    np.testing.assert_allclose(trg[:, 2:], tro[:, 2:], rtol=1e-3)


@pytest.mark.parametrize("solver", [0, 3])
def test_numeric_failure_is_reported_per_subband(cal, synth_mod, solver):
    """One subband's state made non-finite (calib_set_state with a NaN Jones entry): its LM runs
    stop and CALIB_FIELD_STATUS reports it as CALIB_E_NUMERIC, every other subband's local step is
    bitwise what it is without the NaN, and admm_solve returns CALIB_E_NUMERIC."""
    cfg = tiny_cfg(synth_mod, N=7, P=5, Q=2, K=2, T=3, n_chan=2, lm_iters=4)
    d = synth_mod.generate(cfg)
    cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    J = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    Jbad = J.copy()
    Jbad[2, 1, 3, 0, 0] = np.nan
    a = _ctx(cal, d, 0, lm_iters=4, options=0, **SOLVERS[solver])
    b = _ctx(cal, d, 0, lm_iters=4, options=0, **SOLVERS[solver])
    a.set_state(cuda(J))
    b.set_state(cuda(Jbad))
    a.local_step(1)
    b.local_step(1)
    np.testing.assert_array_equal(a.get(cal.FIELD_STATUS).cpu().numpy(), [0, 0, 0, 0, 0])
    np.testing.assert_array_equal(b.get(cal.FIELD_STATUS).cpu().numpy(), [0, 0, 5, 0, 0])
    Ja, Jb = a.get(cal.FIELD_J).cpu().numpy(), b.get(cal.FIELD_J).cpu().numpy()
    ok = [0, 1, 3, 4]
    np.testing.assert_array_equal(Ja[ok], Jb[ok])
    assert np.any(Ja[ok] != J[ok])   # the other subbands did move
    b.set_state(cuda(Jbad))
    with pytest.raises(cal.CalibError) as e:
        b.solve(1)
    assert e.value.status == 5 and "(2)" in str(e.value)
    a.set_state(cuda(J))
    a.solve(1)
