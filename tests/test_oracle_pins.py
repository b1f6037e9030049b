"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the generator's independent
coding of the visibility model (Section 2), closed forms (the Z least squares of Section 3, the
sufficient-statistics expansion of the cost), finite differences of the oracle's own objective,
textbook library routines (Cholesky, least squares, SVD polar factor, SciPy's trust-region least
squares), invariances (the unitary ambiguity of Section 3) and the special cases the method has
(noise-free data, truth inside the basis span, rho = 0 = normal calibration).
"""
import numpy as np
import pytest

from conftest import rand_jones, tiny_cfg


def _unitary(rng):
    A = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def _noise_pair(synth, cfg):
    """Same seed with and without noise: everything but the noise draws is identical."""
    import dataclasses
    clean = synth.generate(dataclasses.replace(cfg, snr=None), seed=12345)
    noisy = synth.generate(cfg, seed=12345)
    return clean, noisy


def test_predict_matches_generator_model(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=3, K=3, snr=None)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    model = pb.predict(d["jones_true"])
    assert np.max(np.abs(model - d["vis"])) <= 1e-13 * np.max(np.abs(d["vis"]))


def test_cost_zero_noise_free_and_noise_energy(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=3, K=2)
    clean, noisy = _noise_pair(synth_mod, cfg)
    g0 = oracle_mod.Problem(clean).subband_cost(clean["jones_true"])
    assert np.all(g0 <= 1e-24 * np.sum(np.abs(clean["vis"]) ** 2))
    g = oracle_mod.Problem(noisy).subband_cost(noisy["jones_true"])
    noise = (noisy["vis"] - clean["vis"]).reshape(-1, 4)
    off = noisy["vis_off"]
    energy = [np.sum(np.abs(noise[off[f]:off[f + 1]]) ** 2) for f in range(cfg.P)]
    np.testing.assert_allclose(g, energy, rtol=1e-12)


def test_cost_gauge_invariance(oracle_mod, synth_mod):
    rng = np.random.default_rng(1)
    cfg = tiny_cfg(synth_mod, N=5, P=3, K=2)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    JU = J.copy()
    for f in range(cfg.P):
        for k in range(cfg.K):
            JU[f, k] = J[f, k] @ _unitary(rng)
    np.testing.assert_allclose(pb.subband_cost(JU), pb.subband_cost(J), rtol=1e-13)


def test_cost_sufficient_statistics_identity(oracle_mod, synth_mod):
    """For one direction, sum_s ||V - c M||^2 = E_b - 2 Re tr(M^H D_b) + S_b ||M||^2 per baseline,
    with E_b = sum ||V||^2, D_b = sum conj(c) V, S_b = sum |c|^2 (C = c I2, J time invariant)."""
    rng = np.random.default_rng(2)
    cfg = tiny_cfg(synth_mod, N=6, P=2, K=1, n_chan=3)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = rand_jones(rng, cfg.P, 1, cfg.N)
    g = pb.subband_cost(J)
    p, q = synth_mod.baseline_pairs(cfg.N)
    spb = cfg.T * 3
    for f in range(cfg.P):
        V = d["vis"][d["vis_off"][f]:d["vis_off"][f + 1]].reshape(cfg.B, spb, 2, 2)
        c = d["coh"][d["coh_off"][f]:d["coh_off"][f + 1]].reshape(cfg.B, spb)
        M = J[f, 0, p] @ np.conj(np.swapaxes(J[f, 0, q], -1, -2))
        E = np.sum(np.abs(V) ** 2, axis=(1, 2, 3))
        D = np.einsum("bs,bsij->bij", np.conj(c), V)
        S = np.sum(np.abs(c) ** 2, axis=1)
        ref = np.sum(E - 2 * np.real(np.einsum("bij,bij->b", np.conj(M), D))
                     + S * np.sum(np.abs(M) ** 2, axis=(1, 2)))
        assert abs(g[f] - ref) <= 1e-11 * abs(ref)


def test_gradient_finite_differences(oracle_mod, synth_mod):
    rng = np.random.default_rng(3)
    cfg = tiny_cfg(synth_mod, N=4, P=2, K=2, rho=3.0)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    Y = 0.3 * (rng.normal(size=J.shape) + 1j * rng.normal(size=J.shape))
    BZ = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    f, k = 1, 1
    L0, G = pb.dir_objective(J, Y, BZ, f, k)
    h = 1e-5
    fd = np.zeros(8 * cfg.N)
    for i in range(4 * cfg.N):
        for ri, step in enumerate((h, 1j * h)):
            Jp = J[f, k].copy().reshape(-1)
            Jm = Jp.copy()
            Jp[i] += step
            Jm[i] -= step
            fd[2 * i + ri] = (pb.dir_objective(J, Y, BZ, f, k, Jp.reshape(cfg.N, 2, 2), grad=False)
                              - pb.dir_objective(J, Y, BZ, f, k, Jm.reshape(cfg.N, 2, 2), grad=False)) / (2 * h)
    g = np.stack([G.reshape(-1).real, G.reshape(-1).imag], axis=1).reshape(-1)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)


def _fd_jacobian(pb, d, J, f, h=1e-6):
    """Central-difference Jacobian of the real/imag parts of the model of subband f with respect to
    the real parameters of direction 0 (one direction, so model = c J_p J_q^H)."""
    N = J.shape[2]
    o0, o1 = d["vis_off"][f], d["vis_off"][f + 1]
    cols = []
    for i in range(4 * N):
        for step in (h, 1j * h):
            Jp, Jm = J.copy(), J.copy()
            Jp[f, 0].reshape(-1)[i] += step
            Jm[f, 0].reshape(-1)[i] -= step
            dm = (pb.predict(Jp)[o0:o1] - pb.predict(Jm)[o0:o1]).reshape(-1) / (2 * h)
            cols.append(np.concatenate([dm.real, dm.imag]))
    return np.stack(cols, axis=1)


def test_gauss_newton_matches_fd_jacobian(oracle_mod, synth_mod):
    rng = np.random.default_rng(4)
    cfg = tiny_cfg(synth_mod, N=4, P=2, K=1)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = rand_jones(rng, cfg.P, 1, cfg.N)
    f = 1
    Jac = _fd_jacobian(pb, d, J, f)
    H = pb.dir_gn_hessian(f, 0, J[f, 0])
    ref = 2 * Jac.T @ Jac
    assert np.linalg.norm(H - ref) <= 1e-8 * np.linalg.norm(ref)
    # the unitary ambiguity leaves a 4-dimensional null space
    ev = np.linalg.eigvalsh(H)
    assert np.sum(ev < 1e-9 * ev[-1]) == 4


def test_full_hessian_equals_gn_at_zero_residual(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=4, P=2, K=1, snr=None, rho=0.0)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d, rho=np.zeros(1))
    J = d["jones_true"].copy()
    Y = np.zeros_like(J)
    f = 0
    H = pb.dir_gn_hessian(f, 0, J[f, 0])
    h = 1e-6
    n = 8 * cfg.N
    Hfd = np.zeros((n, n))
    for i in range(4 * cfg.N):
        for ri, step in enumerate((h, 1j * h)):
            Jp, Jm = J[f, 0].copy().reshape(-1), J[f, 0].copy().reshape(-1)
            Jp[i] += step
            Jm[i] -= step
            gp = pb.dir_objective(J, Y, Y, f, 0, Jp.reshape(-1, 2, 2))[1].reshape(-1)
            gm = pb.dir_objective(J, Y, Y, f, 0, Jm.reshape(-1, 2, 2))[1].reshape(-1)
            dg = (gp - gm) / (2 * h)
            Hfd[:, 2 * i + ri] = np.stack([dg.real, dg.imag], axis=1).reshape(-1)
    assert np.linalg.norm(H - Hfd) <= 1e-6 * np.linalg.norm(H)


def test_textbook_helpers(oracle_mod):
    rng = np.random.default_rng(5)
    A = rng.normal(size=(30, 30))
    A = A @ A.T + 30 * np.eye(30)
    np.testing.assert_allclose(oracle_mod.cholesky(A), np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    assert oracle_mod.cholesky(-np.eye(3)) is None
    M = rng.normal(size=(9, 4))
    X = rng.normal(size=(9, 5)) + 1j * rng.normal(size=(9, 5))
    np.testing.assert_allclose(oracle_mod.lstsq(M, X), np.linalg.lstsq(M, X, rcond=None)[0],
                               rtol=1e-12, atol=1e-12)
    assert oracle_mod.lstsq(np.ones((5, 2)), X[:5]) is None
    for _ in range(20):
        B = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        W, s, Vh = np.linalg.svd(B)
        np.testing.assert_allclose(oracle_mod.polar2(B), W @ Vh, atol=1e-13)


def _vander(d, Q, fsel=None):
    x = (np.asarray(d["freq"]) - d["f0"]) / d["f0"]
    if fsel is not None:
        x = x[fsel]
    return np.vander(x, Q, increasing=True)


def test_z_update_closed_form_and_invariants(oracle_mod, synth_mod):
    rng = np.random.default_rng(6)
    cfg = tiny_cfg(synth_mod, N=3, P=6, Q=3, K=2, rho=2.5)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    Y0 = 0.1 * (rng.normal(size=J.shape) + 1j * rng.normal(size=J.shape))
    Zold = np.zeros(pb.zshape(), np.complex128)
    Y, Z, BZ, pr, du = pb.consensus(J, Y0, Zold)
    Bv = _vander(d, cfg.Q)
    rho = 2.5
    for k in range(cfg.K):
        # the paper's closed form: Z = (1/rho) ((sum b b^T)^+ kron I) sum_f b_f kron (Y_f + rho J_f)
        R = np.einsum("fl,fx->lx", Bv, (Y0[:, k] + rho * J[:, k]).reshape(cfg.P, -1))
        Zref = (np.linalg.pinv(Bv.T @ Bv) @ R) / rho
        np.testing.assert_allclose(Z[k].reshape(cfg.Q, -1), Zref, rtol=1e-10, atol=1e-12)
        # stationarity of M2: sum_f b_f (-Y_f - rho (J_f - B_f Z)) = 0
        grad = np.einsum("fl,fx->lx", Bv, (-Y0[:, k] - rho * (J[:, k] - BZ[:, k])).reshape(cfg.P, -1))
        assert np.max(np.abs(grad)) < 1e-12 * np.max(np.abs(R))
        # after the dual update the multipliers are orthogonal to the basis
        inv = np.einsum("fl,fx->lx", Bv, Y[:, k].reshape(cfg.P, -1))
        assert np.max(np.abs(inv)) < 1e-12 * (1 + np.max(np.abs(Y)))
    # residual definitions of Section 4
    ref_pr = np.mean([np.linalg.norm(J[f, k] - BZ[f, k]) / np.sqrt(4 * cfg.N)
                      for f in range(cfg.P) for k in range(cfg.K)])
    assert abs(pr - ref_pr) < 1e-12
    ref_du = np.mean([np.linalg.norm(Z[k]) / np.sqrt(4 * cfg.Q * cfg.N) for k in range(cfg.K)])
    assert abs(du - ref_du) < 1e-12


def test_rank_condition(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=3, P=2, Q=3, K=1)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    J = synth_mod.identity_jones(2, 1, 3)
    with pytest.raises(ValueError):
        pb.consensus(J, np.zeros_like(J), np.zeros(pb.zshape(), np.complex128))


def test_truth_in_span_is_fixed_point(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=5, Q=3, K=2, snr=None, lm_iters=5)
    d = synth_mod.generate(cfg, truth_in_span=True)
    pb = oracle_mod.Problem(d)
    Jt = d["jones_true"]
    Y = np.zeros_like(Jt)
    J1 = pb.local_step(Jt, Y, Jt)
    assert np.max(np.abs(J1 - Jt)) < 1e-10
    Y1, Z, BZ, pr, du = pb.consensus(J1, Y, np.zeros(pb.zshape(), np.complex128))
    assert pr < 1e-12 and np.max(np.abs(Y1)) < 1e-10
    np.testing.assert_allclose(BZ, Jt, atol=1e-12)


def test_admm_noise_free_reaches_zero_cost(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=6, P=5, Q=3, K=2, snr=None, lm_iters=10)
    d = synth_mod.generate(cfg, truth_in_span=True)
    pb = oracle_mod.Problem(d)
    out = pb.admm_solve(synth_mod.identity_jones(cfg.P, cfg.K, cfg.N), 12)
    tr = out["trace"]
    # the consensus penalty keeps a small per-subband gauge mismatch, so the data cost falls by
    # five to six orders of magnitude rather than to rounding level within a dozen iterations
    assert tr[-1, 0] < 1e-4 * tr[0, 0]
    assert tr[-1, 2] < 2e-2 * tr[0, 2]


def test_rho_zero_is_normal_calibration(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=5, P=4, Q=2, K=2, rho=0.0, lm_iters=6)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d, options=0)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    out = pb.admm_solve(J0, 3)
    J = J0.copy()
    zero = np.zeros_like(J0)
    for _ in range(3):
        J = pb.local_step(J, zero, zero)
    np.testing.assert_allclose(out["J"], J, rtol=0, atol=1e-13)
    assert np.max(np.abs(out["Y"])) == 0.0


def test_lm_converges_noise_free(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=5, P=1, Q=1, K=1, snr=None, rho=0.0, lm_iters=30)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d, rho=np.zeros(1))
    rng = np.random.default_rng(7)
    J0 = d["jones_true"] + 0.05 * (rng.normal(size=d["jones_true"].shape)
                                   + 1j * rng.normal(size=d["jones_true"].shape))
    z = np.zeros_like(J0)
    J, tr = pb.local_step(J0, z, z, trace=True)
    g0 = pb.subband_cost(J0)[0]
    assert pb.subband_cost(J)[0] < 1e-20 * g0
    objective = tr[0, 0, 0, :, 0]
    assert np.all(np.diff(objective) <= 0)


def test_lm_matches_scipy_least_squares(oracle_mod, synth_mod):
    scipy_opt = pytest.importorskip("scipy.optimize")
    cfg = tiny_cfg(synth_mod, N=4, P=1, Q=1, K=1, rho=0.0, lm_iters=60)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d, rho=np.zeros(1))
    J0 = synth_mod.identity_jones(1, 1, cfg.N)
    z = np.zeros_like(J0)
    J = pb.local_step(J0, z, z)
    V = d["vis"].reshape(-1)

    def resid(theta):
        Jt = (theta[0::2] + 1j * theta[1::2]).reshape(1, 1, cfg.N, 2, 2)
        r = V - pb.predict(Jt).reshape(-1)
        return np.concatenate([r.real, r.imag])

    th0 = np.stack([J0.reshape(-1).real, J0.reshape(-1).imag], 1).reshape(-1)
    sol = scipy_opt.least_squares(resid, th0, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
    ref = np.sum(sol.fun ** 2)
    assert abs(pb.subband_cost(J)[0] - ref) <= 1e-9 * ref


def test_gpa_alignment(oracle_mod, synth_mod):
    rng = np.random.default_rng(8)
    cfg = tiny_cfg(synth_mod, N=5, P=5, K=1)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    base = rand_jones(rng, 1, 1, cfg.N)[0, 0]
    J = np.zeros((cfg.P, 1, cfg.N, 2, 2), np.complex128)
    for f in range(cfg.P):
        J[f, 0] = (base + 0.01 * rng.normal(size=base.shape)) @ _unitary(rng)
    Ja = pb.gpa(J, rounds=3)
    np.testing.assert_allclose(pb.subband_cost(Ja), pb.subband_cost(J), rtol=1e-12)
    spread_before = np.mean([np.linalg.norm(J[f, 0] - J[0, 0]) for f in range(cfg.P)])
    spread_after = np.mean([np.linalg.norm(Ja[f, 0] - Ja[0, 0]) for f in range(cfg.P)])
    assert spread_after < 0.1 * spread_before
    # Procrustes optimality: J_f^H mean is Hermitian positive semi-definite after alignment
    mean = Ja[:, 0].mean(axis=0)
    for f in range(cfg.P):
        A = np.einsum("pji,pjk->ik", np.conj(Ja[f, 0]), mean)
        np.testing.assert_allclose(A, A.conj().T, atol=1e-3 * np.abs(A).max())


def test_admm_trends_with_rho(oracle_mod, synth_mod):
    """Section 4.1 trends: the primal residual falls with iterations and is lower for larger rho."""
    cfg = tiny_cfg(synth_mod, N=8, P=6, Q=3, K=1, T=4, n_chan=1, lm_iters=6)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, 1, cfg.N)
    res = {}
    for rho in (0.5, 50.0):
        pb = oracle_mod.Problem(d, rho=np.array([rho]))
        res[rho] = pb.admm_solve(J0, 15)["trace"]
    assert res[50.0][-1, 2] < res[50.0][1, 2]
    assert res[50.0][-1, 2] < res[0.5][-1, 2]


def test_lm_stopping_rule_truncates_the_run(oracle_mod, synth_mod):
    # the stopping rule only ends the run: the trace up to the stop equals the fixed-iteration
    # trace, the rows after it repeat (F, lambda) with no accepted step, and a tolerance no step
    # can meet (the predicted decrease of a step is positive) changes nothing
    cfg = tiny_cfg(synth_mod, N=6, P=3, K=2, T=3, n_chan=2, lm_iters=12)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    z = np.zeros_like(J0)
    _, t0 = oracle_mod.Problem(d, lm_iters=12).local_step(J0, z, z, trace=True)
    _, tn = oracle_mod.Problem(d, lm_iters=12, lm_tol=1e-300).local_step(J0, z, z, trace=True)
    np.testing.assert_array_equal(tn, t0)
    _, ts = oracle_mod.Problem(d, lm_iters=12, lm_tol=1e-7).local_step(J0, z, z, trace=True)
    # direction 0 of every subband starts from the same state in both runs (later directions
    # start from whatever the earlier directions' runs left)
    stopped = 0
    for f in range(cfg.P):
        for k in (0,):
            a, b = t0[f, 0, k], ts[f, 0, k]
            # first row where the runs differ: the stop happened in the row before it
            diff = np.nonzero(np.any(a != b, axis=1))[0]
            if len(diff) == 0:
                continue
            s = diff[0]
            assert s >= 1
            np.testing.assert_array_equal(b[:s], a[:s])
            assert np.all(b[s:, 0] == b[s - 1, 0]) and np.all(b[s:, 1] == b[s - 1, 1])
            assert np.all(b[s:, 2] == 0)
            stopped += 1
    assert stopped >= 2


def test_gradient_is_twice_the_papers_printed_gradient(oracle_mod, synth_mod):
    """Section 3 prints the gradient of the augmented Lagrangian as grad g + Y/2 + rho/2 (J - B Z),
    with grad g = -sum_pq [A_p^T R A_q J C^H + A_q^T R^H A_p J C], R = V - A_p J C J^H A_q^T, J the
    2N x 2 stack of the stations' Jones matrices and A_p the 2 x 2N selector of station p (the
    Riemannian gradient under the inner product tr(x^H y + y^H x) of Appendix A).  The oracle's
    Euclidean gradient over the real parameters (d/dRe + i d/dIm per entry) is exactly twice it:
    this fixes the scale of the Y and rho terms, which finite differences of the oracle's own
    objective cannot tell apart from a consistent slip in objective and gradient together."""
    rng = np.random.default_rng(21)
    cfg = tiny_cfg(synth_mod, N=4, P=2, K=2, T=2, n_chan=2, rho=3.0)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    N, K, spb = cfg.N, cfg.K, cfg.T * 2
    J = rand_jones(rng, cfg.P, K, N)
    Y = 0.4 * (rng.normal(size=J.shape) + 1j * rng.normal(size=J.shape))
    BZ = rand_jones(rng, cfg.P, K, N)
    pairs = list(zip(*synth_mod.baseline_pairs(N)))
    I2 = np.eye(2)
    A = []
    for p in range(N):
        a = np.zeros((2, 2 * N))
        a[:, 2 * p:2 * p + 2] = I2
        A.append(a)
    for f, k in ((0, 1), (1, 0)):
        _, G = pb.dir_objective(J, Y, BZ, f, k)
        V = d["vis"][d["vis_off"][f]:d["vis_off"][f + 1]]
        c = d["coh"][d["coh_off"][f]:d["coh_off"][f + 1]].reshape(K, -1)
        Js = [J[f, l].reshape(2 * N, 2) for l in range(K)]
        grad_g = np.zeros((2 * N, 2), np.complex128)
        for b, (p, q) in enumerate(pairs):
            for s in range(b * spb, (b + 1) * spb):
                # the SAGE expectation of direction k (Section 3): the other directions' models
                # removed from the data
                Vk = V[s] - sum(c[l, s] * A[p] @ Js[l] @ Js[l].conj().T @ A[q].T
                                for l in range(K) if l != k)
                C = c[k, s] * I2
                R = Vk - A[p] @ Js[k] @ C @ Js[k].conj().T @ A[q].T
                grad_g -= (A[p].T @ R @ A[q] @ Js[k] @ C.conj().T
                           + A[q].T @ R.conj().T @ A[p] @ Js[k] @ C)
        grad_L = (grad_g + 0.5 * Y[f, k].reshape(2 * N, 2)
                  + 0.5 * 3.0 * (Js[k] - BZ[f, k].reshape(2 * N, 2)))
        assert np.linalg.norm(G.reshape(2 * N, 2) - 2 * grad_L) <= 1e-12 * np.linalg.norm(grad_L)


def test_trace_lagrangian_column(oracle_mod, synth_mod):
    """Trace row n holds the data cost sum_f g_f after the local step of iteration n and the
    augmented Lagrangian of Section 3 (linear term in the trace form of Appendix A) at that J with
    the multipliers and B_f Z of the previous consensus update.  Tied to the per-direction
    objectives of the local step (each direction's objective after the SAGE expectation holds the
    whole residual, so sum_k L_fk = K_f g_f + sum_k penalty_fk) and to the trace form summed
    directly; per-direction rho_k (Section 3 allows one per direction) of 2 and 7."""
    cfg = tiny_cfg(synth_mod, N=5, P=4, Q=2, K=2, T=2, n_chan=2, lm_iters=4)
    d = synth_mod.generate(cfg)
    rho = np.array([2.0, 7.0])
    pb = oracle_mod.Problem(d, lm_iters=4, rho=rho)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    one = pb.admm_solve(J0, 1)
    two = pb.admm_solve(J0, 2)
    J2 = pb.local_step(one["J"], one["Y"], one["BZ"])
    np.testing.assert_array_equal(J2, two["J"])
    Y1, BZ1 = one["Y"], one["BZ"]
    g = pb.subband_cost(J2)
    via_dirs = sum(pb.dir_objective(J2, Y1, BZ1, f, k, grad=False)
                   for f in range(cfg.P) for k in range(cfg.K)) - (cfg.K - 1) * g.sum()
    e = J2 - BZ1
    direct = g.sum() + sum(np.sum(np.real(np.conj(Y1[:, k]) * e[:, k]))
                           + 0.5 * rho[k] * np.sum(np.abs(e[:, k]) ** 2) for k in range(cfg.K))
    L = two["trace"][1, 1]
    assert abs(two["trace"][1, 0] - g.sum()) <= 1e-13 * g.sum()
    assert abs(L - via_dirs) <= 1e-12 * abs(L)
    assert abs(L - direct) <= 1e-12 * abs(L)


def test_admm_continues_from_a_carried_state(oracle_mod, synth_mod):
    """Section 3 starts a new interval from the previous one's solution: continuing a run from its
    own state after n iterations reproduces the uninterrupted run (the iteration depends on the
    state only), and a zero carried state is the cold start."""
    cfg = tiny_cfg(synth_mod, N=6, P=4, Q=2, K=2, T=3, n_chan=2, lm_iters=4)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d, lm_iters=4, options=0)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    whole = pb.admm_solve(J0, 5)
    first = pb.admm_solve(J0, 2)
    rest = pb.admm_solve(first["J"], 3, first["Y"], first["Z"], first["BZ"])
    np.testing.assert_array_equal(rest["J"], whole["J"])
    # the dual residual of the first continued iteration uses the carried Z, the rest is identical
    np.testing.assert_array_equal(rest["trace"][:, :3], whole["trace"][2:, :3])
    zero = np.zeros(pb.jshape(), np.complex128)
    cold = pb.admm_solve(J0, 2, zero, np.zeros(pb.zshape(), np.complex128), zero)
    np.testing.assert_array_equal(cold["trace"], first["trace"])


def test_lm_damping_schedule_on_an_exact_quadratic(oracle_mod, synth_mod):
    """Nielsen's damping (Madsen, Nielsen & Tingleff 2004, Sec. 3.2) in closed form.  With every
    coherency zero the data term of M1 is the constant sum ||V||^2 and H_GN = 0, so the objective
    is the quadratic penalty with Euclidean gradient G = Y + rho (J - B Z) and Hessian rho I.  The
    LM step delta = -G / (rho + lambda) then decreases the objective by exactly the predicted
    amount, |G|^2 (rho + 2 lambda) / (2 (rho + lambda)^2), so the gain ratio is 1: each step is
    accepted, lambda starts at tau max diag = 1e-3 rho and falls by the rule's floor factor 1/3,
    G shrinks by lambda / (rho + lambda), and each step lowers the objective by the fall of
    |G|^2 / (2 rho), leaving J at |G| / rho from the minimiser B Z - Y / rho.  Within a few steps
    the next step's true decrease falls below the objective's rounding; such steps are rejected
    and lambda grows by nu = 2, 4, 8, ... (the reject branch)."""
    rng = np.random.default_rng(23)
    rho, iters = 3.0, 8
    cfg = tiny_cfg(synth_mod, N=4, P=2, K=1, T=2, n_chan=2, rho=rho, lm_iters=iters)
    d = synth_mod.generate(cfg)
    d = dict(d, coh=np.zeros_like(d["coh"]))
    pb = oracle_mod.Problem(d)
    J0 = rand_jones(rng, cfg.P, 1, cfg.N)
    Y = rand_jones(rng, cfg.P, 1, cfg.N, scale=0.5) - J0
    BZ = rand_jones(rng, cfg.P, 1, cfg.N)
    J, tr = pb.local_step(J0, Y, BZ, trace=True)
    eps = np.finfo(float).eps
    for f in range(cfg.P):
        t = tr[f, 0, 0]
        F_scale = abs(t[0, 0])
        # closed-form accepted phase
        lam = 1e-3 * rho
        G = Y[f, 0] + rho * (J0[f, 0] - BZ[f, 0])
        g2, lams = [np.sum(np.abs(G) ** 2)], []
        for _ in range(iters):
            G = G * lam / (rho + lam)
            g2.append(np.sum(np.abs(G) ** 2))
            lam /= 3.0
            lams.append(lam)
        rejected = np.nonzero(t[:, 2] == 0)[0]
        n_acc = int(rejected[0]) if len(rejected) else iters
        assert n_acc >= 2
        assert np.all(t[:n_acc, 2] == 1)
        np.testing.assert_allclose(t[:n_acc, 1], lams[:n_acc], rtol=1e-14)
        for i in range(1, n_acc):
            want = (g2[i] - g2[i + 1]) / (2 * rho)
            assert abs((t[i - 1, 0] - t[i, 0]) - want) <= 64 * eps * F_scale
        # the distance from the minimiser B Z - Y / rho after the accepted steps: |G| / rho
        Jstar = BZ[f, 0] - Y[f, 0] / rho
        dist = np.sqrt(np.sum(np.abs(J[f, 0] - Jstar) ** 2))
        assert abs(dist - np.sqrt(g2[n_acc]) / rho) <= 1e-13 * np.max(np.abs(Jstar))
        # the first rejected step's true decrease is below the objective's rounding, and each
        # rejection in a row multiplies lambda by the next power of two
        if n_acc < iters:
            assert (g2[n_acc] - g2[n_acc + 1]) / (2 * rho) <= 8 * eps * F_scale
            lam, nu = t[n_acc - 1, 1], 2.0
            for i in range(n_acc, iters):
                if t[i, 2] == 1:
                    break
                lam *= nu
                nu *= 2.0
                assert t[i, 1] == lam
                assert t[i, 0] == t[n_acc - 1, 0]
