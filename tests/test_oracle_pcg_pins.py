"""Pins of the oracle's matrix-free reading of the local solve: Levenberg-Marquardt whose damped
normal equations (H_GN + (rho + lambda) I) delta = -G are solved by block-Jacobi preconditioned
conjugate gradients instead of a Cholesky factorisation (Section 3 minimises M1 iteratively with
an operator-form Hessian; this replaces only the linear solve inside each LM step).

Pinned against: NumPy's dense solve (the CG iterate approaches it as the tolerance goes to zero,
within n iterations), the Galerkin property of CG iterates (delta.(A delta) = b.delta at every
tolerance, which keeps the LM predicted-decrease formula exact), a block-diagonal system (one
iteration with the exact block preconditioner), the closed form of the preconditioner blocks (the
8x8 diagonal block of station p of the Gauss-Newton matrix is v -> 2 v Q_p, Q_p = sum_q S_pq J_q^H
J_q, so the GPU's 2x2 form of it is the same matrix), and whole LM traces against the Cholesky
reading at a tight tolerance.
"""
import numpy as np

from conftest import rand_jones, tiny_cfg


def _system(oracle_mod, synth_mod, N=9, seed=41, lamf=1e-3, rho=5.0):
    cfg = tiny_cfg(synth_mod, N=N, P=1, Q=1, K=1, T=3, n_chan=2, rho=rho)
    d = synth_mod.generate(cfg)
    pb = oracle_mod.Problem(d)
    rng = np.random.default_rng(seed)
    J = rand_jones(rng, 1, 1, N, scale=0.15)
    z = np.zeros_like(J)
    _, G = pb.dir_objective(J, z, z, 0, 0)
    g = np.stack([G.reshape(-1).real, G.reshape(-1).imag], 1).reshape(-1)
    H = pb.dir_gn_hessian(0, 0, J[0, 0]) + rho * np.eye(8 * N)
    A = H + lamf * np.max(np.diag(H)) * np.eye(8 * N)
    return cfg, d, pb, J, A, -g


def test_pcg_approaches_the_dense_solve(oracle_mod, synth_mod):
    for lamf in (1e-3, 1e-6):
        _, _, _, _, A, b = _system(oracle_mod, synth_mod, lamf=lamf)
        exact = np.linalg.solve(A, b)
        errs = []
        for tol in (1e-3, 1e-6, 1e-9, 1e-12):
            x, it = oracle_mod.pcg(A, b, tol)
            assert it <= A.shape[0]
            assert np.linalg.norm(b - A @ x) <= 1.0001 * tol * np.linalg.norm(b)
            errs.append(np.linalg.norm(x - exact) / np.linalg.norm(exact))
            # Galerkin: the residual of a CG iterate is orthogonal to the iterate
            assert abs(x @ (A @ x) - b @ x) <= 1e-12 * abs(b @ x)
        assert errs[-1] < 1e-8 and errs[-1] < errs[0]


def test_pcg_on_block_diagonal_system_is_one_step(oracle_mod):
    rng = np.random.default_rng(42)
    n = 8 * 6
    A = np.zeros((n, n))
    for s in range(6):
        B = rng.normal(size=(8, 8))
        A[8 * s:8 * s + 8, 8 * s:8 * s + 8] = B @ B.T + 8 * np.eye(8)
    b = rng.normal(size=n)
    x, it = oracle_mod.pcg(A, b, 1e-14)
    assert it == 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12)
    assert oracle_mod.pcg(-np.eye(16), np.ones(16), 1e-10) is None


def test_preconditioner_blocks_closed_form(oracle_mod, synth_mod):
    cfg, d, pb, J, A, _ = _system(oracle_mod, synth_mod, N=7, seed=43)
    N = cfg.N
    H = pb.dir_gn_hessian(0, 0, J[0, 0])
    spb = cfg.T * 2
    c = d["coh"].reshape(cfg.B, spb)
    S = np.sum(np.abs(c) ** 2, axis=1)
    p_of, q_of = synth_mod.baseline_pairs(N)
    Sd = np.zeros((N, N))
    Sd[p_of, q_of] = S
    Sd[q_of, p_of] = S
    Jd = J[0, 0]
    for p in range(N):
        Qp = sum(Sd[p, o] * Jd[o].conj().T @ Jd[o] for o in range(N) if o != p)
        blk = np.zeros((8, 8))
        for col in range(8):   # real representation of v -> 2 v Q_p, column by column
            v = np.zeros(8)
            v[col] = 1.0
            V = (v[0::2] + 1j * v[1::2]).reshape(2, 2)
            W = 2 * V @ Qp
            blk[:, col] = np.stack([W.reshape(-1).real, W.reshape(-1).imag], 1).reshape(-1)
        np.testing.assert_allclose(H[8 * p:8 * p + 8, 8 * p:8 * p + 8], blk, rtol=1e-12,
                                   atol=1e-12 * np.abs(blk).max())


def test_lm_with_pcg_follows_the_cholesky_trace(oracle_mod, synth_mod):
    cfg = tiny_cfg(synth_mod, N=8, P=3, K=2, T=3, n_chan=2, lm_iters=8)
    d = synth_mod.generate(cfg)
    J0 = synth_mod.identity_jones(cfg.P, cfg.K, cfg.N)
    z = np.zeros_like(J0)
    Jc, tc = oracle_mod.Problem(d, lm_iters=8).local_step(J0, z, z, trace=True)
    Jp, tp = oracle_mod.Problem(d, lm_iters=8, solver=oracle_mod.SOLVE_PCG,
                                cg_tol=1e-13).local_step(J0, z, z, trace=True)
    # accept decisions agree wherever the step moves the objective by more than rounding (near
    # convergence the last iterations change it by ~1e-16 relative: a tie either way)
    prev = np.concatenate([np.full(tc.shape[:-2] + (1,), np.inf), tc[..., :-1, 0]], axis=-1)
    decisive = np.abs(tc[..., 0] - prev) > 1e-12 * np.abs(tc[..., 0])
    np.testing.assert_array_equal(tp[..., 2][decisive], tc[..., 2][decisive])
    assert decisive.sum() > 0.6 * decisive.size
    np.testing.assert_allclose(tp[..., 0], tc[..., 0], rtol=1e-11)
    # a step taken or refused at a rounding tie near the optimum, where the objective is quadratic,
    # has size ~sqrt(eps) relative: J agrees to that
    assert np.max(np.abs(Jp - Jc)) < 1e-7
    # a loose tolerance changes the steps, not the way the iteration behaves: still descending
    _, tl = oracle_mod.Problem(d, lm_iters=8, solver=oracle_mod.SOLVE_PCG,
                               cg_tol=1e-3).local_step(J0, z, z, trace=True)
    assert np.all(np.diff(tl[..., 0], axis=-1) <= 0)
