"""Pins of the warm-start part of the oracle (network, features, targets, fallback) against
closed forms, finite differences, textbook special cases and independent routes."""
import numpy as np
import pytest

from conftest import rand_jones, tiny_cfg


@pytest.fixture(scope="module")
def mlp_mod():
    from oracle import mlp
    return mlp


@pytest.fixture(scope="module")
def ws_mod(oracle_mod):
    from oracle import warmstart
    return warmstart


# ---- network ------------------------------------------------------------------------------------

def test_bf16_rounding_known_values(mlp_mod):
    # bfloat16 keeps 8 significant bits: the spacing just above 1 is 2^-7
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38, 0.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 2.9908e38, 0.0])
    got = mlp_mod.bf16(x)
    assert np.array_equal(got[:5], want[:5]) and got[6] == 0.0
    assert abs(got[5] - 3.0e38) <= 2 ** -8 * 3.0e38
    # ties go to the even neighbour in both directions
    assert mlp_mod.bf16(1 + 2 ** -7 + 2 ** -8) == 1 + 2 ** -6


def test_gelu_identities(mlp_mod):
    x = np.linspace(-6, 6, 241)
    g = mlp_mod.gelu(x)
    # x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x) = 1)
    assert np.max(np.abs(g - mlp_mod.gelu(-x) - x)) < 1e-14
    assert mlp_mod.gelu(0.0) == 0.0
    assert abs(mlp_mod.gelu(1.0) - 0.8413447460685429) < 1e-15    # Phi(1)
    h = 1e-6
    fd = (mlp_mod.gelu(x + h) - mlp_mod.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp_mod.gelu_grad(x))) < 1e-8


def test_backward_matches_finite_differences(mlp_mod):
    rng = np.random.default_rng(0)
    dims = [5, 7, 6, 3]
    p = rng.normal(0, 0.5, mlp_mod.n_params(dims))
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=(9, 3))
    g, _ = mlp_mod.backward(dims, p, x, t, bf16_ops=False)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp_mod.loss(dims, p + e, x, t, False) - mlp_mod.loss(dims, p - e, x, t, False)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)


def test_single_layer_is_linear_least_squares(mlp_mod):
    # one layer, no activation: y = x W + b and d/dW mean((y-t)^2) = 2 x^T (y - t) / (rows*out)
    rng = np.random.default_rng(1)
    dims = [4, 3]
    p = rng.normal(size=mlp_mod.n_params(dims))
    x = rng.normal(size=(10, 4))
    t = rng.normal(size=(10, 3))
    W, b = p[:12].reshape(4, 3), p[12:]
    y, _ = mlp_mod.forward(dims, p, x, bf16_ops=False)
    assert np.allclose(y, x @ W + b, rtol=0, atol=1e-14)
    g, L = mlp_mod.backward(dims, p, x, t, bf16_ops=False)
    r = x @ W + b - t
    assert np.allclose(g[:12].reshape(4, 3), 2 * x.T @ r / r.size, rtol=1e-13, atol=1e-15)
    assert np.allclose(g[12:], 2 * r.sum(0) / r.size, rtol=1e-13, atol=1e-15)
    assert abs(L - np.mean(r ** 2)) < 1e-14


def test_bf16_mode_rounds_the_gemm_operands(mlp_mod):
    # with bf16-exact inputs and weights, the bf16 mode equals the exact computation
    rng = np.random.default_rng(2)
    dims = [6, 4]
    p = mlp_mod.bf16(rng.normal(size=mlp_mod.n_params(dims)))
    x = mlp_mod.bf16(rng.normal(size=(5, 6)))
    assert np.array_equal(mlp_mod.forward(dims, p, x, True)[0], mlp_mod.forward(dims, p, x, False)[0])
    # and an input off the bf16 grid changes the output by at most the rounding of that input
    x2 = x.copy()
    x2[0, 0] += 2 ** -12 * abs(x2[0, 0])
    y1, y2 = mlp_mod.forward(dims, p, x2, True)[0], mlp_mod.forward(dims, p, x2, False)[0]
    W = p[:24].reshape(6, 4)
    assert np.max(np.abs(y1 - y2)) <= abs(x2[0, 0] - mlp_mod.bf16(x2[0, 0])) * np.max(np.abs(W)) + 1e-15


def test_adam_first_step_closed_form(mlp_mod):
    # after one step m_hat = g, v_hat = g^2, so the update is lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, -1.0, 0.5])
    opt = mlp_mod.Adam(4, lr=0.01)
    p1 = opt.step(p0, g)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    for _ in range(5):
        p2 = opt.step(p1, g)
        assert np.allclose(p2 - p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
        p1 = p2


# ---- features, targets, fallback -----------------------------------------------------------------

def test_gn_step_feature_solves_the_diagonal_gauss_newton_block(oracle_mod, synth_mod, ws_mod):
    # independent route: the explicit-Jacobian Gauss-Newton matrix of the oracle; the feature is
    # SCALE * argmin over dJ_p of the quadratic model with the other stations held
    rng = np.random.default_rng(4)
    cfg = tiny_cfg(synth_mod, N=5, P=2, K=2, flag_frac_max=0.2)
    d = synth_mod.generate(cfg)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N, 0.15)
    F = ws_mod.features(d, J).reshape(cfg.P, cfg.K, cfg.N, 32)
    pb = oracle_mod.Problem(d, rho=np.zeros(cfg.K))
    zeros = np.zeros_like(J)
    for f in range(cfg.P):
        for k in range(cfg.K):
            H = pb.dir_gn_hessian(f, k, J[f, k])
            _, G = pb.dir_objective(J, zeros, zeros, f, k)
            g = np.stack([G.reshape(-1).real, G.reshape(-1).imag], 1).reshape(-1)
            for p in range(cfg.N):
                s = slice(8 * p, 8 * p + 8)
                dlt = np.linalg.solve(H[s, s], -g[s])
                assert np.allclose(F[f, k, p, 16:24], ws_mod.SCALE * dlt, rtol=1e-9,
                                   atol=1e-12 * np.max(np.abs(F[f, k, :, 16:24])))
            assert np.allclose(F[f, k, :, 0:8], ws_mod._flat(J[f, k]))


def test_features_vanish_at_the_noise_free_truth(oracle_mod, synth_mod, ws_mod):
    cfg = tiny_cfg(synth_mod, snr=None)
    d = synth_mod.generate(cfg)
    J = d["jones_true"]
    F = ws_mod.features(d, J, J2=J, BZp=J)
    assert np.max(np.abs(F[:, 8:])) < 1e-9 * np.max(np.abs(F[:, :8]))


def test_target_is_gauge_invariant(oracle_mod, synth_mod, ws_mod):
    # Jnew = (Jprev + dJ) U for a unitary U per (f, k): the target is SCALE * dJ aligned, and for
    # dJ = 0 it is zero whatever U is
    rng = np.random.default_rng(5)
    cfg = tiny_cfg(synth_mod)
    d = synth_mod.generate(cfg)
    Jp = rand_jones(rng, cfg.P, cfg.K, cfg.N)
    U = np.linalg.qr(rng.normal(size=(cfg.P, cfg.K, 2, 2)) + 1j * rng.normal(size=(cfg.P, cfg.K, 2, 2)))[0]
    Jn = Jp @ U[:, :, None]
    assert np.max(np.abs(ws_mod.target(d, Jn, Jp))) < 1e-12
    # Procrustes by SVD agrees with the oracle's Newton polar iteration
    for _ in range(5):
        A = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        assert np.allclose(ws_mod.procrustes(A), oracle_mod.polar2(A), atol=1e-12)


def test_fallback_keeps_only_cost_lowering_corrections(oracle_mod, synth_mod, ws_mod):
    cfg = tiny_cfg(synth_mod, snr=None)
    d = synth_mod.generate(cfg)
    J0 = d["jones_true"] + 0.05
    # delta toward the truth for even subbands, away from it for odd ones
    toward = ws_mod.SCALE * ws_mod._flat(d["jones_true"] - J0)
    toward[1::2] *= -3
    delta = toward.reshape(-1, 8).astype(np.float32)
    J1, keep, c0, c1 = ws_mod.apply(d, J0, delta)
    assert list(keep) == [True, False] * (cfg.P // 2)
    assert np.all(oracle_mod.Problem(d).subband_cost(J1) <= c0)
    assert np.array_equal(J1[1::2], J0[1::2])
