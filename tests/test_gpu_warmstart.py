"""Learned warm start on the GPU against the FP64 oracle: features, training targets, the cost
fallback, and the BF16 network's forward, gradients and Adam step; then what a network trained by
the library's own kernels gains over the previous-interval start.

Network tolerances.  The kernels and the oracle round the same values to BF16 at the same points
and differ only in how they accumulate (FP32 on the matrix cores against FP64): for one GEMM that
is at most (K + 2) 2^-24 sum_i |x_i w_i| per output.  Deeper, an accumulation difference can move
a hidden activation across a BF16 rounding boundary (probability ~K 2^-24 / 2^-8 per element),
which shifts it by one BF16 unit, 2^-8 relative; each such flip moves an output by about
2^-8 |h w|, a few 1e-4 of the output scale at most.
"""
import numpy as np
import pytest

from conftest import rand_jones, tiny_cfg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


@pytest.fixture(scope="module")
def ws_or(oracle_mod):
    from oracle import warmstart
    return warmstart


@pytest.fixture(scope="module")
def mlp_or():
    from oracle import mlp
    return mlp


def _ctx(cal, d, precision=0, jones0=None, **kw):
    vis, coh, flags = cal.device_inputs(d, precision)
    J0 = None if jones0 is None else torch.from_numpy(np.ascontiguousarray(jones0)).cuda()
    return cal.Calib(d, vis, coh, flags, J0, precision=precision, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ragged(synth_mod, **kw):
    return tiny_cfg(synth_mod, N=6, P=4, K=3, T=3, n_chan=2, Q=2, flag_frac_max=0.25,
                    n_dirs=[3, 1, 2, 3], **kw)


# ---- features, targets, fallback -----------------------------------------------------------------

def test_features_match_oracle(cal, ws_or, synth_mod):
    cfg = _ragged(synth_mod)
    d = synth_mod.generate(cfg)
    rng = np.random.default_rng(21)
    J = rand_jones(rng, cfg.P, cfg.K, cfg.N, 0.1)
    J2 = rand_jones(rng, cfg.P, cfg.K, cfg.N, 0.1)
    BZ = rand_jones(rng, cfg.P, cfg.K, cfg.N, 0.1)
    c = _ctx(cal, d, 0, jones0=J)
    print(f"features: N={cfg.N} P={cfg.P} K={cfg.K} n_dirs={list(cfg.n_dirs)}", flush=True)
    for j2, bz in ((J2, BZ), (None, None)):
        got = c.warmstart_features(None if j2 is None else _dev(j2),
                                   None if bz is None else _dev(bz)).cpu().numpy()
        want = ws_or.features(d, J, j2, bz)
        scale = np.max(np.abs(want), axis=0)
        # FP32 rounding of the FP64 value, plus FP64 reduction-order differences in the gradient
        assert np.all(np.abs(got - want) <= 2 * U32 * np.abs(want) + 1e-10 * scale + 1e-300)
    # J is untouched and the absent directions' rows are zero
    assert np.array_equal(c.get(cal.FIELD_J).cpu().numpy(), J)
    rows = got.reshape(cfg.P, cfg.K, cfg.N, 32)
    for f, kf in enumerate(cfg.n_dirs):
        assert np.all(rows[f, kf:] == 0)


def test_target_matches_oracle(cal, ws_or, synth_mod):
    cfg = _ragged(synth_mod)
    d = synth_mod.generate(cfg)
    rng = np.random.default_rng(22)
    Jp = rand_jones(rng, cfg.P, cfg.K, cfg.N, 0.1)
    U = np.linalg.qr(rng.normal(size=(cfg.P, cfg.K, 2, 2)) + 1j * rng.normal(size=(cfg.P, cfg.K, 2, 2)))[0]
    Jn = (Jp + 0.02 * (rng.normal(size=Jp.shape) + 1j * rng.normal(size=Jp.shape))) @ U[:, :, None]
    c = _ctx(cal, d, 0, jones0=Jn)
    got = c.warmstart_target(_dev(Jp)).cpu().numpy()
    want = ws_or.target(d, Jn, Jp)
    for f, kf in enumerate(cfg.n_dirs):
        want.reshape(cfg.P, cfg.K, cfg.N, 8)[f, kf:] = 0.0
    assert np.all(np.abs(got - want) <= 2 * U32 * np.abs(want) + 1e-11 * np.max(np.abs(want)))
    # a pure gauge change gives a zero target
    c.set_jones(_dev(Jp @ U[:, :, None]))
    z = c.warmstart_target(_dev(Jp)).cpu().numpy()
    assert np.max(np.abs(z)) < 1e-10


def test_apply_matches_oracle_bitwise(cal, ws_or, synth_mod, oracle_mod):
    cfg = _ragged(synth_mod)
    d = synth_mod.generate(cfg)
    J0 = d["jones_true"] + 0.03
    for f, kf in enumerate(cfg.n_dirs):
        J0[f, kf:] = 0.0
    # toward the truth in subbands 0 and 2, away from it in 1 and 3
    delta = ws_or.SCALE * ws_or._flat(d["jones_true"] - J0)
    delta[[1, 3]] *= -4
    delta = delta.reshape(-1, 8).astype(np.float32)
    c = _ctx(cal, d, 0, jones0=J0)
    kept = c.warmstart_apply(_dev(delta)).cpu().numpy()
    J1, keep, c0, c1 = ws_or.apply(d, J0, delta)
    assert list(keep) == [True, False, True, False]
    np.testing.assert_array_equal(kept, keep.astype(np.int32))
    np.testing.assert_array_equal(c.get(cal.FIELD_J).cpu().numpy(), J1)


def test_apply_never_raises_the_cost(cal, synth_mod, oracle_mod):
    cfg = _ragged(synth_mod)
    d = synth_mod.generate(cfg)
    J0 = rand_jones(np.random.default_rng(23), cfg.P, cfg.K, cfg.N, 0.05)
    c = _ctx(cal, d, 0, jones0=J0)
    before = c.get(cal.FIELD_COST).cpu().numpy()
    garbage = np.random.default_rng(24).normal(0, 50, (cfg.P * cfg.K * cfg.N, 8)).astype(np.float32)
    kept = c.warmstart_apply(_dev(garbage)).cpu().numpy()
    assert not kept.any()
    np.testing.assert_array_equal(c.get(cal.FIELD_J).cpu().numpy(), J0)
    np.testing.assert_array_equal(c.get(cal.FIELD_COST).cpu().numpy(), before)


# ---- network -------------------------------------------------------------------------------------

def _params(dims, seed, bias=0.1):
    from paper_1502_00858_amd import synth
    p = synth.mlp_init_params(dims, seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    o = 0
    for i in range(len(dims) - 1):
        o += dims[i] * dims[i + 1]
        p[o:o + dims[i + 1]] = rng.normal(0, bias, dims[i + 1])
        o += dims[i + 1]
    return p.astype(np.float32)


def test_single_gemm_layer_within_fp32_accumulation_bound(cal, mlp_or):
    # one layer spanning several 64x64 output tiles and 16-deep k steps, all ragged
    dims = [40, 72]
    rows = 1000
    p = _params(dims, 31)
    x = np.random.default_rng(32).normal(size=(rows, dims[0])).astype(np.float32)
    net = cal.MLP(dims, p, rows)
    y = net.forward(_dev(x)).cpu().numpy()
    want, _ = mlp_or.forward(dims, p, x)
    W = mlp_or.bf16(p[:40 * 72].reshape(40, 72))
    bound = (dims[0] + 2) * U32 * (np.abs(mlp_or.bf16(x)) @ np.abs(W) + np.abs(p[40 * 72:]))
    assert np.all(np.abs(y - want) <= bound)
    net.close()


def test_forward_matches_oracle(cal, mlp_or):
    from paper_1502_00858_amd import warmstart
    dims = warmstart.DIMS
    rows = 777
    p = _params(dims, 33)
    x = np.random.default_rng(34).normal(size=(rows, dims[0])).astype(np.float32)
    net = cal.MLP(dims, p, 1024)
    y = net.forward(_dev(x)).cpu().numpy()
    want, _ = mlp_or.forward(dims, p, x)
    s = np.max(np.abs(want))
    err = np.abs(y - want)
    print(f"forward: max err {err.max() / s:.2e}, mean err {err.mean() / s:.2e} of max |y|", flush=True)
    assert err.max() <= 4e-3 * s and err.mean() <= 1e-4 * s
    net.close()


def test_gradients_match_oracle(cal, mlp_or):
    from paper_1502_00858_amd import warmstart
    dims = warmstart.DIMS
    rows = 640
    p = _params(dims, 35)
    rng = np.random.default_rng(36)
    x = rng.normal(size=(rows, dims[0])).astype(np.float32)
    t = rng.normal(size=(rows, dims[-1])).astype(np.float32)
    net = cal.MLP(dims, p, rows)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(_dev(x), _dev(t), 0.0, loss)
    g = net.grads()
    assert np.array_equal(net.params(), p)          # lr = 0 leaves the parameters alone
    want, L = mlp_or.backward(dims, p, x, t)
    assert abs(loss.item() - L) <= 1e-3 * L
    o = 0
    for i in range(len(dims) - 1):
        for n in (dims[i] * dims[i + 1], dims[i + 1]):
            a, b = g[o:o + n], want[o:o + n]
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            print(f"grad layer {i} block of {n}: rel err {rel:.2e}", flush=True)
            assert rel <= 1e-2
            o += n
    net.close()


def test_adam_step_on_exact_gradients(cal, mlp_or):
    # dyadic inputs, weights and targets make every product and sum exact in FP32 and BF16, so
    # both sides hold the same gradient and differ only by FP32 rounding inside Adam
    dims = [16, 8]
    rows = 64
    rng = np.random.default_rng(37)
    # |y - t| < 8 in steps of 1/16: at most 7 significant bits, exact in BF16 after scaling
    x = rng.integers(-1, 2, (rows, 16)).astype(np.float32)
    W = (rng.integers(-4, 5, (16, 8)) / 16.0).astype(np.float32)
    b = (rng.integers(-4, 5, 8) / 16.0).astype(np.float32)
    t = (rng.integers(-32, 33, (rows, 8)) / 16.0).astype(np.float32)
    p = np.concatenate([W.reshape(-1), b])
    net = cal.MLP(dims, p, rows)
    net.train_step(_dev(x), _dev(t), 0.0)
    g, L = mlp_or.backward(dims, p, x, t)
    np.testing.assert_array_equal(net.grads(), g.astype(np.float32))
    lr = 1e-2
    net.train_step(_dev(x), _dev(t), lr)
    want = mlp_or.Adam(p.size, lr).step(p.astype(np.float64), g)
    got = net.params()
    assert np.all(np.abs(got - want) <= 2 * U32 * 2 * np.abs(want) + 8 * U32 * lr)
    net.close()


def test_training_follows_the_oracle_and_fits(cal, mlp_or):
    # teacher network targets; the GPU and the oracle train the same student from the same start
    dims = [8, 32, 32, 4]
    rows = 256
    rng = np.random.default_rng(38)
    x = rng.normal(size=(rows, 8)).astype(np.float32)
    teacher = _params(dims, 39, bias=0.3)
    t, _ = mlp_or.forward(dims, teacher, x, bf16_ops=False)
    t = t.astype(np.float32)
    p = _params(dims, 40)
    net = cal.MLP(dims, p, rows)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    opt = mlp_or.Adam(p.size, 3e-3)
    po = p.astype(np.float64)
    lg, lo = [], []
    for _ in range(150):
        net.train_step(_dev(x), _dev(t), 3e-3, loss)
        lg.append(loss.item())
        g, L = mlp_or.backward(dims, po, x, t)
        lo.append(L)
        po = opt.step(po, g)
    lg, lo = np.array(lg), np.array(lo)
    print(f"training: loss {lo[0]:.3e} -> {lo[-1]:.3e} (oracle), {lg[-1]:.3e} (GPU)", flush=True)
    assert lo[-1] < 0.1 * lo[0]
    assert np.all(np.abs(lg - lo) <= 0.05 * lo)
    net.close()


# ---- gain of the trained network -----------------------------------------------------------------

def test_learned_warm_start_gains_over_previous_solution(cal, synth_mod):
    """Episodes of consecutive intervals of the 62-station, 32-subband, 5-direction observation
    (FP32 streaming): train on two short episodes, then start interval 2 of a held-out episode
    from (b) the previous interval's whole C-ADMM state and (c) the same state with the learned
    correction of J and the cost fallback.  Target: the median data cost over the second half of an
    80-iteration run from (b)."""
    from paper_1502_00858_amd import warmstart
    cfg = synth_mod.named_config("c2")
    prec, chain_iters, n_ref = cal.CALIB_FP32_MIXED, 20, 80
    train_iv = []
    for e in range(2):
        print(f"gain: solving training episode {e}", flush=True)
        train_iv += warmstart.solve_episode(cfg, e, 4, prec, chain_iters)
    X, Y = warmstart.stack_rows(train_iv)
    del train_iv
    net = warmstart.WarmStartNet(max_rows=16384)
    secs = net.train(X, Y, epochs=30, batch=512, lr=2e-3, lr_final=2e-4)
    zero = float(np.mean(Y.astype(np.float64) ** 2))
    print(f"gain: {X.shape[0]} rows, {secs:.1f} s, loss {net.history[0]:.3e} -> "
          f"{net.history[-1]:.3e} (predicting zero: {zero:.3e})", flush=True)
    assert net.history[-1] < 0.2 * zero
    te = warmstart.solve_episode(cfg, 9, 4, prec, chain_iters, count=2)
    d = synth_mod.episode_interval(cfg, 9, 2, 4)
    vis, coh, flags = cal.device_inputs(d, prec)
    ctx = cal.Calib(d, vis, coh, flags, precision=prec, options=0)
    ctx.set_state(te[1].J, te[1].Y, te[1].Z, te[1].BZ)
    c_plain = ctx.get(cal.FIELD_COST).cpu().numpy()
    tr_plain = ctx.solve(n_ref)
    ctx.set_state(te[1].J, te[1].Y, te[1].Z, te[1].BZ)
    feats = ctx.warmstart_features(te[0].J, te[1].BZ)
    kept = ctx.warmstart_apply(net.predict(feats)).cpu().numpy()
    c_learned = ctx.get(cal.FIELD_COST).cpu().numpy()
    tr_learned = ctx.solve(n_ref)
    ctx.close()
    net.close()
    g_inf = float(np.median(tr_plain[n_ref // 2:, 0]))
    ip = warmstart.iters_to_target(tr_plain, g_inf)
    il = warmstart.iters_to_target(tr_learned, g_inf)
    ex_p, ex_l = c_plain.sum() / g_inf - 1, c_learned.sum() / g_inf - 1
    print(f"gain: kept {kept.sum()}/{cfg.P}; start excess cost over the target: plain {ex_p:.2e}, "
          f"learned {ex_l:.2e}; iterations to 1e-6 of the target: plain {ip}, learned {il}; "
          f"primal residual there: plain {tr_plain[ip - 1, 2]:.3e}, "
          f"learned {tr_learned[(il or n_ref) - 1, 2]:.3e}", flush=True)
    assert np.all(c_learned <= c_plain)           # the fallback guarantee, per subband
    assert ex_l < 0.3 * ex_p
    assert il is not None and il < ip
    assert tr_learned[il - 1, 2] <= 1.05 * tr_plain[ip - 1, 2]
