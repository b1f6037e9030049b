"""The large array at full size: N=128 stations (8128 baselines), K=10 directions, T=20 slots,
64 subbands x 8 channels, 6-term polynomial basis, one launch over all 64 subbands in each
precision, the benchmark's solver (matrix-free conjugate gradients in the one-launch local step,
here at cg_tol 1e-10 on both sides so that the step is the exact one to rounding).

Per precision, the first local step (Y = Z = 0, so subbands are independent) of two sampled
subbands is checked against the oracle's reading of the same iteration, and the fusion-centre
update of all 64 subbands (Q = 6 on the 115-185 MHz grid, cond(B^T B) ~ 1e9) against the oracle's
least-squares fit.  Bounds: FP64 against the oracle on the same inputs: the data cost at the GPU's
own Jones matrices within 1e-10 of the oracle's cost there (the statistics-based energy against the
per-sample sum); accept decisions equal where the step is not a rounding tie; per-LM-iteration
objectives and visibilities after the step within the larger of 1e-10 and 20 x the oracle's own
change when its visibilities are perturbed by 1e-15 relative, or, when a decision taken at a
rounding tie (a step that moves the objective by less than 1e-12 relative) went the other way,
within the size of such a step: ~sqrt(eps) relative in J near the optimum, so 1e-7 on the
visibilities and 1e-9 on the objectives that follow (first order in that change of J).  FP32
streaming against the oracle on the FP32-rounded inputs within 1e-5.  The error of
each precision against the FP64 oracle on the FP64 inputs is printed per result (data cost,
visibilities, Jones matrices, B_f Z).
"""
import threading

import numpy as np
import pytest

from conftest import subset
from parity_tol import FLIP_MARGIN, FP64_VIS_TOL, FP32_TOL, PERTURB

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAMPLE = [0, 63]


@pytest.fixture(scope="module")
def cal():
    from paper_1502_00858_amd import calib
    calib.load()
    return calib


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_c5_first_local_step_and_consensus(cal, oracle_mod, synth_mod):
    cfg = synth_mod.named_config("c5")
    print("c5: generating the full-size inputs", flush=True)
    d = synth_mod.generate(cfg)
    P, K, N = cfg.P, cfg.K, cfg.N
    J0 = synth_mod.identity_jones(P, K, N)
    gpu = {}
    for prec in (1, 0):
        print(f"c5: precision {prec}, first local step and consensus update of all {P} subbands",
              flush=True)
        vis, coh, flags = cal.device_inputs(d, prec)
        c = cal.Calib(d, vis, coh, flags, precision=prec, solver=3, cg_tol=1e-10, options=0)
        del vis, coh
        c.local_step(0)
        J = c.get(cal.FIELD_J).cpu().numpy()
        lm = c.get(cal.FIELD_LM_TRACE).cpu().numpy()
        cost = c.get(cal.FIELD_COST).cpu().numpy()
        c.consensus_update(0)
        bz = c.get(cal.FIELD_BZ).cpu().numpy()
        z = c.get(cal.FIELD_Z).cpu().numpy()
        c.close()
        torch.cuda.empty_cache()
        gpu[prec] = dict(J=J, lm=lm, cost=cost, bz=bz, z=z)

    print(f"c5: oracle first local step of subbands {SAMPLE} on the FP64 and the FP32-rounded "
          f"inputs", flush=True)
    sub64 = subset(d, SAMPLE)
    sub32 = synth_mod.as_fp32_inputs(sub64)
    Js = J0[SAMPLE]
    zs = np.zeros_like(Js)
    res = {}

    def run(name, data):
        pb = oracle_mod.Problem(data, solver=oracle_mod.SOLVE_PCG, cg_tol=1e-10)
        Jo, tro = pb.local_step(Js, zs, zs, trace=True)
        res[name] = (pb, Jo, tro[:, 0])
    rng = np.random.default_rng(1000)
    subp = dict(sub64, vis=sub64["vis"] * (1.0 + PERTURB * rng.standard_normal(sub64["vis"].shape)))
    threads = [threading.Thread(target=run, args=a)
               for a in (("64", sub64), ("32", sub32), ("64p", subp))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    pb64, Jo64, tro64 = res["64"]
    pb32, Jo32, tro32 = res["32"]
    _, Jop, trop = res["64p"]
    vis_o64 = pb64.predict(Jo64)
    sens_f = _rel(trop[..., 0], tro64[..., 0])
    sens_v = _rel(pb64.predict(Jop), vis_o64)
    tol_f = max(FP64_VIS_TOL, FLIP_MARGIN * sens_f)
    tol_v = max(FP64_VIS_TOL, FLIP_MARGIN * sens_v)
    print(f"  oracle sensitivity to a {PERTURB:g} perturbation: LM objectives {sens_f:.2e}, "
          f"visibilities {sens_v:.2e}; bounds {tol_f:.2e}, {tol_v:.2e}", flush=True)

    # FP64 path against the oracle on the same inputs
    g = gpu[0]
    trg = g["lm"][SAMPLE]
    prev = np.concatenate([np.full(tro64.shape[:-2] + (1,), np.inf), tro64[..., :-1, 0]], axis=-1)
    decisive = np.abs(tro64[..., 0] - prev) > 1e-12 * np.abs(tro64[..., 0])
    np.testing.assert_array_equal(trg[..., 2][decisive], tro64[..., 2][decisive])
    e_f = _rel(trg[..., 0], tro64[..., 0])
    same = np.array_equal(trg[..., 2], tro64[..., 2])
    e_vis64 = _rel(pb64.predict(g["J"][SAMPLE]), vis_o64)
    print(f"  FP64 GPU: LM objectives {e_f:.2e}, visibilities {e_vis64:.2e} (accept sequences "
          f"equal: {same}), "
          f"J {_rel(g['J'][SAMPLE], Jo64):.2e}, cost {_rel(g['cost'][SAMPLE], pb64.subband_cost(Jo64)):.2e}",
          flush=True)
    # the GPU's data cost against the oracle's at the GPU's own Jones matrices (bookkeeping of the
    # statistics-based energy, independent of where the two trajectories went)
    e_cost_own = _rel(g["cost"][SAMPLE], pb64.subband_cost(g["J"][SAMPLE]))
    bad = np.argwhere(np.abs(trg[..., 0] - tro64[..., 0]) > 1e-10 * np.abs(tro64[..., 0]))
    first = tuple(bad[0]) if len(bad) else None
    print(f"  FP64 GPU cost at its own J vs the oracle's cost there: {e_cost_own:.2e}; first LM "
          f"trace entry off by > 1e-10 (subband, direction, iteration): {first}", flush=True)
    if first is not None:
        fs, fk, fi = first
        print(f"    GPU {trg[fs, fk, :, 0]}\n    oracle {tro64[fs, fk, :, 0]}\n    GPU accept "
              f"{trg[fs, fk, :, 2]}\n    oracle accept {tro64[fs, fk, :, 2]}", flush=True)
    assert e_cost_own < FP64_VIS_TOL
    if not same:
        tol_f, tol_v = max(tol_f, 1e-9), max(tol_v, 1e-7)
    assert e_f < tol_f and e_vis64 < tol_v

    # FP32 streaming against the oracle on the FP32-rounded inputs (the parity bar), and against
    # the oracle on the FP64 inputs (the error the FP32 path carries, printed)
    g32 = gpu[1]
    np.testing.assert_allclose(g32["cost"][SAMPLE], pb32.subband_cost(Jo32), rtol=FP32_TOL)
    np.testing.assert_allclose(g32["lm"][SAMPLE][..., 0], tro32[..., 0], rtol=FP32_TOL)
    e_vis32 = _rel(pb32.predict(g32["J"][SAMPLE]), pb32.predict(Jo32))
    e_j32 = _rel(g32["J"][SAMPLE], Jo32)
    print(f"  FP32 GPU vs oracle on FP32-rounded inputs: visibilities {e_vis32:.2e}, J {e_j32:.2e}",
          flush=True)
    assert e_vis32 < FP32_TOL and e_j32 < FP32_TOL
    print(f"  FP32 GPU vs oracle on FP64 inputs: visibilities "
          f"{_rel(pb64.predict(g32['J'][SAMPLE]), vis_o64):.2e}, J {_rel(g32['J'][SAMPLE], Jo64):.2e}, "
          f"cost {_rel(g32['cost'][SAMPLE], pb64.subband_cost(Jo64)):.2e}; FP32 vs FP64 GPU: "
          f"J {_rel(g32['J'], g['J']):.2e}, cost {_rel(g32['cost'], g['cost']):.2e}", flush=True)

    # fusion centre at Q = 6 over the 64 subbands, from each precision's own local step
    print("c5: oracle consensus fit of the GPU's Jones matrices", flush=True)
    pbf = oracle_mod.Problem(d)
    zero_y = np.zeros_like(J0)
    zero_z = np.zeros((K, cfg.Q, N, 2, 2), np.complex128)
    for prec in (0, 1):
        _, Zo, BZo, _, _ = pbf.consensus(gpu[prec]["J"], zero_y, zero_z)
        e_bz, e_z = _rel(gpu[prec]["bz"], BZo), _rel(gpu[prec]["z"], Zo)
        print(f"  precision {prec}: B_f Z {e_bz:.2e}, Z {e_z:.2e}", flush=True)
        assert e_bz < 1e-10
        # Z itself carries cond(B^T B) ~ 1e9 times the rounding of the fit
        assert e_z < 1e-5
    print(f"  FP32 vs FP64 GPU: B_f Z {_rel(gpu[1]['bz'], gpu[0]['bz']):.2e}", flush=True)
