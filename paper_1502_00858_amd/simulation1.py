"""Simulation I of Section 4 on the GPU: one direction, distributed against normal calibration.

    python -m paper_1502_00858_amd.simulation1 [--iters 50] [--json OUT]

Set-up of Section 4 (Simulation I) with this package's synthetic stand-ins: N = 47 stations,
P = 32 single-channel subbands over 115-185 MHz, T = 20 time slots, K = 1 direction, true Jones
matrices that vary with frequency as a cubic polynomial (G = 4 terms), complex Gaussian noise.
Distributed calibration: 50 C-ADMM iterations with 10 LM iterations per local step, for every
pair of smoothing-polynomial terms Q in {2, 5} (the paper's F) and penalty rho in {0.5, 5, 50}.
Normal calibration: each subband alone (rho = 0, no consensus), one run of 30 LM iterations.

Per run: the primal and dual residuals of every C-ADMM iteration (the library's trace; Section 4
defines both, normalised per parameter), and the error per parameter of the local solutions J_f
(and of the consensus values B_f Z) against the true Jones matrices after removing the unitary
ambiguity: min over unitary U of ||J_f - J^_f U|| / sqrt(4N),
U from the polar factor of J^_f^H J_f (the matrix Procrustes problem), per frequency and averaged
over the frequencies.  This is an evaluation of results, not part of the method.

The paper reports the trends, not values: primal residual lower (and falling faster) for larger
rho, dual residual lower for the smaller Q, distributed error below normal calibration.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

RHOS = (0.5, 5.0, 50.0)
QS = (2, 5)


def config(Q: int = 2):
    from . import synth
    return synth.SynthConfig("sim1", N=47, P=32, Q=Q, K=1, T=20, n_chan=1, rho=5.0,
                             admm_iters=50, lm_iters=10, config_index=6)


def procrustes_error(J_est: np.ndarray, J_true: np.ndarray) -> np.ndarray:
    """[P] error per parameter: ||J_f - J^_f U_f|| / sqrt(4 N) over the directions' stations, with
    U_f the unitary 2x2 matrix closest to J^_f^H J_f (polar factor through the SVD)."""
    P, K, N = J_true.shape[:3]
    err = np.zeros(P)
    for f in range(P):
        A = J_est[f].reshape(-1, 2)       # stacked rows of every direction and station
        Bm = J_true[f].reshape(-1, 2)
        u, _, vh = np.linalg.svd(A.conj().T @ Bm)
        U = u @ vh
        err[f] = np.linalg.norm(Bm - A @ U) / np.sqrt(4 * N * K)
    return err


def run(iters: int = 50, precision: int = 0, solver: int = 3, cg_tol: float = 1e-10,
        log=print) -> dict:
    import torch
    from . import calib, synth
    out = {"N": 47, "P": 32, "T": 20, "K": 1, "iters": iters, "runs": []}
    base = synth.generate(config())
    truth = base["jones_true"]
    for Q in QS:
        for rho in RHOS:
            d = dict(base, Q=Q, rho=np.full(1, rho))
            vis, coh, flags = calib.device_inputs(d, precision)
            c = calib.Calib(d, vis, coh, flags, precision=precision, lm_iters=10, solver=solver,
                            cg_tol=cg_tol)
            tr = c.solve(iters)
            J = c.get(calib.FIELD_J).cpu().numpy()
            BZ = c.get(calib.FIELD_BZ).cpu().numpy()
            c.close()
            e, ebz = procrustes_error(J, truth), procrustes_error(BZ, truth)
            out["runs"].append({"Q": Q, "rho": rho, "primal": tr[:, 2].tolist(),
                                "dual": tr[:, 3].tolist(), "cost": tr[:, 0].tolist(),
                                "error_per_freq": e.tolist(), "error": float(e.mean()),
                                "error_bz": float(ebz.mean())})
            log(f"Q={Q} rho={rho:5.1f}: primal {tr[-1, 2]:.3e}, dual {tr[-1, 3]:.3e}, "
                f"error {e.mean():.4e} (B_f Z {ebz.mean():.4e})")
    # normal calibration: no consensus term, 30 LM iterations per subband
    d = dict(base, Q=2, rho=np.zeros(1))
    vis, coh, flags = calib.device_inputs(d, precision)
    c = calib.Calib(d, vis, coh, flags, precision=precision, lm_iters=30, solver=solver,
                    cg_tol=cg_tol, options=0)
    c.local_step(0)
    J = c.get(calib.FIELD_J).cpu().numpy()
    c.close()
    torch.cuda.synchronize()
    e = procrustes_error(J, truth)
    out["normal"] = {"error_per_freq": e.tolist(), "error": float(e.mean())}
    log(f"normal calibration: error {e.mean():.4e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    res = run(args.iters)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main()
