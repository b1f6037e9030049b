"""FP64 reference of the warm-start features, training targets and cost fallback (test
infrastructure only).

The paper starts a new solution interval's C-ADMM iteration from the previous interval's
solution (Section 3).  The learned warm start corrects that start per station; its inputs are
plain functions of the previous solution and the new data, written out here from their
definitions:

* the data gradient G_p of direction k at J (the Euclidean gradient of the least-squares cost of
  Section 2 with the other directions held, the SAGE expectation of Section 3), taken from the
  oracle's ``dir_objective`` with rho = 0 and Y = 0;
* the Gauss-Newton block of station p: the data cost changes to second order by
  tr(dJ_p Q_p dJ_p^H) with Q_p = sum over unflagged baselines (p, q) of S_pq J_q^H J_q and
  S_pq = sum over samples of |c|^2 (the coherency is c I2, Section 2), so the minimiser of the
  quadratic model in dJ_p alone is -1/2 G_p Q_p^-1;
* the gauge: solutions are unique up to a common right unitary factor per (subband, direction);
  the target aligns the new solution to the previous one with the unitary polar factor of
  sum_p J_new,p^H J_prev,p (orthogonal Procrustes), here computed by an SVD.
"""
from __future__ import annotations

import numpy as np

from . import Problem as _Problem

SCALE = 10.0
N_FEATURES = 32
N_OUTPUTS = 8


def _flat(M):
    """[..., 2, 2] complex -> [..., 8] real (row-major, re/im interleaved)."""
    M = np.asarray(M, np.complex128)
    out = np.empty(M.shape[:-2] + (8,))
    out[..., 0::2] = M.real.reshape(M.shape[:-2] + (4,))
    out[..., 1::2] = M.imag.reshape(M.shape[:-2] + (4,))
    return out


def gn_blocks(data, J, f, k):
    """Q_p [N, 2, 2] of direction k of subband f at J (definition above)."""
    N, B, T = int(data["N"]), int(data["B"]), int(data["T"])
    spb = T * int(data["n_chan"][f])
    flags = np.asarray(data["flags"]).reshape(-1, B)[f]
    c0 = int(data["coh_off"][f]) + k * B * spb
    coh = np.asarray(data["coh"])[c0:c0 + B * spb].reshape(B, spb)
    S = np.sum(np.abs(coh) ** 2, axis=1)
    Q = np.zeros((N, 2, 2), np.complex128)
    b = 0
    for p in range(N):
        for q in range(p + 1, N):
            if not flags[b]:
                Jp, Jq = J[f, k, p], J[f, k, q]
                Q[p] += S[b] * (Jq.conj().T @ Jq)
                Q[q] += S[b] * (Jp.conj().T @ Jp)
            b += 1
    return Q


def features(data, J, J2=None, BZp=None):
    """Features [P*K*N, 32] of the new interval's data at J (the previous solution)."""
    P, K, N = int(data["P"]), int(data["K"]), int(data["N"])
    prob = _Problem(data, rho=np.zeros(K))
    J = np.asarray(J, np.complex128)
    zeros = np.zeros_like(J)
    out = np.zeros((P, K, N, N_FEATURES))
    for f in range(P):
        for k in range(int(data["n_dirs"][f])):
            _, G = prob.dir_objective(J, zeros, zeros, f, k)
            Q = gn_blocks(data, J, f, k)
            step = np.zeros((N, 2, 2), np.complex128)
            for p in range(N):
                det = (Q[p, 0, 0] * Q[p, 1, 1] - Q[p, 0, 1] * Q[p, 1, 0]).real
                if det > 0.0:
                    step[p] = -0.5 * G[p] @ np.linalg.inv(Q[p])
            out[f, k, :, 0:8] = _flat(J[f, k])
            if J2 is not None:
                out[f, k, :, 8:16] = SCALE * _flat(J[f, k] - J2[f, k])
            out[f, k, :, 16:24] = SCALE * _flat(step)
            if BZp is not None:
                out[f, k, :, 24:32] = SCALE * _flat(BZp[f, k] - J[f, k])
    return out.reshape(P * K * N, N_FEATURES)


def procrustes(A):
    """Unitary U maximising Re tr(U^H A) (the polar factor of A), by the SVD."""
    W, _, Vh = np.linalg.svd(A)
    return W @ Vh


def target(data, Jnew, Jprev):
    """Training target [P*K*N, 8]: SCALE (Jnew_p U - Jprev_p), U the polar factor of
    sum_p Jnew_p^H Jprev_p."""
    P, K, N = int(data["P"]), int(data["K"]), int(data["N"])
    out = np.zeros((P, K, N, N_OUTPUTS))
    for f in range(P):
        for k in range(int(data["n_dirs"][f])):
            A = sum(Jnew[f, k, p].conj().T @ Jprev[f, k, p] for p in range(N))
            U = procrustes(A)
            out[f, k] = SCALE * _flat(Jnew[f, k] @ U - Jprev[f, k])
    return out.reshape(P * K * N, N_OUTPUTS)


def unflat(x, shape):
    """[..., 8] real rows -> complex [..., 2, 2] of the given leading shape."""
    x = np.asarray(x, np.float64).reshape(shape + (8,))
    return (x[..., 0::2] + 1j * x[..., 1::2]).reshape(shape + (2, 2))


def apply(data, J, delta):
    """J + delta/SCALE per subband where that does not raise the data cost (Section 2), else J.
    Returns the new J and the per-subband keep flags."""
    P, K, N = int(data["P"]), int(data["K"]), int(data["N"])
    prob = _Problem(data)
    d = unflat(np.asarray(delta, np.float64) / SCALE, (P, K, N))
    for f in range(P):
        d[f, int(data["n_dirs"][f]):] = 0.0
    Jl = J + d
    c0, c1 = prob.subband_cost(J), prob.subband_cost(Jl)
    keep = np.isfinite(c1) & (c1 <= c0)
    out = np.where(keep[:, None, None, None, None], Jl, J)
    return out, keep, c0, c1
