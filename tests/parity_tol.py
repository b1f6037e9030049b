"""Tolerances of the GPU-against-oracle parity tests and where they come from.

FP64_VIS_TOL is the required agreement of FP64 results with the oracle (relative, on predicted
visibilities and costs).  A single local step from identical state meets it with room to spare:
the oracle's own visibilities move by ~1e-15 when its inputs are perturbed by 1e-15 relative
(recorded by tests/test_oracle_sensitivity.py), so nothing in the step amplifies rounding.

Over a multi-iteration C-ADMM trajectory an LM accept decision can be taken at a gain ratio of
rounding size.  Two FP64 codes that sum in different orders can then take different decisions,
and the trajectories separate by the effect of one LM step, whatever the size of the rounding
that flipped it.  traj_vis_tol() measures that effect for a given case: it reruns the oracle on
inputs perturbed by 1e-15 relative and returns the larger of FP64_VIS_TOL and
FLIP_MARGIN x the largest change it sees in the predicted visibilities.
"""
import numpy as np

FP64_VIS_TOL = 1e-10     # FP64 path, relative, predicted visibilities and per-iteration cost
FP32_TOL = 1e-5          # FP32-streaming path against the oracle on FP32-rounded inputs
FLIP_MARGIN = 20.0       # trajectories: factor over the oracle's own flip-induced change
PERTURB = 1e-15


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_sensitivity(oracle_mod, d, run, seeds=(0, 1, 2)):
    """Largest relative change of the predicted visibilities of run(problem) (a function returning
    J) when d's visibilities are perturbed by PERTURB relative, over a few perturbation seeds."""
    pa = oracle_mod.Problem(d, **run.problem_kw)
    ref = pa.predict(run(pa))
    worst = 0.0
    for s in seeds:
        rng = np.random.default_rng(1000 + s)
        d2 = dict(d, vis=d["vis"] * (1.0 + PERTURB * rng.standard_normal(d["vis"].shape)))
        pb = oracle_mod.Problem(d2, **run.problem_kw)
        worst = max(worst, rel(pa.predict(run(pb)), ref))
    return worst


def traj_vis_tol(oracle_mod, d, run):
    return max(FP64_VIS_TOL, FLIP_MARGIN * oracle_sensitivity(oracle_mod, d, run))


class AdmmRun:
    """run(problem) = J after `iters` C-ADMM iterations from identity (problem options as given)."""

    def __init__(self, P, K, N, iters, **problem_kw):
        self.shape = (P, K, N)
        self.iters = iters
        self.problem_kw = problem_kw

    def __call__(self, pb):
        P, K, N = self.shape
        J0 = np.zeros((P, K, N, 2, 2), np.complex128)
        J0[..., 0, 0] = 1
        J0[..., 1, 1] = 1
        return pb.admm_solve(J0, self.iters)["J"]


class LocalStepRun:
    """run(problem) = J after one local step from identity with Y = B Z = 0."""

    def __init__(self, P, K, N, **problem_kw):
        self.shape = (P, K, N)
        self.problem_kw = problem_kw

    def __call__(self, pb):
        P, K, N = self.shape
        J0 = np.zeros((P, K, N, 2, 2), np.complex128)
        J0[..., 0, 0] = 1
        J0[..., 1, 1] = 1
        z = np.zeros_like(J0)
        return pb.local_step(J0, z, z)
