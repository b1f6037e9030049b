import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def synth_mod():
    from paper_1502_00858_amd import synth
    return synth


def tiny_cfg(synth, **kw):
    base = dict(name="tiny", N=5, P=4, Q=2, K=2, T=3, n_chan=2, rho=5.0, lm_iters=8,
                admm_iters=5, config_index=7)
    base.update(kw)
    return synth.SynthConfig(**base)


def rand_jones(rng, P, K, N, scale=0.2):
    J = np.zeros((P, K, N, 2, 2), np.complex128)
    J[..., 0, 0] = 1
    J[..., 1, 1] = 1
    return J + scale * (rng.normal(size=J.shape) + 1j * rng.normal(size=J.shape))


def subset(data, fs):
    """The generator's arrays restricted to subbands fs (plain slicing of the inputs), for oracle
    checks of per-subband quantities at full problem sizes."""
    fs = [int(f) for f in fs]
    B = int(data["B"])
    vo, co = data["vis_off"], data["coh_off"]
    out = dict(data)
    out["P"] = len(fs)
    for key in ("n_chan", "n_dirs", "freq", "noise_power"):
        out[key] = np.asarray(data[key])[fs]
    out["vis"] = np.concatenate([data["vis"][vo[f]:vo[f + 1]] for f in fs])
    out["coh"] = np.concatenate([data["coh"][co[f]:co[f + 1]] for f in fs])
    out["flags"] = np.concatenate([data["flags"][f * B:(f + 1) * B] for f in fs])
    out["jones_true"] = data["jones_true"][fs]
    spb = int(data["T"]) * out["n_chan"]
    out["vis_off"] = np.concatenate([[0], np.cumsum(B * spb)]).astype(np.int64)
    out["coh_off"] = np.concatenate([[0], np.cumsum(out["n_dirs"] * B * spb)]).astype(np.int64)
    return out
