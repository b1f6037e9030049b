"""Seeded synthetic observations for multi-frequency direction-dependent calibration.

This module only *simulates data*: station layouts, uvw tracks, a point-source sky, true Jones
matrices that vary smoothly with frequency, and noisy visibilities drawn from the measurement
equation of Section 2 (the visibility model and the scalar-times-identity coherency of an
unpolarised point source).  It contains none of the calibration arithmetic (no residuals against
a solution, no gradients, no least squares, no consensus); both the CPU oracle and the GPU
library consume its arrays as plain inputs.

The recipe follows the simulation set-up of Section 4 where the paper fixes it (115-185 MHz band,
0.2 MHz channels, pointing at the north celestial pole, spectral indices uniform in (-1, 1),
complex Gaussian noise with equal real/imaginary variance, polynomial frequency variation of the
Jones terms with reference frequency 150 MHz) and substitutes seeded stand-ins where the paper's
inputs are not available (station layout: uniform in a 2 km-diameter disk instead of the LOFAR
layout; sky: K point sources within +-0.05 rad instead of the NCP sky model).

Array layouts (all complex arrays are numpy complex128 unless ``dtype`` asks for complex64):

* ``vis``  [sum_f B*T*n_chan[f], 2, 2]; per subband, sample s = (b*T + t)*n_chan[f] + ch,
  baseline b enumerates pairs p<q in row-major order.
* ``coh``  [sum_f K_f*B*T*n_chan[f]]; per subband, index (k*B + b)*T*n_chan[f] + (t*n_chan[f]+ch).
  One complex scalar per sample and direction: the coherency matrix is that scalar times I2.
* ``flags`` [P*B] uint8, 1 = the whole baseline is flagged in that subband.
* ``jones_true`` [P, K, N, 2, 2]; rows of directions k >= K_f are zero.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

C_LIGHT = 299_792_458.0
F0_HZ = 150e6
CHAN_WIDTH_HZ = 0.2e6
BAND_HZ = (115e6, 185e6)
LATITUDE_RAD = np.deg2rad(52.9)
SEED_BASE = 150200858
INTERVAL_SLOT_RAD = 2 * np.pi / 1440   # hour angle of one time slot of an episode (1 minute)


@dataclasses.dataclass
class SynthConfig:
    name: str
    N: int                      # stations
    P: int                      # subbands (one compute agent each in the paper)
    Q: int                      # polynomial terms of the frequency basis
    K: int                      # maximum number of directions
    T: int                      # time slots per solution interval
    n_chan: Sequence[int] | int = 1          # channels per subband (int = all equal)
    n_dirs: Optional[Sequence[int]] = None   # K_f per subband (None = K everywhere)
    flag_frac_max: float = 0.0               # per-subband flagged-baseline fraction ~ U(0, max)
    rho: float = 5.0
    admm_iters: int = 20
    lm_iters: int = 10
    snr: Optional[float] = 20.0              # signal/noise power per subband; None = noise free
    jones_sigma: float = 0.1
    jones_degree: int = 3                    # highest power of x in the true Jones polynomial
    disk_radius_m: float = 1000.0
    lm_box: float = 0.05                     # |l|,|m| bound of the sources (rad)
    flux_range: tuple = (1.0, 20.0)
    config_index: int = 0
    # each subband's noise from its own stream seeded by (seed[, interval], subband), so that the
    # subbands can be simulated in parallel threads (the large array); False: one stream for all
    noise_per_subband: bool = False

    @property
    def B(self) -> int:
        return self.N * (self.N - 1) // 2


def named_config(name: str) -> SynthConfig:
    """The workloads the library is exercised on (sizes of the benchmark configurations)."""
    if name == "c1":   # plain ADMM, FP64
        return SynthConfig("c1", N=16, P=8, Q=3, K=2, T=10, n_chan=1, rho=5.0,
                           admm_iters=20, lm_iters=10, config_index=1)
    if name == "c2":   # FP32 streaming with FP64 solve / cost / Z
        return SynthConfig("c2", N=62, P=32, Q=4, K=5, T=10, n_chan=4, rho=5.0,
                           admm_iters=30, lm_iters=10, config_index=2)
    if name == "c3":   # batched uneven subbands
        return SynthConfig("c3", N=62, P=256, Q=4, K=10, T=10, n_chan=-1, n_dirs=None,
                           flag_frac_max=0.3, rho=5.0, admm_iters=30, lm_iters=10,
                           config_index=3, noise_per_subband=True)
    if name == "c5":   # large array
        return SynthConfig("c5", N=128, P=64, Q=6, K=10, T=20, n_chan=8, rho=5.0,
                           admm_iters=30, lm_iters=10, config_index=5, noise_per_subband=True)
    raise KeyError(name)


def baseline_pairs(N: int):
    p, q = np.triu_indices(N, k=1)
    return p.astype(np.int32), q.astype(np.int32)


def _stations(rng, N, radius):
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, N))
    a = rng.uniform(0.0, 2 * np.pi, N)
    east, north = r * np.cos(a), r * np.sin(a)
    return np.stack([east, north, np.zeros(N)], axis=1)


def _uvw(enu_b, hour_angles):
    """uvw (metres) of ENU baseline vectors for a phase centre at the north celestial pole."""
    e, n, u = enu_b[:, 0], enu_b[:, 1], enu_b[:, 2]
    sl, cl = np.sin(LATITUDE_RAD), np.cos(LATITUDE_RAD)
    X = -sl * n + cl * u
    Y = e
    Z = cl * n + sl * u
    H = hour_angles[None, :]
    # declination +90 deg: sin(dec)=1, cos(dec)=0
    uu = np.sin(H) * X[:, None] + np.cos(H) * Y[:, None]
    vv = -np.cos(H) * X[:, None] + np.sin(H) * Y[:, None]
    ww = np.broadcast_to(Z[:, None], uu.shape)
    return uu, vv, ww


def generate(cfg: SynthConfig, seed: Optional[int] = None, episode: int = 0,
             dtype=np.complex128, truth_in_span: bool = False,
             jones_time_factor: Optional[np.ndarray] = None,
             interval: Optional[int] = None) -> dict:
    """Draw one seeded solution interval.

    ``truth_in_span``: true Jones = I + polynomial of degree Q-1 in x=(f-f0)/f0, so that it lies
    exactly in the span of the calibration basis (used for fixed-point checks).
    ``jones_time_factor``: optional complex [N, K] multiplier of the perturbation (solution
    intervals that drift in time).
    ``interval``: index of the solution interval within a longer observation.  Everything drawn
    from ``seed`` (stations, sky, Jones polynomial, flags) stays fixed; the T time slots become
    consecutive slots of INTERVAL_SLOT_RAD hour angle starting at interval*T, and the noise is
    drawn from a generator seeded by (seed, interval).
    """
    if seed is None:
        seed = SEED_BASE + 1000 * cfg.config_index + episode
    rng = np.random.default_rng(seed)
    N, P, K, T = cfg.N, cfg.P, cfg.K, cfg.T
    B = cfg.B
    p_idx, q_idx = baseline_pairs(N)

    if isinstance(cfg.n_chan, int) and cfg.n_chan > 0:
        n_chan = np.full(P, cfg.n_chan, np.int32)
    elif isinstance(cfg.n_chan, int):
        n_chan = rng.integers(1, 17, P).astype(np.int32)
    else:
        n_chan = np.asarray(cfg.n_chan, np.int32)
    if cfg.n_dirs is not None:
        n_dirs = np.asarray(cfg.n_dirs, np.int32)
    elif cfg.name == "c3":
        n_dirs = rng.integers(3, 11, P).astype(np.int32)
    else:
        n_dirs = np.full(P, K, np.int32)
    freq = np.linspace(BAND_HZ[0], BAND_HZ[1], P) if P > 1 else np.array([F0_HZ])
    x = (freq - F0_HZ) / F0_HZ

    st = _stations(rng, N, cfg.disk_radius_m)
    enu_b = st[q_idx] - st[p_idx]
    hour = np.sort(rng.uniform(-np.pi / 3, np.pi / 3, T))   # +-4 h
    if interval is not None:
        hour = -np.pi / 3 + (interval * T + np.arange(T)) * INTERVAL_SLOT_RAD
    uu, vv, ww = _uvw(enu_b, hour)                            # [B, T]

    l = rng.uniform(-cfg.lm_box, cfg.lm_box, K)
    m = rng.uniform(-cfg.lm_box, cfg.lm_box, K)
    flux = rng.uniform(cfg.flux_range[0], cfg.flux_range[1], K)
    alpha = rng.uniform(-1.0, 1.0, K)
    order = np.argsort(-flux)
    l, m, flux, alpha = l[order], m[order], flux[order], alpha[order]
    nn = np.sqrt(1.0 - l * l - m * m)

    deg = (cfg.Q - 1) if truth_in_span else cfg.jones_degree
    A = (rng.normal(0, cfg.jones_sigma, (deg + 1, K, N, 2, 2))
         + 1j * rng.normal(0, cfg.jones_sigma, (deg + 1, K, N, 2, 2)))
    if jones_time_factor is not None:
        A = A * np.asarray(jones_time_factor).T[None, :, :, None, None]
    jones_true = np.zeros((P, K, N, 2, 2), np.complex128)
    for f in range(P):
        pert = sum(A[d] * x[f] ** d for d in range(deg + 1))
        jones_true[f] = np.eye(2)[None, None] + pert
        jones_true[f, n_dirs[f]:] = 0.0

    flags = np.zeros((P, B), np.uint8)
    if cfg.flag_frac_max > 0:
        for f in range(P):
            frac = rng.uniform(0.0, cfg.flag_frac_max)
            nf = int(round(frac * B))
            if nf:
                flags[f, rng.choice(B, nf, replace=False)] = 1

    spb = T * n_chan                                   # samples per baseline
    vis_off = np.concatenate([[0], np.cumsum(B * spb)]).astype(np.int64)
    coh_off = np.concatenate([[0], np.cumsum(n_dirs * B * spb)]).astype(np.int64)
    vis = np.empty((int(vis_off[-1]), 2, 2), dtype)
    coh = np.empty(int(coh_off[-1]), dtype)
    noise_power = np.zeros(P)
    nrng = rng if interval is None else np.random.default_rng([seed, interval])

    def subband(f, frng):
        nch = int(n_chan[f])
        Kf = int(n_dirs[f])
        fch = freq[f] + (np.arange(nch) - (nch - 1) / 2.0) * CHAN_WIDTH_HZ   # [nch]
        # coherency scalars c[k, b, t, ch]
        phase_geo = (uu[None, :, :] * l[:Kf, None, None] + vv[None, :, :] * m[:Kf, None, None]
                     + ww[None, :, :] * (nn[:Kf, None, None] - 1.0))            # [K,B,T] metres
        ph = -2.0 * np.pi * phase_geo[..., None] * (fch / C_LIGHT)[None, None, None, :]
        amp = flux[:Kf, None] * (fch[None, :] / F0_HZ) ** alpha[:Kf, None]     # [K,nch]
        c = amp[:, None, None, :] * np.exp(1j * ph)                             # [K,B,T,nch]
        c[:, flags[f] == 1] = 0.0
        Jp = jones_true[f, :Kf][:, p_idx]                                        # [K,B,2,2]
        Jq = jones_true[f, :Kf][:, q_idx]
        Mb = Jp @ np.conj(np.swapaxes(Jq, -1, -2))                               # [K,B,2,2]
        sig = np.einsum("kbtc,kbij->btcij", c, Mb, optimize=True)                # [B,T,nch,2,2]
        if cfg.snr is not None:
            live = flags[f] == 0
            spow = np.mean(np.abs(sig[live]) ** 2) if live.any() else 0.0
            npow = spow / cfg.snr                    # per complex entry
            noise = (frng.normal(0, np.sqrt(npow / 2), sig.shape)
                     + 1j * frng.normal(0, np.sqrt(npow / 2), sig.shape))
            noise[flags[f] == 1] = 0.0
            sig = sig + noise
            noise_power[f] = npow
        vis[vis_off[f]:vis_off[f + 1]] = sig.reshape(-1, 2, 2)
        coh[coh_off[f]:coh_off[f + 1]] = c.reshape(-1)

    if cfg.noise_per_subband:
        import concurrent.futures
        import os
        key = [seed] if interval is None else [seed, interval]
        with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(lambda f: subband(f, np.random.default_rng(key + [1000003, f])), range(P)))
    else:
        for f in range(P):
            subband(f, nrng)

    return dict(
        name=cfg.name, N=N, P=P, Q=cfg.Q, K=K, T=T, B=B,
        n_chan=n_chan, n_dirs=n_dirs, freq=freq, f0=F0_HZ,
        rho=np.full(K, cfg.rho), admm_iters=cfg.admm_iters, lm_iters=cfg.lm_iters,
        vis=vis, coh=coh, flags=flags.reshape(-1), jones_true=jones_true,
        vis_off=vis_off, coh_off=coh_off, noise_power=noise_power,
        sources=dict(l=l, m=m, flux=flux, alpha=alpha), seed=seed,
    )


def time_factor(cfg: SynthConfig, episode: int, interval: int, n_intervals: int) -> np.ndarray:
    """Complex [N, K] drift of the Jones perturbation over the solution intervals of an episode:
    sin(a1 tau + 2 pi b1) + j sin(a2 tau + 2 pi b2) with a, b ~ U(0, 1) per station and direction
    (the time variation of the simulated gains in Section 4), tau = pi * interval / n_intervals so
    that an episode covers about half a period."""
    rng = np.random.default_rng([SEED_BASE, 7, cfg.config_index, episode])
    a1, b1, a2, b2 = rng.uniform(0.0, 1.0, (4, cfg.N, cfg.K))
    tau = np.pi * interval / max(n_intervals, 1)
    return np.sin(a1 * tau + 2 * np.pi * b1) + 1j * np.sin(a2 * tau + 2 * np.pi * b2)


def episode_interval(cfg: SynthConfig, episode: int, interval: int, n_intervals: int,
                     dtype=np.complex128) -> dict:
    """Solution interval ``interval`` of episode ``episode``: one sky, array and Jones polynomial
    per episode, perturbation scaled by the episode's time factor, consecutive time slots."""
    seed = SEED_BASE + 1000 * cfg.config_index + 100 * (episode + 1)
    return generate(cfg, seed=seed, dtype=dtype,
                    jones_time_factor=time_factor(cfg, episode, interval, n_intervals),
                    interval=interval)


def mlp_init_params(dims: Sequence[int], seed: int = SEED_BASE) -> np.ndarray:
    """Seeded initial parameters of a fully connected network, float32, packed per layer as
    W [dims[l]][dims[l+1]] then b [dims[l+1]]: W ~ N(0, 1/dims[l]), b = 0."""
    rng = np.random.default_rng([seed, 11])
    parts = []
    for i in range(len(dims) - 1):
        parts.append(rng.normal(0.0, 1.0 / np.sqrt(dims[i]), dims[i] * dims[i + 1]))
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def identity_jones(P: int, K: int, N: int) -> np.ndarray:
    """Initial Jones: identity blocks for every subband, direction and station."""
    J = np.zeros((P, K, N, 2, 2), np.complex128)
    J[..., 0, 0] = 1.0
    J[..., 1, 1] = 1.0
    return J


def as_fp32_inputs(data: dict) -> dict:
    """Round the streamed inputs to single precision and widen them back (same values an FP32
    pipeline sees), so that an FP64 computation on the result is comparable to an FP32 one."""
    out = dict(data)
    out["vis"] = data["vis"].astype(np.complex64).astype(np.complex128)
    out["coh"] = data["coh"].astype(np.complex64).astype(np.complex128)
    return out
