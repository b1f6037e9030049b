// Per-subband pieces of the Levenberg-Marquardt local step (minimisation M1 of Section 3), shared
// by the kernels that run one piece per launch over all subbands (lm_kernels.hip,
// stream_kernels.hip) and the fused local-step kernel that runs a subband's whole local step in
// one workgroup (pcg_kernel.hip), so that both run the same arithmetic in the same order.
//
// The objective of direction k is the augmented Lagrangian
//   L(J) = sum_b sum_s ||V_k - c_s J_p J_q^H||^2 + Re tr(Y^H (J - BZ)) + rho/2 ||J - BZ||^2
// (linear term in the trace form of Appendix A).  The residual enters only through per-baseline
// sums (the coherency is a scalar times I2 and J is constant over a baseline's samples): D_b =
// sum_s conj(c_s) r_s per direction and the residual's energy, kept per streaming tile.
#pragma once

#include "calib_internal.h"
#include "wave_reduce.h"

namespace calib {
namespace lmd {

// m = a b^H for 2x2 complex matrices stored as 8 doubles (row-major, re/im interleaved)
__device__ inline void jjh(const double *__restrict__ a, const double *__restrict__ b, double *m) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double ar = a[(i * 2 + t) * 2], ai = a[(i * 2 + t) * 2 + 1];
        const double br = b[(j * 2 + t) * 2], bi = b[(j * 2 + t) * 2 + 1];
        re += ar * br + ai * bi;
        im += ai * br - ar * bi;
      }
      m[(i * 2 + j) * 2] = re;
      m[(i * 2 + j) * 2 + 1] = im;
    }
}

// d -= x m for the complex scalar x (re, im) and the 2x2 complex matrix m (8 reals)
__device__ inline void sub_scaled(double *d, double xr, double xi, const double *m) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    d[2 * e] -= xr * m[2 * e] - xi * m[2 * e + 1];
    d[2 * e + 1] -= xr * m[2 * e + 1] + xi * m[2 * e];
  }
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce NV values per thread over the workgroup in a fixed order; result in v[] of every
// thread (broadcast through LDS).
template <int NV, int NT = kBlock>
__device__ inline void block_sum_vec(double *v, double (*red)[NT / 64]) {
  const int w = threadIdx.x >> 6;
  wave_sum_vec<NV>(v);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i][w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int j = 0; j < NT / 64; ++j) s += red[i][j];
    v[i] = s;
  }
  __syncthreads();
}

__device__ inline const double *jdir(const Buffers &B, const Problem &pb, int f, int k) {
  return B.J + ((int64_t)f * pb.K + k) * pb.N * 8;
}

// data cost of subband f from its tiles' partials (fixed order) + consensus terms at Jx; the data
// cost alone in *data when given (whole workgroup of kBlock threads)
__device__ inline double objective(const Problem &pb, const Layout &L, const Buffers &B, int f,
                                   int k, int unreg, const double *Jx, double (*red)[kBlock / 64],
                                   double *data = nullptr) {
  double acc[1] = {0.0};
  for (int t = L.tile_off[f] + threadIdx.x; t < L.tile_off[f + 1]; t += kBlock) acc[0] += B.cost_part[t];
  double pen = 0.0;
  if (!unreg) {
    const double rho = B.rho[k];
    const int64_t o = ((int64_t)f * pb.K + k) * pb.N * 8;
    for (int e = threadIdx.x; e < 8 * pb.N; e += kBlock) {
      const double d = Jx[e] - B.BZ[o + e];
      pen += B.Y[o + e] * d + 0.5 * rho * d * d;
    }
  }
  double v[2] = {acc[0], pen};
  block_sum_vec<2>(v, red);
  if (data) *data = v[0];
  return v[0] + v[1];
}

// Largest diagonal entry of H_GN + rho I of direction k of subband f at J (whole workgroup of
// NT threads; result in every thread; J at a stride of js doubles per station):
// 2 sum_c S_pc (|J_c[0][j]|^2 + |J_c[1][j]|^2), from the column norms of the stations' Jones
// matrices and the dense S.  Wavefront w sums the rows q of its share for every column p
// (coalesced: lane p reads column p of row q, S being symmetric), the shares are added in LDS.
template <int NT = kBlock>
__device__ inline double max_diag(const Problem &pb, const Buffers &B, int f, int k, const double *J, int js) {
  constexpr int kW = NT / 64;
  __shared__ double nrm[2][kMaxStations];
  __shared__ double part[kW][2][kMaxStations];
  __shared__ double mx[NT / 64];
  for (int p = threadIdx.x; p < pb.N; p += NT) {
    const double *Jp = J + js * p;
    nrm[0][p] = Jp[0] * Jp[0] + Jp[1] * Jp[1] + Jp[4] * Jp[4] + Jp[5] * Jp[5];
    nrm[1][p] = Jp[2] * Jp[2] + Jp[3] * Jp[3] + Jp[6] * Jp[6] + Jp[7] * Jp[7];
  }
  __syncthreads();
  const double *Sd = B.Sd + ((int64_t)f * pb.K + k) * pb.N * pb.N;
  {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qn = (pb.N + kW - 1) / kW, q0 = w * qn, q1 = min(pb.N, q0 + qn);
    for (int p = lane; p < pb.N; p += 64) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll 8
      for (int q = q0; q < q1; ++q) {
        const double S = Sd[(int64_t)q * pb.N + p];
        d0 = fma(S, nrm[0][q], d0);
        d1 = fma(S, nrm[1][q], d1);
      }
      part[w][0][p] = d0;
      part[w][1][p] = d1;
    }
  }
  __syncthreads();
  double dmax = 0.0;
  for (int p = threadIdx.x; p < pb.N; p += NT) {
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
      d0 += part[w][0][p];
      d1 += part[w][1][p];
    }
    dmax = fmax(dmax, 2.0 * fmax(d0, d1));
  }
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = dmax;
  __syncthreads();
  double m = 0.0;
  for (int i = 0; i < NT / 64; ++i) m = fmax(m, mx[i]);
  return m;
}

// State at the start of direction k's LM run (one thread): objective F and data cost E0 at the
// start point, lambda_0 = tau * max diag(H_GN + rho I), nu = 2.  A state that is not finite ends
// the run at once and reports the subband.  With own, the run's direction, sweep and phase are
// recorded.
__device__ inline void begin_state(const Buffers &B, int f, LmState *st, double F, double E0,
                                   double maxdiag, bool own, int cur, int sweep) {
  st->F = F;
  st->E0 = E0;
  st->lambda = kLmTau * maxdiag;
  st->lambda0 = st->lambda;
  st->nu = 2.0;
  st->accepted = 0;
  st->chol_ok = 0;
  st->ell = 0.0;
  st->done = 0;
  if (!isfinite(F)) {   // a state that is not finite: the run does nothing, the subband is reported
    st->done = 1;
    if (B.status) B.status[f] = 5;   // CALIB_E_NUMERIC
  }
  if (own) {
    st->cur = cur;
    st->sweep = sweep;
    st->phase = kPhaseLm;
    st->itc = 0;
  }
}

// Start of direction k's LM run of subband f (whole workgroup of kBlock threads): objective F at
// J, the residual's energy E0, lambda_0, nu = 2, start point Jstart.
// With own, the run's direction, sweep and phase are recorded in the LM state.
__device__ inline void begin_dir(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                 int unreg, bool own, int cur, int sweep) {
  __shared__ double red[2][kBlock / 64];
  LmState *st = B.lm + f;
  const double *J = jdir(B, pb, f, k);
  double E0 = 0.0;
  const double F = objective(pb, L, B, f, k, unreg, J, red, &E0);
  const double m = max_diag(pb, B, f, k, J, 8) + (unreg ? 0.0 : B.rho[k]);
  for (int e = threadIdx.x; e < 8 * pb.N; e += kBlock) B.Jstart[(int64_t)f * pb.N * 8 + e] = J[e];
  if (threadIdx.x == 0) begin_state(B, f, st, F, E0, m, own, cur, sweep);
}

// Data cost and D_b at the LM trial point from the start point's statistics (one wavefront per
// tile, one lane per baseline).  The coherency is a scalar per sample and J_p J_q^H is the same
// for every sample of a baseline, so with the residual R at the start point J0 and
// dM = Jt_p Jt_q^H - J0_p J0_q^H (4 complex entries e),
//     sum_s ||R_s - c_s dM||^2 = sum_s ||R_s||^2 - 2 Re sum_e conj(dM_e) D0_e + S_b sum_e |dM_e|^2,
//     D_b(trial) = sum_s conj(c_s) (R_s - c_s dM) = D0 - S_b dM,
// with D0 = sum_s conj(c_s) R_s and S_b = sum_s |c_s|^2.  The first term, summed over the
// subband, is the data cost at the start point (LmState::E0), added by the subband's first tile;
// the tile partials sum to the data cost at the trial point as the streaming pass's do.
__device__ inline void trial_tile(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                  int tile, int lane) {
  const int nb = L.nb[f], bi = L.tile_b0[tile] + lane;
  double part = 0.0;
  if (lane < pb.bpt && bi < nb) {
    const int64_t gb = (int64_t)L.bl_off[f] + bi;
    const int p = L.bl_p[gb], q = L.bl_q[gb];
    const double *Jt = B.Jtrial + (int64_t)f * pb.N * 8, *J0 = B.Jstart + (int64_t)f * pb.N * 8;
    double m1[8], m0[8];
    jjh(Jt + 8 * p, Jt + 8 * q, m1);
    jjh(J0 + 8 * p, J0 + 8 * q, m0);
    const double S = B.Sb[L.sb_off[f] + (int64_t)k * nb + bi];
    const double *D0 = B.Dstart + 8 * gb;
    double *Dt = d_trial(B, f) + 8 * gb;
    double cross = 0.0, norm = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double dm = m1[e] - m0[e], d0 = D0[e];
      cross = fma(dm, d0, cross);   // Re conj(dM_e) D0_e over the real and imaginary parts
      norm = fma(dm, dm, norm);
      Dt[e] = fma(-S, dm, d0);
    }
    part = fma(S, norm, -2.0 * cross);
  }
  part = wave_sum(part);
  if (lane == 0) B.cost_part[tile] = part + (tile == L.tile_off[f] ? B.lm[f].E0 : 0.0);
}

// End of direction k's LM run (the SAGE commit) over one tile without a pass over the samples
// (one wavefront, one lane per baseline): with dM = J_kp J_kq^H - J0_p J0_q^H (J0 the run's start
// point), the residual R - c_k dM has D_l - X_lk dM for every direction l, and energy
// E - 2 Re sum_e conj(dM_e) D_k,e + X_kk ||dM||^2 (the tile's energy and cost partial).  Each lane
// forms dM once and walks the directions, the next direction's D_l and X_lk requested before the
// current one's are stored.  The next direction's D becomes the accepted and start point of its
// LM run.  Unless all is set only the directions after k are updated: within one SAGE sweep no
// other is read again before the next local step's refresh rebuilds them all.
__device__ inline void commit_tile(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                   int all, int tile, int lane) {
  const int Kf = L.ndir[f], nb = L.nb[f];
  const int K = pb.K, N = pb.N, next = k + 1 < Kf ? k + 1 : 0;
  const int bi = L.tile_b0[tile] + lane;
  const bool live = lane < pb.bpt && bi < nb;
  double part = 0.0;
  if (live) {
    const int64_t gb = (int64_t)L.bl_off[f] + bi;
    const int p = L.bl_p[gb], q = L.bl_q[gb];
    const int64_t nbt = pb.nbt;
    const int l0 = all ? 0 : k;
    // D_l and X_lk of direction l, requested ahead of their use
    double dn[8], xn[2];
    auto request = [&](int l) {
      const double *X = B.Xcoh + (((int64_t)l * K + k) * nbt + gb) * 2;
      const double *D = B.Dall + ((int64_t)l * nbt + gb) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) dn[e] = D[e];
      xn[0] = X[0];
      xn[1] = X[1];
    };
    request(l0);
    const double *J1 = B.J + ((int64_t)f * K + k) * N * 8, *J0 = B.Jstart + (int64_t)f * N * 8;
    double m1[8], m0[8], dm[8];
    jjh(J1 + 8 * p, J1 + 8 * q, m1);
    jjh(J0 + 8 * p, J0 + 8 * q, m0);
#pragma unroll
    for (int e = 0; e < 8; ++e) dm[e] = m1[e] - m0[e];
    for (int l = l0; l < Kf; ++l) {
      double d[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) d[e] = dn[e];
      const double x0 = xn[0], x1 = xn[1];
      if (l + 1 < Kf) request(l + 1);
      if (l == k) {
        double cross = 0.0, norm = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          cross = fma(dm[e], d[e], cross);
          norm = fma(dm[e], dm[e], norm);
        }
        part = fma(x0, norm, -2.0 * cross);
      }
      if (all || l > k) {
        sub_scaled(d, x0, x1, dm);
        double *D = B.Dall + ((int64_t)l * nbt + gb) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) D[e] = d[e];
        if (l == next) {
          double *Da = d_accepted(B, f) + 8 * gb;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            Da[e] = d[e];
            B.Dstart[8 * gb + e] = d[e];
          }
        }
      }
    }
  }
  part = wave_sum(part);
  if (lane == 0) {
    const double e = B.Epart[tile] + part;
    B.Epart[tile] = e;
    B.cost_part[tile] = e;
  }
}

// Trace rows [from, to) of a run that has stopped (one thread): the final objective and damping.
__device__ inline void stopped_rows(const Problem &pb, int f, int k, const LmState *st, double *lm_trace,
                                    int from, int to, int lm_iters) {
  for (int i2 = from; lm_trace && i2 < to; ++i2) {
    double *tn = lm_trace + 3 * ((int64_t)(f * pb.K + k) * lm_iters + i2);
    tn[0] = st->F;
    tn[1] = st->lambda;
    tn[2] = 0;
  }
}

// Gain ratio, accept / reject and damping after the trial point of LM iteration `it` (one thread),
// Nielsen's rule; the stopping rule on the step's predicted decrease; numeric failure; the LM
// trace row(s).  ok: the step was solved; Fn: the objective at the trial point.  Returns whether
// the step was accepted (the trial point's D_b then becomes the accepted one).
__device__ inline int update_state(const Problem &pb, const Buffers &B, int f, int k, LmState *st, int ok,
                                   double Fn, double *lm_trace, int it, int lm_iters, bool own) {
  int a = 0;
  if (ok) {
    const double ell = st->ell, F = st->F;
    if (pb.lm_tol > 0.0 && ell <= pb.lm_tol * F) st->done = 1;
    if (ell > 0.0 && F - Fn > 0.0) {
      const double gain = (F - Fn) / ell;
      const double t = 2.0 * gain - 1.0;
      st->lambda *= fmax(1.0 / 3.0, 1.0 - t * t * t);
      st->nu = 2.0;
      st->F = Fn;
      st->accepted += 1;
      st->dsel ^= 1;   // the trial point's D_b becomes the accepted one
      a = 1;
    }
  }
  if (!a) {
    st->lambda *= st->nu;
    st->nu *= 2.0;
    // normal equations that cannot be solved even with overwhelming damping: not finite
    if (!ok && !(st->lambda <= kLmFailFactor * st->lambda0)) {
      st->done = 1;
      if (B.status) B.status[f] = 5;   // CALIB_E_NUMERIC
    }
  }
  st->Fnew = Fn;
  if (lm_trace) {
    double *tr = lm_trace + 3 * ((int64_t)(f * pb.K + k) * lm_iters + it);
    tr[0] = st->F;
    tr[1] = st->lambda;
    tr[2] = a;
    // a run that stops here: the rows of its remaining iterations, which the host may not
    // launch, get what their updates would write (the final objective and damping)
    if (st->done) stopped_rows(pb, f, k, st, lm_trace, it + 1, lm_iters, lm_iters);
  }
  if (own) {
    st->itc = it + 1;
    if (st->done || it + 1 >= lm_iters) st->phase = kPhaseAdvance;
  }
  return a;
}

// Gain ratio, accept / reject and damping after the trial point of LM iteration `it` of direction
// k of subband f (whole workgroup of kBlock threads).  With own, the run's iteration count and
// phase are advanced in the LM state.
__device__ inline void update_dir(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                  int unreg, double *lm_trace, int it, int lm_iters, bool own) {
  __shared__ double red[2][kBlock / 64];
  __shared__ int acc;
  LmState *st = B.lm + f;
  if (st->done) {
    // the run has stopped: the trace repeats the final objective and damping
    if (own && threadIdx.x == 0) st->phase = kPhaseAdvance;
    if (threadIdx.x == 0) stopped_rows(pb, f, k, st, lm_trace, it, it + 1, lm_iters);
    return;
  }
  const int ok = st->chol_ok;
  double Fn = 0.0;
  if (ok) Fn = objective(pb, L, B, f, k, unreg, B.Jtrial + (int64_t)f * pb.N * 8, red);
  if (threadIdx.x == 0) acc = update_state(pb, B, f, k, st, ok, Fn, lm_trace, it, lm_iters, own);
  __syncthreads();
  if (acc) {
    double *J = B.J + ((int64_t)f * pb.K + k) * pb.N * 8;
    for (int e = threadIdx.x; e < 8 * pb.N; e += kBlock) J[e] = B.Jtrial[(int64_t)f * pb.N * 8 + e];
  }
}

}  // namespace lmd
}  // namespace calib
