// Matrix-free solve of the damped Gauss-Newton normal equations of the Levenberg-Marquardt step:
// (H_GN + (rho + lambda) I) delta = -G by preconditioned conjugate gradients, one workgroup per
// subband (eight wavefronts for N <= 64, four for N <= 128), without forming H.
//
// The coherency is a scalar times I2 (Section 2) and J is time invariant, so the Gauss-Newton
// matrix depends on the data only through S_pq = sum_s |c_s|^2 of each baseline, and its product
// with a direction v (N 2x2 complex blocks) is, per station p,
//     (H_GN v)_p = 2 (v_p Q_p + J_p W_p),   Q_p = sum_q S_pq J_q^H J_q,   W_p = sum_q S_pq v_q^H J_q
// (the operator form of the Hessian in Section 3 and Appendix A, without the residual term: the
// Gauss-Newton part).  Both sums are products of the symmetric N x N table S with a stack of
// per-station 2x2 matrices.  The preconditioner is block Jacobi: the diagonal block of station p
// is v_p -> v_p (2 Q_p + mu I) (the J_p W_p term only couples other stations), inverted in closed
// form as a 2x2 Hermitian matrix acting from the right.  Same iteration as the oracle's reading
// (x0 = 0, stop once ||r|| <= tol ||G|| or after 8N iterations; non-positive curvature fails the
// step like a failed factorisation).
//
// Work layout.  Wavefront 0 owns the vectors: lane l holds x, r, the search direction d, J_p, Q_p
// and the preconditioner of stations p = l + 64 s (s < SPL), so every dot product is a wavefront
// sum and the CG recurrences need no barrier.  The table products are split by columns: wavefront
// w of W takes stations q in [w C, w C + C), C = ceil(N / W), keeps S_pq of those columns for its rows
// p = l + 64 s in registers for the whole solve (read coalesced through the symmetry of S), reads
// each column's u_q = d_q^H J_q from LDS (every lane the same words: a broadcast) and leaves its
// partial sums in LDS, component-major so that lanes touch consecutive words, which wavefront 0
// adds in a fixed order.  One CG iteration: wavefront 0 writes u | all wavefronts their partial W
// | wavefront 0 finishes H d and the recurrences.
#include <type_traits>

#include "calib_internal.h"
#include "lm_device.h"
#include "wave_reduce.h"

namespace calib {
namespace {

// threads of the one-launch local step: eight wavefronts (two per SIMD) for N <= 64, four for
// N <= 128 (whose per-lane state, two stations per lane, leaves room for one wavefront per SIMD)
template <int SPL>
constexpr int pcg_threads() { return SPL == 1 ? 512 : 256; }

// c = a b for 2x2 complex matrices (8 doubles, row-major re/im)
__device__ inline void cmul(const double *a, const double *b, double *c) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double ar = a[(i * 2 + t) * 2], ai = a[(i * 2 + t) * 2 + 1];
        const double br = b[(t * 2 + j) * 2], bi = b[(t * 2 + j) * 2 + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      c[(i * 2 + j) * 2] = re;
      c[(i * 2 + j) * 2 + 1] = im;
    }
}

// c = a^H b
__device__ inline void chmul(const double *a, const double *b, double *c) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double ar = a[(t * 2 + i) * 2], ai = -a[(t * 2 + i) * 2 + 1];
        const double br = b[(t * 2 + j) * 2], bi = b[(t * 2 + j) * 2 + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      c[(i * 2 + j) * 2] = re;
      c[(i * 2 + j) * 2 + 1] = im;
    }
}

// c = a h for the Hermitian h = [[h0, h2 + i h3], [h2 - i h3, h1]] (4 reals)
__device__ inline void hmul(const double *a, const double *h, double *c) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double a0r = a[(i * 2) * 2], a0i = a[(i * 2) * 2 + 1];
    const double a1r = a[(i * 2 + 1) * 2], a1i = a[(i * 2 + 1) * 2 + 1];
    c[(i * 2) * 2] = a0r * h[0] + a1r * h[2] + a1i * h[3];
    c[(i * 2) * 2 + 1] = a0i * h[0] + a1i * h[2] - a1r * h[3];
    c[(i * 2 + 1) * 2] = a0r * h[2] - a0i * h[3] + a1r * h[1];
    c[(i * 2 + 1) * 2 + 1] = a0r * h[3] + a0i * h[2] + a1i * h[1];
  }
}

// J_q^H J_q as a Hermitian (q00, q11, Re q01, Im q01)
__device__ inline void gram(const double *Jq, double *v) {
  v[0] = Jq[0] * Jq[0] + Jq[1] * Jq[1] + Jq[4] * Jq[4] + Jq[5] * Jq[5];
  v[1] = Jq[2] * Jq[2] + Jq[3] * Jq[3] + Jq[6] * Jq[6] + Jq[7] * Jq[7];
  v[2] = Jq[0] * Jq[2] + Jq[1] * Jq[3] + Jq[4] * Jq[6] + Jq[5] * Jq[7];
  v[3] = Jq[0] * Jq[3] - Jq[1] * Jq[2] + Jq[4] * Jq[7] - Jq[5] * Jq[6];
}

// Per-station 2x2 complex matrices in LDS take kJS doubles (8 + 2 of padding): at a stride of
// 20 dwords, 16 stations fall in 16 different 4-bank groups of the 64 LDS banks, so a wavefront's
// 16-byte reads at scattered stations (baselines' p and q, adjacency lists) rarely conflict; at a
// stride of 16 dwords every fourth station shares its banks.
constexpr int kJS = 10;

// LDS of one solve; SPL: stations per lane of wavefront 0 (1 for N <= 64, 2 for N <= 128)
template <int SPL, int NW = pcg_threads<SPL>() / 64>
struct PcgLds {
  double Js[64 * SPL * kJS];                // J of the direction
  double Us[64 * SPL * kJS];                // u_q = d_q^H J_q
  double Wp[NW][8][64 * SPL];               // per-wavefront partials over its columns,
                                            // component-major (lane-consecutive, no bank conflicts)
  double Gs[8][64 * SPL];                   // the gradient, component-major, for the record
  int ctl[2];                               // continue, failed
};

// The gradient and the solve of direction k of subband f (whole workgroup) at the
// current J (sh.Js), with the direction's Y and B_f Z in LDS (Ys, BZs, 8 doubles per station): G
// and the step delta to the record (CALIB_FIELD_LM_STEP), the trial point J + delta into jt_lds,
// the predicted decrease into the LM state st (chol_ok = 0 on a failed solve).  The other
// wavefronts return before wavefront 0 writes the results.
template <int SPL>
__device__ inline void pcg_solve(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                 int unreg, double tol, PcgLds<SPL> &sh, double *jt_lds, LmState *st,
                                 const double *Ys, const double *BZs, bool first) {
  constexpr int kPcgWaves = pcg_threads<SPL>() / 64;
  constexpr int kRows = 64 * SPL;               // stations covered
  constexpr int kC = kRows / kPcgWaves;          // columns per wavefront (at most)
  constexpr int kBatch = 32 / (SPL * kPcgWaves); // baselines of the gradient in flight per lane
  double *Js = sh.Js, *Us = sh.Us;
  auto &Wp = sh.Wp;
  int *ctl = sh.ctl;
  const int N = pb.N, nf = pb.nf;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int C = (N + kPcgWaves - 1) / kPcgWaves, c0 = w * C;
  double lam = st->lambda;   // at the run's first solve set below from Q
  const double rho = unreg ? 0.0 : B.rho[k];
  double mu = rho + lam;
  const double *Sd = B.Sd + ((int64_t)f * pb.K + k) * N * N;

  // gradient of the data term, gathered over station p's baselines (wavefront w takes every
  // W-th one, from the w-th): G_p = -2 sum_{q>p} D_pq J_q - 2 sum_{c<p} D_cp^H J_c (+ Y_p + rho (J_p - BZ_p)
  // below).  The first batch's adjacency entries and D_b are requested before S, so that their two
  // dependent latencies overlap the loads of S.
  const double *Dacc = d_accepted(B, *st);
  int gb[kBatch], oraw[kBatch];
  double d[kBatch][8];
  auto request = [&](int s, int ab) {
    const int p = lane + 64 * s;
    const int a1 = p < N ? L.adj_off[f * N + p + 1] : 0;
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int a = ab + kPcgWaves * i;
      gb[i] = a < a1 ? L.adj_b[a] : -1;
      oraw[i] = a < a1 ? L.adj_o[a] : 0;
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      if (gb[i] >= 0) {
        const double2 *D2 = reinterpret_cast<const double2 *>(Dacc + 8 * (int64_t)gb[i]);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const double2 x = D2[h];
          d[i][2 * h] = x.x;
          d[i][2 * h + 1] = x.y;
        }
      }
    }
  };
  double gp[SPL][8];
  auto consume = [&](int s) {
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      if (gb[i] < 0) continue;
      const bool first = oraw[i] >= 0;
      const int o = first ? oraw[i] : -1 - oraw[i];
      double t[8];
      if (first) cmul(d[i], Js + kJS * o, t);
      else chmul(d[i], Js + kJS * o, t);
#pragma unroll
      for (int e = 0; e < 8; ++e) gp[s][e] = fma(-2.0, t[e], gp[s][e]);
    }
  };
  int a_first[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int p = lane + 64 * s;
    a_first[s] = p < N ? L.adj_off[f * N + p] + w : 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) gp[s][e] = 0.0;
  }
  request(0, a_first[0]);

  // S_pq for rows p = lane + 64 s and this wavefront's columns q = c0 + j; S is symmetric, so
  // the read goes down column p of row q (consecutive lanes, consecutive addresses)
  double S[SPL][kC];
#pragma unroll
  for (int s = 0; s < SPL; ++s)
#pragma unroll
    for (int j = 0; j < kC; ++j) {
      const int p = lane + 64 * s, q = c0 + j;
      S[s][j] = (p < N && j < C && q < N) ? Sd[(int64_t)q * N + p] : 0.0;
    }

  // the rest of the gradient, the next batch in flight while the current one is used (and,
  // after the first, while the Q partials are formed)
  int cs = 0, ab = a_first[0];
  bool more = true;
  auto advance = [&]() {
    consume(cs);
    const int p = lane + 64 * cs;
    const int a1 = p < N ? L.adj_off[f * N + p + 1] : 0;
    ab += kPcgWaves * kBatch;
    if (ab < a1) {
      request(cs, ab);
    } else if (cs + 1 < SPL) {
      ++cs;
      ab = a_first[cs];
      request(cs, ab);
    } else {
      more = false;
    }
  };
  advance();
  // Q_p partials over this wavefront's columns: J_q^H J_q of column q = c0 + j from LDS (the
  // same words for every lane: broadcast reads); columns past N have S = 0
  {
    double qp[SPL][4];
#pragma unroll
    for (int s = 0; s < SPL; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) qp[s][c] = 0.0;
#pragma unroll
    for (int j = 0; j < kC; ++j) {
      double vq[4];
      gram(Js + kJS * (c0 + j), vq);   // past N: zeros; past this wavefront's columns: S = 0
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int s = 0; s < SPL; ++s) qp[s][c] = fma(S[s][j], vq[c], qp[s][c]);
    }
#pragma unroll
    for (int s = 0; s < SPL; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) Wp[w][c][lane + 64 * s] = qp[s][c];
  }
  while (more) advance();
  __syncthreads();   // Q partials in Wp
  double Qp[SPL][4], Jp[SPL][8];
  if (w == 0) {
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < kPcgWaves; ++i) v += Wp[i][c][lane + 64 * s];
        Qp[s][c] = v;
      }
    }
    if (first) {
      // the run's initial damping lambda_0 = tau max diag(H_GN + rho I): the diagonal of H_GN
      // at station p holds 2 Q_p[0][0] and 2 Q_p[1][1] (the squared column norms of the J_q
      // weighted by S_pq)
      double m = 0.0;
#pragma unroll
      for (int s = 0; s < SPL; ++s)
        if (lane + 64 * s < N) m = fmax(m, fmax(Qp[s][0], Qp[s][1]));
      m = lmd::wave_max(m);
      lam = kLmTau * (2.0 * m + rho);
      mu = rho + lam;
      if (lane == 0) {
        st->lambda = lam;
        st->lambda0 = lam;
      }
    }
  }
  __syncthreads();   // Q read; the gradient partials go to Wp
#pragma unroll
  for (int s = 0; s < SPL; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) Wp[w][e][lane + 64 * s] = gp[s][e];
  __syncthreads();

  // wavefront 0: right-hand side b = -G, preconditioner (2 Q_p + mu I)^-1, x = 0, r = b, d = z
  double x[SPL][8], r[SPL][8], dv[SPL][8], Mi[SPL][4];
  double bb = 0.0, rz = 0.0, stop = 0.0;
  int failed = 0;
  const int maxit = 8 * N;
  if (w == 0) {
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const int p = lane + 64 * s;
      const bool live = p < N;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < kPcgWaves; ++i) v += Wp[i][e][p];
        if (live && !unreg) v += Ys[8 * p + e] + rho * (Js[kJS * p + e] - BZs[8 * p + e]);
        const double gv = live ? v : 0.0;
        sh.Gs[e][p] = gv;
        Jp[s][e] = live ? Js[kJS * p + e] : 0.0;
        x[s][e] = 0.0;
        r[s][e] = -gv;
        bb = fma(r[s][e], r[s][e], bb);
      }
      const double a = 2.0 * Qp[s][0] + mu, dd = 2.0 * Qp[s][1] + mu;
      const double br = 2.0 * Qp[s][2], bi = 2.0 * Qp[s][3];
      const double det = a * dd - (br * br + bi * bi);
      if (live && (!(a > 0.0) || !(det > 0.0) || !isfinite(det))) failed = 1;
      const double id = live ? 1.0 / det : 0.0;
      Mi[s][0] = dd * id;
      Mi[s][1] = a * id;
      Mi[s][2] = -br * id;
      Mi[s][3] = -bi * id;
      hmul(r[s], Mi[s], dv[s]);
#pragma unroll
      for (int e = 0; e < 8; ++e) rz = fma(r[s][e], dv[s][e], rz);
    }
    double v2[2] = {bb, rz};
    wave_sum_vec<2>(v2);
    bb = v2[0];
    rz = v2[1];
    stop = tol * tol * bb;
    failed = __any(failed) ? 1 : 0;
  }
  int iters_run = 0;
  for (int it = 0;; ++it) {
    // wavefront 0: u_p = d_p^H J_p for the partial products, and whether to iterate
    if (w == 0) {
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        double u[8];
        chmul(dv[s], Jp[s], u);
        double2 *u2 = reinterpret_cast<double2 *>(Us + kJS * (lane + 64 * s));
#pragma unroll
        for (int h = 0; h < 4; ++h) u2[h] = make_double2(u[2 * h], u[2 * h + 1]);
      }
      if (lane == 0) {
        ctl[0] = (!failed && bb > 0.0 && it < maxit) ? 1 : 0;
        ctl[1] = failed;
      }
    }
    __syncthreads();
    if (!ctl[0]) break;
    ++iters_run;
    // partial W_p over this wavefront's columns: u of column c0 + j read from LDS by every lane
    // (broadcast)
    {
      double W[SPL][8];
#pragma unroll
      for (int s = 0; s < SPL; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) W[s][e] = 0.0;
#pragma unroll
      for (int j = 0; j < kC; ++j) {
        // past N: zeros; past this wavefront's columns: S = 0
        const double2 *u2 = reinterpret_cast<const double2 *>(Us + kJS * (c0 + j));
        double uq[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const double2 t = u2[h];
          uq[2 * h] = t.x;
          uq[2 * h + 1] = t.y;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int s = 0; s < SPL; ++s) W[s][e] = fma(S[s][j], uq[e], W[s][e]);
      }
#pragma unroll
      for (int s = 0; s < SPL; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) Wp[w][e][lane + 64 * s] = W[s][e];
    }
    __syncthreads();
    if (w != 0) continue;
    // wavefront 0: (H d)_p = 2 (d_p Q_p + J_p W_p) + mu d_p, then the CG recurrences
    double Hd[SPL][8], pq = 0.0;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const int p = lane + 64 * s;
      double W[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < kPcgWaves; ++i)
#pragma unroll
        for (int e = 0; e < 8; ++e) W[e] += Wp[i][e][p];
      double t1[8], t2[8];
      hmul(dv[s], Qp[s], t1);
      cmul(Jp[s], W, t2);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        Hd[s][e] = 2.0 * (t1[e] + t2[e]) + mu * dv[s][e];
        pq = fma(dv[s][e], Hd[s][e], pq);
      }
    }
    pq = wave_sum(pq);
    if (!(pq > 0.0) || !isfinite(pq)) {
      failed = 1;
      continue;   // the next pass through the loop head stops every wavefront
    }
    const double alpha = rz / pq;
    double z[SPL][8], v2[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        x[s][e] = fma(alpha, dv[s][e], x[s][e]);
        r[s][e] = fma(-alpha, Hd[s][e], r[s][e]);
        v2[1] = fma(r[s][e], r[s][e], v2[1]);
      }
      hmul(r[s], Mi[s], z[s]);
#pragma unroll
      for (int e = 0; e < 8; ++e) v2[0] = fma(r[s][e], z[s][e], v2[0]);
    }
    wave_sum_vec<2>(v2);
    if (v2[1] <= stop) {
      bb = 0.0;   // converged: the loop head stops
      continue;
    }
    const double beta = v2[0] / rz;
    rz = v2[0];
#pragma unroll
    for (int s = 0; s < SPL; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) dv[s][e] = fma(beta, dv[s][e], z[s][e]);
  }
  if (w != 0) return;
  if (lane == 0 && B.work) {
    B.work[2 * f] += iters_run;
    B.work[2 * f + 1] += 1.0;
  }
  if (ctl[1]) {
    if (lane == 0) st->chol_ok = 0;
    return;
  }
  // delta, trial point, gradient for the record, predicted decrease ell = delta.(lambda delta - G)/2
  double ell = 0.0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int p = lane + 64 * s;
    if (p >= N) continue;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = 8 * p + e;
      const double gv = sh.Gs[e][p];
      B.delta[(int64_t)f * nf + c] = x[s][e];
      B.G[(int64_t)f * nf + c] = gv;
      jt_lds[kJS * p + e] = Jp[s][e] + x[s][e];
      ell = fma(x[s][e], fma(lam, x[s][e], -gv), ell);
    }
  }
  ell = wave_sum(ell);
  if (lane == 0) {
    st->ell = 0.5 * ell;
    st->chol_ok = 1;
  }
}

// Per-baseline passes of the one-workgroup local step.  Four lanes share a baseline, lane h
// holding complex entry h = (i, j) of its 2x2 matrices (D_b, M = J_p J_q^H), so that the
// wavefront's loads and stores of D_b cover 16 consecutive baselines (1 KiB, whole cache lines)
// per instruction; 64 baselines per round of the workgroup, kU rounds with every load issued
// together (a single workgroup has only its own loads in flight, so each batch pays one memory
// latency).  The Jones matrices are read from LDS.  Energy partials are summed over the workgroup
// and kept in the subband's first tile (the objective adds the tiles of a subband).
constexpr int kQuad = 4;                    // lanes per baseline
template <int NT>
constexpr int rounds() { return 2048 / NT; }   // rounds per batch: 512 baselines per batch

// entry (i, j) of a_p a_q^H for the stations' 2x2 complex matrices in LDS (kJS doubles each)
__device__ inline double2 jjh_entry(const double *A, int p, int q, int i, int j) {
  const double *a = A + kJS * p + 4 * i, *b = A + kJS * q + 4 * j;
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const double ar = a[2 * t], ai = a[2 * t + 1], br = b[2 * t], bi = b[2 * t + 1];
    re += ar * br + ai * bi;
    im += ai * br - ar * bi;
  }
  return make_double2(re, im);
}

// Data cost (returned to every thread) and D_b at the trial point Jt from the start point J0's
// statistics (lmd::trial_tile); st: the subband's LM state; NT threads
template <int NT>
__device__ inline double fused_trial(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                     const double *Jt, const double *J0, const LmState *st,
                                     double (*red)[NT / 64]) {
  constexpr int kBpr = NT / kQuad;   // baselines per round
  constexpr int kU = rounds<NT>();
  const int nb = L.nb[f];
  const int64_t b0 = L.bl_off[f];
  const double *Sb = B.Sb + L.sb_off[f] + (int64_t)k * nb;
  double2 *Dt = reinterpret_cast<double2 *>(d_trial(B, *st));
  const double2 *D0 = reinterpret_cast<const double2 *>(B.Dstart);
  const int h = threadIdx.x & 3, ei = h >> 1, ej = h & 1, sub = threadIdx.x >> 2;
  double part = 0.0;
  // a full batch runs without per-baseline guards (and the branches they cost); the last one
  // may be partial
  auto batch = [&](int base, auto full) {
    constexpr bool kFull = decltype(full)::value;
    int p[kU], q[kU];
    double S[kU];
    double2 d0[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int bi = base + sub + kBpr * u;
      if (kFull || bi < nb) {
        const int64_t gb = b0 + bi;
        p[u] = L.bl_p[gb];
        q[u] = L.bl_q[gb];
        S[u] = Sb[bi];
        d0[u] = D0[4 * gb + h];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int bi = base + sub + kBpr * u;
      if (!kFull && bi >= nb) continue;
      const double2 m1 = jjh_entry(Jt, p[u], q[u], ei, ej), m0 = jjh_entry(J0, p[u], q[u], ei, ej);
      const double dr = m1.x - m0.x, di = m1.y - m0.y;
      const double cross = fma(dr, d0[u].x, di * d0[u].y), norm = fma(dr, dr, di * di);
      Dt[4 * (b0 + bi) + h] = make_double2(fma(-S[u], dr, d0[u].x), fma(-S[u], di, d0[u].y));
      part += fma(S[u], norm, -2.0 * cross);
    }
  };
  for (int base = 0; base < nb; base += kBpr * kU) {
    if (base + kBpr * kU <= nb) batch(base, std::true_type{});
    else batch(base, std::false_type{});
  }
  double v[1] = {part};
  lmd::block_sum_vec<1, NT>(v, red);
  return v[0] + st->E0;
}

// SAGE commit of direction k (lmd::commit_tile): with dM = J1_p J1_q^H - J0_p J0_q^H (J1 the run's
// final J, J0 its start, both in LDS), every later direction l (every direction, k's own included,
// with several sweeps) updates D_l -= X_lk dM.  The residual's energy after the run needs no pass:
// it is the data cost of the run's last accepted trial point.  dM is formed once per baseline; the
// directions are walked with the next one's D_l and X_lk requested before the current one's are
// stored.
template <int NT>
__device__ inline void fused_commit(const Problem &pb, const Layout &L, const Buffers &B, int f, int k,
                                    int all, const double *J1, const double *J0, const LmState *st) {
  constexpr int kBpr = NT / kQuad;   // baselines per round
  constexpr int kU = rounds<NT>();
  const int Kf = L.ndir[f], nb = L.nb[f], K = pb.K, next = k + 1 < Kf ? k + 1 : 0;
  const int64_t b0 = L.bl_off[f], nbt = pb.nbt;
  const int l0 = all ? 0 : k + 1;
  if (l0 >= Kf) return;
  const int h = threadIdx.x & 3, ei = h >> 1, ej = h & 1, sub = threadIdx.x >> 2;
  double2 *Dall = reinterpret_cast<double2 *>(B.Dall);
  const double2 *X = reinterpret_cast<const double2 *>(B.Xcoh);
  double2 *Da = reinterpret_cast<double2 *>(d_accepted(B, *st));
  double2 *Ds = reinterpret_cast<double2 *>(B.Dstart);
  // a full batch runs without per-baseline guards; the last one may be partial
  auto batch = [&](int base, auto full) {
    constexpr bool kFull = decltype(full)::value;
    double2 dm[kU], dn[kU], xn[kU];
    auto request = [&](int l) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int bi = base + sub + kBpr * u;
        if (kFull || bi < nb) {
          const int64_t gb = b0 + bi;
          dn[u] = Dall[4 * ((int64_t)l * nbt + gb) + h];
          xn[u] = X[((int64_t)l * K + k) * nbt + gb];
        }
      }
    };
    request(l0);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int bi = base + sub + kBpr * u;
      if (kFull || bi < nb) {
        const int64_t gb = b0 + bi;
        const int p = L.bl_p[gb], q = L.bl_q[gb];
        const double2 m1 = jjh_entry(J1, p, q, ei, ej), m0 = jjh_entry(J0, p, q, ei, ej);
        dm[u] = make_double2(m1.x - m0.x, m1.y - m0.y);
      }
    }
    for (int l = l0; l < Kf; ++l) {
      double2 d[kU], x[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        d[u] = dn[u];
        x[u] = xn[u];
      }
      if (l + 1 < Kf) request(l + 1);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int bi = base + sub + kBpr * u;
        if (!kFull && bi >= nb) continue;
        const int64_t gb = b0 + bi;
        const double2 t = make_double2(d[u].x - (x[u].x * dm[u].x - x[u].y * dm[u].y),
                                       d[u].y - (x[u].x * dm[u].y + x[u].y * dm[u].x));
        Dall[4 * ((int64_t)l * nbt + gb) + h] = t;
        if (l == next) {
          Da[4 * gb + h] = t;
          Ds[4 * gb + h] = t;
        }
      }
    }
  };
  for (int base = 0; base < nb; base += kBpr * kU) {
    if (base + kBpr * kU <= nb) batch(base, std::true_type{});
    else batch(base, std::false_type{});
  }
}

// Re tr(Y^H (J - BZ)) + rho/2 ||J - BZ||^2 of the direction (whole workgroup of NT threads;
// result in every thread): J in LDS at kJS doubles per station, Y and B_f Z in LDS at 8
template <int NT>
__device__ inline double penalty_lds(int N, double rho, const double *Jx, const double *Ys,
                                     const double *BZs, double (*red)[NT / 64]) {
  double pen = 0.0;
  for (int e = threadIdx.x; e < 8 * N; e += NT) {
    const double d = Jx[kJS * (e >> 3) + (e & 7)] - BZs[e];
    pen += Ys[e] * d + 0.5 * rho * d * d;
  }
  double v[1] = {pen};
  lmd::block_sum_vec<1, NT>(v, red);
  return v[0];
}

// A subband's whole local step in one workgroup: for every SAGE sweep and direction, the LM run
// (start, then per iteration the gradient and solve, the trial point's statistics, the update
// with the stopping rule) and the SAGE commit, in the order of the launches of the lockstep local
// step.  Nothing is launched or read back between LM iterations, and what an LM iteration reads
// besides the per-baseline statistics stays in LDS for the whole run: the LM state, the current
// and the start point J, the direction's Y and B_f Z, the residual's energy (from the refresh's
// per-(direction, tile) terms at the start, then moved by each commit).  The LM state and the energy are
// written back at the end (the energy into the subband's first tile, the others zero).
template <int SPL>
__global__ __launch_bounds__(pcg_threads<SPL>()) void k_local_step(Problem pb, Layout L, Buffers B, int unreg,
                                                                   double *lm_trace, int lm_iters, int sweeps) {
  constexpr int NT = pcg_threads<SPL>();
  constexpr int kRows = 64 * SPL;
  __shared__ __align__(16) PcgLds<SPL> sh;
  __shared__ __align__(16) double J0s[kRows * kJS];   // the run's start point
  __shared__ __align__(16) double Ys[kRows * 8], BZs[kRows * 8];
  __shared__ double red[1][NT / 64];
  __shared__ LmState lst;
  __shared__ int acc;
  const int f = blockIdx.x;
  const int Kf = L.ndir[f], N = pb.N, n8 = 8 * N;
  const int all = sweeps > 1;
  const int t0 = L.tile_off[f], t1 = L.tile_off[f + 1];
  if (threadIdx.x == 0) lst = B.lm[f];
  double E;   // energy of the current residual, from the statistics' per-(direction, tile) terms
  {
    double v[1] = {0.0};
    for (int t = t0 + threadIdx.x; t < t1; t += NT)
      for (int l = 0; l < Kf; ++l) v[0] += B.Epl[(int64_t)l * pb.ntiles + t];
    lmd::block_sum_vec<1, NT>(v, red);
    E = v[0];
  }
  for (int sw = 0; sw < sweeps; ++sw)
    for (int k = 0; k < Kf; ++k) {
      const double rho = unreg ? 0.0 : B.rho[k];
      const int64_t jo = ((int64_t)f * pb.K + k) * n8;
      for (int e = threadIdx.x; e < 8 * kRows; e += NT) {
        const double j = e < n8 ? B.J[jo + e] : 0.0;   // zero past the last station
        sh.Js[kJS * (e >> 3) + (e & 7)] = j;
        J0s[kJS * (e >> 3) + (e & 7)] = j;
        if (e < n8) {
          Ys[e] = B.Y[jo + e];
          BZs[e] = B.BZ[jo + e];
        }
      }
      __syncthreads();
      const double F = E + (unreg ? 0.0 : penalty_lds<NT>(N, rho, sh.Js, Ys, BZs, red));
      // lambda_0 comes from the first solve's Q blocks (pcg_solve)
      if (threadIdx.x == 0) lmd::begin_state(B, f, &lst, F, E, 0.0, false, 0, 0);
      __syncthreads();
      if (lst.done && threadIdx.x == 0)   // a run that cannot start (non-finite state): trace rows only
        lmd::stopped_rows(pb, f, k, &lst, lm_trace, 0, lm_iters, lm_iters);
      double Ecur = E;   // data cost at the run's current point
      for (int it = 0; it < lm_iters && !lst.done; ++it) {
        pcg_solve<SPL>(pb, L, B, f, k, unreg, pb.cg_tol, sh, sh.Us, &lst, Ys, BZs, it == 0);
        __syncthreads();
        const int ok = lst.chol_ok;
        double En = 0.0, Fn = 0.0;
        if (ok) {
          En = fused_trial<NT>(pb, L, B, f, k, sh.Us, J0s, &lst, red);
          Fn = En + (unreg ? 0.0 : penalty_lds<NT>(N, rho, sh.Us, Ys, BZs, red));
        }
        if (threadIdx.x == 0) acc = lmd::update_state(pb, B, f, k, &lst, ok, Fn, lm_trace, it, lm_iters, false);
        __syncthreads();
        if (acc) Ecur = En;
        if (acc)   // the trial point is the new J
          for (int e = threadIdx.x; e < n8; e += NT) {
            const double j = sh.Us[kJS * (e >> 3) + (e & 7)];
            sh.Js[kJS * (e >> 3) + (e & 7)] = j;
            B.J[jo + e] = j;
          }
        __syncthreads();
      }
      // the commit updates the later directions' D_l (the last direction of a single sweep has none
      // to update); the residual's energy after the run is the data cost of its last accepted
      // trial point (the same sum as the energy change the commit would form, at the same points)
      fused_commit<NT>(pb, L, B, f, k, all, sh.Js, J0s, &lst);
      E = Ecur;
      __syncthreads();
    }
  if (threadIdx.x == 0) B.lm[f] = lst;
  for (int t = t0 + threadIdx.x; t < t1; t += NT) {
    const double v = t == t0 ? E : 0.0;
    B.Epart[t] = v;
    B.cost_part[t] = v;
  }
}

}  // namespace

hipError_t launch_local_step(const Problem &pb, const Layout &L, const Buffers &B, int unreg,
                             double *lm_trace, int lm_iters, int sweeps, hipStream_t s) {
  if (pb.N > kMaxStations || pb.bpt > 64) return hipErrorInvalidValue;
  if (pb.N <= 64)
    hipLaunchKernelGGL(k_local_step<1>, dim3(pb.P), dim3(pcg_threads<1>()), 0, s, pb, L, B, unreg, lm_trace,
                       lm_iters, sweeps);
  else
    hipLaunchKernelGGL(k_local_step<2>, dim3(pb.P), dim3(pcg_threads<2>()), 0, s, pb, L, B, unreg, lm_trace,
                       lm_iters, sweeps);
  return hipGetLastError();
}

}  // namespace calib
