// Levenberg-Marquardt kernels of the local step (minimisation M1 of Section 3), one subband per
// workgroup except where stated, all in FP64.
//
// Real parameters of one direction: theta[p*8 + (i*2+j)*2 + {0:Re,1:Im}] for the entries
// J_p[i][j].  The objective is the augmented Lagrangian
//   L(J) = sum_b sum_s ||V_k - c_s J_p J_q^H||^2 + Re tr(Y^H (J - BZ)) + rho/2 ||J - BZ||^2
// (linear term as in the trace form of Appendix A).  Its Euclidean gradient, packed as
// d/dRe + i d/dIm per entry, is
//   G_p = -2 sum_{q>p} D_pq J_q - 2 sum_{c<p} D_cp^H J_c + Y_p + rho (J_p - BZ_p),
// with D_b = sum_s conj(c_s) r_s from the streaming pass.  Because the coherency is a scalar
// times I2 (Section 2) and J is time invariant, the Gauss-Newton matrix 2 Jac^T Jac depends on
// the data only through S_b = sum_s |c_s|^2:
//   diagonal block of station p: for each row i of J_p, the real 4x4 form of
//       2 Q_p,  Q_p = sum_{c adjacent p} S_pc J_c^H J_c
//   off-diagonal block of baseline (a,b), a<b, entry (u of J_a, v of J_b):
//       2 S_ab * [[Re w, Im w], [Im w, -Re w]][ri_u][ri_v],  w = J_a[i_u][j_v] J_b[i_v][j_u].
// The damped system (H + (rho + lambda) I) delta = -G is solved by a Cholesky factorisation
// of the matrix augmented with -G^T as an extra row (so the forward substitution falls out of
// the factorisation), followed by a blocked back substitution.
#include "calib_internal.h"
#include "lm_device.h"
#include "wave_reduce.h"

namespace calib {

namespace {

using lmd::block_sum_vec;
using lmd::jdir;

__global__ __launch_bounds__(kBlock) void k_lm_begin(Problem pb, Layout L, Buffers B, int k, int unreg,
                                                     int sweeps) {
  const int f = blockIdx.x;
  LmState *st = B.lm + f;
  // k < 0: the subband's own direction.  A subband whose run has ended (and been committed) moves
  // to its next direction, wrapping to the next SAGE sweep, and starts that direction's run.
  const bool own = k < 0;
  int cur = 0, sweep = 0;
  if (own) {
    int ph = st->phase;
    cur = st->cur;
    sweep = st->sweep;
    if (ph == kPhaseAdvance) {
      if (++cur >= L.ndir[f]) {
        cur = 0;
        ++sweep;
      }
      ph = (L.ndir[f] == 0 || sweep >= sweeps) ? kPhaseFinished : kPhaseBegin;
    }
    __syncthreads();   // every wavefront has read the state before thread 0 moves it on
    if (ph != kPhaseBegin) {
      if (ph == kPhaseFinished && threadIdx.x == 0) st->phase = kPhaseFinished;
      return;
    }
    k = cur;
  } else if (k >= L.ndir[f]) {
    return;
  }
  lmd::begin_dir(pb, L, B, f, k, unreg, own, cur, sweep);
}

// One workgroup of two wavefronts per (subband, station row-block), so that all of them are resident
// at once; blockIdx.y == 0 writes the padding rows, then the stations from the last (whose rows
// are the longest) to the first, so that the longest workgroups are dispatched first.
constexpr int kAsmBlock = 128;
__global__ __launch_bounds__(kAsmBlock) void k_assemble(Problem pb, Layout L, Buffers B, int k, int unreg) {
  __shared__ double red[12][kAsmBlock / 64];
  __shared__ double qg[12];
  const int f = blockIdx.x, p = blockIdx.y == 0 ? pb.N : pb.N - (int)blockIdx.y;
  if (!lm_live(B, L.ndir, f, k)) return;
  k = lm_dir(B, f, k);
  const int N = pb.N, nf = pb.nf, npad = pb.npad;
  double *A = B.H + (int64_t)f * npad * nf;
  const double lam = B.lm[f].lambda;
  const double rho = unreg ? 0.0 : B.rho[k];
  if (p == N) {
    // identity on padded factor columns, zero padding rows below the right-hand side row
    for (int r = 8 * N; r < nf; ++r)
      for (int c = threadIdx.x; c < nf; c += kAsmBlock) A[(int64_t)r * nf + c] = (c == r) ? 1.0 : 0.0;
    for (int c = 8 * N + threadIdx.x; c < nf; c += kAsmBlock) A[(int64_t)nf * nf + c] = 0.0;
    for (int r = nf + 1; r < npad; ++r)
      for (int c = threadIdx.x; c < nf; c += kAsmBlock) A[(int64_t)r * nf + c] = 0.0;
    return;
  }
  // Station p's baselines, one per thread: the adjacency entry and D_b of the accepted point, and
  // the consensus terms of the gradient, requested before the staging below so that the loads
  // overlap
  static_assert(kMaxStations <= kAsmBlock, "at most one baseline of station p per thread");
  const int a = L.adj_off[f * N + p] + threadIdx.x;
  const bool has = a < L.adj_off[f * N + p + 1];
  int gb = 0, oraw = 0;
  double d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (has) {
    gb = L.adj_b[a];
    oraw = L.adj_o[a];
    const double2 *D2 = reinterpret_cast<const double2 *>(d_accepted(B, f) + 8 * (int64_t)gb);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const double2 x = D2[h];
      d[2 * h] = x.x;
      d[2 * h + 1] = x.y;
    }
  }
  double yv = 0.0, bzv = 0.0;
  if (threadIdx.x >= 4 && threadIdx.x < 12 && !unreg) {
    const int64_t o = ((int64_t)f * pb.K + k) * N * 8 + 8 * p + (threadIdx.x - 4);
    yv = B.Y[o];
    bzv = B.BZ[o];
  }
  // the direction's Jones matrices and S of station p's pairs (row p of the dense table) in LDS:
  // everything below reads them
  __shared__ double Js[8 * kMaxStations];
  __shared__ double Sp[kMaxStations];
  {
    const double *Jg = jdir(B, pb, f, k);
    const double *Sd = B.Sd + (((int64_t)f * pb.K + k) * N + p) * N;
    for (int e = threadIdx.x; e < 8 * N; e += kAsmBlock) Js[e] = Jg[e];
    for (int e = threadIdx.x; e < N; e += kAsmBlock) Sp[e] = Sd[e];
  }
  __syncthreads();
  const double *J = Js;
  // Q_p (q00, q11, Re q01, Im q01) and the data part of the gradient of station p
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (has) {
    const bool first = oraw >= 0;
    const int o = first ? oraw : -1 - oraw;
    const double S = Sp[o];
    const double *Jo = J + 8 * o;
    v[0] += S * (Jo[0] * Jo[0] + Jo[1] * Jo[1] + Jo[4] * Jo[4] + Jo[5] * Jo[5]);
    v[1] += S * (Jo[2] * Jo[2] + Jo[3] * Jo[3] + Jo[6] * Jo[6] + Jo[7] * Jo[7]);
    // (J^H J)[0][1] = conj(J00) J01 + conj(J10) J11
    v[2] += S * (Jo[0] * Jo[2] + Jo[1] * Jo[3] + Jo[4] * Jo[6] + Jo[5] * Jo[7]);
    v[3] += S * (Jo[0] * Jo[3] - Jo[1] * Jo[2] + Jo[4] * Jo[7] - Jo[5] * Jo[6]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          // first: (D J_o)[i][j] = sum_t D[i][t] J_o[t][j];
          // second: (D^H J_o)[i][j] = sum_t conj(D[t][i]) J_o[t][j]
          const double dr = first ? d[(i * 2 + t) * 2] : d[(t * 2 + i) * 2];
          const double di = first ? d[(i * 2 + t) * 2 + 1] : -d[(t * 2 + i) * 2 + 1];
          const double jr = Jo[(t * 2 + j) * 2], ji = Jo[(t * 2 + j) * 2 + 1];
          re += dr * jr - di * ji;
          im += dr * ji + di * jr;
        }
        v[4 + (i * 2 + j) * 2] += -2.0 * re;
        v[4 + (i * 2 + j) * 2 + 1] += -2.0 * im;
      }
  }
  block_sum_vec<12, kAsmBlock>(v, red);
  if (threadIdx.x < 12) {
    double x = v[threadIdx.x];
    if (threadIdx.x >= 4 && !unreg) x += yv + rho * (J[8 * p + threadIdx.x - 4] - bzv);
    qg[threadIdx.x] = x;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    B.G[(int64_t)f * nf + 8 * p + threadIdx.x] = qg[4 + threadIdx.x];
    A[(int64_t)nf * nf + 8 * p + threadIdx.x] = -qg[4 + threadIdx.x];
  }
  const double q00 = qg[0], q11 = qg[1], q01r = qg[2], q01i = qg[3];
  const int ncol = 8 * p + 8;
  const double *Jp = J + 8 * p;
  // 16 threads per row v of station p's 8 rows, stepping through its columns two at a time
  // (columns c, c+1 differ only in real / imaginary part: one complex product, one 16-byte store;
  // coalesced, no division)
  static_assert(kAsmBlock == 8 * 16, "one row per 16 threads");
  const int v8 = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  const int iv = v8 >> 2, jv = (v8 >> 1) & 1, rv = v8 & 1;
  double2 *row = reinterpret_cast<double2 *>(A + (int64_t)(8 * p + v8) * nf);   // nf is even
#pragma unroll 2
  for (int c = 2 * l16; c < ncol; c += 32) {
    double2 val;
    const int u = c & 7;   // even: ru = 0 at c, 1 at c+1
    const int iu = u >> 2, ju = (u >> 1) & 1;
    if (c < 8 * p) {
      // baseline (a, p): S of the pair (zero without an unflagged baseline)
      const int a = c >> 3;
      const double *Ja = J + 8 * a;
      const double ar = Ja[(iu * 2 + jv) * 2], ai = Ja[(iu * 2 + jv) * 2 + 1];
      const double br = Jp[(iv * 2 + ju) * 2], bi = Jp[(iv * 2 + ju) * 2 + 1];
      const double wr = ar * br - ai * bi, wi = ar * bi + ai * br;
      const double s2 = 2.0 * Sp[a];
      val.x = s2 * (rv == 0 ? wr : wi);
      val.y = s2 * (rv == 0 ? wi : -wr);
    } else if (iu != iv) {
      val.x = val.y = 0.0;
    } else {
      // g' = Q[jv][ju] (row index v, column index u)
      double gr, gi;
      if (jv == ju) { gr = (jv == 0) ? q00 : q11; gi = 0.0; }
      else if (jv == 0) { gr = q01r; gi = q01i; }      // Q[0][1]
      else { gr = q01r; gi = -q01i; }                  // Q[1][0] = conj(Q[0][1])
      val.x = 2.0 * ((rv == 0) ? gr : -gi);
      val.y = 2.0 * ((rv == 0) ? gi : gr);
      if (u == v8) val.x += rho + lam;
      if (u + 1 == v8) val.y += rho + lam;
    }
    row[c >> 1] = val;
  }
}

__global__ __launch_bounds__(kBlock) void k_lm_update(Problem pb, Layout L, Buffers B, int k, int unreg,
                                                      double *lm_trace, int it, int lm_iters) {
  const int f = blockIdx.x;
  LmState *st = B.lm + f;
  const bool own = k < 0;   // the subband's own direction and iteration count
  if (own) {
    if (st->phase != kPhaseLm) return;
    k = st->cur;
    it = st->itc;
    __syncthreads();   // every wavefront has read the phase before thread 0 moves it on
  } else if (k >= L.ndir[f]) {
    return;
  }
  lmd::update_dir(pb, L, B, f, k, unreg, lm_trace, it, lm_iters, own);
}

// Dense S_b per (subband, direction): entry (p, q) and (q, p) of the baseline of stations p, q,
// zero on the diagonal and for pairs without an unflagged baseline (grid: subband x direction)
__global__ __launch_bounds__(kBlock) void k_dense_s(Problem pb, Layout L, Buffers B) {
  const int f = blockIdx.x, k = blockIdx.y, N = pb.N;
  double *Sd = B.Sd + ((int64_t)f * pb.K + k) * N * N;
  const int nb = L.nb[f];
  for (int e = threadIdx.x; e < N * N; e += kBlock) {
    const int p = e / N, q = e % N;
    double v = 0.0;
    if (k < L.ndir[f] && p != q) {
      const int gb = L.bidx[((int64_t)f * N + min(p, q)) * N + max(p, q)];
      if (gb >= 0) v = B.Sb[L.sb_off[f] + (int64_t)k * nb + (gb - L.bl_off[f])];
    }
    Sd[e] = v;
  }
}

// Whether every subband has finished its local step after the current LM iteration (*flag = 1,
// else 0), each subband on its own direction: it is done, or its run ends now (stopping rule or
// last LM iteration) and that run is the last direction of the last sweep.  Launched right after
// the solve: the stopping rule needs only the step's predicted decrease and the objective before
// it (k_lm_update applies the same test), so the host can enqueue the next step while the trial
// point and the update still run.
__global__ __launch_bounds__(kBlock) void k_lm_stopped(Problem pb, Layout L, Buffers B, int *flag,
                                                       int lm_iters, int sweeps) {
  int running = 0;
  for (int f = threadIdx.x; f < pb.P; f += kBlock) {
    const LmState &st = B.lm[f];
    if (st.phase == kPhaseFinished) continue;
    const bool stops = st.done || (st.chol_ok && pb.lm_tol > 0.0 && st.ell <= pb.lm_tol * st.F);
    const bool ends = st.phase == kPhaseLm && (stops || st.itc + 1 >= lm_iters);
    const bool last = st.cur + 1 >= L.ndir[f] && st.sweep + 1 >= sweeps;
    running |= (ends && last) ? 0 : 1;
  }
  running = __syncthreads_or(running);
  if (threadIdx.x == 0) *flag = running ? 0 : 1;
}

// Start of a local step whose subbands move on their own: no direction yet, first sweep
__global__ void k_dir_reset(Problem pb, Buffers B) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= pb.P) return;
  LmState *st = B.lm + f;
  st->cur = -1;
  st->itc = 0;
  st->sweep = 0;
  st->phase = kPhaseAdvance;
}

}  // namespace

hipError_t launch_dense_s(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_s, dim3(pb.P, pb.K), dim3(kBlock), 0, s, pb, L, B);
  return hipGetLastError();
}

hipError_t launch_lm_stopped(const Problem &pb, const Layout &L, const Buffers &B, int *flag,
                             int lm_iters, int sweeps, hipStream_t s) {
  hipLaunchKernelGGL(k_lm_stopped, dim3(1), dim3(kBlock), 0, s, pb, L, B, flag, lm_iters, sweeps);
  return hipGetLastError();
}

hipError_t launch_dir_reset(const Problem &pb, const Buffers &B, hipStream_t s) {
  hipLaunchKernelGGL(k_dir_reset, dim3((pb.P + 63) / 64), dim3(64), 0, s, pb, B);
  return hipGetLastError();
}

hipError_t launch_lm_begin(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                           hipStream_t s, int sweeps) {
  hipLaunchKernelGGL(k_lm_begin, dim3(pb.P), dim3(kBlock), 0, s, pb, L, B, k, unreg, sweeps);
  return hipGetLastError();
}

hipError_t launch_assemble(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(pb.P, pb.N + 1), dim3(kAsmBlock), 0, s, pb, L, B, k, unreg);
  return hipGetLastError();
}

hipError_t launch_lm_update_tr(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                               double *lm_trace, int it, int lm_iters, hipStream_t s) {
  hipLaunchKernelGGL(k_lm_update, dim3(pb.P), dim3(kBlock), 0, s, pb, L, B, k, unreg, lm_trace, it,
                     lm_iters);
  return hipGetLastError();
}

}  // namespace calib
