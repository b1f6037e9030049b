// Fusion-centre kernels (steps D2/D3 of Section 3) and bookkeeping, all FP64.
//
//   basis_setup : b_l(f) = ((f - f0)/f0)^(l-1) (the example polynomial of Section 3) and, per
//                 direction, the least-squares operator W_k = R^-1 Q^T of the basis matrix of the
//                 subbands that carry the direction (thin QR by twice-iterated classical
//                 Gram-Schmidt).  Z_k = W_k (J + Y/rho) equals the closed-form minimiser
//                 (sum b b^T)^+ sum b kron (Y + rho J) / rho of Section 3 when the basis matrix
//                 has full column rank (the paper's condition P >= F).
//   gpa         : first-iteration alignment of the unitary ambiguity (Section 3,
//                 initialisation): generalised Procrustes to the mean over subbands.
//   z_fit       : Z_k per direction and the dual-residual partials.
//   y_update    : B_f Z_k, Y_fk += rho_k (J_fk - B_f Z_k) (minimisation M3) and primal partials
//                 (and, except on the alignment's iteration, the trace row's penalty partials).
//   residuals   : primal and dual residuals of Section 4.1 averaged over (f, k) and k, and the
//                 trace row's data cost and augmented Lagrangian.
#include "calib_internal.h"
#include "wave_reduce.h"
#include "device_math.h"

namespace calib {

namespace {


template <int NV>
__device__ inline void block_sum_vec(double *v, double (*red)[kBlock / 64]) {
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
    for (int j = 0; j < kBlock / 64; ++j) s += red[i][j];
    v[i] = s;
  }
  __syncthreads();
}

// one thread per direction
__global__ void k_basis_setup(int P, int Q, int K, const double *freq, double f0,
                              const int32_t *ndir, double *basis, double *fitw, int *rank_fail) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0)
    for (int f = 0; f < P; ++f) {
      const double x = (freq[f] - f0) / f0;
      double v = 1.0;
      for (int l = 0; l < Q; ++l) { basis[f * Q + l] = v; v *= x; }
    }
  if (k >= K) return;
  double *W = fitw + (int64_t)k * Q * P;   // row l = column l of the basis matrix, then of Q
  double R[8][8];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) R[i][j] = 0.0;
  for (int l = 0; l < Q; ++l)
    for (int f = 0; f < P; ++f) {
      const double x = (freq[f] - f0) / f0;
      double v = 1.0;
      for (int e = 0; e < l; ++e) v *= x;
      W[l * P + f] = (ndir[f] > k) ? v : 0.0;
    }
  for (int l = 0; l < Q; ++l) {
    double n0 = 0.0;
    for (int f = 0; f < P; ++f) n0 += W[l * P + f] * W[l * P + f];
    n0 = sqrt(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < l; ++j) {
        double r = 0.0;
        for (int f = 0; f < P; ++f) r += W[j * P + f] * W[l * P + f];
        R[j][l] += r;
        for (int f = 0; f < P; ++f) W[l * P + f] -= r * W[j * P + f];
      }
    double nrm = 0.0;
    for (int f = 0; f < P; ++f) nrm += W[l * P + f] * W[l * P + f];
    nrm = sqrt(nrm);
    if (!(nrm > 1e-12 * n0)) { atomicOr(rank_fail, 1); return; }
    R[l][l] = nrm;
    for (int f = 0; f < P; ++f) W[l * P + f] /= nrm;
  }
  for (int f = 0; f < P; ++f) {
    double w[8];
    for (int l = Q - 1; l >= 0; --l) {
      double s = W[l * P + f];
      for (int j = l + 1; j < Q; ++j) s -= R[l][j] * w[j];
      w[l] = s / R[l][l];
    }
    for (int l = 0; l < Q; ++l) W[l * P + f] = w[l];
  }
}

// Trace row's data cost sum_f g_f (from the tile partials of the final residual) and augmented
// Lagrangian sum_f [g_f + sum_k Re tr(Y^H (J - BZ)) + rho_k/2 ||J - BZ||^2]: per-subband cost and
// per-(subband, direction) penalty partials, which k_residuals adds in a fixed order.  Taken here
// when the first iteration's alignment runs between the local step and the Y update; otherwise
// k_y_update takes them from the J, Y and B_f Z it reads anyway.
__device__ inline double *cost_partials(const Problem &pb, const Buffers &B) {
  return B.scratch + (int64_t)pb.P * pb.K + (int64_t)pb.K * kZChunks;
}
__device__ inline double *penalty_partials(const Problem &pb, const Buffers &B) {
  return cost_partials(pb, B) + pb.P;
}

__device__ inline double subband_cost_sum(const Layout &L, const Buffers &B, int f) {
  double v = 0.0;
  for (int t = L.tile_off[f] + threadIdx.x; t < L.tile_off[f + 1]; t += kBlock) v += B.cost_part[t];
  return v;
}

// one workgroup per subband
__global__ __launch_bounds__(kBlock) void k_penalty_part(Problem pb, Layout L, Buffers B) {
  __shared__ double red[1][kBlock / 64];
  const int f = blockIdx.x, n8 = 8 * pb.N, Kf = L.ndir[f];
  double v[1] = {subband_cost_sum(L, B, f)};
  block_sum_vec<1>(v, red);
  if (threadIdx.x == 0) cost_partials(pb, B)[f] = v[0];
  for (int k = 0; k < pb.K; ++k) {   // the directions f carries; zero for the others
    const int64_t o = ((int64_t)f * pb.K + k) * n8;
    double pen[1] = {0.0};
    if (k < Kf)
      for (int e = threadIdx.x; e < n8; e += kBlock) {
        const double d = B.J[o + e] - B.BZ[o + e];
        pen[0] += B.Y[o + e] * d + 0.5 * B.rho[k] * d * d;
      }
    block_sum_vec<1>(pen, red);
    if (threadIdx.x == 0) penalty_partials(pb, B)[(int64_t)f * pb.K + k] = pen[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_subband_cost(Problem pb, Layout L, Buffers B, double *out) {
  __shared__ double red[1][kBlock / 64];
  const int f = blockIdx.x;
  double v[1] = {0.0};
  for (int t = L.tile_off[f] + threadIdx.x; t < L.tile_off[f + 1]; t += kBlock) v[0] += B.cost_part[t];
  block_sum_vec<1>(v, red);
  if (threadIdx.x == 0) out[f] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_gpa(Problem pb, Layout L, Buffers B, int rounds) {
  extern __shared__ double ref[];   // [N*8]
  __shared__ double red[8][kBlock / 64];
  __shared__ double U[8];
  const int k = blockIdx.x, N = pb.N, P = pb.P;
  int cnt = 0, mid = -1;
  for (int f = 0; f < P; ++f) cnt += (L.ndir[f] > k);
  if (cnt == 0) return;
  for (int f = 0, c = 0; f < P; ++f)
    if (L.ndir[f] > k) { if (c == cnt / 2) mid = f; ++c; }
  for (int e = threadIdx.x; e < 8 * N; e += kBlock)
    ref[e] = B.J[((int64_t)mid * pb.K + k) * N * 8 + e];
  __syncthreads();
  for (int r = 0; r < rounds; ++r) {
    for (int f = 0; f < P; ++f) {
      if (L.ndir[f] <= k) continue;
      double *Jf = B.J + ((int64_t)f * pb.K + k) * N * 8;
      // A = J_f^H ref = sum_p J_fp^H ref_p
      double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int p = threadIdx.x; p < N; p += kBlock) {
        const double *x = Jf + 8 * p, *y = ref + 8 * p;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int t = 0; t < 2; ++t) {
              const double xr = x[(t * 2 + i) * 2], xi = -x[(t * 2 + i) * 2 + 1];
              const double yr = y[(t * 2 + j) * 2], yi = y[(t * 2 + j) * 2 + 1];
              v[(i * 2 + j) * 2] += xr * yr - xi * yi;
              v[(i * 2 + j) * 2 + 1] += xr * yi + xi * yr;
            }
      }
      block_sum_vec<8>(v, red);
      if (threadIdx.x == 0) polar2(v, U);
      __syncthreads();
      for (int p = threadIdx.x; p < N; p += kBlock) {
        double x[8], y[8];
        for (int e = 0; e < 8; ++e) x[e] = Jf[8 * p + e];
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < 2; ++t) {
              const double xr = x[(i * 2 + t) * 2], xi = x[(i * 2 + t) * 2 + 1];
              const double ur = U[(t * 2 + j) * 2], ui = U[(t * 2 + j) * 2 + 1];
              re += xr * ur - xi * ui;
              im += xr * ui + xi * ur;
            }
            y[(i * 2 + j) * 2] = re;
            y[(i * 2 + j) * 2 + 1] = im;
          }
        for (int e = 0; e < 8; ++e) Jf[8 * p + e] = y[e];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < 8 * N; e += kBlock) {
      double s = 0.0;
      for (int f = 0; f < P; ++f)
        if (L.ndir[f] > k) s += B.J[((int64_t)f * pb.K + k) * N * 8 + e] / cnt;
      ref[e] = s;
    }
    __syncthreads();
  }
}

// grid (K, kZChunks) of one wavefront each: Z_k = W_k (J + Y/rho) for 64 of the direction's 8N
// real Jones parameters (N <= 128), one per lane, the subbands taken in order in batches of kF.
// Per block of 64 subbands the block's fit weights go to LDS with one coalesced load per basis
// term and the subbands carrying the direction to a wave-uniform bit mask (per-subband scalar loads
// would each wait on their own).  The next batch's J and Y are requested before the current one
// is summed, and the old Z before anything (the workgroup is one wavefront, whose LDS accesses
// are ordered without a barrier that would wait for those loads).  The chunk's part of
// ||Z_new - Z_old||^2 goes to the dual-residual partials (chunks past 8N write zero).
__global__ __launch_bounds__(64) void k_z_fit(Problem pb, Layout L, Buffers B) {
  __shared__ __align__(16) double sw[64][8];   // [subband of the block][basis term]
  if (B.rank_fail && *B.rank_fail) return;
  const int k = blockIdx.x, c = blockIdx.y, N = pb.N, P = pb.P, Q = pb.Q, t = threadIdx.x;
  double *dz_out = B.scratch + (int64_t)pb.P * pb.K + (int64_t)k * kZChunks + c;
  if (c * 64 >= 8 * N) {
    if (t == 0) *dz_out = 0.0;
    return;
  }
  const int e = c * 64 + t;
  const bool live = e < 8 * N;
  const int ec = min(e, 8 * N - 1);   // lanes past 8N load in bounds and store nothing
  const double rho = B.rho[k];
  const double *W = B.fitw + (int64_t)k * Q * P;
  constexpr int kF = 16;
  static_assert(64 % kF == 0, "a batch of subbands stays inside its block");
  double zo[8], z[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    zo[l] = B.Z[((int64_t)k * Q + min(l, Q - 1)) * N * 8 + ec];
    z[l] = 0.0;
  }
  auto fetch = [&](int b, double *jj, double *yy) {
#pragma unroll
    for (int u = 0; u < kF; ++u) {
      const int64_t o = ((int64_t)min(b * kF + u, P - 1) * pb.K + k) * N * 8 + ec;
      jj[u] = B.J[o];
      yy[u] = B.Y[o];
    }
  };
  const int nbatch = (P + kF - 1) / kF;
  double jv[kF], yv[kF], jn[kF], yn[kF];
  uint64_t mask = 0;
  fetch(0, jv, yv);
  for (int b = 0; b < nbatch; ++b) {
    const int fb = (b * kF) & ~63, f0 = b * kF - fb;
    if (f0 == 0) {   // a new block of 64 subbands: its weights and carrying mask
      const int fl = fb + t, fc = min(fl, P - 1);
      const bool carried = fl < P && L.ndir[fc] > k;
      double wl[8];
#pragma unroll
      for (int l = 0; l < 8; ++l) {   // terms past Q repeat the last one and are never stored
        const double w = W[min(l, Q - 1) * P + fc];
        wl[l] = carried ? w : 0.0;
      }
      wave_lds_sync();   // the previous block's weights have been read
#pragma unroll
      for (int l = 0; l < 8; ++l) sw[t][l] = wl[l];
      mask = __ballot(carried);
      wave_lds_sync();
    }
    if (b + 1 < nbatch) fetch(b + 1, jn, yn);
#pragma unroll
    for (int u = 0; u < kF; ++u) {   // f0 + u < 64: kF divides 64
      const int f = f0 + u;
      const double x0 = (rho > 0.0) ? jv[u] + yv[u] / rho : jv[u];
      const double x = ((mask >> f) & 1) ? x0 : 0.0;   // past the last subband or not carrying k
#pragma unroll
      for (int l = 0; l < 8; ++l) z[l] += sw[f][l] * x;
    }
#pragma unroll
    for (int u = 0; u < kF; ++u) {
      jv[u] = jn[u];
      yv[u] = yn[u];
    }
  }
  double dz = 0.0;
  if (live)
#pragma unroll
    for (int l = 0; l < 8; ++l)
      if (l < Q) {
        const double d = z[l] - zo[l];
        dz += d * d;
        B.Z[((int64_t)k * Q + l) * N * 8 + e] = z[l];
      }
  dz = wave_sum(dz);
  if (t == 0) *dz_out = dz;
}

// grid (P, K): B_f Z_k, dual ascent, primal partial ||J - BZ||^2; with with_penalty also the
// trace row's partials of k_penalty_part, from J and the old Y and B_f Z before they are replaced
__global__ __launch_bounds__(kBlock) void k_y_update(Problem pb, Layout L, Buffers B, int with_penalty) {
  __shared__ double red[3][kBlock / 64];
  if (B.rank_fail && *B.rank_fail) return;
  const int f = blockIdx.x, k = blockIdx.y, N = pb.N, Q = pb.Q;
  const int64_t slot = (int64_t)f * pb.K + k;
  if (with_penalty && k == 0) {   // every subband carries direction 0
    double v[1] = {subband_cost_sum(L, B, f)};
    block_sum_vec<1>(v, red);
    if (threadIdx.x == 0) cost_partials(pb, B)[f] = v[0];
  }
  if (k >= L.ndir[f]) {
    if (threadIdx.x == 0) {
      B.scratch[slot] = -1.0;
      if (with_penalty) penalty_partials(pb, B)[slot] = 0.0;
    }
    return;
  }
  const double rho = B.rho[k];
  double bf[8];   // the subband's basis row, read once (the stores below could alias it)
#pragma unroll
  for (int l = 0; l < 8; ++l) bf[l] = l < Q ? B.basis[f * Q + l] : 0.0;
  double pr = 0.0, pen = 0.0;
  for (int e = threadIdx.x; e < 8 * N; e += kBlock) {
    double bz = 0.0;
#pragma unroll
    for (int l = 0; l < 8; ++l)
      if (l < Q) bz += bf[l] * B.Z[((int64_t)k * Q + l) * N * 8 + e];
    const int64_t o = slot * N * 8 + e;
    const double j = B.J[o], y = B.Y[o];
    if (with_penalty) {
      const double d = j - B.BZ[o];
      pen += y * d + 0.5 * rho * d * d;
    }
    B.BZ[o] = bz;
    const double t = j - bz;
    B.Y[o] = y + rho * t;
    pr += t * t;
  }
  double v[2] = {pr, pen};
  block_sum_vec<2>(v, red);
  if (threadIdx.x == 0) {
    B.scratch[slot] = v[0];
    if (with_penalty) penalty_partials(pb, B)[slot] = v[1];
  }
}

// Trace row of the current iteration: primal and dual residual norms from the per-(subband,
// direction) and per-direction partials, and (with_penalty) the data cost and augmented Lagrangian
// from the per-subband cost and per-(subband, direction) penalty partials; 64 threads take strided
// shares, summed in a
// fixed order. Advances the iteration counter, so that a replayed graph writes the next row.
__global__ __launch_bounds__(64) void k_residuals(Problem pb, Buffers B, int with_penalty) {
  __shared__ double sg[64], sa[64], sps[64], sdz[kMaxDirs];
  __shared__ int spc[64];
  const int t = threadIdx.x;
  const int64_t PK = (int64_t)pb.P * pb.K;
  double g = 0.0, a = 0.0;
  if (with_penalty) {
    const double *cost = cost_partials(pb, B), *pen = penalty_partials(pb, B);
    for (int f = t; f < pb.P; f += 64) g += cost[f];
    for (int64_t i = t; i < PK; i += 64) a += pen[i];
  }
  double ps = 0.0;
  int pc = 0;
  const double pn = sqrt(4.0 * pb.N);
  for (int64_t i = t; i < PK; i += 64) {
    const double x = B.scratch[i];
    if (x >= 0.0) {
      ps += sqrt(x) / pn;
      ++pc;
    }
  }
  if (t < pb.K) {   // direction t's dual-residual partials, in chunk order
    double dz = 0.0;
    for (int c = 0; c < kZChunks; ++c) dz += B.scratch[PK + (int64_t)t * kZChunks + c];
    sdz[t] = sqrt(dz) / sqrt(4.0 * pb.Q * pb.N);
  }
  sg[t] = g;
  sa[t] = a;
  sps[t] = ps;
  spc[t] = pc;
  __syncthreads();
  if (t != 0) return;
  const int iter = B.iter[0];
  if (with_penalty) {
    g = 0.0;
    a = 0.0;
    for (int i = 0; i < 64; ++i) {
      g += sg[i];
      a += sa[i];
    }
    B.trace[4 * iter] = g;
    B.trace[4 * iter + 1] = g + a;
  }
  if (B.rank_fail && *B.rank_fail) return;
  ps = 0.0;
  pc = 0;
  for (int i = 0; i < 64; ++i) {
    ps += sps[i];
    pc += spc[i];
  }
  double ds = 0.0;
  for (int k = 0; k < pb.K; ++k) ds += sdz[k];
  B.trace[4 * iter + 2] = pc ? ps / pc : 0.0;
  B.trace[4 * iter + 3] = pb.K ? ds / pb.K : 0.0;
  B.iter[0] = iter + 1;
}

__global__ void k_set_iter(int *p, int v) {
  if (threadIdx.x == 0) p[0] = v;
}

__global__ void k_fill_identity(double *J, int64_t nblocks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblocks) return;
  double *b = J + 8 * i;
  b[0] = 1.0; b[1] = 0.0; b[2] = 0.0; b[3] = 0.0;
  b[4] = 0.0; b[5] = 0.0; b[6] = 1.0; b[7] = 0.0;
}

__global__ void k_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_zero_int(int *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_basis_setup(const Problem &pb, const double *freq, double f0, const int32_t *ndir,
                              double *basis, double *fitw, int *rank_fail, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_setup, dim3(1), dim3(64), 0, s, pb.P, pb.Q, pb.K, freq, f0, ndir, basis,
                     fitw, rank_fail);
  return hipGetLastError();
}

hipError_t launch_set_iter(const Buffers &B, int iter, hipStream_t s) {
  hipLaunchKernelGGL(k_set_iter, dim3(1), dim3(64), 0, s, B.iter, iter);
  return hipGetLastError();
}

hipError_t launch_penalty_part(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s) {
  hipLaunchKernelGGL(k_penalty_part, dim3(pb.P), dim3(kBlock), 0, s, pb, L, B);
  return hipGetLastError();
}

hipError_t launch_subband_cost(const Problem &pb, const Layout &L, const Buffers &B, double *out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_subband_cost, dim3(pb.P), dim3(kBlock), 0, s, pb, L, B, out);
  return hipGetLastError();
}

hipError_t launch_gpa(const Problem &pb, const Layout &L, const Buffers &B, int rounds, hipStream_t s) {
  const size_t lds = (size_t)pb.N * 8 * sizeof(double);
  hipLaunchKernelGGL(k_gpa, dim3(pb.K), dim3(kBlock), lds, s, pb, L, B, rounds);
  return hipGetLastError();
}

hipError_t launch_consensus(const Problem &pb, const Layout &L, const Buffers &B, int penalty,
                             hipStream_t s) {
  if (pb.N > kMaxStations) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_z_fit, dim3(pb.K, kZChunks), dim3(64), 0, s, pb, L, B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_y_update, dim3(pb.P, pb.K), dim3(kBlock), 0, s, pb, L, B,
                     penalty == kPenaltyInYUpdate ? 1 : 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residuals, dim3(1), dim3(64), 0, s, pb, B, penalty != kPenaltyNone ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill_identity(double *J, int64_t nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_identity, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0, s, J, nblocks);
  return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace calib
