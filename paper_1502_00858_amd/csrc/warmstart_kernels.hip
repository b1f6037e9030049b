// Warm start of a new solution interval from the previous one (Section 3 notes that the previous
// time slot's solutions can initialise the C-ADMM iteration); the learned form predicts the
// converged Jones matrices of the new interval from per-station features, and a per-subband cost
// comparison keeps the plain initialisation whenever the prediction is worse.
//
// Features of row (f, k, p), 32 floats:
//   [0,8)   J_prev,p                          previous interval's solution (current J)
//   [8,16)  s (J_prev,p - J_prev2,p)          its change over the last interval (0 if absent)
//   [16,24) s (-1/2) G_p Q_p^-1                block-Jacobi Gauss-Newton step of the new data at
//                                             J_prev (G_p: data gradient of station p;
//                                             Q_p = sum S_pq J_q^H J_q, the station's GN block)
//   [24,32) s (B_f Z_prev,p - J_prev,p)       previous consensus value minus J_prev (0 if absent)
// with s = kWsScale; the network output is s (J_new - J_prev) per station (8 floats).
//
// Training target of row (f, k, p): s (J_new,p U - J_prev,p) with U the unitary polar factor of
// sum_p J_new,p^H J_prev,p, i.e. the converged solution moved to the unitary gauge closest to the
// previous one (the solutions are unique only up to a common right unitary factor, Section 3).
#include "calib_internal.h"
#include "wave_reduce.h"
#include "device_math.h"

namespace calib {

namespace {


// One wavefront per row (f, k, p), four rows per workgroup: the lanes stride over station p's
// baselines (at most N - 1 <= 127) for Q_p and the data gradient G_p, a wavefront sum leaves the
// twelve sums in every lane, and lane e < 8 writes features e, 8 + e, 16 + e and 24 + e.
__global__ __launch_bounds__(kBlock) void k_ws_features(Problem pb, Layout L, Buffers B,
                                                        const double *J2, const double *BZp,
                                                        float *feat) {
  const int lane = threadIdx.x & 63, N = pb.N;
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= (int64_t)pb.P * pb.K * N) return;   // uniform per wavefront
  const int p = (int)(row % N);
  const int64_t fk = row / N;
  const int k = (int)(fk % pb.K), f = (int)(fk / pb.K);
  float *o = feat + row * kWsFeatures;
  if (k >= L.ndir[f]) {
    if (lane < kWsFeatures) o[lane] = 0.f;
    return;
  }
  const double *J = B.J + ((int64_t)f * pb.K + k) * N * 8;
  const int nb = L.nb[f];
  const double *Sb = B.Sb + L.sb_off[f] + (int64_t)k * nb - L.bl_off[f];
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = L.adj_off[f * N + p] + lane; a < L.adj_off[f * N + p + 1]; a += 64) {
    const int gb = L.adj_b[a];
    const bool first = L.adj_o[a] >= 0;
    const int q = first ? L.adj_o[a] : -1 - L.adj_o[a];
    const double S = Sb[gb];
    const double *Jo = J + 8 * q;
    v[0] += S * (Jo[0] * Jo[0] + Jo[1] * Jo[1] + Jo[4] * Jo[4] + Jo[5] * Jo[5]);
    v[1] += S * (Jo[2] * Jo[2] + Jo[3] * Jo[3] + Jo[6] * Jo[6] + Jo[7] * Jo[7]);
    v[2] += S * (Jo[0] * Jo[2] + Jo[1] * Jo[3] + Jo[4] * Jo[6] + Jo[5] * Jo[7]);
    v[3] += S * (Jo[0] * Jo[3] - Jo[1] * Jo[2] + Jo[4] * Jo[7] - Jo[5] * Jo[6]);
    const double *D = B.Dall + ((int64_t)k * pb.nbt + gb) * 8;   // D_k at the current J
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        double re = 0.0, im = 0.0;
        for (int t = 0; t < 2; ++t) {
          const double jr = Jo[(t * 2 + j) * 2], ji = Jo[(t * 2 + j) * 2 + 1];
          double dr, di;
          if (first) { dr = D[(i * 2 + t) * 2]; di = D[(i * 2 + t) * 2 + 1]; }         // D J_q
          else { dr = D[(t * 2 + i) * 2]; di = -D[(t * 2 + i) * 2 + 1]; }             // D^H J_q
          re += dr * jr - di * ji;
          im += dr * ji + di * jr;
        }
        v[4 + (i * 2 + j) * 2] += -2.0 * re;
        v[4 + (i * 2 + j) * 2 + 1] += -2.0 * im;
      }
  }
  wave_sum_vec<12>(v);   // every lane holds the sums
  if (lane >= 8) return;
  const double q00 = v[0], q11 = v[1], qr = v[2], qi = v[3];
  const double det = q00 * q11 - (qr * qr + qi * qi);
  // Q^-1 = [[q11, -q01], [-conj(q01), q00]] / det
  double inv[8] = {q11, 0.0, -qr, -qi, -qr, qi, q00, 0.0};
  const double sc = (det > 0.0) ? 1.0 / det : 0.0;
  for (int e = 0; e < 8; ++e) inv[e] *= sc;
  const double *G = v + 4;
  const double *Jp = J + 8 * p;
  const double ws = kWsScale;
  const int e = lane;
  o[e] = (float)Jp[e];
  o[8 + e] = J2 ? (float)(ws * (Jp[e] - J2[row * 8 + e])) : 0.f;
  o[24 + e] = BZp ? (float)(ws * (BZp[row * 8 + e] - Jp[e])) : 0.f;
  const int i = e >> 2, j = (e >> 1) & 1;
  double re = 0.0, im = 0.0;   // (G Q^-1)[i][j]
  for (int m = 0; m < 2; ++m) {
    const double gr = G[(i * 2 + m) * 2], gi = G[(i * 2 + m) * 2 + 1];
    const double ir = inv[(m * 2 + j) * 2], ii = inv[(m * 2 + j) * 2 + 1];
    re += gr * ir - gi * ii;
    im += gr * ii + gi * ir;
  }
  o[16 + e] = (float)(-0.5 * ws * ((e & 1) ? im : re));
}

// J <- J + delta / s for the directions each subband carries; the previous J is kept in Jsave
__global__ void k_ws_add(Problem pb, Layout L, Buffers B, const float *delta, double *Jsave) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)pb.P * pb.K * pb.N * 8;
  if (e >= n) return;
  const int k = (int)((e / ((int64_t)pb.N * 8)) % pb.K);
  const int f = (int)(e / ((int64_t)pb.K * pb.N * 8));
  Jsave[e] = B.J[e];
  if (k < L.ndir[f]) B.J[e] += (double)delta[e] / kWsScale;
}

// per subband, keep the learned initialisation only if it does not raise the data cost
__global__ void k_ws_choose(Problem pb, Buffers B, const double *cost0, const double *cost1,
                            const double *Jsave, int32_t *kept) {
  const int f = blockIdx.x;
  const bool keep = isfinite(cost1[f]) && cost1[f] <= cost0[f];
  if (!keep) {
    const int64_t n = (int64_t)pb.K * pb.N * 8, o = (int64_t)f * n;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) B.J[o + e] = Jsave[o + e];
  }
  if (kept && threadIdx.x == 0) kept[f] = keep ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_ws_target(Problem pb, Layout L, Buffers B,
                                                      const double *Jprev, float *target) {
  __shared__ double red[8][kBlock / 64];
  __shared__ double U[8];
  const int f = blockIdx.x, k = blockIdx.y, N = pb.N;
  const int64_t base = ((int64_t)f * pb.K + k) * N;
  float *o = target + base * kWsOutputs;
  if (k >= L.ndir[f]) {
    for (int e = threadIdx.x; e < N * kWsOutputs; e += kBlock) o[e] = 0.f;
    return;
  }
  const double *Jn = B.J + base * 8, *Jp = Jprev + base * 8;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // A = sum_p Jn_p^H Jp_p
  for (int p = threadIdx.x; p < N; p += kBlock) {
    const double *x = Jn + 8 * p, *y = Jp + 8 * p;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int t = 0; t < 2; ++t) {
          const double xr = x[(t * 2 + i) * 2], xi = -x[(t * 2 + i) * 2 + 1];   // conj(Jn[t][i])
          const double yr = y[(t * 2 + j) * 2], yi = y[(t * 2 + j) * 2 + 1];
          v[(i * 2 + j) * 2] += xr * yr - xi * yi;
          v[(i * 2 + j) * 2 + 1] += xr * yi + xi * yr;
        }
  }
  const int w = threadIdx.x >> 6;
  wave_sum_vec<8>(v);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) red[e][w] = v[e];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a[8];
    for (int e = 0; e < 8; ++e) a[e] = red[e][0] + red[e][1] + red[e][2] + red[e][3];
    polar2(a, U);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < N; p += kBlock) {
    const double *x = Jn + 8 * p, *y = Jp + 8 * p;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        double re = 0.0, im = 0.0;
        for (int t = 0; t < 2; ++t) {
          const double xr = x[(i * 2 + t) * 2], xi = x[(i * 2 + t) * 2 + 1];
          const double ur = U[(t * 2 + j) * 2], ui = U[(t * 2 + j) * 2 + 1];
          re += xr * ur - xi * ui;
          im += xr * ui + xi * ur;
        }
        o[p * kWsOutputs + (i * 2 + j) * 2] = (float)(kWsScale * (re - y[(i * 2 + j) * 2]));
        o[p * kWsOutputs + (i * 2 + j) * 2 + 1] = (float)(kWsScale * (im - y[(i * 2 + j) * 2 + 1]));
      }
  }
}

}  // namespace

hipError_t launch_ws_target(const Problem &pb, const Layout &L, const Buffers &B, const double *Jprev,
                            float *target, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_target, dim3(pb.P, pb.K), dim3(kBlock), 0, s, pb, L, B, Jprev, target);
  return hipGetLastError();
}

hipError_t launch_ws_features(const Problem &pb, const Layout &L, const Buffers &B,
                              const double *J2, const double *BZp, float *feat, hipStream_t s) {
  const int64_t rows = (int64_t)pb.P * pb.K * pb.N, per = kBlock / 64;
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ws_features, dim3((unsigned)((rows + per - 1) / per)), dim3(kBlock), 0, s, pb, L, B, J2,
                     BZp, feat);
  return hipGetLastError();
}

hipError_t launch_ws_add(const Problem &pb, const Layout &L, const Buffers &B, const float *delta,
                         double *Jsave, hipStream_t s) {
  const int64_t n = (int64_t)pb.P * pb.K * pb.N * 8;
  hipLaunchKernelGGL(k_ws_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pb, L, B, delta, Jsave);
  return hipGetLastError();
}

hipError_t launch_ws_choose(const Problem &pb, const Buffers &B, const double *cost0,
                            const double *cost1, const double *Jsave, int32_t *kept, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_choose, dim3(pb.P), dim3(kBlock), 0, s, pb, B, cost0, cost1, Jsave, kept);
  return hipGetLastError();
}

}  // namespace calib
