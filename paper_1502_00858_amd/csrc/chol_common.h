// Device pieces shared by the two Cholesky solvers of the damped normal equations
// (chol_kernel.hip: one workgroup per matrix; chol_blocked.hip: panel launches spread over many
// workgroups per matrix): MFMA tile helpers, the 16x16 diagonal-tile factorisation with its
// inverse, and the back substitution that finishes the Levenberg-Marquardt step.
#pragma once

#include "calib_internal.h"

namespace calib {
namespace chol {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kWaves = 8;
constexpr int kColsPerThread = 2;   // back substitution: nf <= kColsPerThread * kThreads
constexpr int kThreads = 64 * kWaves;

__device__ inline double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// The accumulator element r of lane l of v_mfma_f64_16x16x4f64 holds D[4r + l/16][l%16].
__device__ inline d4 load_tile(const double *A, int ld, int I, int J, int lane) {
  d4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = A[(int64_t)(I * 16 + 4 * r + (lane >> 4)) * ld + J * 16 + (lane & 15)];
  return v;
}
__device__ inline void store_tile(double *A, int ld, int I, int J, int lane, d4 v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) A[(int64_t)(I * 16 + 4 * r + (lane >> 4)) * ld + J * 16 + (lane & 15)] = v[r];
}

__device__ inline void load4(const double *p, double &a0, double &a1, double &a2, double &a3) {
  const double2 x = reinterpret_cast<const double2 *>(p)[0];
  const double2 y = reinterpret_cast<const double2 *>(p)[1];
  a0 = x.x; a1 = x.y; a2 = y.x; a3 = y.y;
}

// 1/sqrt(d) for d > 0: the hardware estimate v_rsq_f64 (about 2^-29 relative) refined by two
// Newton-Raphson steps y <- y + y (1 - d y^2) / 2, which square the relative error each time.
__device__ inline double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// 1/d for d != 0: the hardware estimate v_rcp_f64 refined by two Newton-Raphson steps
// y <- y + y (1 - d y), which square the relative error each time.
__device__ inline double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-d, y, 1.0), y);
  return y;
}

// Inverse of a 16x16 lower-triangular tile T (row-major in LDS, leading dimension 16, 1/T_ii in
// the diagonal slots, entries above the diagonal never read) by forward substitution on one
// wavefront: lane c < 16 solves T x = e_c with four partial sums per row, the next row of T
// prefetched while the current one is used.  The inverse (row-major) goes to out_lds (which may
// be T itself: every read of T precedes the first write) and to out_global, each when not null.
__device__ inline void tri_inverse16(const double *T, double *out_lds, double *out_global, int lane) {
  double x[16], row[16], nxt[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) row[m] = (m == 0) ? T[0] : 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i + 1 < 16) {
#pragma unroll
      for (int m = 0; m <= i + 1; ++m) nxt[m] = T[(i + 1) * 16 + m];
    }
    double p[4] = {(i == lane) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < i; ++m) p[m & 3] -= row[m] * x[m];
    x[i] = ((p[0] + p[1]) + (p[2] + p[3])) * row[i];
    __asm__ __volatile__("" : "+v"(x[i]) :: "memory");
#pragma unroll
    for (int m = 0; m < 16; ++m) row[m] = nxt[m];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (out_lds) out_lds[i * 16 + lane] = x[i];
      if (out_global) out_global[i * 16 + lane] = x[i];
    }
  }
}

// One full wavefront factors the 16x16 SPD tile D (row-major, leading dimension ld, lower
// triangle read) and inverts the factor.  Lane i < 16 keeps row i of the reduced matrix; every
// lane also keeps the whole reduced diagonal (dg, identical in all lanes), so the pivot of each
// column is at hand without an exchange.  Column c of L is exchanged through the LDS scratch
// xch (32 doubles; a wavefront's LDS accesses complete in order), no value goes through scalar
// registers, and each finished column goes to inv at once with 1/L_ii in the diagonal slot of
// row i.  The inverse (tri_inverse16) is written to inv (16x16 row-major, LDS) and, when Li_out
// is not null, to Li_out.  Straight-line code (no early exit); a non-positive or non-finite pivot
// only makes the result false (wave-uniform).  The empty asm statements emit no instruction:
// they pin values and LDS accesses to their column so that the unrolled loop keeps few registers
// live.
__device__ inline bool factor16(const double *D, int ld, double *inv, double *xch, double *Li_out,
                                int lane) {
  double a[16], dg[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = (lane < 16 && c <= lane) ? D[lane * ld + c] : 0.0;
    dg[c] = D[c * ld + c];
  }
  int okv = 1;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const double d = dg[c];
    okv &= (d > 0.0 && isfinite(d)) ? 1 : 0;
    const double rl = rsqrt_nr(fmax(d, 1e-300));
    const double lv = (lane > c) ? a[c] * rl : 0.0;
    if (lane < 16) {
      xch[16 + lane] = lv;
      inv[lane * 16 + c] = (lane == c) ? rl : lv;   // finished column c of row lane
    }
    __builtin_amdgcn_wave_barrier();
    // entries right of a row's diagonal also change here; they are never read
#pragma unroll
    for (int c2 = c + 1; c2 < 16; ++c2) {
      const double l2 = xch[16 + c2];
      a[c2] = a[c2] - lv * l2;
      dg[c2] = dg[c2] - l2 * l2;
    }
#pragma unroll
    for (int c2 = c + 1; c2 < 16; ++c2) __asm__ __volatile__("" : "+v"(a[c2]), "+v"(dg[c2]));
    __asm__ __volatile__("" : "+v"(okv) :: "memory");
  }
  const bool ok = okv != 0;
  if (ok) {
    __builtin_amdgcn_wave_barrier();
    tri_inverse16(inv, inv, Li_out, lane);
  }
  return ok;
}

// Back substitution L^T delta = y of a factored augmented matrix A (row nf holds y^T, the
// strictly-lower tiles hold L, Li the inverses of the diagonal tiles), then delta, the predicted
// decrease ell = delta.(lambda delta - G)/2, the trial point and chol_ok.  All kThreads threads
// of the workgroup; tb, xb: 16 doubles of LDS each; red: kWaves doubles of LDS.
__device__ inline void backsub_tail(const Problem &pb, const Buffers &B, int f, int k,
                                    const double *A, const double *Li, double *tb, double *xb,
                                    double *red) {
  const int nf = pb.nf, nct = nf >> 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  LmState *st = B.lm + f;
  // thread tid owns columns tid + u * kThreads
  double t[kColsPerThread], lc[kColsPerThread][16], ln[kColsPerThread][16];
#pragma unroll
  for (int u = 0; u < kColsPerThread; ++u) {
    const int c = tid + u * kThreads;
    t[u] = (c < nf) ? A[(int64_t)nf * nf + c] : 0.0;
    const int j0 = nf - 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) ln[u][r] = (c < j0) ? A[(int64_t)(j0 + r) * nf + c] : 0.0;
  }
  double lin[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) lin[i] = (tid < 16) ? Li[(nct - 1) * 256 + i * 16 + tid] : 0.0;
  for (int jb = nct - 1; jb >= 0; --jb) {
    const int j0 = jb * 16;
#pragma unroll
    for (int u = 0; u < kColsPerThread; ++u) {
      const int c = tid + u * kThreads;
#pragma unroll
      for (int r = 0; r < 16; ++r) lc[u][r] = ln[u][r];
      if (jb > 0) {
        const int j1 = j0 - 16;
#pragma unroll
        for (int r = 0; r < 16; ++r) ln[u][r] = (c < j1) ? A[(int64_t)(j1 + r) * nf + c] : 0.0;
      }
      if (c >= j0 && c < j0 + 16) tb[c - j0] = t[u];
    }
    __syncthreads();
    if (tid < 16) {
      // x = L_jj^-T t_blk: x_r = sum_i (L_jj^-1)[i][r] t_i; the next block's column prefetched
      double lic[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) lic[i] = lin[i];
      if (jb > 0) {
#pragma unroll
        for (int i = 0; i < 16; ++i) lin[i] = Li[(jb - 1) * 256 + i * 16 + tid];
      }
      double x = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) x += lic[i] * tb[i];
      xb[tid] = x;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kColsPerThread; ++u) {
      const int c = tid + u * kThreads;
      if (c < j0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) t[u] -= lc[u][r] * xb[r];
      } else if (c < j0 + 16) {
        t[u] = xb[c - j0];
      }
    }
  }
  // delta, predicted decrease ell = delta.(lambda delta - G)/2, trial point
  const double lam = st->lambda;
  const int n8 = 8 * pb.N;
  double ell = 0.0;
#pragma unroll
  for (int u = 0; u < kColsPerThread; ++u) {
    const int c = tid + u * kThreads;
    if (c < n8) {
      const double g = B.G[(int64_t)f * nf + c];
      ell += t[u] * (lam * t[u] - g);
      B.delta[(int64_t)f * nf + c] = t[u];
      B.Jtrial[(int64_t)f * n8 + c] = B.J[((int64_t)f * pb.K + k) * n8 + c] + t[u];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ell += __shfl_xor(ell, o, 64);
  if (lane == 0) red[w] = ell;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int i = 0; i < kWaves; ++i) sum += red[i];
    st->ell = 0.5 * sum;
    st->chol_ok = 1;
  }
}


}  // namespace chol
}  // namespace calib
