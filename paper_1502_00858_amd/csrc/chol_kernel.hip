// Batched FP64 Cholesky factorisation and solve of the damped Gauss-Newton normal equations
// (H_GN + (rho + lambda) I) delta = -G of the Levenberg-Marquardt step, one workgroup of
// 8 wavefronts per subband (256-register budget: no spills).
//
// The matrix is the lower triangle of a row-major npad x nf array (nf = 8N rounded up to 16,
// identity on padded columns) whose row nf holds -G^T, so the forward substitution L y = -G is
// carried out by the factorisation itself (row nf of the factor is y^T).  Left-looking over
// 16-column panels:
//   1. every 16x16 tile (I, j) of panel j, I >= j, is updated with
//      A[I,j] - sum_{k<j} L[I,k] L[j,k]^T on v_mfma_f64_16x16x4f64, operands read from L2; the
//      k range is split across wavefronts when the panel has fewer tiles than wavefronts and the
//      partial tiles are summed in a fixed order (run-to-run deterministic);
//   2. one wavefront factors the diagonal tile and forms its inverse L_jj^-1;
//   3. the tiles below are finished as L[I,j] = A'[I,j] L_jj^-T (an MFMA product).
// The back substitution L^T delta = y runs 16 rows at a time with the stored L_jj^-1, two
// columns per thread, the next block of L prefetched into registers.
#include "chol_common.h"

namespace calib {

namespace {

using namespace chol;
constexpr int kCholWaves = kWaves;
constexpr int kCholThreads = kThreads;
constexpr int kGroup = 3;           // panel tiles a wavefront updates together

__global__ __launch_bounds__(kCholThreads) void k_chol_solve(Problem pb, Buffers B, int k,
                                                             const int32_t *ndir) {
  __shared__ double part[kCholWaves][256];
  __shared__ double diag[256];
  __shared__ double inv[256];
  __shared__ double xch[32];
  __shared__ double tb[16];
  __shared__ double xb[16];
  __shared__ double red[kCholWaves];
  __shared__ int fail;
  const int f = blockIdx.x;
  if (!lm_live(B, ndir, f, k)) return;
  k = lm_dir(B, f, k);
  const int nf = pb.nf, npad = pb.npad, nct = nf >> 4, nrt = npad >> 4;
  double *A = B.H + (int64_t)f * npad * nf;
  double *Li = B.Linv + (int64_t)f * nct * 256;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront index, uniform
  const int li = lane & 15, lq = lane >> 4;
  if (tid == 0) fail = 0;
  __syncthreads();

  for (int j = 0; j < nct; ++j) {
    const int T = nrt - j;                 // row tiles of this panel
    int s = 1;                             // k-range split factor
    if (T < kCholWaves && j > 0) {
      s = kCholWaves / T;
      if (s > j) s = j;
    }
    // tile m of this wavefront is row tile t0 + m * kCholWaves (m < ntile)
    int ntile = 0, chunk = 0, kb = 0, ke = j, t0 = j + w;
    if (s == 1) {
      ntile = (w < T) ? (T - w + kCholWaves - 1) / kCholWaves : 0;
    } else if (w / s < T) {
      t0 = j + w / s;
      ntile = 1;
      chunk = w % s;
      kb = chunk * j / s;
      ke = (chunk + 1) * j / s;
    }
    // Phase 1, in groups of kGroup tiles per wavefront; the operands of k-tile kt+1 are in
    // flight while the MFMAs of k-tile kt run
    for (int g0 = 0; g0 < ntile; g0 += kGroup) {
      d4 acc[kGroup], acc2[kGroup];
#pragma unroll
      for (int g = 0; g < kGroup; ++g) acc2[g] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
        acc[g] = (g0 + g < ntile && chunk == 0) ? load_tile(A, nf, t0 + (g0 + g) * kCholWaves, j, lane)
                                                : d4{0.0, 0.0, 0.0, 0.0};
      const double *brow = A + (int64_t)(j * 16 + li) * nf + 4 * lq;
      const double *arow[kGroup];
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
        arow[g] = A + (int64_t)((t0 + (g0 + g) * kCholWaves) * 16 + li) * nf + 4 * lq;
      // k-tiles in pairs; the operands of the next pair are in flight while the MFMAs of the
      // current pair run (two k-tiles of prefetch distance hide the L2/MALL latency)
      double bn[2][4], an[2][kGroup][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kt = kb + h;
        if (kt < ke) {
          load4(brow + kt * 16, bn[h][0], bn[h][1], bn[h][2], bn[h][3]);
#pragma unroll
          for (int g = 0; g < kGroup; ++g)
            if (g0 + g < ntile) load4(arow[g] + kt * 16, an[h][g][0], an[h][g][1], an[h][g][2], an[h][g][3]);
        }
      }
      for (int kt0 = kb; kt0 < ke; kt0 += 2) {
        double b[2][4], a[2][kGroup][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int q = 0; q < 4; ++q) b[h][q] = bn[h][q];
#pragma unroll
          for (int g = 0; g < kGroup; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[h][g][q] = an[h][g][q];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kt = kt0 + 2 + h;
          if (kt < ke) {
            load4(brow + kt * 16, bn[h][0], bn[h][1], bn[h][2], bn[h][3]);
#pragma unroll
            for (int g = 0; g < kGroup; ++g)
              if (g0 + g < ntile) load4(arow[g] + kt * 16, an[h][g][0], an[h][g][1], an[h][g][2], an[h][g][3]);
          }
        }
        // independent accumulator chains back to back: tiles of the group, and two partial
        // sums per tile
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (kt0 + h < ke) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int g = 0; g < kGroup; ++g)
                if (g0 + g < ntile) {
                  if (h == 0) acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[h][g][q], b[h][q], acc[g], 0, 0, 0);
                  else acc2[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[h][g][q], b[h][q], acc2[g], 0, 0, 0);
                }
          }
        }
      }
#pragma unroll
      for (int g = 0; g < kGroup; ++g) acc[g] += acc2[g];
      if (s == 1) {
        // updated panel tiles go back to the matrix (the factor overwrites them below); the
        // diagonal tile (first tile of wavefront 0) also goes to LDS
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
          if (g0 + g < ntile) store_tile(A, nf, t0 + (g0 + g) * kCholWaves, j, lane, acc[g]);
        if (w == 0 && g0 == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) diag[(4 * r + lq) * 16 + li] = acc[0][r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) part[w][(4 * r + lq) * 16 + li] = acc[0][r];
      }
    }
    const bool owner = ntile > 0 && chunk == 0;
    if (s > 1) {
      // k-split partials of one tile, summed in a fixed order by the chunk-0 wavefront
      __syncthreads();
      if (owner) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < s; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] += part[w + c][(4 * r + lq) * 16 + li];
        store_tile(A, nf, t0, j, lane, acc);
        if (w == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) diag[(4 * r + lq) * 16 + li] = acc[r];
        }
      }
    }
    __syncthreads();
    // diagonal tile: one wavefront factors and inverts it
    if (w == 0) {
      const bool ok = factor16(diag, 16, inv, xch, Li + j * 256, lane);
      if (!ok && lane == 0) fail = 1;
    }
    __syncthreads();
    if (fail) break;
    // tiles below the diagonal: L[I,j] = A'[I,j] L_jj^-T, A' read back in the MFMA A layout
    double iv0 = inv[li * 16 + 4 * lq], iv1 = inv[li * 16 + 4 * lq + 1];
    double iv2 = inv[li * 16 + 4 * lq + 2], iv3 = inv[li * 16 + 4 * lq + 3];
#pragma unroll
    for (int m = 0; m < kCholMaxTilesPerWave; ++m) {
      const int I = t0 + m * kCholWaves;
      if (owner && m < ntile && I > j) {
        double x0, x1, x2, x3;
        load4(A + (int64_t)(I * 16 + li) * nf + j * 16 + 4 * lq, x0, x1, x2, x3);
        d4 d = {0.0, 0.0, 0.0, 0.0};
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, iv0, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, iv1, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, iv2, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(x3, iv3, d, 0, 0, 0);
        store_tile(A, nf, I, j, lane, d);
      }
    }
    __syncthreads();
  }
  LmState *st = B.lm + f;
  if (fail) {
    if (tid == 0) st->chol_ok = 0;
    return;
  }
  backsub_tail(pb, B, f, k, A, Li, tb, xb, red);
}

}  // namespace

hipError_t launch_chol_solve_nd(const Problem &pb, const Buffers &B, int k, const int32_t *ndir,
                                hipStream_t s) {
  if (pb.nf > kColsPerThread * kCholThreads || (pb.npad >> 4) > kCholWaves * kCholMaxTilesPerWave)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_solve, dim3(pb.P), dim3(kCholThreads), 0, s, pb, B, k, ndir);
  return hipGetLastError();
}

}  // namespace calib
