// Blocked FP64 Cholesky solve of the damped normal equations spread over many workgroups per
// matrix, for batches too small to fill the chip with one workgroup per matrix (c2: 32 subbands
// on 256 compute units).  Same augmented matrix as chol_kernel.hip (row nf holds -G^T, so the
// factorisation also performs the forward substitution) and the same back substitution.
//
// Right-looking over 64-column panels p (tile columns 4p .. 4p+wp-1), one launch per panel
// (grid: subband x (64-row chunks below the panel's diagonal block + 64x64 blocks of the trailing
// lower triangle)):
//   panel workgroups load the panel's diagonal block and their chunk of rows into LDS, apply the
//          pending rank-64 update of the previous panel there, and factor the block (left-looking
//          over its 16x16 tiles: diagonal tile factor + inverse on one wavefront, the tiles below
//          as MFMA products with the inverse, then the rank-16 update of the block's later tile
//          columns) - redundantly, so that no workgroup waits for another - applying the same
//          steps to their own rows: L[I, panel] = A[I, panel] L_pp^-T.  The workgroup of chunk 0
//          also keeps the diagonal tiles' inverses (for the back substitution) and the block's
//          strictly-lower tiles (in a side buffer: the other workgroups are still reading the
//          block from the matrix);
//   trailing workgroups apply the previous panel's update to the lower triangle right of the
//          panel (right-hand-side row included): A[I,K] -= sum_t L[I,t] L[K,t]^T on
//          v_mfma_f64_16x16x4f64.
// Both roles read only the previous panel's L and write disjoint regions; launch boundaries order
// the panels and nothing spins.  A 1024-thread back substitution follows.  A non-positive pivot
// sets a per-subband flag that makes the later launches skip the subband and the back
// substitution report chol_ok = 0 (and clear the flag).
#include "chol_common.h"

namespace calib {

namespace {

using namespace chol;

constexpr int kPanelTiles = 4;            // 16-column tiles per panel
constexpr int kPB = 64;                   // panel width in columns
constexpr int kLd = kPB + 1;              // LDS row stride of a 64x64 block (doubles)
constexpr int kBThreads = 256;            // panel and trail workgroups: 4 wavefronts

struct PanelGeom {
  int c0, wp, c1;                         // first tile column, tile columns, first trailing tile
};

__device__ inline PanelGeom panel_geom(int p, int nct) {
  PanelGeom g;
  g.c0 = kPanelTiles * p;
  g.wp = min(kPanelTiles, nct - g.c0);
  g.c1 = g.c0 + g.wp;
  return g;
}

// T (16x16 tile in LDS, stride kLd) <- T - X Y^T, X and Y 16x16 tiles in LDS (v_mfma operands:
// lane l supplies row l%16, columns 4(l/16)..4(l/16)+3 of X and of Y)
__device__ inline void tile_update_lds(double *T, const double *X, const double *Y, int li, int lq) {
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = T[(4 * r + lq) * kLd + li];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-X[li * kLd + 4 * lq + q], Y[li * kLd + 4 * lq + q],
                                               acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(4 * r + lq) * kLd + li] = acc[r];
}

// Trailing update of one 4x4-tile block (rb, kb) of the lower triangle that starts at tile rs:
// A[I,K] -= sum_{t in panel src} L[I,t] L[K,t]^T; each wavefront owns 2x2 tiles and has all
// operands of the panel in flight at once.
__device__ __attribute__((always_inline)) inline void trail_block(double *A, int nf, int nct, int nrt, const PanelGeom &src, int rs,
                                   int rb, int kb, int w, int lane) {
  const int li = lane & 15, lq = lane >> 4;
  const int i0 = rs + kPanelTiles * rb + 2 * (w >> 1);
  const int k0 = rs + kPanelTiles * kb + 2 * (w & 1);
  bool valid[2][2];
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int I = i0 + a, K = k0 + b;
      valid[a][b] = I < nrt && K < nct && K <= I;
      acc[a][b] = valid[a][b] ? load_tile(A, nf, I, K, lane) : d4{0.0, 0.0, 0.0, 0.0};
    }
  const bool rowok[2] = {i0 < nrt, i0 + 1 < nrt};
  const bool colok[2] = {k0 < nct, k0 + 1 < nct};
  double x[kPanelTiles][2][4], y[kPanelTiles][2][4];
#pragma unroll
  for (int t = 0; t < kPanelTiles; ++t) {
    const int tc = (src.c0 + t) * 16 + 4 * lq;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (t < src.wp && rowok[a]) load4(A + (int64_t)((i0 + a) * 16 + li) * nf + tc, x[t][a][0], x[t][a][1], x[t][a][2], x[t][a][3]);
      else x[t][a][0] = x[t][a][1] = x[t][a][2] = x[t][a][3] = 0.0;
      if (t < src.wp && colok[a]) load4(A + (int64_t)((k0 + a) * 16 + li) * nf + tc, y[t][a][0], y[t][a][1], y[t][a][2], y[t][a][3]);
      else y[t][a][0] = y[t][a][1] = y[t][a][2] = y[t][a][3] = 0.0;
    }
  }
#pragma unroll
  for (int t = 0; t < kPanelTiles; ++t) {
    if (t < src.wp) {
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x[t][a][qq], y[t][b][qq], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      if (valid[a][b]) store_tile(A, nf, i0 + a, k0 + b, lane, acc[a][b]);
}

// T (16x16 tile in LDS, stride kLd) <- T - sum_{t < wsrc} X_t Y_t^T with X_t, Y_t the 16x16 tiles
// at column offset 16t of the LDS row blocks X and Y
__device__ __attribute__((always_inline)) inline void tile_update_lds_panel(double *T, const double *X, const double *Y, int wsrc,
                                             int li, int lq) {
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = T[(4 * r + lq) * kLd + li];
#pragma unroll
  for (int t = 0; t < kPanelTiles; ++t) {
    if (t < wsrc) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-X[li * kLd + 16 * t + 4 * lq + q],
                                                   Y[li * kLd + 16 * t + 4 * lq + q], acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(4 * r + lq) * kLd + li] = acc[r];
}

// One step p of the blocked factorisation (grid: subband x (nchunk panel workgroups + trailing
// workgroups)).  Panel workgroups (blockIdx.y < nchunk, dispatched first) apply the pending
// rank-64 update of panel p-1 to their LDS copies of panel p's diagonal block and of their chunk
// of rows, then factor panel p.  Trailing workgroups apply the same update of panel p-1 to the
// lower triangle right of panel p.  Both roles only read panel p-1's L and write disjoint regions,
// so one launch per panel suffices and nothing waits across workgroups.
__global__ __launch_bounds__(kBThreads) void k_chol_panel(Problem pb, Buffers B, int k,
                                                          const int32_t *ndir, int p, double *Ld,
                                                          int *cfail) {
  __shared__ double Dl[kPB * kLd];    // the panel's diagonal block
  __shared__ double Xl[kPB * kLd];    // this workgroup's rows of the panel
  __shared__ double Pd[kPB * kLd];    // L of panel p-1 at the diagonal block's rows
  __shared__ double Px[kPB * kLd];    // L of panel p-1 at this workgroup's rows
  __shared__ double inv[256];
  __shared__ double xch[32];
  __shared__ int bad;
  const int f = blockIdx.x;
  if (k >= ndir[f] || B.lm[f].done || cfail[f]) return;
  const int nf = pb.nf, nct = nf >> 4, nrt = pb.npad >> 4;
  const PanelGeom g = panel_geom(p, nct);
  double *A = B.H + (int64_t)f * pb.npad * nf;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lq = lane >> 4;
  const PanelGeom gs = panel_geom(p > 0 ? p - 1 : 0, nct);   // source of the pending update
  const int nchunk = (nrt - g.c1 + kPanelTiles - 1) / kPanelTiles;
  if ((int)blockIdx.y >= nchunk) {
    // trailing role: the region right of panel p, rows and columns from tile g.c1
    const int bb = blockIdx.y - nchunk;
    const int nkb = (nct - g.c1 + kPanelTiles - 1) / kPanelTiles;
    const int rb = bb / nkb, kb = bb % nkb;
    if (kb > rb) return;
    trail_block(A, nf, nct, nrt, gs, g.c1, rb, kb, w, lane);
    return;
  }
  const int q = blockIdx.y;
  const int r0 = g.c1 + kPanelTiles * q;            // first row tile of this chunk
  const int nr = min(kPanelTiles, nrt - r0);
  const int wcol = 16 * g.wp, wsrc = (p > 0) ? 16 * gs.wp : 0;

  // fixed-count loops over the 64x64 footprints: each block pair's loads are all issued before
  // its first LDS store
  {
    double dv[kPB * kPB / kBThreads], xv[kPB * kPB / kBThreads];
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      dv[it] = (row < wcol && col < wcol && (col >> 4) <= (row >> 4))
                   ? A[(int64_t)(g.c0 * 16 + row) * nf + g.c0 * 16 + col] : 0.0;
      xv[it] = (row < 16 * nr && col < wcol) ? A[(int64_t)(r0 * 16 + row) * nf + g.c0 * 16 + col] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      Dl[row * kLd + col] = dv[it];
      Xl[row * kLd + col] = xv[it];
    }
  }
  if (p > 0) {
    double dv[kPB * kPB / kBThreads], xv[kPB * kPB / kBThreads];
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      dv[it] = (row < wcol && col < wsrc) ? A[(int64_t)(g.c0 * 16 + row) * nf + gs.c0 * 16 + col] : 0.0;
      xv[it] = (row < 16 * nr && col < wsrc) ? A[(int64_t)(r0 * 16 + row) * nf + gs.c0 * 16 + col] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      Pd[row * kLd + col] = dv[it];
      Px[row * kLd + col] = xv[it];
    }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  if (p > 0) {
    // pending rank-64 update of panel p-1: the diagonal block's lower tiles, then the chunk's
    int cnt = 0;
    for (int s2 = 0; s2 < g.wp; ++s2)
      for (int t2 = 0; t2 <= s2; ++t2, ++cnt)
        if ((cnt & 3) == w)
          tile_update_lds_panel(Dl + s2 * 16 * kLd + t2 * 16, Pd + s2 * 16 * kLd, Pd + t2 * 16 * kLd,
                                gs.wp, li, lq);
    for (int r = 0; r < nr; ++r)
      for (int t2 = 0; t2 < g.wp; ++t2, ++cnt)
        if ((cnt & 3) == w)
          tile_update_lds_panel(Xl + r * 16 * kLd + t2 * 16, Px + r * 16 * kLd, Pd + t2 * 16 * kLd,
                                gs.wp, li, lq);
    __syncthreads();
  }
  for (int t = 0; t < g.wp; ++t) {
    if (w == 0) {
      double *Li = (q == 0) ? B.Linv + ((int64_t)f * nct + g.c0 + t) * 256 : nullptr;
      const bool ok = factor16(Dl + t * 16 * kLd + t * 16, kLd, inv, xch, Li, lane);
      if (!ok && lane == 0) bad = 1;
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) cfail[f] = 1;
      return;
    }
    // tiles below diagonal tile t: the block's tiles (s, t), s > t, then the chunk's tiles
    const double iv0 = inv[li * 16 + 4 * lq], iv1 = inv[li * 16 + 4 * lq + 1];
    const double iv2 = inv[li * 16 + 4 * lq + 2], iv3 = inv[li * 16 + 4 * lq + 3];
    const int nbelow = g.wp - 1 - t;
    for (int m = w; m < nbelow + nr; m += 4) {
      double *T = (m < nbelow) ? Dl + (t + 1 + m) * 16 * kLd + t * 16 : Xl + (m - nbelow) * 16 * kLd + t * 16;
      const double x0 = T[li * kLd + 4 * lq], x1 = T[li * kLd + 4 * lq + 1];
      const double x2 = T[li * kLd + 4 * lq + 2], x3 = T[li * kLd + 4 * lq + 3];
      d4 d = {0.0, 0.0, 0.0, 0.0};
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, iv0, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, iv1, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, iv2, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(x3, iv3, d, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(4 * r + lq) * kLd + li] = d[r];
    }
    __syncthreads();
    // rank-16 update of the later tile columns t' > t: the block's tiles (s, t'), s >= t', then
    // the chunk's tiles
    int cnt = 0;
    for (int tp = t + 1; tp < g.wp; ++tp)
      for (int s = tp; s < g.wp; ++s, ++cnt)
        if ((cnt & 3) == w)
          tile_update_lds(Dl + s * 16 * kLd + tp * 16, Dl + s * 16 * kLd + t * 16,
                          Dl + tp * 16 * kLd + t * 16, li, lq);
    for (int r = 0; r < nr; ++r)
      for (int tp = t + 1; tp < g.wp; ++tp, ++cnt)
        if ((cnt & 3) == w)
          tile_update_lds(Xl + r * 16 * kLd + tp * 16, Xl + r * 16 * kLd + t * 16,
                          Dl + tp * 16 * kLd + t * 16, li, lq);
    __syncthreads();
  }

  {
    double *dst = Ld + ((int64_t)f * ((nct + kPanelTiles - 1) / kPanelTiles) + p) * kPB * kPB;
    double xv[kPB * kPB / kBThreads], dv[kPB * kPB / kBThreads];
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      xv[it] = Xl[row * kLd + col];
      dv[it] = Dl[row * kLd + col];
    }
#pragma unroll
    for (int it = 0; it < kPB * kPB / kBThreads; ++it) {
      const int e = tid + it * kBThreads, row = e >> 6, col = e & 63;
      if (row < 16 * nr && col < wcol) A[(int64_t)(r0 * 16 + row) * nf + g.c0 * 16 + col] = xv[it];
      if (q == 0 && row < wcol && col < wcol && (col >> 4) < (row >> 4)) dst[row * kPB + col] = dv[it];
    }
  }
}


// Back substitution L^T delta = y with one thread per column (nf <= 1024): per 16-row block,
// from the last, x_J = (L_JJ^-1)^T t_J on 16 threads, then t -= L_J^T x_J on every column left
// of the block.  The rows of L of the next block are in flight while a block is used (the
// matrix streams from memory once, so the loads are what the loop waits on).
constexpr int kBsThreads = 1024;
constexpr int kBsWaves = kBsThreads / 64;

__global__ __launch_bounds__(kBsThreads) void k_chol_backsub(Problem pb, Buffers B, int k,
                                                             const int32_t *ndir, const double *Ld,
                                                             int *cfail) {
  __shared__ double tb[2][16];
  __shared__ double xb[2][16];
  __shared__ double liS[2][256];   // L_JJ^-1 of the current and the next block
  __shared__ double red[kBsWaves];
  __shared__ int failed;
  const int f = blockIdx.x;
  if (k >= ndir[f] || B.lm[f].done) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid == 0) failed = cfail[f];
  __syncthreads();
  LmState *st = B.lm + f;
  if (failed) {
    if (tid == 0) {
      st->chol_ok = 0;
      cfail[f] = 0;
    }
    return;
  }
  const int nf = pb.nf, nct = nf >> 4;
  const int np = (nct + kPanelTiles - 1) / kPanelTiles;
  double *A = B.H + (int64_t)f * pb.npad * nf;
  const double *Li = B.Linv + (int64_t)f * nct * 256;
  // the diagonal blocks' strictly-lower tiles go back into the matrix
  const double *src = Ld + (int64_t)f * np * kPB * kPB;
  for (int e = tid; e < np * kPB * kPB; e += kBsThreads) {
    const int p = e / (kPB * kPB), row = (e / kPB) % kPB, col = e % kPB;
    const PanelGeom g = panel_geom(p, nct);
    if ((col >> 4) < (row >> 4) && (row >> 4) < g.wp)
      A[(int64_t)(g.c0 * 16 + row) * nf + g.c0 * 16 + col] = src[e];
  }
  __syncthreads();

  const int c = tid;
  double t = (c < nf) ? A[(int64_t)nf * nf + c] : 0.0;
  // rows of blocks jb (cur), jb-1 (n1) and jb-2 (n2) at this thread's column, zero where the
  // column is not left of the block
  // rows of block jb at this thread's column (zero where the column is not left of the block):
  // two buffers rotated by name, so that the next block's loads stay in flight while a block is
  // used
  double b0[16], b1[16];
  auto load_rows = [&](int jb, double (&dst)[16]) {
    const int j0 = jb * 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) dst[r] = (jb >= 0 && c < j0) ? A[(int64_t)(j0 + r) * nf + c] : 0.0;
  };
  // the last wavefront stages L_JJ^-1 of the next block in LDS from registers loaded a step
  // earlier, then loads the one after (no wave waits on a load before a barrier)
  const bool stager = w == kBsWaves - 1;
  double lireg[4];
  auto step = [&](int jb, const double (&use)[16], double (&fill)[16]) {
    const int j0 = jb * 16, buf = jb & 1;
    load_rows(jb - 1, fill);
    if (stager) {
      if (jb > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) liS[buf ^ 1][lane + 64 * u] = lireg[u];
      }
      if (jb > 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) lireg[u] = Li[(jb - 2) * 256 + lane + 64 * u];
      }
    }
    if (c >= j0 && c < j0 + 16) tb[buf][c - j0] = t;
    __syncthreads();
    if (tid < 16) {
      // x_r = sum_i (L_JJ^-1)[i][r] t_i
      double x0 = 0.0, x1 = 0.0;
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        x0 += liS[buf][i * 16 + tid] * tb[buf][i];
        x1 += liS[buf][(i + 1) * 16 + tid] * tb[buf][i + 1];
      }
      xb[buf][tid] = x0 + x1;
    }
    __syncthreads();
    if (c < j0) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        s0 += use[r] * xb[buf][r];
        s1 += use[r + 1] * xb[buf][r + 1];
      }
      t -= s0 + s1;
    } else if (c < j0 + 16) {
      t = xb[buf][c - j0];
    }
  };
  load_rows(nct - 1, b0);
  if (stager) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      liS[(nct - 1) & 1][lane + 64 * u] = Li[(nct - 1) * 256 + lane + 64 * u];
      lireg[u] = (nct > 1) ? Li[(nct - 2) * 256 + lane + 64 * u] : 0.0;
    }
  }
  for (int jb = nct - 1; jb >= 0; jb -= 2) {
    step(jb, b0, b1);
    if (jb >= 1) step(jb - 1, b1, b0);
  }
  // delta, predicted decrease ell = delta.(lambda delta - G)/2, trial point
  const double lam = st->lambda;
  const int n8 = 8 * pb.N;
  double ell = 0.0;
  if (c < n8) {
    const double gc = B.G[(int64_t)f * nf + c];
    ell = t * (lam * t - gc);
    B.delta[(int64_t)f * nf + c] = t;
    B.Jtrial[(int64_t)f * n8 + c] = B.J[((int64_t)f * pb.K + k) * n8 + c] + t;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ell += __shfl_xor(ell, o, 64);
  if (lane == 0) red[w] = ell;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int i = 0; i < kBsWaves; ++i) sum += red[i];
    st->ell = 0.5 * sum;
    st->chol_ok = 1;
  }
}

}  // namespace

int chol_blocked_panels(const Problem &pb) { return (pb.nf / 16 + kPanelTiles - 1) / kPanelTiles; }

hipError_t launch_chol_blocked(const Problem &pb, const Buffers &B, int k, const int32_t *ndir,
                               double *Ld, int *cfail, hipStream_t s) {
  const int nct = pb.nf >> 4, nrt = pb.npad >> 4;
  if (pb.nf > kBsThreads || nrt != nct + 1) return hipErrorInvalidValue;
  const int np = chol_blocked_panels(pb);
  for (int p = 0; p < np; ++p) {
    const int c1 = min(kPanelTiles * (p + 1), nct);
    const int nchunk = (nrt - c1 + kPanelTiles - 1) / kPanelTiles;
    const int nrb = (nrt - c1 + kPanelTiles - 1) / kPanelTiles;
    const int nkb = (nct - c1 + kPanelTiles - 1) / kPanelTiles;
    const int ntrail = (p > 0) ? nrb * nkb : 0;
    hipLaunchKernelGGL(k_chol_panel, dim3(pb.P, nchunk + ntrail), dim3(kBThreads), 0, s, pb, B, k,
                       ndir, p, Ld, cfail);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_chol_backsub, dim3(pb.P), dim3(kBsThreads), 0, s, pb, B, k, ndir, Ld, cfail);
  return hipGetLastError();
}

}  // namespace calib
