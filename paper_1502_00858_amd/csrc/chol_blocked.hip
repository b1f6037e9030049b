// Blocked FP64 Cholesky solve of the damped normal equations spread over many workgroups per
// matrix, for batches too small to fill the chip with one workgroup per matrix (c2: 32 subbands
// on 256 compute units).  Same augmented matrix as chol_kernel.hip (row nf holds -G^T, so the
// factorisation also performs the forward substitution) and the same back substitution.
//
// Over 64-column panels p (tile columns 4p .. 4p+wp-1), one launch per panel (grid: subband x
// (64-row chunks below the panel's diagonal block, one workgroup for the previous panel's
// diagonal block, the block rows of the next panel's column strip)):
//   panel workgroups hold the panel's diagonal block and their chunk of rows (a 128x64 stack) in
//          registers, apply the pending rank-64 update of the previous panel on MFMA, and
//          eliminate the panel's columns two at a time across the whole workgroup: the stack's
//          values of the next two columns are published in LDS, every lane forms the 2x2 pivot
//          block's elimination itself, the owners of the following pair update it first and
//          publish it, one barrier per pair, the rest of the update on MFMA inside the next pair's
//          pivot latency.  Every panel workgroup factors the diagonal block redundantly, so none
//          waits for another; the chunk rows come out as L[I, panel] = A[I, panel] L_pp^-T.  The
//          workgroup of chunk 0 keeps the block's lower tiles in a side buffer (the other
//          workgroups are still reading the block from the matrix);
//   the diagonal-block workgroup moves the previous panel's block from the side buffer into the
//          matrix and inverts its diagonal 16x16 tiles for the back substitution;
//   strip workgroups bring the next panel's column strip up to date with every panel before this
//          one (left-looking: A[I,K] -= sum_s L[I,s] L[K,s]^T on v_mfma_f64_16x16x4f64), so that
//          the next launch only has its pending rank-64 update left.
// All roles read only finished panels' L and write disjoint regions; launch boundaries order the
// panels and nothing spins.  A back substitution follows.  A non-positive pivot sets a per-subband
// flag that makes the later launches skip the subband and the back substitution report
// chol_ok = 0 (and clear the flag).
#include "chol_common.h"

namespace calib {

namespace {

using namespace chol;

constexpr int kPanelTiles = 4;            // 16-column tiles per panel
constexpr int kPB = 64;                   // panel width in columns
constexpr int kPs = kPB + 2;              // LDS row stride of the previous panel's L (16-byte rows)
constexpr int kStack = 2 * kPB;           // rows of a panel workgroup's stack: diagonal block + chunk
constexpr int kBThreads = 512;            // panel and trailing workgroups: 8 wavefronts

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

// Left-looking update of half of one 64x64 block of panel p+1's column strip (block row rb of
// the strip, whose first tile row and column is rs = 4(p+1); half h holds its tile rows 2h and
// 2h+1): A[I,K] -= sum over the source panels s < nsrc of L[I,s] L[K,s]^T (panel p's own update is
// the pending update that panel p+1's workgroups apply).  Eight wavefronts, one tile each.  Per
// source panel the workgroup stages the operands it needs once in LDS (L at its 2 tile rows and at
// the strip's 4 tile columns: 48 KB, where eight wavefronts loading their own would move 128 KB
// through the compute unit), the next panel's operands in flight in registers while the current
// one's are multiplied.  Four accumulators per tile keep consecutive products independent.
__device__ inline double2 lds2(const double *p) { return *reinterpret_cast<const double2 *>(p); }
constexpr int kSRows = 6 * 16;   // staged rows: 2 tile rows of the block half + 4 of the strip
__device__ __attribute__((always_inline)) inline void strip_half(double *A, double *lds, int nf,
                                                                 int nct, int nrt, int nsrc, int rs,
                                                                 int rb, int h, int w, int lane) {
  const int li = lane & 15, lq = lane >> 4, tid = threadIdx.x;
  const int I0 = rs + kPanelTiles * rb + 2 * h;
  const int I = I0 + (w >> 2), K = rs + (w & 3);
  const bool valid = I < nrt && K < nct && K <= I;
  d4 acc[4] = {valid ? load_tile(A, nf, I, K, lane) : d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0},
               d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
  // thread tid stages elements e = 2 tid + 2 kBThreads it (pairs of columns) of the 96 x 64 operand
  // block: rows 0-31 the block half's tile rows, rows 32-95 the strip's tile rows
  constexpr int kPer = kSRows * kPB / (2 * kBThreads);
  double2 reg[kPer];
  auto load = [&](int s) {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = 2 * tid + 2 * kBThreads * it, r = e >> 6, col = e & 63;
      const int tr = (r < 32) ? I0 + (r >> 4) : rs + ((r - 32) >> 4);   // tile row
      const int grow = (r < 32) ? 16 * I0 + r : 16 * rs + (r - 32);
      const bool ok = (r < 32) ? tr < nrt : tr < nct;
      reg[it] = ok ? *reinterpret_cast<const double2 *>(A + (int64_t)grow * nf + s * kPB + col)
                   : double2{0.0, 0.0};
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = 2 * tid + 2 * kBThreads * it, r = e >> 6, col = e & 63;
      *reinterpret_cast<double2 *>(lds + r * kPs + col) = reg[it];
    }
  };
  const double *xr = lds + (16 * (w >> 2) + li) * kPs + 4 * lq;
  const double *yr = lds + (32 + 16 * (w & 3) + li) * kPs + 4 * lq;
  load(0);
  for (int s = 0; s < nsrc; ++s) {
    stage();
    __syncthreads();
    if (s + 1 < nsrc) load(s + 1);
    if (valid) {
#pragma unroll
      for (int t = 0; t < kPanelTiles; ++t) {
        const double2 a0 = lds2(xr + 16 * t), a1 = lds2(xr + 16 * t + 2);
        const double2 b0 = lds2(yr + 16 * t), b1 = lds2(yr + 16 * t + 2);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0.x, b0.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0.y, b0.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1.x, b1.x, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1.y, b1.y, acc[3], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (valid) store_tile(A, nf, I, K, lane, (acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// A panel workgroup's stack: wavefront w owns stack tile row w (0-3: the panel's diagonal block,
// 4-7: the chunk rows) across the panel's four tile columns, in the v_mfma_f64_16x16x4f64
// accumulator layout: element r of lane l of tile J is stack row 16w + 4r + l/16 at panel column
// 16J + l%16.
typedef d4 Stack[kPanelTiles];

__device__ inline int stack_row(int w, int r, int lq) { return 16 * w + 4 * r + lq; }

// The value of the even lane of this lane's pair of lanes (DPP quad_perm [0,0,2,2])
__device__ inline double quad_even(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0xA0, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xA0, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 1/d: the v_rcp_f64 estimate (relative error below 2^-24) refined by one third-order step
// y (1 + e + e^2), e = 1 - d y, which cubes the relative error.
__device__ inline double rcp3(double d) {
  const double y = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

// What the eliminations of two consecutive pairs leave for the next odd step: this lane's
// v_mfma operands of their rank-2 updates of the tile columns right of their priority tiles, the
// pair of an even step in lanes l < 32 (k = 0, 1), the pair of an odd step in lanes l >= 32
// (k = 2, 3), so one product applies both.  A: the pair's column k & 1 at stack row 16w + l%16;
// B, formed when the product is issued: row k & 1 of M^-1 [a[j][c] a[j][c+1]]^T at column
// j = 16J + l%16, from the carried coefficients al, be and the pair's values v0, v1 at row j.
struct PairCarry {
  double aval, al, be, v0[kPanelTiles], v1[kPanelTiles];
};

// The two carried pairs' update of tile columns JD.. on v_mfma_f64_16x16x4f64 (the tile columns
// past the panel's width hold padding that is never read).  The empty asm emits
// nothing; it keeps the products ahead of the publication that follows in the same step.
template <int JD>
__device__ __attribute__((always_inline)) inline void pair_rest(Stack &acc, const PairCarry &cy) {
#pragma unroll
  for (int j2 = JD; j2 < kPanelTiles; ++j2) {
    const double bval = fma(cy.al, cy.v0[j2], cy.be * cy.v1[j2]);
    acc[j2] = __builtin_amdgcn_mfma_f64_16x16x4f64(-cy.aval, bval, acc[j2], 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) __asm__ __volatile__("" : "+v"(acc[j2][r]));
  }
}

// Elimination of the column pair c, c+1 (c even, in tile column J; JP = (c+2)/16 holds the next
// pair).  hist[c/2]: the stack's values of columns c and c+1 ([row][2], updated through column
// c-1); hist[c/2 + 1]: where the next pair goes.  With the pivot block M = [a00 a10; a10 a11]
// (a00 = a[c][c], a10 = a[c+1][c], a11 = a[c+1][c+1]) and d = det M, two steps of the
// right-looking Cholesky update of column j > c+1 are
//     a[i][j] -= [a[i][c] a[i][c+1]] M^-1 [a[j][c] a[j][c+1]]^T
//              = (a[i][c] (a11 a[j][c] - a10 a[j][c+1]) + a[i][c+1] (a00 a[j][c+1] - a10 a[j][c])) / d,
// and every lane forms it from hist itself.  The step: this pair's reads, d and the hardware
// estimate of 1/d, on odd steps (kOdd: the second pair of a tile column's four column groups) the
// two previous pairs' update of the tile columns right of J on MFMA (independent of this pair's
// pivots, it runs inside the estimate's latency), the refinement of 1/d, this pair's update of
// tile JP on the vector unit and the publication of the pair c+2, c+3, the carry, the barrier
// (sched_barrier keeps the compiler from interleaving the groups otherwise).  Deferred updates
// commute with the vector unit's; every pair reaches tile J+1 before its first column is published
// (the last, odd, step of tile column J applies the pending two).
// Columns stay unscaled: L is formed from hist after the last pair.  Entries above the diagonal
// block's diagonal are carried along and never read; finished columns are left alone (their
// lanes add zero).
template <int J, int JP, bool kOdd>
__device__ __attribute__((always_inline)) inline void elim_pair(Stack &acc, double *hist,
                                                                PairCarry &cy, int c, int wcol,
                                                                int w, int lane) {
  const int li = lane & 15, lq = lane >> 4;
  const double *cb = hist + (c >> 1) * 2 * kStack;
  double *cn = hist + ((c >> 1) + 1) * 2 * kStack;
  const double a00 = cb[2 * c];
  const double2 p1 = lds2(cb + 2 * (c + 1));
  const double a10 = p1.x, a11 = p1.y;
  double u0[4], u1[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double2 v = lds2(cb + 2 * stack_row(w, r, lq));
    u0[r] = v.x;
    u1[r] = v.y;
  }
  const double arow = cb[2 * (16 * w + li) + (lq & 1)];
  double v0[kPanelTiles], v1[kPanelTiles];
#pragma unroll
  for (int j2 = 0; j2 < kPanelTiles; ++j2) {
    if (j2 >= JP) {
      const double2 v = lds2(cb + 2 * (16 * j2 + li));
      v0[j2] = v.x;
      v1[j2] = v.y;
    } else {
      v0[j2] = v1[j2] = 0.0;
    }
  }
  const double det = fma(a00, a11, -(a10 * a10));
  double y0 = __builtin_amdgcn_rcp(det);
  __asm__ __volatile__("" : "+v"(y0));
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (kOdd) pair_rest<J + 1>(acc, cy);
  __builtin_amdgcn_sched_barrier(0);
  const double e0 = fma(-det, y0, 1.0);
  const double rdet = fma(y0, fma(e0, e0, e0), y0);   // third-order refinement, as in rcp3
  if constexpr (JP < kPanelTiles) {
    const bool upd = 16 * JP + li > c + 1;
    const double pn = upd ? fma(a11, v0[JP], -(a10 * v1[JP])) : 0.0;
    const double qn = upd ? fma(a00, v1[JP], -(a10 * v0[JP])) : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[JP][r] = fma(-fma(u0[r], pn, u1[r] * qn), rdet, acc[JP][r]);
    const int cc = (c + 2) & 15;
    if (c + 2 < wcol && (li == cc || li == cc + 1)) {
#pragma unroll
      for (int r = 0; r < 4; ++r) cn[2 * stack_row(w, r, lq) + (li - cc)] = acc[JP][r];
    }
  }
  const bool mine = kOdd ? lq >= 2 : lq < 2;
  const double al = ((lq & 1) == 0 ? a11 : -a10) * rdet, be = ((lq & 1) == 0 ? -a10 : a00) * rdet;
  cy.aval = mine ? arow : cy.aval;
  cy.al = mine ? al : cy.al;
  cy.be = mine ? be : cy.be;
#pragma unroll
  for (int j2 = 0; j2 < kPanelTiles; ++j2) {
    cy.v0[j2] = mine ? v0[j2] : cy.v0[j2];
    cy.v1[j2] = mine ? v1[j2] : cy.v1[j2];
  }
  __syncthreads();
}

// The eight column pairs of tile column J, even and odd steps alternating
template <int J>
__device__ __attribute__((always_inline)) inline void elim_tile(Stack &acc, double *hist,
                                                                PairCarry &cy, int wcol, int w,
                                                                int lane) {
#pragma unroll 1
  for (int s = 0; s < 6; s += 2) {
    elim_pair<J, J, false>(acc, hist, cy, 16 * J + 2 * s, wcol, w, lane);
    elim_pair<J, J, true>(acc, hist, cy, 16 * J + 2 * s + 2, wcol, w, lane);
  }
  elim_pair<J, J, false>(acc, hist, cy, 16 * J + 12, wcol, w, lane);
  elim_pair<J, J + 1, true>(acc, hist, cy, 16 * J + 14, wcol, w, lane);
}

// One step p of the blocked factorisation (grid: subband x (nchunk panel workgroups; for p > 0 one
// workgroup for panel p-1's diagonal block and two per block row of panel p+1's column strip)).
// Panel workgroups (blockIdx.y < nchunk, dispatched first) apply the pending rank-64 update of
// panel p-1 to their stack (panel p's diagonal block and their chunk of rows), then factor panel p.
// Every role reads only finished panels and writes a region no other workgroup of the launch
// touches, so one launch per panel suffices and nothing waits across workgroups.
__global__ __launch_bounds__(kBThreads) void k_chol_panel(Problem pb, Buffers B, int k,
                                                          const int32_t *ndir, int p, double *Ld,
                                                          int *cfail) {
  // L of panel p-1 at the diagonal block's rows (Pd) and at this workgroup's rows (Px); after the
  // pending update, the history of published column pairs (hist, [pair][row][2]); at the end, the
  // diagonal tiles to invert
  __shared__ __align__(16) double lds[2 * kPB * kPs];
  static_assert(kPB / 2 * 2 * kStack <= 2 * kPB * kPs, "column history fits");
  double *Pd = lds, *Px = lds + kPB * kPs, *hist = lds;
  const int f = blockIdx.x;
  if (!lm_live(B, ndir, f, k) || cfail[f]) return;
  const int nf = pb.nf, nct = nf >> 4, nrt = pb.npad >> 4;
  const PanelGeom g = panel_geom(p, nct);
  double *A = B.H + (int64_t)f * pb.npad * nf;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lq = lane >> 4;
  const PanelGeom gs = panel_geom(p > 0 ? p - 1 : 0, nct);   // source of the pending update
  const int np = (nct + kPanelTiles - 1) / kPanelTiles;
  const int nchunk = (nrt - g.c1 + kPanelTiles - 1) / kPanelTiles;
  if (p > 0 && (int)blockIdx.y == nchunk) {
    // panel p-1's diagonal block: its strictly-lower tiles from the side buffer into the matrix
    // (no workgroup of this launch reads them there) and its diagonal tiles inverted for the back
    // substitution, one wavefront per tile
    const PanelGeom gp = panel_geom(p - 1, nct);
    const double *src = Ld + ((int64_t)f * np + p - 1) * kPB * kPB;
#pragma unroll 4
    for (int e = tid; e < kPB * kPB; e += kBThreads) {
      const int row = e >> 6, col = e & 63, ti = row >> 4, tj = col >> 4;
      if (ti < gp.wp && tj < ti) A[(int64_t)(gp.c0 * 16 + row) * nf + gp.c0 * 16 + col] = src[e];
    }
    if (w < gp.wp) {
      double *T = lds + w * 256;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        T[e] = src[(16 * w + (e >> 4)) * kPB + 16 * w + (e & 15)];
      }
      __builtin_amdgcn_wave_barrier();
      tri_inverse16(T, nullptr, B.Linv + ((int64_t)f * nct + gp.c0 + w) * 256, lane);
    }
    return;
  }
  const int side = (p > 0) ? 1 : 0;
  if ((int)blockIdx.y >= nchunk + side) {
    // strip role: panel p+1's column strip, half a 64x64 block row each, panels 0 .. p-1
    const int rs = kPanelTiles * (p + 1);
    const int e = (int)blockIdx.y - nchunk - side, rb = e >> 1;
    if (p + 1 >= np || rb >= (nrt - rs + kPanelTiles - 1) / kPanelTiles) return;
    strip_half(A, lds, nf, nct, nrt, p, rs, rb, e & 1, w, lane);
    return;
  }
  const int q = blockIdx.y;
  const int r0 = g.c1 + kPanelTiles * q;            // first row tile of this chunk
  const int nr = min(kPanelTiles, nrt - r0);
  const int wp = g.wp, wcol = 16 * wp, wsrc = (p > 0) ? 16 * gs.wp : 0;
  // this wavefront's stack tile row: its first matrix row, and whether it holds rows of the
  // block or the chunk
  const bool in_block = w < kPanelTiles;
  const bool live = in_block ? w < wp : w - kPanelTiles < nr;
  const int64_t row0 = in_block ? 16 * (g.c0 + w) : 16 * (r0 + w - kPanelTiles);

  Stack acc;
#pragma unroll
  for (int J = 0; J < kPanelTiles; ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = 4 * r + lq;
      const bool v = live && J < wp && (!in_block || J < w || (J == w && li <= rr));
      acc[J][r] = v ? A[(row0 + rr) * nf + 16 * (g.c0 + J) + li] : 0.0;
    }
  if (p > 0) {
    // L of panel p-1 at the block's rows and at the chunk's rows (fixed-count loops: each pair's
    // loads are all issued before its first LDS store)
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
      Pd[row * kPs + col] = dv[it];
      Px[row * kPs + col] = xv[it];
    }
    __syncthreads();
    // pending rank-64 update: stack tile (w, J) -= P_w P_J^T, P_w the previous panel's L at the
    // tile's rows (v_mfma operands: lane l supplies row l%16, columns 16t + 4(l/16) + qq)
    const double *xrow = (in_block ? Pd + (16 * w + li) * kPs : Px + (16 * (w - kPanelTiles) + li) * kPs) + 4 * lq;
    // (every tile of the row: those above the block's diagonal, past the panel's width or in
    // padding rows hold values that are never read; gs.wp = 4 for every source panel)
#pragma unroll
    for (int t = 0; t < kPanelTiles; ++t) {
      {
        double xa[4], yb[kPanelTiles][4];
        {
          const double2 a = lds2(xrow + 16 * t), b = lds2(xrow + 16 * t + 2);
          xa[0] = a.x; xa[1] = a.y; xa[2] = b.x; xa[3] = b.y;
        }
#pragma unroll
        for (int J = 0; J < kPanelTiles; ++J) {
          const double *src = Pd + (16 * J + li) * kPs + 16 * t + 4 * lq;
          const double2 a = lds2(src), b = lds2(src + 2);
          yb[J][0] = a.x; yb[J][1] = a.y; yb[J][2] = b.x; yb[J][3] = b.y;
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
#pragma unroll
          for (int J = 0; J < kPanelTiles; ++J)
            acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xa[qq], yb[J][qq], acc[J], 0, 0, 0);
      }
    }
  }
  __syncthreads();   // the pending update's reads of Pd and Px are done
  // columns 0 and 1 published, then the pairs
  if (li < 2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) hist[2 * stack_row(w, r, lq) + li] = acc[0][r];
  }
  __syncthreads();
  PairCarry cy{};   // the odd slot holds no pair before the first odd step: it adds zero
  elim_tile<0>(acc, hist, cy, wcol, w, lane);
  if (wp > 1) elim_tile<1>(acc, hist, cy, wcol, w, lane);
  if (wp > 2) elim_tile<2>(acc, hist, cy, wcol, w, lane);
  if (wp > 3) elim_tile<3>(acc, hist, cy, wcol, w, lane);

  // L: column c of pair (c, c+1) is L[.][c] sqrt(a00), column c+1 is
  // (a[.][c+1] - a[.][c] a10 / a00) / sqrt(det / a00); 1/L_jj in the diagonal slots.  A column is
  // never updated after its publication, so each lane's stack already holds its column as the
  // history does; an odd column takes its even neighbour's value from the adjacent lane (DPP
  // quad_perm [0,0,2,2]) and only the pivots come from the history.  Each lane checks the pivots
  // of its columns' pairs (all pairs are covered).
  int okv = 1;
#pragma unroll
  for (int J = 0; J < kPanelTiles; ++J) {
    const int cpair = 16 * J + (li & ~1);
    const double *h = hist + (cpair >> 1) * 2 * kStack;
    const double a00 = J < wp ? h[2 * cpair] : 1.0;
    const double2 p1 = lds2(h + 2 * (cpair + 1));
    const double a10 = J < wp ? p1.x : 0.0, a11 = J < wp ? p1.y : 1.0;
    const double det = fma(a00, a11, -(a10 * a10));
    okv &= (a00 > 0.0 && det > 0.0 && isfinite(a00) && isfinite(det)) ? 1 : 0;
    const double inv0 = rcp3(a00);
    const double l10 = a10 * inv0;
    const bool odd = li & 1;
    const double rs = rsqrt_nr(odd ? det * inv0 : a00);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double own = acc[J][r];
      const double ev = quad_even(own);
      const double v = odd ? fma(-ev, l10, own) : own;
      acc[J][r] = (in_block && stack_row(w, r, lq) == 16 * J + li) ? rs : v * rs;
    }
  }
  if (!__syncthreads_and(okv)) {
    if (tid == 0) cfail[f] = 1;
    return;
  }

  // the chunk's rows of L go back into the matrix
  if (!in_block && live) {
#pragma unroll
    for (int J = 0; J < kPanelTiles; ++J)
      if (J < wp) {
#pragma unroll
        for (int r = 0; r < 4; ++r) A[(row0 + 4 * r + lq) * nf + 16 * (g.c0 + J) + li] = acc[J][r];
      }
  }
  if (q == 0 && p < np - 1 && in_block && live) {
    // the block's lower tiles (diagonal tiles included) to the side buffer: the other workgroups
    // are still reading the block from the matrix (the next launch moves them and inverts the
    // diagonal tiles)
    double *dst = Ld + ((int64_t)f * np + p) * kPB * kPB;
#pragma unroll
    for (int J = 0; J < kPanelTiles; ++J)
      if (J <= w) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(16 * w + 4 * r + lq) * kPB + 16 * J + li] = acc[J][r];
      }
  }
  if (p == np - 1) {
    // the last panel has one workgroup, chunk 0 (its chunk is the right-hand-side row): the
    // block's strictly-lower tiles go straight into the matrix, its diagonal tiles are inverted
    if (in_block && live) {
#pragma unroll
      for (int J = 0; J < kPanelTiles; ++J) {
        if (J < w) {
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(row0 + 4 * r + lq) * nf + 16 * (g.c0 + J) + li] = acc[J][r];
        } else if (J == w) {
#pragma unroll
          for (int r = 0; r < 4; ++r) lds[w * 256 + (4 * r + lq) * 16 + li] = acc[J][r];
        }
      }
    }
    __syncthreads();
    if (w < wp) tri_inverse16(lds + w * 256, nullptr, B.Linv + ((int64_t)f * nct + g.c0 + w) * 256, lane);
  }
}

// Back substitution L^T delta = y with one thread per column (nf <= 1024): per 16-row block,
// from the last, x_J = (L_JJ^-1)^T t_J on 16 threads, then t -= L_J^T x_J on every column left
// of the block.  The rows of L of the next block are in flight while a block is used (the
// matrix streams from memory once, so the loads are what the loop waits on).
constexpr int kBsThreads = 1024;
constexpr int kBsWaves = kBsThreads / 64;

__global__ __launch_bounds__(kBsThreads) void k_chol_backsub(Problem pb, Buffers B, int k,
                                                             const int32_t *ndir, int *cfail) {
  __shared__ double tb[2][16];
  __shared__ double xb[2][16];
  __shared__ double liS[2][256];   // L_JJ^-1 of the current and the next block
  __shared__ double red[kBsWaves];
  __shared__ int failed;
  const int f = blockIdx.x;
  if (!lm_live(B, ndir, f, k)) return;
  k = lm_dir(B, f, k);
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
  double *A = B.H + (int64_t)f * pb.npad * nf;
  const double *Li = B.Linv + (int64_t)f * nct * 256;

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

// Back substitution L^T delta = y for nf <= 512, one thread per column: per 16-row block J, from
// the last, the 16 lanes that own the block's columns form x_J = (L_JJ^-1)^T t_J inside their
// wavefront (t_J exchanged through LDS; each lane holds its column of L_JJ^-1 from the start) and
// publish it; after one barrier every column left of the block takes t -= L_J^T x_J.  The rows of
// L stream from memory once, up to kBsAhead blocks ahead of their use, in a ring of register
// buffers indexed at compile time (the block loop is unrolled by kBsAhead).  Only lanes whose
// column is left of a block load its rows, so wavefronts right of it issue no loads: the step is
// bound by the vector-memory instructions the compute unit issues, not by their latency.
constexpr int kBrThreads = 512;
constexpr int kBrWaves = kBrThreads / 64;
constexpr int kBsAhead = 4;

__global__ __launch_bounds__(kBrThreads) void k_chol_backsub_ring(Problem pb, Buffers B, int k,
                                                                  const int32_t *ndir, int *cfail) {
  __shared__ double tx[kBrWaves][16];   // per wavefront: the right-hand side of its block
  __shared__ double xs[2][16];          // the current block's solution
  __shared__ double red[kBrWaves];
  __shared__ int failed;
  const int f = blockIdx.x;
  if (!lm_live(B, ndir, f, k)) return;
  k = lm_dir(B, f, k);
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
  const double *A = B.H + (int64_t)f * pb.npad * nf;
  const int c = tid, myblk = c >> 4, r16 = c & 15;
  double t = (c < nf) ? A[(int64_t)nf * nf + c] : 0.0;
  double lic[16];   // column r16 of L_JJ^-1, J = this lane's block
#pragma unroll
  for (int i = 0; i < 16; ++i) lic[i] = (c < nf) ? B.Linv[((int64_t)f * nct + myblk) * 256 + i * 16 + r16] : 0.0;
  auto load_rows = [&](int jb, double (&dst)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) dst[r] = (jb >= 0 && c < 16 * jb) ? A[(int64_t)(16 * jb + r) * nf + c] : 0.0;
  };
  double ring[kBsAhead][16];
#pragma unroll
  for (int u = 0; u < kBsAhead; ++u) load_rows(nct - 1 - u, ring[u]);
  auto step = [&](int jb, double (&use)[16]) {
    if (myblk == jb) {
      tx[w][r16] = t;
      __builtin_amdgcn_wave_barrier();
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 16; ++i) s4[i & 3] = fma(lic[i], tx[w][i], s4[i & 3]);
      t = (s4[0] + s4[1]) + (s4[2] + s4[3]);
      xs[jb & 1][r16] = t;
    }
    __syncthreads();
    if (c < 16 * jb) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 16; ++r) s4[r & 3] = fma(use[r], xs[jb & 1][r], s4[r & 3]);
      t -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    load_rows(jb - kBsAhead, use);
  };
  for (int jb = nct - 1; jb >= 0; jb -= kBsAhead) {
#pragma unroll
    for (int u = 0; u < kBsAhead; ++u)
      if (jb - u >= 0) step(jb - u, ring[u]);
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
    for (int i = 0; i < kBrWaves; ++i) sum += red[i];
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
    // for p > 0: one workgroup for panel p-1's diagonal block, then (unless p is the last panel)
    // two per 64x64 block row of panel p+1's column strip
    const int rs = kPanelTiles * (p + 1);
    const int nstrip = (p > 0 && p + 1 < np) ? 2 * ((nrt - rs + kPanelTiles - 1) / kPanelTiles) : 0;
    const int nextra = (p > 0) ? 1 + nstrip : 0;
    hipLaunchKernelGGL(k_chol_panel, dim3(pb.P, nchunk + nextra), dim3(kBThreads), 0, s, pb, B, k,
                       ndir, p, Ld, cfail);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (pb.nf <= kBrThreads)
    hipLaunchKernelGGL(k_chol_backsub_ring, dim3(pb.P), dim3(kBrThreads), 0, s, pb, B, k, ndir, cfail);
  else
    hipLaunchKernelGGL(k_chol_backsub, dim3(pb.P), dim3(kBsThreads), 0, s, pb, B, k, ndir, cfail);
  return hipGetLastError();
}

}  // namespace calib
