// Kernels of the local step over the packed visibilities and coherencies (baseline-major).
//
// The coherency of an unpolarised source is a scalar times I2 (Section 2) and the Jones matrices
// are constant over a baseline's samples, so everything the Levenberg-Marquardt runs need from
// the residual R = V - sum_l c_l J_lp J_lq^H (Section 2 visibility model) is per-baseline sums:
// D_l = sum_s conj(c_ls) R_s for every direction l, and the energy sum_s ||R_s||^2.
//   k_pack_stats   (per interval)      packed V, C and U_l = sum conj(c_l) V, X_lm = sum conj(c_l) c_m,
//                                      sum ||V||^2 per baseline
//   refresh        (start of a local step) the energy, streaming V and the coherencies once
//                  (k_stream), and every D_l = U_l - sum_m X_lm M_m (k_dall); for the one-launch
//                  local step D_l and the energy both from the statistics (k_dall<true>)
//   k_trial_stats  (each LM trial point) cost and D_b of r = R - c_k (M_trial - M_start) (the
//                  SAGE expectation V_k = R + c_k M_start of Section 3 minus the trial model)
//   k_commit_stats (end of direction k)  R <- R - c_k (M_final - M_start) as an update of every
//                  D_l and of the energy
//
// The coherency of an unpolarised source is a scalar times I2 (Section 2), so one complex value
// per sample and direction is streamed.  The Jones matrices are time invariant over the interval
// (Section 2), so the 2x2 products M = J_p J_q^H are formed once per baseline in FP64.
//
// Work decomposition: a tile is a run of kBlock/G consecutive baselines of one subband.  In the
// streaming pass G lanes of a wavefront share a baseline and stride over its T*n_chan samples, so
// consecutive lanes read consecutive 32-byte (float) or 64-byte (double) samples; the per-tile
// energy is reduced into one FP64 partial per tile, summed later in a fixed order (run-to-run
// deterministic).  The per-baseline kernels run one wavefront per tile, one lane per baseline.
#include <type_traits>

#include "calib_internal.h"
#include "lm_device.h"
#include "wave_reduce.h"

namespace calib {

namespace {


using lmd::jjh;
using lmd::sub_scaled;

template <typename T>
__device__ inline void load8(const T *__restrict__ p, T *v);
template <>
__device__ inline void load8<float>(const float *__restrict__ p, float *v) {
  const float4 a = reinterpret_cast<const float4 *>(p)[0];
  const float4 b = reinterpret_cast<const float4 *>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <>
__device__ inline void load8<double>(const double *__restrict__ p, double *v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 a = reinterpret_cast<const double2 *>(p)[i];
    v[2 * i] = a.x; v[2 * i + 1] = a.y;
  }
}
template <typename T>
__device__ inline void store8(T *__restrict__ p, const T *v);
template <>
__device__ inline void store8<float>(float *__restrict__ p, const float *v) {
  reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
  reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
}
template <>
__device__ inline void store8<double>(double *__restrict__ p, const double *v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) reinterpret_cast<double2 *>(p)[i] = make_double2(v[2 * i], v[2 * i + 1]);
}

template <typename T>
__device__ inline void load2(const T *__restrict__ p, T &re, T &im) {
  re = p[0];
  im = p[1];
}


// Sum over the workgroup in a fixed order; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) s += red[i];
  return s;
}

// Energy of the residual R = V - sum_l c_l J_lp J_lq^H over one tile (one FP64 partial per
// tile); R itself is not stored.  G lanes share a baseline and stride over its samples.
template <typename T, int G>
__device__ inline void stream_tile(const Problem &pb, const Layout &L, const Buffers &B, int tile,
                                   T (*Msh)[kMaxDirs][8], double *red) {
  const int f = L.tile_f[tile];
  const int Kf = L.ndir[f];
  const int nb = L.nb[f], spb = L.spb[f];
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int bi = L.tile_b0[tile] + grp;
  const bool live = bi < nb;
  const int N = pb.N, K = pb.K;
  const int64_t gb = (int64_t)L.bl_off[f] + bi;
  const int64_t s0 = L.samp_off[f] + (int64_t)bi * spb;
  const T *C = static_cast<const T *>(B.C);
  if (live) {
    const int p = L.bl_p[gb], q = L.bl_q[gb];
    for (int l = lane; l < Kf; l += G) {
      double m[8];
      const double *Jl = B.J + ((int64_t)f * K + l) * N * 8;
      jjh(Jl + 8 * p, Jl + 8 * q, m);
#pragma unroll
      for (int e = 0; e < 8; ++e) Msh[grp][l][e] = (T)m[e];
    }
  }
  __syncthreads();
  double cost = 0.0;
  if (live) {
    const T *V = static_cast<const T *>(B.V);
    const T *Cb = C + 2 * (L.coh_off[f] + (int64_t)bi * spb);
    const int64_t cstride = 2 * (int64_t)nb * spb;   // between directions
    for (int s = lane; s < spb; s += G) {
      T r[8], c[kMaxDirs][2];
      load8<T>(V + 8 * (s0 + s), r);
      // every direction's coherency requested before the first is used
#pragma unroll
      for (int l = 0; l < kMaxDirs; ++l)
        if (l < Kf) load2<T>(Cb + l * cstride + 2 * s, c[l][0], c[l][1]);
#pragma unroll
      for (int l = 0; l < kMaxDirs; ++l) {
        if (l < Kf) {
          const T cr = c[l][0], ci = c[l][1];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const T mr = Msh[grp][l][2 * e], mi = Msh[grp][l][2 * e + 1];
            r[2 * e] -= cr * mr - ci * mi;
            r[2 * e + 1] -= cr * mi + ci * mr;
          }
        }
      }
      T ss = 0;
#pragma unroll
      for (int e = 0; e < 8; ++e) ss += r[e] * r[e];
      cost += (double)ss;
    }
  }
  const double tot = block_sum(cost, red);
  if (threadIdx.x == 0) {
    B.cost_part[tile] = tot;
    B.Epart[tile] = tot;
  }
}

// Data cost and D_b at the LM trial point (lmd::trial_tile), one wavefront per tile.
constexpr int kStatTiles = 4;   // tiles per workgroup of the per-baseline kernels, one per wavefront
__global__ __launch_bounds__(64 * kStatTiles) void k_trial_stats(Problem pb, Layout L, Buffers B, int k) {
  const int tile = kStatTiles * blockIdx.x + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (tile >= pb.ntiles) return;   // uniform per wavefront
  const int f = L.tile_f[tile];
  if (!lm_live(B, L.ndir, f, k) || !B.lm[f].chol_ok) return;   // uniform
  k = lm_dir(B, f, k);
  lmd::trial_tile(pb, L, B, f, k, tile, lane);
}

// Every direction's D_l at the current point from the coherency statistics, one workgroup per tile
// and four lanes per baseline: lane h of a baseline's four holds the entry (h>>1, h&1) of its 2x2
// matrices, so that a wavefront's loads and stores of the per-baseline tables are contiguous.
// The entry of M_m = J_p J_q^H of every direction m is formed once, then each direction's
// D_l = U_l - sum_m X_lm M_m is streamed (U_l and the row X_l. read, D_l written); direction 0's D
// also becomes the accepted and start point of the next LM run.  kL >= K directions are unrolled;
// the loads of a row X_l. take every m < kL at a clamped index (in bounds, never used past K_f),
// so that they are issued together.
// With kEnergy, also the residual's energy from the statistics, with R = V - sum_m c_m M_m:
//   sum_s ||R_s||^2 = sum_s ||V_s||^2 - 2 Re sum_m <M_m, U_m> + sum_lm X_lm <M_l, M_m>
//                   = Ev - Re sum_l <M_l, U_l + D_l>     (<A, B> = tr(A^H B), D_l = U_l - sum_m X_lm M_m)
// the tile's terms of direction l (direction 0 with Ev) summed in a fixed order into Epl[l][tile]
// (zero for the directions l >= K_f of its subband).  In FP64 the expansion cancels by about the
// ratio of the data's energy to the residual's (~SNR), far inside the double's precision; at a
// perfect fit it leaves an absolute error of order eps * sum ||V||^2.
constexpr int kDallThreads = 256;   // one tile of up to 64 baselines, four lanes each
template <bool kEnergy, int kL>
__global__ __launch_bounds__(kDallThreads) void k_dall(Problem pb, Layout L, Buffers B) {
  __shared__ double red[kL][kDallThreads / 64];
  const int tile = blockIdx.x, tid = threadIdx.x, w = tid >> 6;
  const int h = tid & 3, ei = h >> 1, ej = h & 1, bl = tid >> 2;
  const int f = L.tile_f[tile];
  const int Kf = L.ndir[f], nb = L.nb[f], K = pb.K;
  const int bi = L.tile_b0[tile] + bl;
  const bool live = bl < pb.bpt && bi < nb;
  double part[kL];
#pragma unroll
  for (int l = 0; l < kL; ++l) part[l] = 0.0;
  if (live) {
    const int N = pb.N;
    const int64_t gb = (int64_t)L.bl_off[f] + bi, nbt = pb.nbt;
    const int p = L.bl_p[gb], q = L.bl_q[gb];
    // entry (ei, ej) of J_p J_q^H = sum_t J_p[ei][t] conj(J_q[ej][t]) per direction
    double2 M[kL];
#pragma unroll
    for (int m = 0; m < kL; ++m) {
      const int mc = min(m, Kf - 1);
      const double2 *a = reinterpret_cast<const double2 *>(B.J + (((int64_t)f * K + mc) * N + p) * 8 + 4 * ei);
      const double2 *b = reinterpret_cast<const double2 *>(B.J + (((int64_t)f * K + mc) * N + q) * 8 + 4 * ej);
      const double2 a0 = a[0], a1 = a[1], b0 = b[0], b1 = b[1];
      double re = 0.0, im = 0.0;
      re += a0.x * b0.x + a0.y * b0.y;
      im += a0.y * b0.x - a0.x * b0.y;
      re += a1.x * b1.x + a1.y * b1.y;
      im += a1.y * b1.x - a1.x * b1.y;
      M[m] = make_double2(re, im);
    }
    const double2 *U2 = reinterpret_cast<const double2 *>(B.Ucoh);
    const double2 *X2 = reinterpret_cast<const double2 *>(B.Xcoh);
    double2 *D2 = reinterpret_cast<double2 *>(B.Dall);
    const double ev = (kEnergy && h == 0) ? B.Ev[gb] : 0.0;
#pragma unroll
    for (int l = 0; l < kL; ++l) {
      if (l >= Kf) continue;   // uniform per workgroup
      const double2 u = U2[((int64_t)l * nbt + gb) * 4 + h];
      double2 x[kL];
#pragma unroll
      for (int m = 0; m < kL; ++m) x[m] = X2[((int64_t)l * K + min(m, Kf - 1)) * nbt + gb];
      double2 d = u;
#pragma unroll
      for (int m = 0; m < kL; ++m) {
        if (m < Kf) {
          d.x -= x[m].x * M[m].x - x[m].y * M[m].y;
          d.y -= x[m].x * M[m].y + x[m].y * M[m].x;
        }
      }
      D2[((int64_t)l * nbt + gb) * 4 + h] = d;
      if (l == 0) {
        reinterpret_cast<double2 *>(d_accepted(B, f))[4 * gb + h] = d;
        reinterpret_cast<double2 *>(B.Dstart)[4 * gb + h] = d;
      }
      if (kEnergy)   // Re <M_l, U_l + D_l> over this lane's entry
        part[l] = (l == 0 ? ev : 0.0) - fma(M[l].x, u.x + d.x, M[l].y * (u.y + d.y));
    }
  }
  if (kEnergy) {
    wave_sum_vec<kL>(part);
    if ((tid & 63) == 0)
#pragma unroll
      for (int l = 0; l < kL; ++l) red[l][w] = part[l];
    __syncthreads();
    if (tid < K) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < kDallThreads / 64; ++i) v += red[tid][i];
      B.Epl[(int64_t)tid * pb.ntiles + tile] = v;
    }
  }
}

template <bool kEnergy>
hipError_t launch_dall(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s) {
  if (pb.bpt > 64 || pb.K < 1 || pb.K > kMaxDirs) return hipErrorInvalidValue;
  const dim3 grid(pb.ntiles), block(kDallThreads);
  if (pb.K <= 4)
    hipLaunchKernelGGL((k_dall<kEnergy, 4>), grid, block, 0, s, pb, L, B);
  else if (pb.K <= 5)
    hipLaunchKernelGGL((k_dall<kEnergy, 5>), grid, block, 0, s, pb, L, B);
  else if (pb.K <= 6)
    hipLaunchKernelGGL((k_dall<kEnergy, 6>), grid, block, 0, s, pb, L, B);
  else if (pb.K <= 8)
    hipLaunchKernelGGL((k_dall<kEnergy, 8>), grid, block, 0, s, pb, L, B);
  else if (pb.K <= 10)
    hipLaunchKernelGGL((k_dall<kEnergy, 10>), grid, block, 0, s, pb, L, B);
  else if (pb.K <= 12)
    hipLaunchKernelGGL((k_dall<kEnergy, 12>), grid, block, 0, s, pb, L, B);
  else
    hipLaunchKernelGGL((k_dall<kEnergy, 16>), grid, block, 0, s, pb, L, B);
  return hipGetLastError();
}

// The tiles' energies (Epart, cost_part) from the statistics' per-(direction, tile) terms, for the
// kernels that read the energy per tile
__global__ __launch_bounds__(kBlock) void k_fold_energy(Problem pb, Buffers B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= pb.ntiles) return;
  double e = 0.0;
  for (int l = 0; l < pb.K; ++l) e += B.Epl[(int64_t)l * pb.ntiles + t];
  B.Epart[t] = e;
  B.cost_part[t] = e;
}

// End of direction k's LM run (the SAGE commit, lmd::commit_tile), one wavefront per tile.
__global__ __launch_bounds__(64 * kStatTiles) void k_commit_stats(Problem pb, Layout L, Buffers B, int k,
                                                                   int all) {
  const int tile = kStatTiles * blockIdx.x + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (tile >= pb.ntiles) return;   // uniform per wavefront
  const int f = L.tile_f[tile];
  if (k < 0) {   // the subband's own direction, if its run has just ended
    if (B.lm[f].phase != kPhaseAdvance || B.lm[f].cur < 0) return;
    k = B.lm[f].cur;
  }
  if (k >= L.ndir[f]) return;   // uniform per wavefront
  lmd::commit_tile(pb, L, B, f, k, all, tile, lane);
}

// One workgroup per tile (grid = ntiles), or a persistent grid that strides over the tiles.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_stream(Problem pb, Layout L, Buffers B) {
  constexpr int BPT = kBlock / G;
  __shared__ T Msh[BPT][kMaxDirs][8];
  __shared__ double red[kBlock / 64];
  for (int tile = blockIdx.x; tile < pb.ntiles; tile += gridDim.x) {
    stream_tile<T, G>(pb, L, B, tile, Msh, red);
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_energy(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s) {
  if (pb.ntiles == 0) return hipSuccess;
  dim3 grid(pb.stream_grid > 0 && pb.stream_grid < pb.ntiles ? pb.stream_grid : pb.ntiles), block(kBlock);
  switch (pb.group) {
    case 4: hipLaunchKernelGGL((k_stream<T, 4>), grid, block, 0, s, pb, L, B); break;
    case 8: hipLaunchKernelGGL((k_stream<T, 8>), grid, block, 0, s, pb, L, B); break;
    case 16: hipLaunchKernelGGL((k_stream<T, 16>), grid, block, 0, s, pb, L, B); break;
    case 32: hipLaunchKernelGGL((k_stream<T, 32>), grid, block, 0, s, pb, L, B); break;
    case 64: hipLaunchKernelGGL((k_stream<T, 64>), grid, block, 0, s, pb, L, B); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Per solution interval: pack the caller's visibilities and coherencies into the library's
// baseline-major layout (flagged baselines dropped) and form every baseline's coherency statistics
// and the energy of its visibilities in the same pass, in FP64 from the element type:
//   S_b,l = sum_s |c_ls|^2,   U_l = sum_s conj(c_ls) V_s,   X_lm = sum_s conj(c_ls) c_ms,
//   Ev_b = sum_s ||V_s||^2.
// With the scalar coherency and J constant over a baseline's samples, everything the local steps
// need from the samples besides the residual's energy follows from these: at a point with models
// M_m, D_l = sum_s conj(c_ls) R_s = U_l - sum_m X_lm M_m.
//
// One workgroup per (run of TB = kBlock / G compact baselines, subband); group j of G lanes (one
// wavefront holds 64 / G groups) takes baseline j and walks its samples in chunks of SC.  Per chunk
// the group copies the baseline's V and coherency rows of the chunk, lane l taking elements
// l, l + G, ... of each row, so that consecutive lanes read consecutive complex values of the
// caller's arrays (each byte read once, in full cache lines per wavefront request), every load of
// the chunk issued before the first is used, into LDS and into the packed arrays; then lane l
// accumulates direction l's sums from LDS (the group's lanes read the same words: broadcasts).
// Only the group's own lanes exchange data through LDS, so the wavefronts never wait for each
// other.  V rows are padded by 16 bytes so that the groups of a wavefront hit different LDS banks;
// a baseline's coherencies are stored [sample][direction], so that the group's lanes, each reading
// its own direction at one sample, read consecutive words (stored direction-major, at a direction
// stride that is a multiple of the bank count, every such read was a K_f-way bank conflict).
// A non-finite input sets *bad (when given) and the subband's status word.
template <typename T>
struct Cplx;
template <>
struct Cplx<float> { using type = float2; };
template <>
struct Cplx<double> { using type = double2; };

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_pack_stats(Problem pb, Layout L, Buffers B, const T *vis,
                                                       const T *coh, T *Vp, T *Cp, double *Sb,
                                                       const int64_t *in_vis_off,
                                                       const int64_t *in_coh_off,
                                                       const int32_t *comp2full, int *bad,
                                                       int *status) {
  using C2 = typename Cplx<T>::type;
  constexpr int TB = kBlock / G;                   // baselines per workgroup
  constexpr int SC = 32 / (int)sizeof(T);          // samples per chunk
  // LDS element: the 16-lane groups (up to 16 directions, K_f/2 + 1 coherency products per sample
  // and lane) keep their rows in FP64, converted once when staged rather than at every read; the
  // 8-lane groups keep the input type (FP64 rows would halve their occupancy)
  using LT = typename std::conditional<G == 16, double, T>::type;
  constexpr int VR = SC * 8 + 16 / (int)sizeof(LT);   // padded LDS row of V (elements)
  // a baseline's chunk of coherencies, [sample][direction] (lanes reading different directions at
  // one sample hit consecutive banks), padded by 128 bytes between the group's baselines
  constexpr int CJ = SC * G * 2 + 128 / (int)sizeof(LT);
  constexpr int NV = 4 * SC / G;                   // V values per lane per chunk
  constexpr int NC = SC;                           // coherency values per lane per chunk (G*SC >= K_f*SC)
  static_assert(NV >= 1 && 4 * SC == NV * G, "chunk of V split evenly over the group");
  __shared__ __align__(16) LT Vs[TB * VR];
  __shared__ __align__(16) LT Cs[TB * CJ];
  const int f = blockIdx.y;
  const int nb = L.nb[f];
  const int bi0 = blockIdx.x * TB;
  if (bi0 >= nb) return;                           // whole workgroup
  // subbands of up to 8 directions go to the 8-lane launch, the others to the 16-lane one
  if (G == 8 ? L.ndir[f] > 8 : L.ndir[f] <= 8) return;   // whole workgroup
  const int j = threadIdx.x / G, l = threadIdx.x % G;
  const int bi = bi0 + j;
  if (bi >= nb) return;                            // whole group (no workgroup barrier below)
  const int spb = L.spb[f], Kf = L.ndir[f];
  const int64_t Bfull = (int64_t)pb.N * (pb.N - 1) / 2;
  const int64_t gb = (int64_t)L.bl_off[f] + bi;
  const int64_t bf = comp2full[gb];
  const C2 *vsrc = reinterpret_cast<const C2 *>(vis + 8 * (in_vis_off[f] + bf * spb));
  const C2 *csrc = reinterpret_cast<const C2 *>(coh + 2 * (in_coh_off[f] + bf * spb));
  // the packed copies (not kept when Vp and Cp are null: the statistics alone)
  const bool keep = Vp != nullptr;
  C2 *vdst = keep ? reinterpret_cast<C2 *>(Vp + 8 * (L.samp_off[f] + (int64_t)bi * spb)) : nullptr;
  C2 *cdst = keep ? reinterpret_cast<C2 *>(Cp + 2 * (L.coh_off[f] + (int64_t)bi * spb)) : nullptr;
  const int64_t cs = Bfull * spb, cd = (int64_t)nb * spb;   // between directions (complex values)
  LT *vl = Vs + j * VR;
  // X is Hermitian (X_ml = conj X_lm): lane l sums X_lm for m = (l + d) mod K_f at distances
  // d = 0 .. K_f/2 (at d = K_f/2 for even K_f only lanes l < K_f/2), so every pair is summed once
  constexpr int kD = G / 2 + 1;
  double u[8] = {0, 0, 0, 0, 0, 0, 0, 0}, x[2 * kD], ev = 0.0;
#pragma unroll
  for (int d = 0; d < 2 * kD; ++d) x[d] = 0.0;
  const int dmax = Kf / 2;                         // largest distance
  const bool half = (Kf & 1) == 0 && l >= dmax;    // lanes that skip distance K_f/2
  bool finite = true;
  // chunk s0's V and coherency values of this lane (complex value e of the chunk's V row; value
  // t of direction m's coherency row)
  auto fetch = [&](int s0, C2 *v, C2 *c) {
    const int n = min(SC, spb - s0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = l + G * i;
      if (e < 4 * n) v[i] = vsrc[4 * s0 + e];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int e = l + G * i, m = e / SC, t = e % SC;
      if (m < Kf && t < n) c[i] = csrc[m * cs + s0 + t];
    }
  };
  C2 v[NV], c[NC];
  fetch(0, v, c);
  for (int s0 = 0; s0 < spb; s0 += SC) {
    const int n = min(SC, spb - s0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e = l + G * i;
      if (e < 4 * n) {
        finite &= isfinite(v[i].x) && isfinite(v[i].y);
        if (keep) vdst[4 * s0 + e] = v[i];
        vl[2 * e] = (LT)v[i].x;
        vl[2 * e + 1] = (LT)v[i].y;
      }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int e = l + G * i, m = e / SC, t = e % SC;
      if (m < Kf && t < n) {
        finite &= isfinite(c[i].x) && isfinite(c[i].y);
        if (keep) cdst[m * cd + s0 + t] = c[i];
        LT *cl = Cs + j * CJ + (t * G + m) * 2;
        cl[0] = (LT)c[i].x;
        cl[1] = (LT)c[i].y;
      }
    }
    wave_lds_sync();
    if (s0 + SC < spb) fetch(s0 + SC, v, c);   // the next chunk in flight during this one's sums
    if (l < Kf) {
      for (int t = 0; t < n; ++t) {
        double vv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) vv[e] = (double)vl[8 * t + e];
        if (l == 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) ev = fma(vv[e], vv[e], ev);   // sum_s ||V_s||^2
        }
        const LT *ct = Cs + j * CJ + t * G * 2;    // direction m's value at ct[2 m]
        const double cr = (double)ct[2 * l], ci = (double)ct[2 * l + 1];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          u[2 * e] = fma(cr, vv[2 * e], fma(ci, vv[2 * e + 1], u[2 * e]));
          u[2 * e + 1] = fma(cr, vv[2 * e + 1], fma(-ci, vv[2 * e], u[2 * e + 1]));
        }
#pragma unroll
        for (int d = 0; d < kD; ++d) {
          if (d <= dmax) {                         // uniform over the workgroup
            const int m = l + d < Kf ? l + d : l + d - Kf;
            const double mr = (double)ct[2 * m], mi = (double)ct[2 * m + 1];
            x[2 * d] = fma(cr, mr, fma(ci, mi, x[2 * d]));
            x[2 * d + 1] = fma(cr, mi, fma(-ci, mr, x[2 * d + 1]));
          }
        }
      }
    }
    wave_lds_sync();   // the chunk's LDS rows are read before the next chunk overwrites them
  }
  if (!finite) {
    if (bad) atomicOr(bad, 1);
    if (status) atomicOr(status + f, 5);   // CALIB_E_NUMERIC
  }
  if (l == 0) B.Ev[gb] = ev;
  if (l >= Kf) return;
  const int64_t nbt = pb.nbt;
  double2 *U2 = reinterpret_cast<double2 *>(B.Ucoh + ((int64_t)l * nbt + gb) * 8);
#pragma unroll
  for (int h = 0; h < 4; ++h) U2[h] = make_double2(u[2 * h], u[2 * h + 1]);
  auto xat = [&](int a, int b) {
    return reinterpret_cast<double2 *>(B.Xcoh + (((int64_t)a * pb.K + b) * nbt + gb) * 2);
  };
#pragma unroll
  for (int d = 0; d < kD; ++d) {
    if (d > dmax || (d == dmax && d > 0 && half)) continue;
    const int m = l + d < Kf ? l + d : l + d - Kf;
    *xat(l, m) = make_double2(x[2 * d], x[2 * d + 1]);
    if (d > 0) *xat(m, l) = make_double2(x[2 * d], -x[2 * d + 1]);
  }
  for (int m = Kf; m < pb.K; ++m) *xat(l, m) = make_double2(0.0, 0.0);   // directions f lacks
  Sb[L.sb_off[f] + (int64_t)l * nb + bi] = x[0];   // X_ll = sum |c_l|^2
}

// Model visibilities in the caller's full layout (zero on flagged baselines).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_model(Problem pb, Layout L, Buffers B, T *out,
                                                  const int64_t *full_off, const int32_t *full_bmap) {
  __shared__ double Msh[kMaxDirs][8];
  const int f = blockIdx.y;
  const int b = blockIdx.x;
  const int Bfull = pb.N * (pb.N - 1) / 2;
  if (b >= Bfull) return;
  const int spb = L.spb[f], Kf = L.ndir[f], nb = L.nb[f];
  const int gb = full_bmap[(int64_t)f * Bfull + b];
  T *o = out + 8 * (full_off[f] + (int64_t)b * spb);
  if (gb < 0) {
    for (int i = threadIdx.x; i < 8 * spb; i += kBlock) o[i] = (T)0;
    return;
  }
  const int bi = gb - L.bl_off[f];
  if (threadIdx.x < Kf) {
    const int l = threadIdx.x;
    const double *Jl = B.J + ((int64_t)f * pb.K + l) * pb.N * 8;
    jjh(Jl + 8 * L.bl_p[gb], Jl + 8 * L.bl_q[gb], Msh[l]);
  }
  __syncthreads();
  const T *C = static_cast<const T *>(B.C);
  for (int s = threadIdx.x; s < spb; s += kBlock) {
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int l = 0; l < Kf; ++l) {
      const T *c = C + 2 * (L.coh_off[f] + ((int64_t)l * nb + bi) * spb + s);
      const double cr = c[0], ci = c[1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        m[2 * e] += cr * Msh[l][2 * e] - ci * Msh[l][2 * e + 1];
        m[2 * e + 1] += cr * Msh[l][2 * e + 1] + ci * Msh[l][2 * e];
      }
    }
    T v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (T)m[e];
    store8<T>(o + 8 * s, v);
  }
}

}  // namespace

template <typename T>
hipError_t launch_refresh(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s) {
  const hipError_t e = launch_energy<T>(pb, L, B, s);
  if (e != hipSuccess || pb.ntiles == 0) return e;
  return launch_dall<false>(pb, L, B, s);
}
hipError_t launch_refresh_stats(const Problem &pb, const Layout &L, const Buffers &B, bool fold,
                                hipStream_t s) {
  if (pb.ntiles == 0) return hipSuccess;
  hipError_t e = launch_dall<true>(pb, L, B, s);
  if (e != hipSuccess || !fold) return e;
  hipLaunchKernelGGL(k_fold_energy, dim3((pb.ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pb, B);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_commit(const Problem &pb, const Layout &L, const Buffers &B, int k, int all,
                         hipStream_t s) {
  if (pb.ntiles == 0) return hipSuccess;
  if (pb.bpt > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_commit_stats, dim3((pb.ntiles + kStatTiles - 1) / kStatTiles),
                     dim3(64 * kStatTiles), 0, s, pb, L, B, k, all);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_model(const Problem &pb, const Layout &L, const Buffers &B, void *model_out,
                        const int64_t *full_off, const int32_t *full_bmap, hipStream_t s) {
  const int Bfull = pb.N * (pb.N - 1) / 2;
  hipLaunchKernelGGL(k_model<T>, dim3(Bfull, pb.P), dim3(kBlock), 0, s, pb, L, B,
                     static_cast<T *>(model_out), full_off, full_bmap);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_pack_stats(const Problem &pb, const Layout &L, const Buffers &B, const void *vis,
                             const void *coh, void *Vp, void *Cp, double *Sb,
                             const int64_t *in_vis_off, const int64_t *in_coh_off,
                             const int32_t *comp_tab, int nb_total, int *bad, int *status,
                             hipStream_t s) {
  if (nb_total == 0) return hipSuccess;
  if (pb.K > kMaxDirs || pb.max_nb <= 0) return hipErrorInvalidValue;
  // comp_tab: the full-layout baseline of each compact baseline (then its subband, unused here)
  const T *v = static_cast<const T *>(vis), *c = static_cast<const T *>(coh);
  T *vp = static_cast<T *>(Vp), *cp = static_cast<T *>(Cp);
  // 8 lanes per baseline for the subbands of up to 8 directions, 16 for the others (each lane
  // sums the statistics of one direction), one launch per lane count
  const dim3 grid8((pb.max_nb + kBlock / 8 - 1) / (kBlock / 8), pb.P);
  hipLaunchKernelGGL((k_pack_stats<T, 8>), grid8, dim3(kBlock), 0, s, pb, L, B, v, c, vp, cp, Sb,
                     in_vis_off, in_coh_off, comp_tab, bad, status);
  if (pb.K <= 8) return hipGetLastError();
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid16((pb.max_nb + kBlock / 16 - 1) / (kBlock / 16), pb.P);
  hipLaunchKernelGGL((k_pack_stats<T, 16>), grid16, dim3(kBlock), 0, s, pb, L, B, v, c, vp, cp, Sb,
                     in_vis_off, in_coh_off, comp_tab, bad, status);
  return hipGetLastError();
}

template hipError_t launch_refresh<float>(const Problem &, const Layout &, const Buffers &, hipStream_t);
template hipError_t launch_refresh<double>(const Problem &, const Layout &, const Buffers &, hipStream_t);
hipError_t launch_trial_stats(const Problem &pb, const Layout &L, const Buffers &B, int k,
                              hipStream_t s) {
  if (pb.ntiles == 0) return hipSuccess;
  if (pb.bpt > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trial_stats, dim3((pb.ntiles + kStatTiles - 1) / kStatTiles), dim3(64 * kStatTiles),
                     0, s, pb, L, B, k);
  return hipGetLastError();
}

template hipError_t launch_commit<float>(const Problem &, const Layout &, const Buffers &, int, int, hipStream_t);
template hipError_t launch_commit<double>(const Problem &, const Layout &, const Buffers &, int, int, hipStream_t);
template hipError_t launch_model<float>(const Problem &, const Layout &, const Buffers &, void *,
                                        const int64_t *, const int32_t *, hipStream_t);
template hipError_t launch_model<double>(const Problem &, const Layout &, const Buffers &, void *,
                                         const int64_t *, const int32_t *, hipStream_t);
template hipError_t launch_pack_stats<float>(const Problem &, const Layout &, const Buffers &, const void *,
                                             const void *, void *, void *, double *, const int64_t *,
                                             const int64_t *, const int32_t *, int, int *, int *,
                                             hipStream_t);
template hipError_t launch_pack_stats<double>(const Problem &, const Layout &, const Buffers &, const void *,
                                              const void *, void *, void *, double *, const int64_t *,
                                              const int64_t *, const int32_t *, int, int *, int *,
                                              hipStream_t);

}  // namespace calib
