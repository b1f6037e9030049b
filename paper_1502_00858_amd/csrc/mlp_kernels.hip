// Kernels of the warm-start network: a fully connected GELU network trained and evaluated on the
// GPU.  GEMMs run on v_mfma_f32_16x16x16bf16_1k (BF16 operands, FP32 accumulation); master
// weights, biases, Adam moments, pre-activations and gradients are FP32.
#include "calib_internal.h"
#include "mlp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace calib {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 32;   // output tile and k step of one workgroup
constexpr int kLdk = kTK + 8;                   // LDS row stride (80 bytes: conflict-free 8-byte reads)

__device__ inline unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// One k step's share of an operand tile (64 rows x 32 k) for one thread: 8 elements, as one
// 16-byte load where the run is whole and aligned.  KC: the operand is stored [rows][K] (k
// contiguous: the thread takes row t/4, k 8(t%4)..+7); else stored [K][rows] (rows contiguous: k
// t/8, rows 8(t%8)..+7).  Elements outside rows < R, k < kend read as zero.
template <bool KC>
__device__ inline uint4 fetch8(const unsigned short *X, int R, int K, int r0, int k0, int kend,
                               bool vec) {
  const int t = threadIdx.x;
  const int r = r0 + (KC ? t >> 2 : (t & 7) * 8), k = k0 + (KC ? (t & 3) * 8 : t >> 3);
  const bool whole = KC ? (r < R && k + 8 <= kend) : (k < kend && r + 8 <= R);
  if (vec && whole)
    return *reinterpret_cast<const uint4 *>(KC ? X + (int64_t)r * K + k : X + (int64_t)k * R + r);
  unsigned short v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int re = KC ? r : r + e, ke = KC ? k + e : k;
    v[e] = (re < R && ke < kend) ? (KC ? X[(int64_t)re * K + ke] : X[(int64_t)ke * R + re]) : 0;
  }
  uint4 u;
  u.x = v[0] | ((unsigned)v[1] << 16);
  u.y = v[2] | ((unsigned)v[3] << 16);
  u.z = v[4] | ((unsigned)v[5] << 16);
  u.w = v[6] | ((unsigned)v[7] << 16);
  return u;
}

// Stores a thread's 8 elements into the [row][k] LDS tile (one 16-byte write when k is contiguous)
template <bool KC>
__device__ inline void put8(unsigned short (*S)[kLdk], uint4 u) {
  const int t = threadIdx.x;
  if (KC) {
    *reinterpret_cast<uint4 *>(&S[t >> 2][(t & 3) * 8]) = u;
  } else {
    const int k = t >> 3, r = (t & 7) * 8;
    const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      S[r + 2 * e][k] = (unsigned short)(w[e] & 0xFFFFu);
      S[r + 2 * e + 1][k] = (unsigned short)(w[e] >> 16);
    }
  }
}

// C[M][N] = A'[M][K] B'[K][N] (FP32 out).  A' = A (stored [M][K]) or A^T (A stored [K][M]);
// B' = B (stored [K][N]) or B^T (B stored [N][K]).  Out-of-range elements load as zero.
// Workgroup z of a split launch sums k in [z kchunk, (z+1) kchunk) into its own slice of ws
// ([splits][M][N]), added in a fixed order afterwards; with one split it writes C.  The next k
// step's operands are fetched into registers while the MFMAs consume the current one from LDS.
// MFMA layouts (16x16x16 bf16): A lane l holds A[l%16][4(l/16)+e], B lane l holds
// B[4(l/16)+e][l%16], accumulator element r of lane l is D[4(l/16)+r][l%16].
template <bool TA, bool TB>
__global__ __launch_bounds__(kBlock) void k_gemm_bf16(const unsigned short *A, const unsigned short *B,
                                                      float *C, float *ws, int M, int N, int K,
                                                      int kchunk, int avec, int bvec) {
  __shared__ __align__(16) unsigned short As[kTM][kLdk];   // [m][k]
  __shared__ __align__(16) unsigned short Bs[kTN][kLdk];   // [n][k]
  const int m0 = blockIdx.x * kTM, n0 = blockIdx.y * kTN;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;   // 2x2 waves, 32x32 each
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  uint4 ra = fetch8<!TA>(A, M, K, m0, kb, ke, avec), rb = fetch8<TB>(B, N, K, n0, kb, ke, bvec);
  for (int k0 = kb; k0 < ke; k0 += kTK) {
    put8<!TA>(As, ra);
    put8<TB>(Bs, rb);
    __syncthreads();
    if (k0 + kTK < ke) {
      ra = fetch8<!TA>(A, M, K, m0, k0 + kTK, ke, avec);
      rb = fetch8<TB>(B, N, K, n0, k0 + kTK, ke, bvec);
    }
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 16) {
      s4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const s4 *>(&As[wm + i * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
        b[i] = *reinterpret_cast<const s4 *>(&Bs[wn + i * 16 + (lane & 15)][ks + 4 * (lane >> 4)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float *out = gridDim.z == 1 ? C : ws + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r, gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) out[(int64_t)gm * N + gn] = acc[i][j][r];
      }
}

// C = sum over the splits of ws, in split order
__global__ void k_splitk_sum(const float *ws, float *C, int64_t n, int splits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = ws[i];
  for (int z = 1; z < splits; ++z) s += ws[(int64_t)z * n + i];
  C[i] = s;
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Z = C + b (kept), out = BF16(GELU(Z)) or, for the last layer, Y = Z
__global__ void k_bias_act(const float *C, const float *b, float *Z, unsigned short *Hb, float *Y,
                           int64_t rows, int n, int act) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * n) return;
  const float z = C[i] + b[i % n];
  if (act) {
    Z[i] = z;
    Hb[i] = bf16_rne(gelu(z));
  } else {
    Y[i] = z;
  }
}

__global__ void k_to_bf16(const float *x, unsigned short *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = bf16_rne(x[i]);
}

// mean-square error loss: dY = 2 (Y - T) / (rows n) as BF16, per-block loss partials (FP64)
__global__ __launch_bounds__(kBlock) void k_mse(const float *Y, const float *T, unsigned short *dYb,
                                                double *part, int64_t total) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const float d = Y[i] - T[i];
    s += (double)d * d;
    dYb[i] = bf16_rne(2.0f * d / (float)total);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one wavefront: lane l sums the partials l, l + 64, ... in order, then a butterfly over lanes
__global__ void k_loss_final(const double *part, int nparts, int64_t total, float *loss) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int i = lane; i < nparts; i += 64) s += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) loss[0] = (float)(s / (double)total);
}

// gb[j] = sum over rows of dZ[r][j] (dZ stored BF16) in two fixed-order stages: workgroup
// (x, y) sums columns 64x..64x+63 over the rows r = 4y + g + 4*kColsumGroups*i (g: wavefront),
// the four wavefronts combine in LDS, then k_colsum_final adds the kColsumGroups partials
constexpr int kColsumGroups = 16;
__global__ __launch_bounds__(kBlock) void k_colsum(const unsigned short *dZb, double *part,
                                                   int64_t rows, int n) {
  __shared__ double red[4][64];
  const int j = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  double s = 0.0;
  if (j < n)
    for (int64_t r = 4 * blockIdx.y + g; r < rows; r += 4 * kColsumGroups) s += bf16_to_f(dZb[r * n + j]);
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && j < n)
    part[(int64_t)blockIdx.y * n + j] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                        (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void k_colsum_final(const double *part, float *gb, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int y = 0; y < kColsumGroups; ++y) s += part[(int64_t)y * n + j];
  gb[j] = (float)s;
}

// dZ = dA * GELU'(Z) stored BF16
__global__ void k_gelu_back(const float *dA, const float *Z, unsigned short *dZb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dZb[i] = bf16_rne(dA[i] * gelu_grad(Z[i]));
}

// Adam on FP32 master parameters; refreshes the BF16 copy of the weights
__global__ void k_adam(float *p, const float *g, float *m, float *v, unsigned short *pb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  const float np = p[i] - upd;
  p[i] = np;
  if (pb) pb[i] = bf16_rne(np);
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int mlp_gemm_scratch() { return 256 * kTM * kTN; }

hipError_t mlp_gemm(const unsigned short *A, bool ta, const unsigned short *B, bool tb, float *C,
                    int M, int N, int K, float *ws, hipStream_t s) {
  if (M < 1 || N < 1 || K < 1) return hipErrorInvalidValue;
  const int tiles_m = (M + kTM - 1) / kTM, tiles_n = (N + kTN - 1) / kTN;
  const int tiles = tiles_m * tiles_n, ksteps = (K + kTK - 1) / kTK;
  // split k over more workgroups when the output tiles alone fill under half the chip, each
  // split keeping at least two k steps; split partial sums fit the scratch by construction
  // (splits <= 256 / tiles and M N <= tiles kTM kTN)
  int splits = 1;
  if (ws && tiles < 128) splits = std::max(1, std::min(ksteps / 2, 256 / tiles));
  const int kchunk = ((ksteps + splits - 1) / splits) * kTK;
  splits = (K + kchunk - 1) / kchunk;
  if (splits > 1 && (int64_t)splits * M * N > mlp_gemm_scratch()) return hipErrorInvalidValue;
  auto aligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const int avec = aligned(A) && ((ta ? M : K) % 8 == 0);
  const int bvec = aligned(B) && ((tb ? K : N) % 8 == 0);
  dim3 grid(tiles_m, tiles_n, splits), block(kBlock);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, block, 0, s, A, B, C, ws, M, N, K, kchunk, avec, bvec);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, block, 0, s, A, B, C, ws, M, N, K, kchunk, avec, bvec);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, block, 0, s, A, B, C, ws, M, N, K, kchunk, avec, bvec);
  else hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, block, 0, s, A, B, C, ws, M, N, K, kchunk, avec, bvec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t n = (int64_t)M * N;
  hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws, C, n, splits);
  return hipGetLastError();
}

hipError_t mlp_bias_act(const float *C, const float *b, float *Z, unsigned short *Hb, float *Y,
                        int64_t rows, int n, bool act, hipStream_t s) {
  hipLaunchKernelGGL(k_bias_act, dim3(blocks(rows * n)), dim3(256), 0, s, C, b, Z, Hb, Y, rows, n, act ? 1 : 0);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *x, unsigned short *y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t mlp_mse(const float *Y, const float *T, unsigned short *dYb, double *part, int nparts,
                   int64_t total, float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(nparts), dim3(kBlock), 0, s, Y, T, dYb, part, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss) return e;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, part, nparts, total, loss);
  return hipGetLastError();
}

int mlp_colsum_scratch(int n) { return kColsumGroups * n; }

hipError_t mlp_colsum(const unsigned short *dZb, float *gb, double *part, int64_t rows, int n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(blocks(n, 64), kColsumGroups), dim3(kBlock), 0, s, dZb, part, rows, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3(blocks(n, 64)), dim3(64), 0, s, part, gb, n);
  return hipGetLastError();
}

hipError_t mlp_gelu_back(const float *dA, const float *Z, unsigned short *dZb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_back, dim3(blocks(n)), dim3(256), 0, s, dA, Z, dZb, n);
  return hipGetLastError();
}

hipError_t mlp_adam(float *p, const float *g, float *m, float *v, unsigned short *pb, int64_t n,
                    float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace calib
