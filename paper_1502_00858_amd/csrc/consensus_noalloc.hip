// Context-free fusion-centre update that allocates no device memory (calib_consensus_noalloc).
//
// It runs the kernels of admm_consensus_update after the first iteration - the least-squares
// operator of the basis matrix, Z_k = argmin sum_f ||J_fk + Y_fk/rho_k - B_f Z_k||^2 (M2 of
// Section 3), B_f Z_k, Y_fk += rho_k (J_fk - B_f Z_k) (M3) and the residuals of Section 4.1 - on
// caller-owned J, Y, Z and B_f Z.  What those kernels keep beyond their inputs and outputs (the
// basis values, the per-direction least-squares operator, the residual partials, the direction
// counts, a rank flag and the iteration counter) lives in one file-scope device array, so the
// call makes no allocation and can be captured into a HIP graph or issued from a serving loop.
//
// Every GPU holds its own copy of the array (until the process ends); its device address is
// taken once per device with hipGetSymbolAddress and used for every kernel argument.  Calls that
// overlap on one GPU share the array and race; each call rewrites everything it reads.
#include "calib.h"
#include "calib_internal.h"

#include <mutex>
#include <string>

namespace calib {
namespace {

// scratch size in doubles (4 MiB): basis P*Q, operator K*Q*P, residual partials P*K + 16K, four
// trace values, then the int region (iteration counter, rank flag, P direction counts)
constexpr int64_t kScratchDoubles = int64_t(1) << 19;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// device address of this device's scratch array (taken on the first call on the device)
hipError_t scratch_address(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double *>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

int64_t scratch_need(int P, int Q, int K) {
  const int64_t ints = 2 + (int64_t)P;
  return (int64_t)P * Q + (int64_t)K * Q * P + (int64_t)P * K + (int64_t)K * kZChunks + 4 + (ints + 1) / 2;
}

// per-call set-up of the scratch's int region: iteration counter 0, rank flag 0, direction counts
// (n_dirs, or K for every subband)
__global__ void k_noalloc_begin(int *ints, const int32_t *n_dirs, int P, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2) ints[i] = 0;
  if (i < P) ints[2 + i] = n_dirs ? n_dirs[i] : K;
}

// the residuals (primal, dual) and the status to the caller
__global__ void k_noalloc_end(const double *trace, const int *rank_fail, double *residuals,
                              int32_t *status) {
  if (threadIdx.x != 0) return;
  const bool fail = *rank_fail != 0;
  if (residuals && !fail) {
    residuals[0] = trace[2];
    residuals[1] = trace[3];
  }
  if (status) *status = fail ? CALIB_E_RANK : CALIB_OK;
}

calib_status fail_msg(calib_status st, const std::string &m) {
  set_context_free_error(m.c_str());
  return st;
}

}  // namespace
}  // namespace calib

using namespace calib;

extern "C" calib_status calib_consensus_noalloc(int32_t n_stations, int32_t n_subbands,
                                                int32_t n_basis, int32_t n_dirs_max,
                                                const int32_t *n_dirs, const double *freq_hz,
                                                double f0_hz, const double *rho,
                                                const double *jones, double *y, double *z,
                                                double *bz, double *residuals, int32_t *status,
                                                void *hip_stream) {
  const int N = n_stations, P = n_subbands, Q = n_basis, K = n_dirs_max;
  if (N < 2 || N > kMaxStations) return fail_msg(CALIB_E_INVAL, "n_stations must be in [2, 128]");
  if (P < 1) return fail_msg(CALIB_E_INVAL, "n_subbands must be >= 1");
  if (Q < 1 || Q > 8) return fail_msg(CALIB_E_INVAL, "n_basis must be in [1, 8]");
  if (K < 1 || K > kMaxDirs) return fail_msg(CALIB_E_INVAL, "n_dirs_max must be in [1, 16]");
  if (!(f0_hz > 0.0)) return fail_msg(CALIB_E_INVAL, "f0_hz must be positive");
  if (!freq_hz || !rho || !jones || !y || !z || !bz)
    return fail_msg(CALIB_E_INVAL, "freq_hz, rho, jones, y, z and bz are required");
  const int64_t need = scratch_need(P, Q, K);
  if (need > kScratchDoubles)
    return fail_msg(CALIB_E_INVAL, "problem too large for the scratch array: needs " +
                                       std::to_string(need) + " doubles, holds " +
                                       std::to_string(kScratchDoubles) +
                                       " (P*(Q + K*Q + K) + 16K + 4 + (P + 3)/2)");
  double *base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return fail_msg(CALIB_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));

  double *basis = base;
  double *fitw = basis + (int64_t)P * Q;
  double *part = fitw + (int64_t)K * Q * P;
  double *trace = part + (int64_t)P * K + (int64_t)K * kZChunks;
  int *ints = reinterpret_cast<int *>(trace + 4);
  int *iter = ints, *rank_fail = ints + 1;
  int32_t *ndir = ints + 2;

  Problem pb{};
  pb.N = N; pb.P = P; pb.Q = Q; pb.K = K;
  Layout L{};
  L.ndir = ndir;
  Buffers B{};
  B.J = const_cast<double *>(jones);
  B.Y = y; B.Z = z; B.BZ = bz;
  B.rho = rho; B.basis = basis; B.fitw = fitw;
  B.scratch = part; B.trace = trace; B.iter = iter;
  B.rank_fail = rank_fail;

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int threads = 256, blocks = (P + 2 + threads - 1) / threads;
  hipLaunchKernelGGL(k_noalloc_begin, dim3(blocks), dim3(threads), 0, s, ints, n_dirs, P, K);
  e = hipGetLastError();
  if (e == hipSuccess) e = launch_basis_setup(pb, freq_hz, f0_hz, ndir, basis, fitw, rank_fail, s);
  if (e == hipSuccess) e = launch_consensus(pb, L, B, kPenaltyNone, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(64), 0, s, trace, rank_fail, residuals, status);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail_msg(CALIB_E_DEVICE, std::string("consensus launch: ") + hipGetErrorString(e));
  return CALIB_OK;
}
