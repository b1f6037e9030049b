// Launchers of the warm-start network kernels (mlp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace calib {

int mlp_gemm_scratch();   // floats of split-k partial sums mlp_gemm may use
// C = A' B' (see k_gemm_bf16); ws (mlp_gemm_scratch() floats, or null: no k split)
hipError_t mlp_gemm(const unsigned short *A, bool ta, const unsigned short *B, bool tb, float *C,
                    int M, int N, int K, float *ws, hipStream_t s);
hipError_t mlp_bias_act(const float *C, const float *b, float *Z, unsigned short *Hb, float *Y,
                        int64_t rows, int n, bool act, hipStream_t s);
hipError_t mlp_to_bf16(const float *x, unsigned short *y, int64_t n, hipStream_t s);
hipError_t mlp_mse(const float *Y, const float *T, unsigned short *dYb, double *part, int nparts,
                   int64_t total, float *loss, hipStream_t s);
int mlp_colsum_scratch(int n);   // doubles of partial sums mlp_colsum needs for n columns
hipError_t mlp_colsum(const unsigned short *dZb, float *gb, double *part, int64_t rows, int n,
                      hipStream_t s);
hipError_t mlp_gelu_back(const float *dA, const float *Z, unsigned short *dZb, int64_t n, hipStream_t s);
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, unsigned short *pb, int64_t n,
                    float lr, int step, hipStream_t s);

}  // namespace calib
