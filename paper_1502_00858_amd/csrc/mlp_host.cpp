// C ABI of the warm-start network: a fully connected GELU network (BF16 GEMM operands, FP32
// accumulation and master weights) evaluated and trained with Adam on the GPU.
#include "calib.h"
#include "mlp_internal.h"

#include <algorithm>
#include <string>
#include <vector>

using namespace calib;

namespace {
constexpr int kLossParts = 256;
thread_local std::string g_mlp_error;
}  // namespace

struct calib_mlp {
  int L = 0;
  std::vector<int> dims;
  int64_t max_rows = 0;
  int maxd = 0;
  hipStream_t stream = nullptr;
  std::vector<void *> allocs;
  std::vector<float *> W, b, gW, gb, mW, vW, mb, vb;
  std::vector<unsigned short *> Wb, Xb;   // BF16 weights; BF16 input of every layer
  std::vector<float *> Z;                 // FP32 pre-activations of the hidden layers
  float *C = nullptr, *Y = nullptr, *dA = nullptr;
  unsigned short *dZ0 = nullptr, *dZ1 = nullptr;
  double *part = nullptr;
  double *cpart = nullptr;   // column-sum partials
  float *ws = nullptr;       // split-k partial sums of the GEMMs
  std::string err;

  template <typename T>
  hipError_t alloc(T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) {
      allocs.push_back(q);
      *p = static_cast<T *>(q);
    }
    return e;
  }
};

namespace {

calib_status mfail(calib_mlp *m, calib_status st, const std::string &msg) {
  if (m) m->err = msg; else g_mlp_error = msg;
  return st;
}

#define MCHK(m, expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return mfail(m, CALIB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

calib_status forward(calib_mlp *m, const float *x, int64_t rows, float *y) {
  hipStream_t s = m->stream;
  MCHK(m, mlp_to_bf16(x, m->Xb[0], rows * m->dims[0], s));
  for (int l = 0; l < m->L; ++l) {
    const int in = m->dims[l], out = m->dims[l + 1];
    MCHK(m, mlp_gemm(m->Xb[l], false, m->Wb[l], false, m->C, (int)rows, out, in, m->ws, s));
    const bool last = (l == m->L - 1);
    MCHK(m, mlp_bias_act(m->C, m->b[l], last ? nullptr : m->Z[l], last ? nullptr : m->Xb[l + 1],
                         last ? (y ? y : m->Y) : nullptr, rows, out, !last, s));
  }
  return CALIB_OK;
}

}  // namespace

extern "C" {

const char *calib_mlp_last_error(const calib_mlp *m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

void calib_mlp_destroy(calib_mlp *m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  for (void *p : m->allocs) (void)hipFree(p);
  delete m;
}

calib_status calib_mlp_create(int32_t n_layers, const int32_t *dims, const float *params,
                              int64_t max_rows, void *hip_stream, calib_mlp **out) {
  g_mlp_error.clear();
  if (!out || !dims || !params || n_layers < 1 || max_rows < 1)
    return mfail(nullptr, CALIB_E_INVAL, "bad arguments");
  *out = nullptr;
  calib_mlp *m = new calib_mlp();
  m->L = n_layers;
  m->dims.assign(dims, dims + n_layers + 1);
  for (int d : m->dims)
    if (d < 1) { delete m; return mfail(nullptr, CALIB_E_INVAL, "layer widths must be >= 1"); }
  m->max_rows = max_rows;
  m->maxd = *std::max_element(m->dims.begin(), m->dims.end());
  m->stream = static_cast<hipStream_t>(hip_stream);
  auto oom = [&]() { calib_mlp_destroy(m); return mfail(nullptr, CALIB_E_NOMEM, "hipMalloc failed"); };
  const float *src = params;
  for (int l = 0; l < m->L; ++l) {
    const int in = m->dims[l], o = m->dims[l + 1];
    float *W, *b, *gW, *gb, *mW, *vW, *mb, *vb;
    unsigned short *Wb;
    if (m->alloc(&W, (size_t)in * o) || m->alloc(&b, o) || m->alloc(&gW, (size_t)in * o) ||
        m->alloc(&gb, o) || m->alloc(&mW, (size_t)in * o) || m->alloc(&vW, (size_t)in * o) ||
        m->alloc(&mb, o) || m->alloc(&vb, o) || m->alloc(&Wb, (size_t)in * o))
      return oom();
    m->W.push_back(W); m->b.push_back(b); m->gW.push_back(gW); m->gb.push_back(gb);
    m->mW.push_back(mW); m->vW.push_back(vW); m->mb.push_back(mb); m->vb.push_back(vb);
    m->Wb.push_back(Wb);
    hipError_t e = hipMemcpyAsync(W, src, sizeof(float) * in * o, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b, src + (size_t)in * o, sizeof(float) * o, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(mW, 0, sizeof(float) * in * o, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(vW, 0, sizeof(float) * in * o, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(mb, 0, sizeof(float) * o, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(vb, 0, sizeof(float) * o, m->stream);
    if (e == hipSuccess) e = mlp_to_bf16(W, Wb, (int64_t)in * o, m->stream);
    if (e != hipSuccess) { calib_mlp_destroy(m); return mfail(nullptr, CALIB_E_DEVICE, hipGetErrorString(e)); }
    src += (size_t)in * o + o;
  }
  for (int l = 0; l < m->L; ++l) {
    unsigned short *xb;
    if (m->alloc(&xb, (size_t)max_rows * m->dims[l])) return oom();
    m->Xb.push_back(xb);
    if (l < m->L - 1) {
      float *z;
      if (m->alloc(&z, (size_t)max_rows * m->dims[l + 1])) return oom();
      m->Z.push_back(z);
    }
  }
  const size_t big = (size_t)max_rows * m->maxd;
  if (m->alloc(&m->C, big) || m->alloc(&m->Y, (size_t)max_rows * m->dims[m->L]) ||
      m->alloc(&m->dA, big) || m->alloc(&m->dZ0, big) || m->alloc(&m->dZ1, big) ||
      m->alloc(&m->part, kLossParts) || m->alloc(&m->cpart, (size_t)mlp_colsum_scratch(m->maxd)) ||
      m->alloc(&m->ws, (size_t)mlp_gemm_scratch()))
    return oom();
  if (hipStreamSynchronize(m->stream) != hipSuccess) {
    calib_mlp_destroy(m);
    return mfail(nullptr, CALIB_E_DEVICE, "stream synchronisation failed");
  }
  *out = m;
  return CALIB_OK;
}

calib_status calib_mlp_forward(calib_mlp *m, const float *x, int64_t rows, float *y) {
  if (!m) return CALIB_E_INVAL;
  if (!x || !y || rows < 1 || rows > m->max_rows) return mfail(m, CALIB_E_INVAL, "bad rows or pointers");
  return forward(m, x, rows, y);
}

calib_status calib_mlp_train_step(calib_mlp *m, const float *x, const float *target, int64_t rows,
                                  float lr, int32_t step, float *loss) {
  if (!m) return CALIB_E_INVAL;
  if (!x || !target || rows < 1 || rows > m->max_rows || step < 1)
    return mfail(m, CALIB_E_INVAL, "bad rows, step or pointers");
  hipStream_t s = m->stream;
  calib_status st = forward(m, x, rows, nullptr);
  if (st != CALIB_OK) return st;
  const int L = m->L;
  MCHK(m, mlp_mse(m->Y, target, m->dZ0, m->part, kLossParts, rows * m->dims[L], loss, s));
  unsigned short *dz = m->dZ0, *dz_next = m->dZ1;
  for (int l = L - 1; l >= 0; --l) {
    const int in = m->dims[l], out = m->dims[l + 1];
    // dW_l = X_l^T dZ_l, db_l = column sums of dZ_l
    MCHK(m, mlp_gemm(m->Xb[l], true, dz, false, m->gW[l], in, out, (int)rows, m->ws, s));
    MCHK(m, mlp_colsum(dz, m->gb[l], m->cpart, rows, out, s));
    if (l > 0) {
      // dX_l = dZ_l W_l^T, then through the GELU of layer l-1
      MCHK(m, mlp_gemm(dz, false, m->Wb[l], true, m->dA, (int)rows, in, out, m->ws, s));
      MCHK(m, mlp_gelu_back(m->dA, m->Z[l - 1], dz_next, rows * in, s));
      std::swap(dz, dz_next);
    }
  }
  if (lr > 0.f)
    for (int l = 0; l < L; ++l) {
      const int64_t nw = (int64_t)m->dims[l] * m->dims[l + 1];
      MCHK(m, mlp_adam(m->W[l], m->gW[l], m->mW[l], m->vW[l], m->Wb[l], nw, lr, step, s));
      MCHK(m, mlp_adam(m->b[l], m->gb[l], m->mb[l], m->vb[l], nullptr, m->dims[l + 1], lr, step, s));
    }
  return CALIB_OK;
}

calib_status calib_mlp_get(calib_mlp *m, int32_t what, float *dst) {
  if (!m) return CALIB_E_INVAL;
  if (!dst || (what != 0 && what != 1)) return mfail(m, CALIB_E_INVAL, "bad field or pointer");
  MCHK(m, hipStreamSynchronize(m->stream));
  float *o = dst;
  for (int l = 0; l < m->L; ++l) {
    const size_t nw = (size_t)m->dims[l] * m->dims[l + 1], nb = m->dims[l + 1];
    MCHK(m, hipMemcpy(o, what == 0 ? m->W[l] : m->gW[l], nw * sizeof(float), hipMemcpyDeviceToHost));
    MCHK(m, hipMemcpy(o + nw, what == 0 ? m->b[l] : m->gb[l], nb * sizeof(float), hipMemcpyDeviceToHost));
    o += nw + nb;
  }
  return CALIB_OK;
}

}  // extern "C"
