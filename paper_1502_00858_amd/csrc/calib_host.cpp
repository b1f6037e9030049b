// Host side of the C ABI: validation, packing, workspace management and the launch sequence of
// the consensus-ADMM iteration (Section 3, steps D1-D3).  Every arithmetic step of the method
// runs in the HIP kernels; this file only prepares index tables and enqueues work.
#include "calib.h"
#include "calib_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace calib;

static_assert(CALIB_WS_FEATURES == kWsFeatures && CALIB_WS_OUTPUTS == kWsOutputs,
              "warm-start row widths of the ABI and the kernels differ");

namespace {
constexpr int kMaxTrace = 4096;
thread_local std::string g_init_error;

struct DevAlloc {
  std::vector<void *> ptrs;
  hipError_t alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};
}  // namespace

void calib::set_context_free_error(const char *msg) { g_init_error = msg; }

struct calib_ctx {
  int N = 0, P = 0, Q = 0, K = 0, T = 0;
  calib_precision precision = CALIB_FP64;
  int lm_iters = 1, sage_sweeps = 1;
  uint32_t options = 0;
  double f0 = 0.0;
  std::vector<int32_t> n_chan, n_dirs;
  std::vector<double> freq, rho;
  hipStream_t stream = nullptr;
  Problem pb{};
  Layout L{};
  Buffers B{};
  DevAlloc mem;
  int64_t total_full_samples = 0;
  int64_t *d_full_off = nullptr;
  int32_t *d_full_bmap = nullptr;
  // packing of a solution interval's inputs (calib_init, calib_set_data)
  int64_t *d_in_vis_off = nullptr, *d_in_coh_off = nullptr;
  int32_t *d_comp = nullptr;   // full-layout baseline of each compact baseline, then its subband
  int nb_total = 0;
  void *Vp = nullptr, *Cp = nullptr;
  double *Sb = nullptr;
  int32_t *d_ndir = nullptr;
  double *lm_trace = nullptr;
  int iters_done = 0;
  std::string err;
  // per-kernel event timing (measurement aid)
  bool timing = false;
  std::vector<hipEvent_t> events;
  std::vector<std::pair<int, size_t>> pending;
  size_t next_event = 0;
  double kms[CALIB_NUM_KERNELS] = {0};
  double kcount[CALIB_NUM_KERNELS] = {0};
  // one captured ADMM iteration (iterations >= 1 share their launch sequence)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // the local step under the LM stopping rule: after each step's solve the device writes here
  // whether every subband has finished its local step, and the host reads it before launching
  // the next step
  int *stop_flag = nullptr;                 // pinned host memory
  // warm start
  double *ws_jsave = nullptr;   // [P][K][N][8]
  double *ws_cost = nullptr;    // [2][P]
};

namespace {

constexpr size_t kMaxPendingEvents = 4096;

hipError_t flush_timing(calib_ctx *c) {
  if (c->pending.empty()) return hipSuccess;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  for (auto &pr : c->pending) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, c->events[pr.second], c->events[pr.second + 1]);
    if (e != hipSuccess) return e;
    c->kms[pr.first] += ms;
    c->kcount[pr.first] += 1.0;
  }
  c->pending.clear();
  c->next_event = 0;
  return hipSuccess;
}

// Launch through `launch`, bracketed by an event pair on the context stream when timing is on.
template <typename F>
hipError_t timed(calib_ctx *c, int id, F &&launch) {
  if (!c->timing) return launch();
  if (c->pending.size() >= kMaxPendingEvents) {
    hipError_t e = flush_timing(c);
    if (e != hipSuccess) return e;
  }
  while (c->next_event + 2 > c->events.size()) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    c->events.push_back(ev);
  }
  const size_t i = c->next_event;
  c->next_event += 2;
  hipError_t e = hipEventRecord(c->events[i], c->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(c->events[i + 1], c->stream);
  c->pending.emplace_back(id, i);
  return e;
}

calib_status fail(calib_ctx *ctx, calib_status st, const std::string &msg) {
  if (ctx) ctx->err = msg; else g_init_error = msg;
  return st;
}

#define HIPCHK(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, CALIB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define ALLOC(ctx, ptr, bytes)                                                                 \
  do {                                                                                         \
    void *p_ = nullptr;                                                                        \
    if ((ctx)->mem.alloc(&p_, (bytes)) != hipSuccess)                                          \
      return fail(ctx, CALIB_E_NOMEM, "hipMalloc failed for " #ptr);                           \
    ptr = reinterpret_cast<decltype(ptr)>(p_);                                                 \
  } while (0)

template <typename V>
calib_status upload(calib_ctx *ctx, V **dst, const std::vector<V> &src) {
  ALLOC(ctx, *dst, sizeof(V) * std::max<size_t>(src.size(), 1));
  if (!src.empty())
    HIPCHK(ctx, hipMemcpyAsync(*dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice,
                               ctx->stream));
  return CALIB_OK;
}

// lanes per baseline for the streaming kernels: the configured value, else the fewest idle
// lane-iterations over the subbands, ties to the larger group
int choose_group(const std::vector<int32_t> &spb, const std::vector<int32_t> &nb, int requested,
                 bool matrix_free) {
  if (requested == 4 || requested == 8 || requested == 16 || requested == 32 || requested == 64)
    return requested;
  // the matrix-free solver's per-baseline kernels take one lane per baseline of a tile: 64
  // baselines per tile fill every lane (its samples are read only by the per-interval pack, whose
  // shape does not depend on the tile)
  if (matrix_free) return 4;
  int best = 16;
  double best_w = 1e300;
  for (int g : {64, 32, 16, 8}) {
    double w = 0.0;
    for (size_t f = 0; f < spb.size(); ++f) {
      const int it = (spb[f] + g - 1) / g;
      w += (double)nb[f] * (double)(it * g - spb[f]);
    }
    if (w < best_w) { best_w = w; best = g; }
  }
  return best;
}

// one LM iteration of direction k (k < 0: of each subband's own direction): normal equations,
// solve, trial point, accept / damping; with flag (own directions only), the stop flag right
// after the solve
template <typename T>
calib_status lm_iteration(calib_ctx *c, int k, int it, int unreg, hipStream_t s, int *flag = nullptr) {
  const Problem &pb = c->pb;
  const Layout &L = c->L;
  const Buffers &B = c->B;
  HIPCHK(c, timed(c, CALIB_KERNEL_ASSEMBLE, [&] { return launch_assemble(pb, L, B, k, unreg, s); }));
  HIPCHK(c, timed(c, CALIB_KERNEL_CHOL_SOLVE, [&] {
    return pb.solver == kSolverBlocked
               ? launch_chol_blocked(pb, B, k, c->d_ndir, B.chol_ld, B.chol_fail, s)
               : launch_chol_solve_nd(pb, B, k, c->d_ndir, s);
  }));
  if (flag) HIPCHK(c, launch_lm_stopped(pb, L, B, flag, c->lm_iters, c->sage_sweeps, s));
  HIPCHK(c, timed(c, CALIB_KERNEL_TRIAL, [&] { return launch_trial_stats(pb, L, B, k, s); }));
  HIPCHK(c, timed(c, CALIB_KERNEL_LM_UPDATE, [&] {
    return launch_lm_update_tr(pb, L, B, k, unreg, c->lm_trace, it, c->lm_iters, s);
  }));
  return CALIB_OK;
}

template <typename T>
calib_status run_local_step(calib_ctx *c, int admm_iter, hipStream_t s) {
  const int unreg = (admm_iter == 0 && (c->options & CALIB_OPT_UNREG_FIRST)) ? 1 : 0;
  const Problem &pb = c->pb;
  const Layout &L = c->L;
  const Buffers &B = c->B;
  if (pb.solver == kSolverPcg) {
    // every D_l and the residual's energy from the coherency statistics (no pass over the
    // samples), then every subband's whole local step in one launch: the LM runs, the stopping
    // rule and the SAGE commits stay on the device
    HIPCHK(c, timed(c, CALIB_KERNEL_REFRESH, [&] { return launch_refresh_stats(pb, L, B, false, s); }));
    HIPCHK(c, timed(c, CALIB_KERNEL_LOCAL_STEP, [&] {
      return launch_local_step(pb, L, B, unreg, c->lm_trace, c->lm_iters, c->sage_sweeps, s);
    }));
    return CALIB_OK;
  }
  HIPCHK(c, timed(c, CALIB_KERNEL_REFRESH, [&] { return launch_refresh<T>(pb, L, B, s); }));
  for (int sw = 0; sw < c->sage_sweeps; ++sw)
    for (int k = 0; k < c->K; ++k) {
      HIPCHK(c, timed(c, CALIB_KERNEL_LM_BEGIN, [&] { return launch_lm_begin(pb, L, B, k, unreg, s); }));
      for (int it = 0; it < c->lm_iters; ++it) {
        const calib_status st = lm_iteration<T>(c, k, it, unreg, s);
        if (st != CALIB_OK) return st;
      }
      HIPCHK(c, timed(c, CALIB_KERNEL_COMMIT, [&] { return launch_commit<T>(pb, L, B, k, c->sage_sweeps > 1, s); }));
    }
  return CALIB_OK;
}

calib_status local_step_on(calib_ctx *c, int admm_iter, hipStream_t s) {
  return c->precision == CALIB_FP64 ? run_local_step<double>(c, admm_iter, s)
                                    : run_local_step<float>(c, admm_iter, s);
}

// The stop flag of the step just enqueued: the stopped kernel overwrites the -1 the host left in
// the pinned word with 0 (running) or 1 (stopped).  The host spins on it, so the next launch
// follows the flag within microseconds; after 50 ms it synchronises the stream instead, which also
// reports a device error.
calib_status wait_stop_flag(calib_ctx *c, hipStream_t s, bool *stopped) {
  volatile int *fl = c->stop_flag;
  const auto t0 = std::chrono::steady_clock::now();
  int v;
  while ((v = *fl) < 0) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
      HIPCHK(c, hipStreamSynchronize(s));
      v = *fl;
      if (v < 0) return fail(c, CALIB_E_DEVICE, "the LM stop flag was not written");
      break;
    }
  }
  *stopped = v == 1;
  return CALIB_OK;
}

// The local step under the LM stopping rule (per subband the same results as run_local_step).
// Every launch of a step takes each subband's own direction: a subband whose LM run has stopped
// commits it and starts its next direction's run in the next step while the others still iterate,
// so a step costs one solve per subband that still works and no launch waits for the slowest
// subband of a direction.  After each step the host reads the stop flag (written right after the
// solve: the host enqueues the next step while the trial point and the update run) and ends the
// loop once every subband has finished its last run.  The kernels are launched directly, not from
// captured graphs (a graph per step was measured slower: the flag would come only at its end).
template <typename T>
calib_status run_local_step_stopping(calib_ctx *c, int admm_iter, hipStream_t s) {
  const int unreg = (admm_iter == 0 && (c->options & CALIB_OPT_UNREG_FIRST)) ? 1 : 0;
  const Problem &pb = c->pb;
  const Layout &L = c->L;
  const Buffers &B = c->B;
  const int sweeps = c->sage_sweeps, all = sweeps > 1;
  HIPCHK(c, timed(c, CALIB_KERNEL_REFRESH, [&] { return launch_refresh<T>(pb, L, B, s); }));
  HIPCHK(c, launch_dir_reset(pb, B, s));
  // each step runs one LM iteration of every unfinished subband: at most sweeps x K x lm_iters
  const int64_t max_steps = (int64_t)sweeps * c->K * c->lm_iters;
  bool stopped = max_steps == 0;
  for (int64_t step = 0; step < max_steps && !stopped; ++step) {
    *reinterpret_cast<volatile int *>(c->stop_flag) = -1;
    HIPCHK(c, timed(c, CALIB_KERNEL_COMMIT, [&] { return launch_commit<T>(pb, L, B, -1, all, s); }));
    HIPCHK(c, timed(c, CALIB_KERNEL_LM_BEGIN, [&] { return launch_lm_begin(pb, L, B, -1, unreg, s, sweeps); }));
    calib_status st = lm_iteration<T>(c, -1, -1, unreg, s, c->stop_flag);
    if (st == CALIB_OK) st = wait_stop_flag(c, s, &stopped);
    if (st != CALIB_OK) return st;
  }
  if (!stopped) return fail(c, CALIB_E_STATE, "the local step did not finish within its LM iterations");
  HIPCHK(c, timed(c, CALIB_KERNEL_COMMIT, [&] { return launch_commit<T>(pb, L, B, -1, all, s); }));
  return CALIB_OK;
}

calib_status local_step_stopping_on(calib_ctx *c, int admm_iter, hipStream_t s) {
  return c->precision == CALIB_FP64 ? run_local_step_stopping<double>(c, admm_iter, s)
                                    : run_local_step_stopping<float>(c, admm_iter, s);
}

// Lagrangian trace row, first-iteration alignment, Z, B_f Z, Y and residuals; the trace row is
// the device iteration counter, which the last kernel advances
calib_status consensus_on(calib_ctx *c, bool gpa, hipStream_t s) {
  HIPCHK(c, timed(c, CALIB_KERNEL_CONSENSUS, [&] {
    hipError_t e = hipSuccess;
    if (gpa) {   // the trace row's penalty at the local step's J, before the alignment rotates it
      e = launch_penalty_part(c->pb, c->L, c->B, s);
      if (e == hipSuccess) e = launch_gpa(c->pb, c->L, c->B, 3, s);
    }
    if (e == hipSuccess)
      e = launch_consensus(c->pb, c->L, c->B, gpa ? kPenaltyTaken : kPenaltyInYUpdate, s);
    return e;
  }));
  return CALIB_OK;
}

// capture the launch sequence of one ADMM iteration >= 1 into a graph (recorded, not run)
calib_status build_iteration_graph(calib_ctx *c) {
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  calib_status st = local_step_on(c, 1, c->cap_stream);
  if (st == CALIB_OK) st = consensus_on(c, false, c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (st != CALIB_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(c, CALIB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  return CALIB_OK;
}

}  // namespace

extern "C" {

const char *calib_last_error(const calib_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

void calib_destroy(calib_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->stop_flag) (void)hipHostFree(ctx->stop_flag);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
  ctx->mem.release();
  delete ctx;
}

calib_status calib_init(const calib_config *cfg, const void *vis, const void *coh,
                        const uint8_t *flags, const void *jones0, void *hip_stream,
                        calib_ctx **out) {
  g_init_error.clear();
  if (!out) return fail(nullptr, CALIB_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !vis || !coh) return fail(nullptr, CALIB_E_INVAL, "cfg, vis and coh are required");
  const int N = cfg->n_stations, P = cfg->n_subbands, Q = cfg->n_basis, K = cfg->n_dirs_max,
            T = cfg->n_times;
  if (N < 2 || N > kMaxStations) return fail(nullptr, CALIB_E_INVAL, "n_stations must be in [2, 128]");
  if (P < 1) return fail(nullptr, CALIB_E_INVAL, "n_subbands must be >= 1");
  if (Q < 1 || Q > 8) return fail(nullptr, CALIB_E_INVAL, "n_basis must be in [1, 8]");
  if (K < 1 || K > kMaxDirs) return fail(nullptr, CALIB_E_INVAL, "n_dirs_max must be in [1, 16]");
  if (T < 1) return fail(nullptr, CALIB_E_INVAL, "n_times must be >= 1");
  if (!cfg->n_chan || !cfg->freq_hz || !cfg->rho)
    return fail(nullptr, CALIB_E_INVAL, "n_chan, freq_hz and rho are required");
  if (!(cfg->f0_hz > 0.0) || !std::isfinite(cfg->f0_hz))
    return fail(nullptr, CALIB_E_INVAL, "f0_hz must be positive");
  if (cfg->precision != CALIB_FP64 && cfg->precision != CALIB_FP32_MIXED)
    return fail(nullptr, CALIB_E_INVAL, "unknown precision");
  if (cfg->lm_iters < 1 || cfg->sage_sweeps < 1)
    return fail(nullptr, CALIB_E_INVAL, "lm_iters and sage_sweeps must be >= 1");
  if (!(cfg->lm_tol >= 0.0) || !std::isfinite(cfg->lm_tol))
    return fail(nullptr, CALIB_E_INVAL, "lm_tol must be finite and >= 0");
  if (cfg->solver < 0 || cfg->solver > 3) return fail(nullptr, CALIB_E_INVAL, "solver must be 0, 1, 2 or 3");
  if ((cfg->options & CALIB_OPT_STATS_ONLY) && cfg->solver != 3)
    return fail(nullptr, CALIB_E_INVAL, "CALIB_OPT_STATS_ONLY needs solver 3");
  if (!(cfg->cg_tol >= 0.0) || !(cfg->cg_tol < 1.0))
    return fail(nullptr, CALIB_E_INVAL, "cg_tol must be in [0, 1)");

  calib_ctx *c = new calib_ctx();
  c->N = N; c->P = P; c->Q = Q; c->K = K; c->T = T;
  c->precision = cfg->precision;
  c->lm_iters = cfg->lm_iters;
  c->sage_sweeps = cfg->sage_sweeps;
  c->options = cfg->options;
  c->f0 = cfg->f0_hz;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->n_chan.assign(cfg->n_chan, cfg->n_chan + P);
  c->freq.assign(cfg->freq_hz, cfg->freq_hz + P);
  c->rho.assign(cfg->rho, cfg->rho + K);
  if (cfg->n_dirs) c->n_dirs.assign(cfg->n_dirs, cfg->n_dirs + P);
  else c->n_dirs.assign(P, K);
  auto bail = [&](calib_status st, const std::string &m) {
    g_init_error = m;
    calib_destroy(c);
    return st;
  };
  for (int f = 0; f < P; ++f) {
    if (c->n_chan[f] < 1) return bail(CALIB_E_INVAL, "n_chan entries must be >= 1");
    if (c->n_dirs[f] < 1 || c->n_dirs[f] > K) return bail(CALIB_E_INVAL, "n_dirs entries must be in [1, K]");
    if (!std::isfinite(c->freq[f])) return bail(CALIB_E_INVAL, "freq_hz must be finite");
  }
  for (int k = 0; k < K; ++k)
    if (!(c->rho[k] >= 0.0) || !std::isfinite(c->rho[k])) return bail(CALIB_E_INVAL, "rho must be finite and >= 0");
  for (int k = 0; k < K; ++k) {
    std::vector<double> fr;
    for (int f = 0; f < P; ++f)
      if (c->n_dirs[f] > k) fr.push_back(c->freq[f]);
    std::sort(fr.begin(), fr.end());
    const size_t distinct = std::unique(fr.begin(), fr.end()) - fr.begin();
    if ((int)distinct < Q)
      return bail(CALIB_E_RANK, "direction " + std::to_string(k) + " is carried by fewer than Q distinct subband frequencies");
  }

  const int Bfull = N * (N - 1) / 2;
  std::vector<uint8_t> hflags((size_t)P * Bfull, 0);
  if (flags) {
    hipError_t e = hipMemcpyAsync(hflags.data(), flags, hflags.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(CALIB_E_DEVICE, std::string("reading flags: ") + hipGetErrorString(e));
  }
  std::vector<int32_t> pair_p(Bfull), pair_q(Bfull);
  for (int a = 0, b = 0; a < N; ++a)
    for (int q = a + 1; q < N; ++q, ++b) { pair_p[b] = a; pair_q[b] = q; }

  std::vector<int64_t> samp_off(P), coh_off(P), sb_off(P), in_vis_off(P), in_coh_off(P), full_off(P);
  std::vector<int32_t> bl_off(P), nb(P), spb(P), bl_p, bl_q, comp2full, comp_f;
  std::vector<int32_t> full_bmap((size_t)P * Bfull, -1), bidx((size_t)P * N * N, -1);
  int64_t so = 0, co = 0, sbo = 0, ivo = 0, ico = 0;
  for (int f = 0; f < P; ++f) {
    spb[f] = T * c->n_chan[f];
    bl_off[f] = (int32_t)bl_p.size();
    samp_off[f] = so; coh_off[f] = co; sb_off[f] = sbo;
    in_vis_off[f] = ivo; in_coh_off[f] = ico; full_off[f] = ivo;
    int cnt = 0;
    for (int b = 0; b < Bfull; ++b) {
      if (hflags[(size_t)f * Bfull + b]) continue;
      const int gb = (int)bl_p.size();
      full_bmap[(size_t)f * Bfull + b] = gb;
      bidx[((size_t)f * N + pair_p[b]) * N + pair_q[b]] = gb;
      bidx[((size_t)f * N + pair_q[b]) * N + pair_p[b]] = gb;
      bl_p.push_back(pair_p[b]);
      bl_q.push_back(pair_q[b]);
      comp2full.push_back(b);
      comp_f.push_back(f);
      ++cnt;
    }
    nb[f] = cnt;
    so += (int64_t)cnt * spb[f];
    co += (int64_t)c->n_dirs[f] * cnt * spb[f];
    sbo += (int64_t)c->n_dirs[f] * cnt;
    ivo += (int64_t)Bfull * spb[f];
    ico += (int64_t)c->n_dirs[f] * Bfull * spb[f];
  }
  const int nb_total = (int)bl_p.size();
  c->total_full_samples = ivo;
  std::vector<int32_t> comp_tab(comp2full);
  comp_tab.insert(comp_tab.end(), comp_f.begin(), comp_f.end());

  const int group = choose_group(spb, nb, cfg->tile_group, cfg->solver == 3);
  const int bpt = kBlock / group;
  std::vector<int32_t> tile_f, tile_b0, tile_off(P + 1);
  for (int f = 0; f < P; ++f) {
    tile_off[f] = (int32_t)tile_f.size();
    for (int b0 = 0; b0 < nb[f]; b0 += bpt) { tile_f.push_back(f); tile_b0.push_back(b0); }
  }
  tile_off[P] = (int32_t)tile_f.size();
  std::vector<int32_t> adj_off((size_t)P * N + 1), adj_b, adj_o;
  for (int f = 0; f < P; ++f)
    for (int p = 0; p < N; ++p) {
      adj_off[(size_t)f * N + p] = (int32_t)adj_b.size();
      for (int o = 0; o < N; ++o) {
        if (o == p) continue;
        const int gb = bidx[((size_t)f * N + p) * N + o];
        if (gb < 0) continue;
        adj_b.push_back(gb);
        adj_o.push_back(o > p ? o : -1 - o);
      }
    }
  adj_off[(size_t)P * N] = (int32_t)adj_b.size();

  Problem &pb = c->pb;
  pb.N = N; pb.P = P; pb.Q = Q; pb.K = K;
  pb.nf = ((8 * N + 15) / 16) * 16;
  pb.npad = pb.nf + 16;
  pb.ntiles = (int)tile_f.size();
  pb.group = group;
  pb.bpt = bpt;
  pb.nbt = nb_total;
  pb.max_nb = P > 0 ? *std::max_element(nb.begin(), nb.end()) : 0;
  pb.stream_grid = cfg->stream_grid > 0 ? cfg->stream_grid : 0;
  pb.lm_tol = cfg->lm_tol;
  pb.solver = cfg->solver == 1 ? kSolverSingle
              : cfg->solver == 2 ? kSolverBlocked
              : cfg->solver == 3 ? kSolverPcg
              : (P < kBlockedSolverMaxSubbands ? kSolverBlocked : kSolverSingle);
  pb.cg_tol = cfg->cg_tol > 0.0 ? cfg->cg_tol : kDefaultCgTol;

  calib_status st = CALIB_OK;
#define UPL(dst, src)                                                                          \
  do {                                                                                         \
    st = upload(c, &dst, src);                                                                 \
    if (st != CALIB_OK) { g_init_error = c->err; calib_destroy(c); return st; }                \
  } while (0)
  int64_t *d_samp, *d_coh, *d_sb, *d_ivo, *d_ico;
  int32_t *d_bl_off, *d_nb, *d_spb, *d_ndir, *d_blp, *d_blq, *d_tf, *d_tb, *d_to, *d_ao, *d_ab, *d_aoth,
      *d_bidx, *d_comp;
  UPL(d_samp, samp_off); UPL(d_coh, coh_off); UPL(d_sb, sb_off); UPL(d_ivo, in_vis_off);
  UPL(d_ico, in_coh_off); UPL(d_bl_off, bl_off); UPL(d_nb, nb); UPL(d_spb, spb);
  UPL(d_ndir, c->n_dirs); UPL(d_blp, bl_p); UPL(d_blq, bl_q); UPL(d_tf, tile_f); UPL(d_tb, tile_b0);
  UPL(d_to, tile_off); UPL(d_ao, adj_off); UPL(d_ab, adj_b); UPL(d_aoth, adj_o); UPL(d_bidx, bidx);
  UPL(d_comp, comp_tab); UPL(c->d_full_off, full_off); UPL(c->d_full_bmap, full_bmap);
  double *d_rho, *d_freq;
  UPL(d_rho, c->rho); UPL(d_freq, c->freq);
  c->d_ndir = d_ndir;
  Layout &L = c->L;
  L.samp_off = d_samp; L.coh_off = d_coh; L.bl_off = d_bl_off; L.nb = d_nb; L.spb = d_spb;
  L.ndir = d_ndir; L.bl_p = d_blp; L.bl_q = d_blq; L.tile_f = d_tf; L.tile_b0 = d_tb;
  L.tile_off = d_to; L.adj_off = d_ao; L.adj_b = d_ab; L.adj_o = d_aoth; L.bidx = d_bidx;
  L.sb_off = d_sb;

  const size_t elt = (c->precision == CALIB_FP64) ? sizeof(double) : sizeof(float);
  Buffers &B = c->B;
  auto fail_alloc = [&](const char *what) {
    g_init_error = std::string("hipMalloc failed for ") + what;
    calib_destroy(c);
    return CALIB_E_NOMEM;
  };
#define DALLOC(ptr, bytes)                                                                     \
  do {                                                                                         \
    void *p_ = nullptr;                                                                        \
    if (c->mem.alloc(&p_, (bytes)) != hipSuccess) return fail_alloc(#ptr);                     \
    ptr = reinterpret_cast<decltype(ptr)>(p_);                                                 \
  } while (0)
  void *Vp = nullptr, *Cp = nullptr;   // the packed samples (none with CALIB_OPT_STATS_ONLY)
  double *Sb;
  if (!(cfg->options & CALIB_OPT_STATS_ONLY)) {
    DALLOC(Vp, (size_t)so * 8 * elt);
    DALLOC(Cp, (size_t)co * 2 * elt);
  }
  DALLOC(Sb, (size_t)sbo * sizeof(double));
  const size_t nj = (size_t)P * K * N * 8, nz = (size_t)K * Q * N * 8;
  DALLOC(B.J, nj * 8); DALLOC(B.Y, nj * 8); DALLOC(B.BZ, nj * 8);
  DALLOC(B.Z, nz * 8); B.Zold = nullptr;
  DALLOC(B.Sd, (size_t)P * K * N * N * 8);
  DALLOC(B.Jstart, (size_t)P * N * 8 * 8); DALLOC(B.Jtrial, (size_t)P * N * 8 * 8);
  DALLOC(B.D0, (size_t)nb_total * 8 * 8); DALLOC(B.D1, (size_t)nb_total * 8 * 8);
  DALLOC(B.Dstart, (size_t)nb_total * 8 * 8);
  B.H = nullptr;
  B.Linv = nullptr;
  if (pb.solver != kSolverPcg) {   // the dense normal equations of the Cholesky solvers
    DALLOC(B.H, (size_t)P * pb.npad * pb.nf * 8);
    DALLOC(B.Linv, (size_t)P * (pb.nf / 16) * 256 * 8);
  }
  DALLOC(B.G, (size_t)P * pb.nf * 8); DALLOC(B.delta, (size_t)P * pb.nf * 8);
  DALLOC(B.cost_part, (size_t)std::max(pb.ntiles, 1) * 8);
  DALLOC(B.Epart, (size_t)std::max(pb.ntiles, 1) * 8);
  DALLOC(B.Ev, (size_t)std::max(nb_total, 1) * 8);
  DALLOC(B.Epl, (size_t)K * std::max(pb.ntiles, 1) * 8);
  DALLOC(B.Ucoh, (size_t)pb.nbt * K * 8 * 8);
  DALLOC(B.Xcoh, (size_t)pb.nbt * K * K * 2 * 8);
  DALLOC(B.Dall, (size_t)pb.nbt * K * 8 * 8);
  DALLOC(B.lm, (size_t)P * sizeof(LmState));
  DALLOC(B.status, (size_t)P * sizeof(int));
  DALLOC(B.work, (size_t)P * 2 * sizeof(double));
  double *basis, *fitw;
  DALLOC(basis, (size_t)P * Q * 8);
  DALLOC(fitw, (size_t)K * Q * P * 8);
  DALLOC(B.trace, (size_t)kMaxTrace * 4 * 8);
  DALLOC(B.scratch, (2 * (size_t)P * K + (size_t)K * kZChunks + P) * 8);   // residual partials, then the trace row's cost and penalty partials
  DALLOC(B.iter, sizeof(int));
  B.chol_fail = nullptr;
  B.chol_ld = nullptr;
  if (pb.solver == kSolverBlocked) {
    DALLOC(B.chol_fail, (size_t)P * sizeof(int));
    DALLOC(B.chol_ld, (size_t)P * chol_blocked_panels(pb) * 64 * 64 * 8);
  }
  DALLOC(c->ws_jsave, nj * 8);
  DALLOC(c->ws_cost, (size_t)2 * P * 8);
  DALLOC(c->lm_trace, (size_t)P * K * c->lm_iters * 3 * 8);
  {
    const hipError_t he = hipHostMalloc(reinterpret_cast<void **>(&c->stop_flag), sizeof(int),
                                        hipHostMallocCoherent);
    if (he != hipSuccess) return bail(CALIB_E_DEVICE, std::string("pinned flag: ") + hipGetErrorString(he));
    *c->stop_flag = 0;
  }
  int *flagbuf;
  DALLOC(flagbuf, 2 * sizeof(int));
  B.V = Vp; B.C = Cp; B.Sb = Sb; B.rho = d_rho; B.basis = basis; B.fitw = fitw;
  c->d_in_vis_off = d_ivo; c->d_in_coh_off = d_ico; c->d_comp = d_comp; c->nb_total = nb_total;
  c->Vp = Vp; c->Cp = Cp; c->Sb = Sb;

  hipStream_t s = c->stream;
  auto dev = [&](hipError_t e, const char *what) -> bool {
    if (e == hipSuccess) return true;
    g_init_error = std::string(what) + ": " + hipGetErrorString(e);
    return false;
  };
  const bool ok =
      dev(hipMemsetAsync(flagbuf, 0, 2 * sizeof(int), s), "clear flags") &&
      dev(c->precision == CALIB_FP64
              ? launch_pack_stats<double>(pb, L, B, vis, coh, Vp, Cp, Sb, d_ivo, d_ico, d_comp, nb_total,
                                          flagbuf, nullptr, s)
              : launch_pack_stats<float>(pb, L, B, vis, coh, Vp, Cp, Sb, d_ivo, d_ico, d_comp, nb_total,
                                         flagbuf, nullptr, s),
          "pack and coherency statistics") &&
      dev(launch_basis_setup(pb, d_freq, c->f0, d_ndir, basis, fitw, flagbuf + 1, s), "basis setup") &&
      dev(launch_dense_s(pb, L, B, s), "dense S") &&
      (!B.H || dev(launch_zero(B.H, (int64_t)P * pb.npad * pb.nf, s), "zero H")) &&
      dev(hipMemsetAsync(B.lm, 0, (size_t)P * sizeof(LmState), s), "zero LM state") &&
      dev(hipMemsetAsync(B.status, 0, (size_t)P * sizeof(int), s), "zero status") &&
      dev(launch_zero(B.work, (int64_t)P * 2, s), "zero work counters") &&
      (!B.chol_fail || dev(hipMemsetAsync(B.chol_fail, 0, (size_t)P * sizeof(int), s), "zero flags")) &&
      dev(launch_zero(B.Y, (int64_t)nj, s), "zero Y") && dev(launch_zero(B.BZ, (int64_t)nj, s), "zero BZ") &&
      dev(launch_zero(B.Z, (int64_t)nz, s), "zero Z") &&
      dev(launch_zero(B.trace, (int64_t)kMaxTrace * 4, s), "zero trace") &&
      dev(launch_set_iter(B, 0, s), "iteration counter") &&
      dev(launch_zero(c->lm_trace, (int64_t)P * K * c->lm_iters * 3, s), "zero lm trace") &&
      dev(jones0 ? hipMemcpyAsync(B.J, jones0, nj * 8, hipMemcpyDeviceToDevice, s)
                 : launch_fill_identity(B.J, (int64_t)P * K * N, s),
          "initial jones");
  if (!ok) { calib_destroy(c); return CALIB_E_DEVICE; }
  int hflag[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(hflag, flagbuf, sizeof hflag, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(CALIB_E_DEVICE, std::string("init: ") + hipGetErrorString(e));
  if (hflag[0]) return bail(CALIB_E_NUMERIC, "non-finite values in vis or coh");
  if (hflag[1]) return bail(CALIB_E_RANK, "basis matrix of the subband frequencies is rank deficient");
  *out = c;
  return CALIB_OK;
}

calib_status admm_local_step(calib_ctx *ctx, int32_t admm_iter) {
  if (!ctx) return CALIB_E_INVAL;
  if (admm_iter < 0 || admm_iter >= kMaxTrace) return fail(ctx, CALIB_E_INVAL, "admm_iter out of range");
  return local_step_on(ctx, admm_iter, ctx->stream);
}

calib_status admm_consensus_update(calib_ctx *ctx, int32_t admm_iter) {
  if (!ctx) return CALIB_E_INVAL;
  if (admm_iter < 0 || admm_iter >= kMaxTrace) return fail(ctx, CALIB_E_INVAL, "admm_iter out of range");
  HIPCHK(ctx, launch_set_iter(ctx->B, admm_iter, ctx->stream));
  const calib_status st =
      consensus_on(ctx, admm_iter == 0 && (ctx->options & CALIB_OPT_GPA_FIRST_ITER), ctx->stream);
  if (st != CALIB_OK) return st;
  ctx->iters_done = std::max(ctx->iters_done, admm_iter + 1);
  return CALIB_OK;
}

calib_status admm_solve(calib_ctx *ctx, int32_t max_iters, double rel_cost_tol, double *trace_out,
                        int32_t *iters_done) {
  if (!ctx) return CALIB_E_INVAL;
  if (max_iters < 0 || max_iters > kMaxTrace) return fail(ctx, CALIB_E_INVAL, "max_iters out of range");
  int n = 0;
  double prev = 0.0;
  // the host-driven local step of the stopping rule (Cholesky solvers); the matrix-free solver
  // applies the rule inside its one-launch local step, so its iterations replay a graph as well
  const bool stopping = ctx->pb.lm_tol > 0.0 && ctx->pb.solver != kSolverPcg;
  for (; n < max_iters; ++n) {
    calib_status st = CALIB_OK;
    if (stopping) {
      const bool eager = n == 0 || ctx->timing;
      st = local_step_stopping_on(ctx, n, ctx->stream);
      if (st == CALIB_OK) {
        if (eager) {
          st = admm_consensus_update(ctx, n);
        } else {
          // the device counter (set by iteration 0) selects the trace row
          st = consensus_on(ctx, false, ctx->stream);
          ctx->iters_done = std::max(ctx->iters_done, n + 1);
        }
      }
    } else if (n == 0 || ctx->timing) {
      st = admm_local_step(ctx, n);
      if (st == CALIB_OK) st = admm_consensus_update(ctx, n);
    } else {
      // iterations >= 1: replay the captured iteration; the device counter (set by iteration 0)
      // selects the trace row
      if (!ctx->graph_exec) st = build_iteration_graph(ctx);
      if (st == CALIB_OK) HIPCHK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
      ctx->iters_done = std::max(ctx->iters_done, n + 1);
    }
    if (st != CALIB_OK) return st;
    if (rel_cost_tol > 0.0) {
      double cur = 0.0;
      HIPCHK(ctx, hipMemcpyAsync(&cur, ctx->B.trace + 4 * n, sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      if (n > 0 && std::fabs(cur - prev) <= rel_cost_tol * std::fabs(prev)) { ++n; break; }
      prev = cur;
    }
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (trace_out && n > 0)
    HIPCHK(ctx, hipMemcpy(trace_out, ctx->B.trace, sizeof(double) * 4 * n, hipMemcpyDeviceToHost));
  if (iters_done) *iters_done = n;
  std::vector<int> status(ctx->P);
  HIPCHK(ctx, hipMemcpy(status.data(), ctx->B.status, sizeof(int) * ctx->P, hipMemcpyDeviceToHost));
  std::string bad;
  int nbad = 0;
  for (int f = 0; f < ctx->P; ++f)
    if (status[f] != CALIB_OK && ++nbad <= 8) bad += (bad.empty() ? "" : ", ") + std::to_string(f);
  if (nbad)
    return fail(ctx, CALIB_E_NUMERIC, std::to_string(nbad) + " subband(s) with a non-finite objective or "
                                      "normal equations that could not be solved (" + bad +
                                      (nbad > 8 ? ", ...)" : ")") + "; see CALIB_FIELD_STATUS");
  return CALIB_OK;
}


calib_status calib_get(calib_ctx *ctx, int32_t field, void *dst) {
  if (!ctx) return CALIB_E_INVAL;
  if (!dst) return fail(ctx, CALIB_E_INVAL, "dst is NULL");
  hipStream_t s = ctx->stream;
  const size_t nj = (size_t)ctx->P * ctx->K * ctx->N * 8 * sizeof(double);
  switch (field) {
    case CALIB_FIELD_J:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.J, nj, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_Y:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.Y, nj, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_BZ:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.BZ, nj, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_Z:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.Z, (size_t)ctx->K * ctx->Q * ctx->N * 8 * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_MODEL_VIS:
      if (!ctx->Vp) return fail(ctx, CALIB_E_STATE, "the context keeps no samples (CALIB_OPT_STATS_ONLY)");
      HIPCHK(ctx, ctx->precision == CALIB_FP64
                      ? launch_model<double>(ctx->pb, ctx->L, ctx->B, dst, ctx->d_full_off, ctx->d_full_bmap, s)
                      : launch_model<float>(ctx->pb, ctx->L, ctx->B, dst, ctx->d_full_off, ctx->d_full_bmap, s));
      return CALIB_OK;
    case CALIB_FIELD_COST:
      if (!ctx->Vp)
        HIPCHK(ctx, launch_refresh_stats(ctx->pb, ctx->L, ctx->B, true, s));
      else
        HIPCHK(ctx, ctx->precision == CALIB_FP64 ? launch_refresh<double>(ctx->pb, ctx->L, ctx->B, s)
                                                 : launch_refresh<float>(ctx->pb, ctx->L, ctx->B, s));
      HIPCHK(ctx, launch_subband_cost(ctx->pb, ctx->L, ctx->B, static_cast<double *>(dst), s));
      return CALIB_OK;
    case CALIB_FIELD_TRACE:
      HIPCHK(ctx, hipStreamSynchronize(s));
      if (ctx->iters_done > 0)
        HIPCHK(ctx, hipMemcpy(dst, ctx->B.trace, sizeof(double) * 4 * ctx->iters_done, hipMemcpyDeviceToHost));
      return CALIB_OK;
    case CALIB_FIELD_LM_TRACE:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->lm_trace,
                                 sizeof(double) * 3 * (size_t)ctx->P * ctx->K * ctx->lm_iters,
                                 hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_KERNEL_TIMES: {
      HIPCHK(ctx, flush_timing(ctx));
      double *o = static_cast<double *>(dst);
      for (int i = 0; i < CALIB_NUM_KERNELS; ++i) { o[2 * i] = ctx->kcount[i]; o[2 * i + 1] = ctx->kms[i]; }
      return CALIB_OK;
    }
    case CALIB_FIELD_WORK:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.work, sizeof(double) * 2 * ctx->P, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_STATUS:
      HIPCHK(ctx, hipMemcpyAsync(dst, ctx->B.status, sizeof(int) * ctx->P, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    case CALIB_FIELD_LM_STEP: {
      const size_t w = (size_t)8 * ctx->N * sizeof(double), sp = (size_t)ctx->pb.nf * sizeof(double);
      char *d = static_cast<char *>(dst);
      HIPCHK(ctx, hipMemcpy2DAsync(d, 2 * w, ctx->B.G, sp, w, ctx->P, hipMemcpyDeviceToDevice, s));
      HIPCHK(ctx, hipMemcpy2DAsync(d + w, 2 * w, ctx->B.delta, sp, w, ctx->P, hipMemcpyDeviceToDevice, s));
      return CALIB_OK;
    }
    default:
      return fail(ctx, CALIB_E_INVAL, "unknown field");
  }
}

calib_status calib_warmstart_features(calib_ctx *ctx, const void *jones_prev2, const void *bz_prev,
                                      float *features) {
  if (!ctx) return CALIB_E_INVAL;
  if (!features) return fail(ctx, CALIB_E_INVAL, "features is NULL");
  hipStream_t s = ctx->stream;
  const Problem &pb = ctx->pb;
  const Layout &L = ctx->L;
  const Buffers &B = ctx->B;
  const double *J2 = static_cast<const double *>(jones_prev2);
  const double *BZp = static_cast<const double *>(bz_prev);
  // every direction's per-baseline sums D_k at the current J (from the coherency statistics),
  // then the features of every (subband, direction, station) in one launch
  HIPCHK(ctx, launch_refresh_stats(pb, L, B, false, s));
  HIPCHK(ctx, launch_ws_features(pb, L, B, J2, BZp, features, s));
  return CALIB_OK;
}

calib_status calib_warmstart_target(calib_ctx *ctx, const void *jones_prev, float *target) {
  if (!ctx) return CALIB_E_INVAL;
  if (!jones_prev || !target) return fail(ctx, CALIB_E_INVAL, "jones_prev or target is NULL");
  HIPCHK(ctx, launch_ws_target(ctx->pb, ctx->L, ctx->B, static_cast<const double *>(jones_prev),
                               target, ctx->stream));
  return CALIB_OK;
}

calib_status calib_warmstart_apply(calib_ctx *ctx, const float *delta, int32_t *kept) {
  if (!ctx) return CALIB_E_INVAL;
  if (!delta) return fail(ctx, CALIB_E_INVAL, "delta is NULL");
  hipStream_t s = ctx->stream;
  const Problem &pb = ctx->pb;
  const Layout &L = ctx->L;
  const Buffers &B = ctx->B;
  double *cost0 = ctx->ws_cost, *cost1 = ctx->ws_cost + ctx->P;
  // data cost per subband from the coherency statistics (no pass over the samples)
  auto cost = [&](double *out) -> hipError_t {
    const hipError_t e = launch_refresh_stats(pb, L, B, true, s);
    return e == hipSuccess ? launch_subband_cost(pb, L, B, out, s) : e;
  };
  HIPCHK(ctx, cost(cost0));
  HIPCHK(ctx, launch_ws_add(pb, L, B, delta, ctx->ws_jsave, s));
  HIPCHK(ctx, cost(cost1));
  HIPCHK(ctx, launch_ws_choose(pb, B, cost0, cost1, ctx->ws_jsave, kept, s));
  ctx->iters_done = 0;
  return CALIB_OK;
}

calib_status calib_set_data(calib_ctx *ctx, const void *vis, const void *coh) {
  if (!ctx) return CALIB_E_INVAL;
  if (!vis || !coh) return fail(ctx, CALIB_E_INVAL, "vis and coh are required");
  hipStream_t s = ctx->stream;
  HIPCHK(ctx, launch_zero_int(ctx->B.status, ctx->P, s));
  HIPCHK(ctx, timed(ctx, CALIB_KERNEL_PACK, [&] {
    hipError_t e = ctx->precision == CALIB_FP64
        ? launch_pack_stats<double>(ctx->pb, ctx->L, ctx->B, vis, coh, ctx->Vp, ctx->Cp, ctx->Sb,
                                    ctx->d_in_vis_off, ctx->d_in_coh_off, ctx->d_comp,
                                    ctx->nb_total, nullptr, ctx->B.status, s)
        : launch_pack_stats<float>(ctx->pb, ctx->L, ctx->B, vis, coh, ctx->Vp, ctx->Cp, ctx->Sb,
                                   ctx->d_in_vis_off, ctx->d_in_coh_off, ctx->d_comp,
                                   ctx->nb_total, nullptr, ctx->B.status, s);
    return e == hipSuccess ? launch_dense_s(ctx->pb, ctx->L, ctx->B, s) : e;
  }));
  ctx->iters_done = 0;
  return CALIB_OK;
}

calib_status calib_set_kernel_timing(calib_ctx *ctx, int32_t enable) {
  if (!ctx) return CALIB_E_INVAL;
  HIPCHK(ctx, flush_timing(ctx));
  ctx->timing = enable != 0;
  for (int i = 0; i < CALIB_NUM_KERNELS; ++i) ctx->kms[i] = ctx->kcount[i] = 0.0;
  if (ctx->timing) HIPCHK(ctx, launch_zero(ctx->B.work, (int64_t)ctx->P * 2, ctx->stream));
  return CALIB_OK;
}

calib_status calib_set_state(calib_ctx *ctx, const void *jones, const void *y, const void *z,
                             const void *bz) {
  if (!ctx) return CALIB_E_INVAL;
  if (!jones) return fail(ctx, CALIB_E_INVAL, "jones is NULL");
  hipStream_t s = ctx->stream;
  const int64_t nj = (int64_t)ctx->P * ctx->K * ctx->N * 8;
  const int64_t nz = (int64_t)ctx->K * ctx->Q * ctx->N * 8;
  HIPCHK(ctx, hipMemcpyAsync(ctx->B.J, jones, nj * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, launch_zero_int(ctx->B.status, ctx->P, s));
  if (y) HIPCHK(ctx, hipMemcpyAsync(ctx->B.Y, y, nj * 8, hipMemcpyDeviceToDevice, s));
  else HIPCHK(ctx, launch_zero(ctx->B.Y, nj, s));
  if (z) HIPCHK(ctx, hipMemcpyAsync(ctx->B.Z, z, nz * 8, hipMemcpyDeviceToDevice, s));
  else HIPCHK(ctx, launch_zero(ctx->B.Z, nz, s));
  if (bz) HIPCHK(ctx, hipMemcpyAsync(ctx->B.BZ, bz, nj * 8, hipMemcpyDeviceToDevice, s));
  else HIPCHK(ctx, launch_zero(ctx->B.BZ, nj, s));
  ctx->iters_done = 0;
  return CALIB_OK;
}

calib_status calib_set_jones(calib_ctx *ctx, const void *jones) {
  if (!ctx) return CALIB_E_INVAL;
  if (!jones) return fail(ctx, CALIB_E_INVAL, "jones is NULL");
  hipStream_t s = ctx->stream;
  const int64_t nj = (int64_t)ctx->P * ctx->K * ctx->N * 8;
  HIPCHK(ctx, hipMemcpyAsync(ctx->B.J, jones, nj * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, launch_zero_int(ctx->B.status, ctx->P, s));
  HIPCHK(ctx, launch_zero(ctx->B.Y, nj, s));
  HIPCHK(ctx, launch_zero(ctx->B.BZ, nj, s));
  HIPCHK(ctx, launch_zero(ctx->B.Z, (int64_t)ctx->K * ctx->Q * ctx->N * 8, s));
  ctx->iters_done = 0;
  return CALIB_OK;
}

}  // extern "C"
