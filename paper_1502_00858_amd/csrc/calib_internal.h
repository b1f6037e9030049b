// Internal declarations shared by the host code and the HIP kernels of the calibration library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace calib {

constexpr int kBlock = 256;        // threads per workgroup of every kernel (4 wave64)
constexpr int kMaxDirs = 16;       // directions per subband
constexpr double kLmTau = 1e-3;    // Nielsen's initial damping factor
constexpr double kLmFailFactor = 1e16;   // a solve still failing at lambda > this x lambda_0 is a
                                         // numeric failure of the subband
constexpr int kCholMaxTilesPerWave = 9;   // 16-row tiles per wavefront in one Cholesky panel
constexpr int kMaxStations = 128;         // the solve keeps one column of 8N per thread
constexpr int kZChunks = 8 * kMaxStations / 64;   // per-direction partials of the dual residual,
                                                  // one per 64 entries of a direction's 8N

// Per-subband tables of the packed, baseline-major layout.  Flagged baselines are dropped at
// init, so "baseline index" below always means the compact index of an unflagged baseline.
struct Layout {
  const int64_t *samp_off;   // [P] first sample of subband f in V and R
  const int64_t *coh_off;    // [P] first coherency of subband f (directions outermost)
  const int32_t *bl_off;     // [P] first compact baseline of subband f
  const int32_t *nb;         // [P] unflagged baselines
  const int32_t *spb;        // [P] samples per baseline = T * n_chan
  const int32_t *ndir;       // [P] directions K_f
  const int32_t *bl_p;       // [sum nb] first station of each compact baseline
  const int32_t *bl_q;       // [sum nb] second station
  const int32_t *tile_f;     // [ntiles] subband of a streaming tile
  const int32_t *tile_b0;    // [ntiles] first compact baseline of the tile
  const int32_t *tile_off;   // [P+1] first tile of subband f
  const int32_t *adj_off;    // [P*N+1] adjacency list of (subband, station)
  const int32_t *adj_b;      // compact baseline index (global, i.e. including bl_off)
  const int32_t *adj_o;      // other station; negative-encoded (-1-q) when the station is second
  const int32_t *bidx;       // [P][N][N] compact baseline (global) of pair a<b or -1
  const int64_t *sb_off;     // [P] first S_b entry of subband f (directions outermost)
};

// State of the Levenberg-Marquardt iteration of the active direction of each subband.
struct LmState {
  double F;        // objective at the accepted point
  double E0;       // data cost at the LM run's start point (the residual's energy)
  double lambda;   // damping
  double nu;       // damping growth factor
  double ell;      // predicted decrease of the last step
  double Fnew;     // objective at the last trial point
  double lambda0;  // damping at the start of the run
  int32_t chol_ok; // last factorisation succeeded
  int32_t accepted;// accepted steps in this LM run
  int32_t done;    // the LM run of the active direction has met its stopping rule
  int32_t dsel;    // D_b of the accepted point is in D1 (1) or D0 (0); the trial pass writes the other
  // A local step whose launches take the direction from each subband (direction argument k < 0):
  // every subband moves through its own SAGE sequence, the direction of its current run, that
  // run's LM iteration, the sweep and the phase below
  int32_t cur, itc, sweep, phase;
};
constexpr int kPhaseLm = 0;        // in an LM run of direction cur
constexpr int kPhaseAdvance = 1;   // the run of cur has ended: commit it, go to the next direction
constexpr int kPhaseFinished = 2;  // every direction of every sweep done
constexpr int kPhaseBegin = 3;     // the run of cur starts (taken inside the LM start launch)

struct Problem {
  int N, P, Q, K;
  int nf;          // factor columns = round_up(8N, 16)
  int npad;        // rows of the augmented matrix = nf + 16 (row nf holds the right-hand side)
  int ntiles;
  int group;       // lanes per baseline in the streaming kernels
  int bpt;         // baselines per tile = kBlock / group
  int nbt;         // unflagged baselines over all subbands (the plane stride of the baseline statistics)
  int max_nb;      // unflagged baselines of the fullest subband
  int stream_grid; // 0 = one workgroup per tile, else persistent grid size
  double lm_tol;   // LM stops once a step's predicted decrease <= lm_tol * F (0 = never)
  int solver;      // normal-equation solver: kSolverSingle, kSolverBlocked or kSolverPcg
  double cg_tol;   // kSolverPcg: relative residual at which conjugate gradients stop
};

constexpr int kSolverSingle = 1;    // one workgroup per matrix (chol_kernel.hip)
constexpr int kSolverBlocked = 2;   // 64-column panels over many workgroups (chol_blocked.hip)
constexpr int kSolverPcg = 3;       // matrix-free conjugate gradients, no dense H (pcg_kernel.hip)
constexpr double kDefaultCgTol = 1e-10;
constexpr int kBlockedSolverMaxSubbands = 128;   // automatic choice: blocked below this batch

struct Buffers {
  const void *V;   // packed visibilities (stream type)
  const void *C;   // packed coherencies (stream type)
  const double *Sb;
  double *Sd;                           // [P][K][N][N] S_b of pair (p, q) in both orders, 0 if none
  double *J, *Y, *BZ, *Z, *Zold;        // FP64 master state
  double *Jstart, *Jtrial;              // [P][N][8] active direction
  double *D0, *D1;                      // [sum nb][8] D_b, accepted and trial point (LmState::dsel)
  double *Dstart;                       // [sum nb][8] D_b at the LM run's start point
  // per-baseline tables, direction-major with the baseline index fastest (a wavefront's lanes,
  // consecutive baselines, read consecutive entries)
  double *Ucoh;                         // [K][sum nb][8] sum_s conj(c_l) V per direction l
  double *Xcoh;                         // [K][K][sum nb][2] sum_s conj(c_l) c_m
  double *Dall;                         // [K][sum nb][8] D_l of the current residual, every l
  double *Epart;                        // [ntiles] energy of the current residual per tile
  double *Ev;                           // [sum nb] sum_s ||V_s||^2 per baseline (per interval)
  double *Epl;                          // [K][ntiles] energy of the residual from the statistics:
                                        // per direction l and tile, direction 0 with the V part
  double *H;                            // [P][npad][nf]
  double *Linv;                         // [P][nf/16][16*16] inverses of the diagonal tiles
  double *G, *delta;                    // [P][nf]
  double *cost_part;                    // [ntiles]
  LmState *lm;                          // [P]
  const double *rho;                    // [K]
  const double *basis;                  // [P][Q] b_l(f)
  const double *fitw;                   // [K][Q][P] least-squares operator per direction
  double *trace;                        // [iters][4]
  double *scratch;                      // [P*K + K*kZChunks] residual partials, [P] cost, [P*K] penalty partials
  int *iter;                            // ADMM iteration whose trace row is being written
  int *chol_fail;                       // [P] blocked solver: a pivot failed in this solve
  double *chol_ld;                      // [P][panels][64*64] blocked solver: diagonal blocks' L
  double *work;                         // [P][2] CG iterations and LM solves of the matrix-free
                                        // solver since kernel timing was enabled (measurement)
  int *status;                          // [P] CALIB_OK or CALIB_E_NUMERIC per subband (a run
                                        // whose objective is not finite, or whose normal
                                        // equations fail past kLmFailFactor lambda_0)
  const int *rank_fail;                 // set by the basis setup of a context-free consensus
                                        // update: the Z fit, Y update and residuals do nothing
                                        // (null in a context, whose rank is checked at init)
};

// The direction a launch works on for subband f: its argument k, or (k < 0) the subband's own
__device__ inline int lm_dir(const Buffers &B, int f, int k) { return k >= 0 ? k : B.lm[f].cur; }
// Whether subband f takes part in a launch of an LM iteration (assembly, solve, trial point)
__device__ inline bool lm_live(const Buffers &B, const int32_t *ndir, int f, int k) {
  return (k >= 0 ? k < ndir[f] : B.lm[f].phase == kPhaseLm) && !B.lm[f].done;
}

// D_b of subband f at its accepted point and at its trial point: an accepted LM step swaps the two
// buffers instead of copying the trial values
__device__ inline double *d_accepted(const Buffers &B, int f) { return B.lm[f].dsel ? B.D1 : B.D0; }
__device__ inline double *d_trial(const Buffers &B, int f) { return B.lm[f].dsel ? B.D0 : B.D1; }
// the same from a copy of the subband's LM state (the one-launch local step keeps it in LDS)
__device__ inline double *d_accepted(const Buffers &B, const LmState &st) { return st.dsel ? B.D1 : B.D0; }
__device__ inline double *d_trial(const Buffers &B, const LmState &st) { return st.dsel ? B.D0 : B.D1; }

// streaming kernels (templated on the stream element type float or double)
template <typename T>
hipError_t launch_refresh(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s);
// the refresh without a pass over the samples: every D_l and the residual's energy from the
// coherency statistics (into Epl; with fold, also into the tiles' Epart and cost_part)
hipError_t launch_refresh_stats(const Problem &pb, const Layout &L, const Buffers &B, bool fold,
                                hipStream_t s);
template <typename T>
hipError_t launch_commit(const Problem &pb, const Layout &L, const Buffers &B, int k, int all,
                         hipStream_t s);
template <typename T>
hipError_t launch_model(const Problem &pb, const Layout &L, const Buffers &B, void *model_out,
                        const int64_t *full_off, const int32_t *full_bmap, hipStream_t s);
// per solution interval: packed V and C, S_b, U_l and X_lm in one pass over the caller's arrays
template <typename T>
hipError_t launch_pack_stats(const Problem &pb, const Layout &L, const Buffers &B, const void *vis,
                             const void *coh, void *Vp, void *Cp, double *Sb,
                             const int64_t *in_vis_off, const int64_t *in_coh_off,
                             const int32_t *comp_tab, int nb_total, int *bad, int *status,
                             hipStream_t s);

// LM kernels
// k < 0: each subband's own next direction (sweeps = SAGE sweeps of the local step)
hipError_t launch_lm_begin(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                           hipStream_t s, int sweeps = 1);
hipError_t launch_assemble(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                           hipStream_t s);
hipError_t launch_chol_solve_nd(const Problem &pb, const Buffers &B, int k, const int32_t *ndir,
                                hipStream_t s);
hipError_t launch_chol_blocked(const Problem &pb, const Buffers &B, int k, const int32_t *ndir,
                               double *Ld, int *cfail, hipStream_t s);
int chol_blocked_panels(const Problem &pb);
// the whole local step of every subband in one launch (after the refresh), solver kSolverPcg
hipError_t launch_local_step(const Problem &pb, const Layout &L, const Buffers &B, int unreg,
                             double *lm_trace, int lm_iters, int sweeps, hipStream_t s);
hipError_t launch_trial_stats(const Problem &pb, const Layout &L, const Buffers &B, int k,
                              hipStream_t s);
hipError_t launch_lm_update_tr(const Problem &pb, const Layout &L, const Buffers &B, int k, int unreg,
                               double *lm_trace, int it, int lm_iters, hipStream_t s);
hipError_t launch_dense_s(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s);
// each subband on its own direction (k < 0 launches): *flag = 1 once all have finished the local step
hipError_t launch_lm_stopped(const Problem &pb, const Layout &L, const Buffers &B, int *flag,
                             int lm_iters, int sweeps, hipStream_t s);
hipError_t launch_dir_reset(const Problem &pb, const Buffers &B, hipStream_t s);

// consensus kernels
hipError_t launch_basis_setup(const Problem &pb, const double *freq, double f0, const int32_t *ndir,
                              double *basis, double *fitw, int *rank_fail, hipStream_t s);
hipError_t launch_set_iter(const Buffers &B, int iter, hipStream_t s);
// the trace row's data cost and penalty partials (per subband, per subband and direction), taken
// before the alignment on its iteration; launch_consensus(kPenaltyTaken) folds them into the row,
// launch_consensus(kPenaltyInYUpdate) takes them in the Y update, kPenaltyNone leaves the row's
// cost and Lagrangian unwritten
hipError_t launch_penalty_part(const Problem &pb, const Layout &L, const Buffers &B, hipStream_t s);
constexpr int kPenaltyNone = 0, kPenaltyTaken = 1, kPenaltyInYUpdate = 2;
hipError_t launch_gpa(const Problem &pb, const Layout &L, const Buffers &B, int rounds, hipStream_t s);
hipError_t launch_consensus(const Problem &pb, const Layout &L, const Buffers &B, int penalty,
                             hipStream_t s);
hipError_t launch_subband_cost(const Problem &pb, const Layout &L, const Buffers &B, double *out,
                               hipStream_t s);
// warm start (warmstart_kernels.hip)
constexpr int kWsFeatures = 32;     // network inputs per (subband, direction, station)
constexpr int kWsOutputs = 8;       // network outputs: scaled change of the station's Jones
constexpr double kWsScale = 10.0;   // scale of the difference features and of the outputs
hipError_t launch_ws_features(const Problem &pb, const Layout &L, const Buffers &B,
                              const double *J2, const double *BZp, float *feat, hipStream_t s);
hipError_t launch_ws_add(const Problem &pb, const Layout &L, const Buffers &B, const float *delta,
                         double *Jsave, hipStream_t s);
hipError_t launch_ws_target(const Problem &pb, const Layout &L, const Buffers &B, const double *Jprev,
                            float *target, hipStream_t s);
hipError_t launch_ws_choose(const Problem &pb, const Buffers &B, const double *cost0,
                            const double *cost1, const double *Jsave, int32_t *kept, hipStream_t s);

hipError_t launch_fill_identity(double *J, int64_t nblocks, hipStream_t s);
// message returned by calib_last_error(NULL) for entry points that take no context
void set_context_free_error(const char *msg);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_zero_int(int *p, int64_t n, hipStream_t s);

}  // namespace calib
