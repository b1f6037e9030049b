/* FP64 CPU oracle for consensus-ADMM distributed calibration (Yatawatta 2015).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct implementation used to check the
 * GPU library.  Nothing in the product path loads it.  It shares no code with the GPU library.
 *
 * Structure follows the paper:
 *   Section 2  visibility model and least-squares cost          -> or_predict, or_subband_cost
 *   Section 3  SAGE expectation for one direction               -> dir_estep
 *              augmented Lagrangian per agent (the trace form of Appendix A is used for the
 *              linear term: Re tr(Y^H (J - B Z)))                -> dir_objective
 *              local minimisation (M1) by Levenberg-Marquardt    -> lm_dir
 *              gauge alignment at the first iteration            -> or_gpa
 *              fusion-centre least squares for Z (M2), B_f Z,
 *              dual ascent (M3), primal/dual residuals (Sec. 4)  -> or_consensus
 * The gradient and Gauss-Newton matrix are formed by the chain rule from the explicit Jacobian
 * of M = J_p J_q^H with respect to the 16 real parameters of (J_p, J_q).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LM_TAU 1e-3
#define GPA_TOL 1e-15
#define OR_KMAX 32   /* directions per subband handled by the fixed-size model tables */

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static int n_baselines(int N) { return N * (N - 1) / 2; }

static void baseline_tables(int N, int *bp, int *bq) {
  int b = 0;
  for (int p = 0; p < N; ++p)
    for (int q = p + 1; q < N; ++q) { bp[b] = p; bq[b] = q; ++b; }
}

static int64_t samples_of(const or_cfg *c, int f) {
  return (int64_t)n_baselines(c->N) * c->T * c->n_chan[f];
}

static int64_t vis_offset(const or_cfg *c, int f) {
  int64_t o = 0;
  for (int g = 0; g < f; ++g) o += samples_of(c, g);
  return o;
}

static int64_t coh_offset(const or_cfg *c, int f) {
  int64_t o = 0;
  for (int g = 0; g < f; ++g) o += (int64_t)c->n_dirs[g] * samples_of(c, g);
  return o;
}

static int flagged(const or_cfg *c, const or_data *d, int f, int b) {
  return d->flags ? d->flags[(int64_t)f * n_baselines(c->N) + b] != 0 : 0;
}

/* ---- 2x2 complex matrices, row-major ---------------------------------------------------- */
static void m2_mul_h(const double complex *A, const double complex *B, double complex *C) {
  /* C = A B^H */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      C[i * 2 + j] = A[i * 2 + 0] * conj(B[j * 2 + 0]) + A[i * 2 + 1] * conj(B[j * 2 + 1]);
}

static void m2_hmul(const double complex *A, const double complex *B, double complex *C) {
  /* C = A^H B */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      C[i * 2 + j] = conj(A[0 * 2 + i]) * B[0 * 2 + j] + conj(A[1 * 2 + i]) * B[1 * 2 + j];
}

static void m2_mul(const double complex *A, const double complex *B, double complex *C) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      C[i * 2 + j] = A[i * 2 + 0] * B[0 * 2 + j] + A[i * 2 + 1] * B[1 * 2 + j];
}

static double m2_norm2(const double complex *A) {
  double s = 0;
  for (int i = 0; i < 4; ++i) s += creal(A[i]) * creal(A[i]) + cimag(A[i]) * cimag(A[i]);
  return s;
}

/* ---- Section 2: visibility model and cost ----------------------------------------------- */
void or_predict(const or_cfg *c, const or_data *d, const double complex *J, double complex *model) {
  const int N = c->N, B = n_baselines(N), K = c->K;
  int *bp = malloc(sizeof(int) * B), *bq = malloc(sizeof(int) * B);
  baseline_tables(N, bp, bq);
#pragma omp parallel for schedule(dynamic)
  for (int f = 0; f < c->P; ++f) {
    const int Kf = c->n_dirs[f];
    const int64_t spb = (int64_t)c->T * c->n_chan[f], S = samples_of(c, f);
    const double complex *coh = d->coh + coh_offset(c, f);
    double complex *out = model + 4 * vis_offset(c, f);
    for (int b = 0; b < B; ++b) {
      double complex M[OR_KMAX][4];
      for (int k = 0; k < Kf; ++k) {
        const double complex *Jk = J + ((int64_t)f * K + k) * N * 4;
        m2_mul_h(Jk + 4 * bp[b], Jk + 4 * bq[b], M[k]);
      }
      for (int64_t s = b * spb; s < (b + 1) * spb; ++s) {
        double complex m[4] = {0, 0, 0, 0};
        if (!flagged(c, d, f, b))
          for (int k = 0; k < Kf; ++k)
            for (int e = 0; e < 4; ++e) m[e] += coh[k * S + s] * M[k][e];
        for (int e = 0; e < 4; ++e) out[4 * s + e] = m[e];
      }
    }
  }
  free(bp); free(bq);
}

void or_subband_cost(const or_cfg *c, const or_data *d, const double complex *J, double *cost) {
  int64_t tot = 0;
  for (int f = 0; f < c->P; ++f) tot += samples_of(c, f);
  double complex *model = malloc(sizeof(double complex) * 4 * tot);
  or_predict(c, d, J, model);
  const int B = n_baselines(c->N);
  for (int f = 0; f < c->P; ++f) {
    const int64_t off = vis_offset(c, f), spb = (int64_t)c->T * c->n_chan[f];
    double g = 0;
    for (int b = 0; b < B; ++b) {
      if (flagged(c, d, f, b)) continue;
      for (int64_t s = b * spb; s < (b + 1) * spb; ++s) {
        double complex r[4];
        for (int e = 0; e < 4; ++e) r[e] = d->vis[4 * (off + s) + e] - model[4 * (off + s) + e];
        g += m2_norm2(r);
      }
    }
    cost[f] = g;
  }
  free(model);
}

/* ---- Section 3: one direction of one subband --------------------------------------------- */
typedef struct {
  int N, B;
  int64_t spb;                  /* samples per baseline */
  const int *bp, *bq;
  const double complex *Vk;     /* [S][4] SAGE expectation for this direction */
  const double complex *ck;     /* [S] coherency scalars of this direction */
  const uint8_t *flag;          /* [B] or NULL */
  const double complex *Y, *BZ; /* [N][4] */
  double rho;
  int solver;                   /* OR_SOLVE_CHOLESKY or OR_SOLVE_PCG */
  double cg_tol;
} dir_problem;

/* SAGE expectation step: V_k = V - sum_{l != k} c_l J_lp J_lq^H */
static void dir_estep(const or_cfg *c, const or_data *d, const double complex *J, int f, int k,
                      const int *bp, const int *bq, double complex *Vk) {
  const int N = c->N, B = n_baselines(N), Kf = c->n_dirs[f];
  const int64_t spb = (int64_t)c->T * c->n_chan[f], S = samples_of(c, f);
  const double complex *V = d->vis + 4 * vis_offset(c, f);
  const double complex *coh = d->coh + coh_offset(c, f);
  for (int b = 0; b < B; ++b) {
    double complex M[OR_KMAX][4];
    for (int l = 0; l < Kf; ++l) {
      const double complex *Jl = J + ((int64_t)f * c->K + l) * N * 4;
      m2_mul_h(Jl + 4 * bp[b], Jl + 4 * bq[b], M[l]);
    }
    for (int64_t s = b * spb; s < (b + 1) * spb; ++s)
      for (int e = 0; e < 4; ++e) {
        double complex v = V[4 * s + e];
        for (int l = 0; l < Kf; ++l)
          if (l != k) v -= coh[l * S + s] * M[l][e];
        Vk[4 * s + e] = v;
      }
  }
}

/* Data term sum ||V_k - c J_p J_q^H||^2 and, optionally, D_b = sum_s conj(c_s) r_s */
static double dir_data_cost(const dir_problem *P, const double complex *Jd, double complex *D) {
  double g = 0;
  for (int b = 0; b < P->B; ++b) {
    if (D) for (int e = 0; e < 4; ++e) D[4 * b + e] = 0;
    if (P->flag && P->flag[b]) continue;
    double complex M[4];
    m2_mul_h(Jd + 4 * P->bp[b], Jd + 4 * P->bq[b], M);
    for (int64_t s = b * P->spb; s < (b + 1) * P->spb; ++s) {
      const double complex cs = P->ck[s];
      for (int e = 0; e < 4; ++e) {
        const double complex r = P->Vk[4 * s + e] - cs * M[e];
        g += creal(r) * creal(r) + cimag(r) * cimag(r);
        if (D) D[4 * b + e] += conj(cs) * r;
      }
    }
  }
  return g;
}

/* Consensus terms Re tr(Y^H (J - BZ)) + rho/2 ||J - BZ||^2 (Appendix A trace form) */
static double dir_penalty(const dir_problem *P, const double complex *Jd) {
  double s = 0;
  for (int i = 0; i < 4 * P->N; ++i) {
    const double complex e = Jd[i] - P->BZ[i];
    s += creal(conj(P->Y[i]) * e) + 0.5 * P->rho * (creal(e) * creal(e) + cimag(e) * cimag(e));
  }
  return s;
}

/* Jacobian of M = J_p J_q^H with respect to the 16 real parameters: first the 8 of J_p
 * (entry (a,b), then Re/Im), then the 8 of J_q.  M_ij = sum_m J_p[i][m] conj(J_q[j][m]). */
static void dM_dtheta(const double complex *Jp, const double complex *Jq, double complex dM[16][4]) {
  for (int a = 0; a < 2; ++a)
    for (int bb = 0; bb < 2; ++bb)
      for (int ri = 0; ri < 2; ++ri) {
        const int idx = (a * 2 + bb) * 2 + ri;
        const double complex unit = ri ? I : 1.0;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) {
            dM[idx][i * 2 + j] = (i == a) ? unit * conj(Jq[j * 2 + bb]) : 0.0;
            dM[8 + idx][i * 2 + j] = (j == a) ? Jp[i * 2 + bb] * conj(unit) : 0.0;
          }
      }
}

/* Euclidean gradient over the real parameters, packed as d/dRe + i d/dIm per entry:
 * data part  -2 sum_b sum_ij Re(conj(dM_ij/dtheta) D_b,ij), plus Y + rho (J - BZ). */
static void dir_gradient(const dir_problem *P, const double complex *Jd, const double complex *D,
                         double complex *G) {
  double *g = calloc(8 * P->N, sizeof(double));
  for (int b = 0; b < P->B; ++b) {
    if (P->flag && P->flag[b]) continue;
    const int p = P->bp[b], q = P->bq[b];
    double complex dM[16][4];
    dM_dtheta(Jd + 4 * p, Jd + 4 * q, dM);
    for (int t = 0; t < 16; ++t) {
      double v = 0;
      for (int e = 0; e < 4; ++e) v += creal(conj(dM[t][e]) * D[4 * b + e]);
      g[(t < 8 ? p * 8 + t : q * 8 + (t - 8))] += -2.0 * v;
    }
  }
  for (int i = 0; i < 4 * P->N; ++i)
    G[i] = g[2 * i] + I * g[2 * i + 1] + P->Y[i] + P->rho * (Jd[i] - P->BZ[i]);
  free(g);
}

/* Gauss-Newton matrix of the data term: 2 sum_b S_b Re<dM/dtheta_u, dM/dtheta_v>, where
 * S_b = sum_s |c_s|^2 (the coherency is a scalar times I2, so the per-sample Jacobian is c_s
 * times the Jacobian of M). */
static void dir_gn(const dir_problem *P, const double complex *Jd, double *H) {
  const int n = 8 * P->N;
  memset(H, 0, sizeof(double) * n * n);
  for (int b = 0; b < P->B; ++b) {
    if (P->flag && P->flag[b]) continue;
    double Sb = 0;
    for (int64_t s = b * P->spb; s < (b + 1) * P->spb; ++s)
      Sb += creal(P->ck[s]) * creal(P->ck[s]) + cimag(P->ck[s]) * cimag(P->ck[s]);
    const int p = P->bp[b], q = P->bq[b];
    double complex dM[16][4];
    dM_dtheta(Jd + 4 * p, Jd + 4 * q, dM);
    for (int u = 0; u < 16; ++u)
      for (int v = 0; v < 16; ++v) {
        double w = 0;
        for (int e = 0; e < 4; ++e) w += creal(conj(dM[u][e]) * dM[v][e]);
        const int ru = u < 8 ? p * 8 + u : q * 8 + u - 8;
        const int rv = v < 8 ? p * 8 + v : q * 8 + v - 8;
        H[(int64_t)ru * n + rv] += 2.0 * Sb * w;
      }
  }
}

int or_cholesky(int n, const double *A, double *L) {
  memset(L, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double s = A[(int64_t)j * n + j];
    for (int m = 0; m < j; ++m) s -= L[(int64_t)j * n + m] * L[(int64_t)j * n + m];
    if (!(s > 0.0) || !isfinite(s)) return -1;
    const double ljj = sqrt(s);
    L[(int64_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(int64_t)i * n + j];
      for (int m = 0; m < j; ++m) t -= L[(int64_t)i * n + m] * L[(int64_t)j * n + m];
      L[(int64_t)i * n + j] = t / ljj;
    }
  }
  return 0;
}

static void chol_solve(int n, const double *L, const double *b, double *x) {
  double *y = malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int m = 0; m < i; ++m) s -= L[(int64_t)i * n + m] * y[m];
    y[i] = s / L[(int64_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int m = i + 1; m < n; ++m) s -= L[(int64_t)m * n + i] * x[m];
    x[i] = s / L[(int64_t)i * n + i];
  }
  free(y);
}

/* Preconditioned conjugate gradients (Hestenes & Stiefel 1952; preconditioned form as in Saad,
 * "Iterative Methods for Sparse Linear Systems", 2nd ed., Algorithm 9.1) for M x = b with M
 * symmetric positive definite, from x = 0.  The preconditioner is block Jacobi: the inverse of
 * each 8x8 diagonal block of M (the real parameters of one station), applied through that block's
 * Cholesky factor.  Iterates until ||r|| <= tol ||b|| (r = b - M x) or n iterations; a search
 * direction with p.Mp <= 0 or a block that is not positive definite is a failure (-1). */
int or_pcg(int n, const double *M, const double *b, double tol, double *x, int *iters) {
  const int nb = n / 8;
  double *Lb = malloc(sizeof(double) * 64 * nb);
  double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
  double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
  int status = 0, it = 0;
  for (int s = 0; s < nb && status == 0; ++s) {
    double blk[64];
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) blk[i * 8 + j] = M[(int64_t)(8 * s + i) * n + 8 * s + j];
    if (or_cholesky(8, blk, Lb + 64 * s) != 0) status = -1;
  }
  double bb = 0;
  for (int i = 0; i < n; ++i) { x[i] = 0; r[i] = b[i]; bb += b[i] * b[i]; }
  if (status == 0 && bb > 0) {
    for (int s = 0; s < nb; ++s) chol_solve(8, Lb + 64 * s, r + 8 * s, z + 8 * s);
    double rz = 0;
    for (int i = 0; i < n; ++i) { p[i] = z[i]; rz += r[i] * z[i]; }
    while (it < n) {
      ++it;
      double pq = 0;
      for (int i = 0; i < n; ++i) {
        double t = 0;
        for (int j = 0; j < n; ++j) t += M[(int64_t)i * n + j] * p[j];
        q[i] = t;
        pq += p[i] * t;
      }
      if (!(pq > 0.0) || !isfinite(pq)) { status = -1; break; }
      const double alpha = rz / pq;
      double rr = 0;
      for (int i = 0; i < n; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
        rr += r[i] * r[i];
      }
      if (rr <= tol * tol * bb) break;
      for (int s = 0; s < nb; ++s) chol_solve(8, Lb + 64 * s, r + 8 * s, z + 8 * s);
      double rzn = 0;
      for (int i = 0; i < n; ++i) rzn += r[i] * z[i];
      const double beta = rzn / rz;
      for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      rz = rzn;
    }
  }
  if (iters) *iters = it;
  free(Lb); free(r); free(z); free(p); free(q);
  return status;
}

/* Levenberg-Marquardt on one direction's augmented Lagrangian (minimisation M1).
 * Damping follows Nielsen's rule (Madsen, Nielsen & Tingleff 2004, Sec. 3.2): lambda_0 =
 * tau * max diag(A), A = H_GN + rho I; step (A + lambda I) delta = -G; predicted decrease
 * ell = delta.(lambda delta - G)/2; accept iff ell > 0 and the objective decreases.  The step is
 * the Cholesky solution, or (solver OR_SOLVE_PCG) the conjugate-gradient iterate at the stated
 * residual tolerance: a CG iterate from zero satisfies delta.(A + lambda I) delta = -G.delta
 * (its residual is orthogonal to the Krylov space holding delta), so ell keeps the same form.
 * Stopping: after an iteration whose step predicts ell <= lm_tol * F (F the objective before
 * the step) the run ends, the trace rows of the iterations not run repeating (F, lambda) with
 * accepted = 0; lm_tol = 0 runs all iterations. */
static void lm_dir(const dir_problem *P, double complex *Jd, int iters, double lm_tol,
                   double *trace) {
  const int N = P->N, n = 8 * N;
  double complex *D = malloc(sizeof(double complex) * 4 * P->B);
  double complex *G = malloc(sizeof(double complex) * 4 * N);
  double complex *Jt = malloc(sizeof(double complex) * 4 * N);
  double *A = malloc(sizeof(double) * n * n), *Mw = malloc(sizeof(double) * n * n);
  double *L = malloc(sizeof(double) * n * n);
  double *rhs = malloc(sizeof(double) * n), *delta = malloc(sizeof(double) * n);

  double F = dir_data_cost(P, Jd, D) + dir_penalty(P, Jd);
  dir_gradient(P, Jd, D, G);
  dir_gn(P, Jd, A);
  for (int i = 0; i < n; ++i) A[(int64_t)i * n + i] += P->rho;
  double dmax = 0;
  for (int i = 0; i < n; ++i) dmax = fmax(dmax, A[(int64_t)i * n + i]);
  double lambda = LM_TAU * dmax, nu = 2.0;

  for (int it = 0; it < iters; ++it) {
    int accepted = 0, stop = 0;
    const double F_before = F;
    memcpy(Mw, A, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) Mw[(int64_t)i * n + i] += lambda;
    for (int i = 0; i < 4 * N; ++i) { rhs[2 * i] = -creal(G[i]); rhs[2 * i + 1] = -cimag(G[i]); }
    int solved;
    if (P->solver == OR_SOLVE_PCG) {
      solved = or_pcg(n, Mw, rhs, P->cg_tol, delta, NULL) == 0;
    } else {
      solved = or_cholesky(n, Mw, L) == 0;
      if (solved) chol_solve(n, L, rhs, delta);
    }
    if (!solved) {
      lambda *= nu; nu *= 2.0;
    } else {
      double ell = 0;
      for (int i = 0; i < 4 * N; ++i)
        ell += delta[2 * i] * (lambda * delta[2 * i] - creal(G[i]))
             + delta[2 * i + 1] * (lambda * delta[2 * i + 1] - cimag(G[i]));
      ell *= 0.5;
      stop = lm_tol > 0.0 && ell <= lm_tol * F_before;
      for (int i = 0; i < 4 * N; ++i) Jt[i] = Jd[i] + delta[2 * i] + I * delta[2 * i + 1];
      const double Fn = dir_data_cost(P, Jt, NULL) + dir_penalty(P, Jt);
      if (ell > 0.0 && F - Fn > 0.0) {
        const double gain = (F - Fn) / ell;
        memcpy(Jd, Jt, sizeof(double complex) * 4 * N);
        F = dir_data_cost(P, Jd, D) + dir_penalty(P, Jd);
        dir_gradient(P, Jd, D, G);
        dir_gn(P, Jd, A);
        for (int i = 0; i < n; ++i) A[(int64_t)i * n + i] += P->rho;
        const double t = 2.0 * gain - 1.0;
        lambda *= fmax(1.0 / 3.0, 1.0 - t * t * t);
        nu = 2.0;
        accepted = 1;
      } else {
        lambda *= nu; nu *= 2.0;
      }
    }
    if (trace) { trace[3 * it] = F; trace[3 * it + 1] = lambda; trace[3 * it + 2] = accepted; }
    if (stop) {
      for (int r = it + 1; trace && r < iters; ++r) {
        trace[3 * r] = F; trace[3 * r + 1] = lambda; trace[3 * r + 2] = 0;
      }
      break;
    }
  }
  free(D); free(G); free(Jt); free(A); free(Mw); free(L); free(rhs); free(delta);
}

static void make_problem(const or_cfg *c, const or_data *d, int f, int k, const int *bp,
                         const int *bq, const double complex *Vk, const double complex *Y,
                         const double complex *BZ, double rho, dir_problem *P) {
  P->N = c->N; P->B = n_baselines(c->N);
  P->spb = (int64_t)c->T * c->n_chan[f];
  P->bp = bp; P->bq = bq; P->Vk = Vk;
  P->ck = d->coh + coh_offset(c, f) + (int64_t)k * samples_of(c, f);
  P->flag = d->flags ? d->flags + (int64_t)f * P->B : NULL;
  P->Y = Y; P->BZ = BZ; P->rho = rho;
  P->solver = c->solver;
  P->cg_tol = c->cg_tol;
}

void or_dir_objective(const or_cfg *c, const or_data *d, const double complex *J,
                      const double complex *Y, const double complex *BZ, int f, int k,
                      const double complex *Jdir, double *L, double complex *grad) {
  const int N = c->N, B = n_baselines(N);
  int *bp = malloc(sizeof(int) * B), *bq = malloc(sizeof(int) * B);
  baseline_tables(N, bp, bq);
  double complex *Vk = malloc(sizeof(double complex) * 4 * samples_of(c, f));
  dir_estep(c, d, J, f, k, bp, bq, Vk);
  const int64_t o = ((int64_t)f * c->K + k) * N * 4;
  dir_problem P;
  make_problem(c, d, f, k, bp, bq, Vk, Y + o, BZ + o, c->rho[k], &P);
  double complex *D = malloc(sizeof(double complex) * 4 * B);
  *L = dir_data_cost(&P, Jdir, D) + dir_penalty(&P, Jdir);
  if (grad) dir_gradient(&P, Jdir, D, grad);
  free(D); free(Vk); free(bp); free(bq);
}

void or_dir_gn_hessian(const or_cfg *c, const or_data *d, int f, int k,
                       const double complex *Jdir, double *H) {
  const int N = c->N, B = n_baselines(N);
  int *bp = malloc(sizeof(int) * B), *bq = malloc(sizeof(int) * B);
  baseline_tables(N, bp, bq);
  dir_problem P;
  make_problem(c, d, f, k, bp, bq, NULL, NULL, NULL, 0.0, &P);
  dir_gn(&P, Jdir, H);
  free(bp); free(bq);
}

int or_local_step(const or_cfg *c, const or_data *d, double complex *J, const double complex *Y,
                  const double complex *BZ, int unregularised, double *lm_trace) {
  const int N = c->N, B = n_baselines(N), K = c->K;
  int *bp = malloc(sizeof(int) * B), *bq = malloc(sizeof(int) * B);
  baseline_tables(N, bp, bq);
  double complex *zeros = calloc(4 * N, sizeof(double complex));
#pragma omp parallel for schedule(dynamic)
  for (int f = 0; f < c->P; ++f) {
    double complex *Vk = malloc(sizeof(double complex) * 4 * samples_of(c, f));
    for (int sw = 0; sw < c->sage_sweeps; ++sw)
      for (int k = 0; k < c->n_dirs[f]; ++k) {
        const int64_t o = ((int64_t)f * K + k) * N * 4;
        dir_estep(c, d, J, f, k, bp, bq, Vk);
        dir_problem P;
        make_problem(c, d, f, k, bp, bq, Vk, unregularised ? zeros : Y + o,
                     unregularised ? zeros : BZ + o, unregularised ? 0.0 : c->rho[k], &P);
        double *tr = lm_trace
            ? lm_trace + 3 * (int64_t)c->lm_iters * ((int64_t)(f * c->sage_sweeps + sw) * K + k)
            : NULL;
        lm_dir(&P, J + o, c->lm_iters, c->lm_tol, tr);
      }
    free(Vk);
  }
  free(zeros); free(bp); free(bq);
  return 0;
}

/* ---- Section 3, initialisation: unitary-ambiguity alignment ----------------------------- */
/* unitary polar factor of a 2x2 complex matrix by the Newton iteration
 * U <- (U + U^{-H}) / 2 (Higham, "Functions of Matrices", Sec. 8.3) */
int or_polar2(const double complex *A, double complex *U) {
  double complex X[4] = {A[0], A[1], A[2], A[3]};
  for (int it = 0; it < 100; ++it) {
    const double complex det = X[0] * X[3] - X[1] * X[2];
    if (cabs(det) == 0.0) return -1;
    /* X^{-H} = (adj X / det)^H */
    double complex inv[4] = {X[3] / det, -X[1] / det, -X[2] / det, X[0] / det};
    double complex Xn[4];
    Xn[0] = 0.5 * (X[0] + conj(inv[0]));
    Xn[1] = 0.5 * (X[1] + conj(inv[2]));
    Xn[2] = 0.5 * (X[2] + conj(inv[1]));
    Xn[3] = 0.5 * (X[3] + conj(inv[3]));
    double diff = 0;
    for (int e = 0; e < 4; ++e) diff += cabs(Xn[e] - X[e]);
    memcpy(X, Xn, sizeof X);
    if (diff < GPA_TOL) break;
  }
  memcpy(U, X, sizeof X);
  return 0;
}

void or_gpa(const or_cfg *c, double complex *J, int rounds) {
  const int N = c->N, K = c->K;
  int *list = malloc(sizeof(int) * c->P);
  double complex *ref = malloc(sizeof(double complex) * 4 * N);
  for (int k = 0; k < K; ++k) {
    int cnt = 0;
    for (int f = 0; f < c->P; ++f)
      if (c->n_dirs[f] > k) list[cnt++] = f;
    if (cnt == 0) continue;
    memcpy(ref, J + ((int64_t)list[cnt / 2] * K + k) * N * 4, sizeof(double complex) * 4 * N);
    for (int r = 0; r < rounds; ++r) {
      for (int i = 0; i < cnt; ++i) {
        double complex *Jf = J + ((int64_t)list[i] * K + k) * N * 4;
        double complex A[4] = {0, 0, 0, 0}, T[4], U[4];
        for (int p = 0; p < N; ++p) {        /* A = J_f^H J_ref */
          m2_hmul(Jf + 4 * p, ref + 4 * p, T);
          for (int e = 0; e < 4; ++e) A[e] += T[e];
        }
        if (or_polar2(A, U) != 0) continue;
        for (int p = 0; p < N; ++p) {
          m2_mul(Jf + 4 * p, U, T);
          memcpy(Jf + 4 * p, T, sizeof T);
        }
      }
      memset(ref, 0, sizeof(double complex) * 4 * N);
      for (int i = 0; i < cnt; ++i)
        for (int e = 0; e < 4 * N; ++e) ref[e] += J[((int64_t)list[i] * K + k) * N * 4 + e] / cnt;
    }
  }
  free(list); free(ref);
}

/* ---- Section 3, fusion centre ---------------------------------------------------------- */
/* least squares min ||A z - x|| for real A (m x n, row-major) and nrhs complex right-hand
 * sides (X is m x nrhs), by Householder QR.  Returns -1 when A is rank deficient. */
int or_lstsq(int m, int n, const double *A, int nrhs, const double complex *X, double complex *Z) {
  if (m < n) return -1;
  double *R = malloc(sizeof(double) * m * n), *v = malloc(sizeof(double) * m);
  double complex *W = malloc(sizeof(double complex) * m * nrhs);
  memcpy(R, A, sizeof(double) * m * n);
  memcpy(W, X, sizeof(double complex) * m * nrhs);
  double amax = 0;
  for (int i = 0; i < m * n; ++i) amax = fmax(amax, fabs(A[i]));
  int status = 0;
  for (int j = 0; j < n; ++j) {
    double nrm = 0;
    for (int i = j; i < m; ++i) nrm += R[i * n + j] * R[i * n + j];
    nrm = sqrt(nrm);
    if (nrm <= 1e-13 * amax) { status = -1; break; }
    const double alpha = R[j * n + j] > 0 ? -nrm : nrm;
    for (int i = 0; i < m; ++i) v[i] = 0;
    for (int i = j; i < m; ++i) v[i] = R[i * n + j];
    v[j] -= alpha;
    double vn = 0;
    for (int i = j; i < m; ++i) vn += v[i] * v[i];
    if (vn == 0) continue;
    for (int col = j; col < n; ++col) {
      double s = 0;
      for (int i = j; i < m; ++i) s += v[i] * R[i * n + col];
      s = 2.0 * s / vn;
      for (int i = j; i < m; ++i) R[i * n + col] -= s * v[i];
    }
    for (int col = 0; col < nrhs; ++col) {
      double complex s = 0;
      for (int i = j; i < m; ++i) s += v[i] * W[(int64_t)i * nrhs + col];
      s = 2.0 * s / vn;
      for (int i = j; i < m; ++i) W[(int64_t)i * nrhs + col] -= s * v[i];
    }
  }
  if (status == 0)
    for (int col = 0; col < nrhs; ++col)
      for (int i = n - 1; i >= 0; --i) {
        double complex s = W[(int64_t)i * nrhs + col];
        for (int j = i + 1; j < n; ++j) s -= R[i * n + j] * Z[(int64_t)j * nrhs + col];
        Z[(int64_t)i * nrhs + col] = s / R[i * n + i];
      }
  free(R); free(v); free(W);
  return status;
}

static double basis_term(const or_cfg *c, int f, int l) {
  /* b_l(f) = ((f - f0)/f0)^(l-1), the example polynomial of Section 3 (l counted from 1) */
  const double x = (c->freq[f] - c->f0) / c->f0;
  double v = 1.0;
  for (int e = 0; e < l; ++e) v *= x;
  return v;
}

int or_consensus(const or_cfg *c, const double complex *J, double complex *Y, double complex *Z,
                 double complex *BZ, double *primal, double *dual) {
  const int N = c->N, K = c->K, Q = c->Q, W = 4 * N;
  int *list = malloc(sizeof(int) * c->P);
  double *A = malloc(sizeof(double) * c->P * Q);
  double complex *X = malloc(sizeof(double complex) * c->P * W);
  double complex *Zn = malloc(sizeof(double complex) * Q * W);
  double psum = 0, dsum = 0;
  int pcnt = 0, dcnt = 0, status = 0;
  for (int k = 0; k < K; ++k) {
    int cnt = 0;
    for (int f = 0; f < c->P; ++f)
      if (c->n_dirs[f] > k) list[cnt++] = f;
    if (cnt == 0) continue;
    if (cnt < Q) { status = -1; break; }
    const double rho = c->rho[k];
    for (int i = 0; i < cnt; ++i) {
      const int f = list[i];
      for (int l = 0; l < Q; ++l) A[i * Q + l] = basis_term(c, f, l);
      const int64_t o = ((int64_t)f * K + k) * W;
      for (int e = 0; e < W; ++e) X[(int64_t)i * W + e] = rho > 0 ? J[o + e] + Y[o + e] / rho : J[o + e];
    }
    /* Z_k = argmin sum_f || (J_f + Y_f/rho) - B_f Z_k ||^2, the minimiser M2 (gradient wrt Z
     * equal to zero, Section 3) */
    if (or_lstsq(cnt, Q, A, W, X, Zn) != 0) { status = -1; break; }
    double dz = 0;
    for (int e = 0; e < Q * W; ++e) {
      const double complex t = Zn[e] - Z[(int64_t)k * Q * W + e];
      dz += creal(t) * creal(t) + cimag(t) * cimag(t);
      Z[(int64_t)k * Q * W + e] = Zn[e];
    }
    dsum += sqrt(dz) / sqrt(4.0 * Q * N); dcnt++;
    for (int i = 0; i < cnt; ++i) {
      const int f = list[i];
      const int64_t o = ((int64_t)f * K + k) * W;
      double pr = 0;
      for (int e = 0; e < W; ++e) {
        double complex bz = 0;
        for (int l = 0; l < Q; ++l) bz += A[i * Q + l] * Zn[(int64_t)l * W + e];
        BZ[o + e] = bz;
        const double complex t = J[o + e] - bz;
        Y[o + e] += rho * t;                       /* dual ascent M3 */
        pr += creal(t) * creal(t) + cimag(t) * cimag(t);
      }
      psum += sqrt(pr) / sqrt(4.0 * N); pcnt++;
    }
  }
  if (primal) *primal = pcnt ? psum / pcnt : 0;
  if (dual) *dual = dcnt ? dsum / dcnt : 0;
  free(list); free(A); free(X); free(Zn);
  return status;
}

static double total_penalty(const or_cfg *c, const double complex *J, const double complex *Y,
                            const double complex *BZ) {
  double s = 0;
  const int N = c->N, K = c->K;
  for (int f = 0; f < c->P; ++f)
    for (int k = 0; k < c->n_dirs[f]; ++k) {
      const int64_t o = ((int64_t)f * K + k) * N * 4;
      for (int e = 0; e < 4 * N; ++e) {
        const double complex t = J[o + e] - BZ[o + e];
        s += creal(conj(Y[o + e]) * t) + 0.5 * c->rho[k] * (creal(t) * creal(t) + cimag(t) * cimag(t));
      }
    }
  return s;
}

int or_admm_solve(const or_cfg *c, const or_data *d, int iters, double complex *J,
                  double complex *Y, double complex *Z, double complex *BZ, double *trace,
                  int carry) {
  const int64_t nj = (int64_t)c->P * c->K * c->N * 4, nz = (int64_t)c->K * c->Q * c->N * 4;
  if (!carry) {   /* Y^0 = Z^0 = 0 (Section 3); carry: continue from the given state */
    memset(Y, 0, sizeof(double complex) * nj);
    memset(BZ, 0, sizeof(double complex) * nj);
    memset(Z, 0, sizeof(double complex) * nz);
  }
  double *g = malloc(sizeof(double) * c->P);
  int status = 0;
  for (int n = 0; n < iters && status == 0; ++n) {
    or_local_step(c, d, J, Y, BZ, n == 0 && (c->options & OR_OPT_UNREG_FIRST), NULL);
    if (n == 0 && (c->options & OR_OPT_GPA_FIRST)) or_gpa(c, J, 3);
    or_subband_cost(c, d, J, g);
    double cost = 0;
    for (int f = 0; f < c->P; ++f) cost += g[f];
    const double L = cost + total_penalty(c, J, Y, BZ);
    double pr = 0, du = 0;
    status = or_consensus(c, J, Y, Z, BZ, &pr, &du);
    if (trace) { trace[4 * n] = cost; trace[4 * n + 1] = L; trace[4 * n + 2] = pr; trace[4 * n + 3] = du; }
  }
  free(g);
  return status;
}
