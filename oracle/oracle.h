/* FP64 CPU oracle for consensus-ADMM distributed calibration (Yatawatta 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately unoptimised implementation of
 * what the GPU library computes, written from the paper's equations.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (shared with the data generator, fixed by the paper's problem statement):
 *   complex values are C99 double complex (interleaved re, im);
 *   baselines b enumerate station pairs p<q row-major; per subband the sample index is
 *   s = (b*T + t)*n_chan[f] + ch; visibilities are 2x2 row-major per sample;
 *   coherencies are one complex scalar c per (k, b, t, ch) (the paper's C = c*I2 for an
 *   unpolarised point source, Section 2);
 *   Jones J[f][k][p] are 2x2 row-major; Z[k][l][p] likewise; Y and BZ have J's layout.
 *   The real parameter vector of one direction is theta[p*8 + (i*2+j)*2 + {0:Re, 1:Im}].
 */
#ifndef CALIB_ORACLE_H
#define CALIB_ORACLE_H

#include <complex.h>
#include <stdint.h>

#define OR_OPT_GPA_FIRST 1u        /* align gauges at the first ADMM iteration (Section 3)   */
#define OR_OPT_UNREG_FIRST 2u      /* first local step without the consensus terms           */

typedef struct {
  int N, P, Q, K, T;
  const int32_t *n_chan;   /* [P] */
  const int32_t *n_dirs;   /* [P] */
  const double *freq;      /* [P] Hz */
  double f0;               /* basis reference frequency, Hz */
  const double *rho;       /* [K] */
  int lm_iters, sage_sweeps;
  uint32_t options;
  double lm_tol;           /* stop a direction's LM once a step's predicted decrease <= lm_tol*F */
  int solver;              /* damped normal equations: OR_SOLVE_CHOLESKY or OR_SOLVE_PCG         */
  double cg_tol;           /* OR_SOLVE_PCG: stop once ||r|| <= cg_tol ||G||                      */
} or_cfg;

#define OR_SOLVE_CHOLESKY 0
#define OR_SOLVE_PCG 1

typedef struct {
  const double complex *vis;    /* [sum_f S_f][2][2] */
  const double complex *coh;    /* [sum_f K_f*S_f]   */
  const uint8_t *flags;         /* [P*B] or NULL     */
} or_data;

/* model visibilities sum_k c J_p J_q^H per sample (Section 2, visibility model) */
void or_predict(const or_cfg *c, const or_data *d, const double complex *J, double complex *model);
/* data cost g_f per subband (Section 2, least-squares cost) */
void or_subband_cost(const or_cfg *c, const or_data *d, const double complex *J, double *cost);
/* one direction's augmented Lagrangian value and Euclidean gradient at Jdir (4N complex), with
 * the SAGE expectation built from the other directions of J (Section 3) */
void or_dir_objective(const or_cfg *c, const or_data *d, const double complex *J,
                      const double complex *Y, const double complex *BZ, int f, int k,
                      const double complex *Jdir, double *L, double complex *grad);
/* Gauss-Newton part 2*Jac^T*Jac of the data term's Hessian, dense (8N)x(8N) row-major */
void or_dir_gn_hessian(const or_cfg *c, const or_data *d, int f, int k,
                       const double complex *Jdir, double *H);
/* one local step (all subbands): SAGE over directions, LM per direction.  lm_trace (optional)
 * receives per (f, sweep, k, it) the triple (objective after the iteration, lambda, accepted). */
int or_local_step(const or_cfg *c, const or_data *d, double complex *J, const double complex *Y,
                  const double complex *BZ, int unregularised, double *lm_trace);
/* first-iteration gauge alignment by generalised Procrustes (Section 3, initialisation) */
void or_gpa(const or_cfg *c, double complex *J, int rounds);
/* fusion-centre Z update, B_f Z, dual update and residuals (Section 3, steps D2-D3) */
int or_consensus(const or_cfg *c, const double complex *J, double complex *Y, double complex *Z,
                 double complex *BZ, double *primal, double *dual);
/* the whole C-ADMM loop; trace [iters][4] = data cost, Lagrangian, primal, dual.  carry = 0
 * starts from Y = Z = B_f Z = 0 (Section 3); carry = 1 continues from the given Y, Z and B_f Z
 * (the previous solution interval's state) */
int or_admm_solve(const or_cfg *c, const or_data *d, int iters, double complex *J,
                  double complex *Y, double complex *Z, double complex *BZ, double *trace,
                  int carry);

/* textbook helpers exposed for pinning */
int or_cholesky(int n, const double *A, double *L);
/* preconditioned conjugate gradients on the SPD system M x = b (block-Jacobi, 8x8 blocks), x0 = 0;
 * returns -1 on a non-positive curvature or block, else 0; *iters receives the iterations run */
int or_pcg(int n, const double *M, const double *b, double tol, double *x, int *iters);
int or_polar2(const double complex *A, double complex *U);
int or_lstsq(int m, int n, const double *A, int nrhs, const double complex *X, double complex *Z);
int or_num_threads(void);
void or_set_num_threads(int n);

#endif
