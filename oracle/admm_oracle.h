/*
 * admm_oracle.h -- plain double-precision CPU oracle for the ADMM iteration of
 * Zhou & Bhattacharya, "Accelerated computational micromechanics"
 * (arXiv 2010.06697).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU path: the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does. It shares no code, header, table or helper with
 * the HIP library.
 *
 * Conventions (chosen here, independent of the GPU library's header):
 *   - grid n1 x n2 x n3, voxel (k1,k2,k3) at linear index (k3*n2 + k2)*n1 + k1,
 *     spacing h = 1 (voxel units);
 *   - fields are component-major: a 3-vector field holds 3*V doubles,
 *     component i at [i*V + idx]; a 3x3 tensor field holds 9*V doubles,
 *     component (i,J) at [(3*i+J)*V + idx] (row-major F_iJ);
 *   - the deformation gradient is stored as F itself (not F - I);
 *   - the DFT is unnormalised forward, exp(-2*pi*i m.k/N), inverse exp(+...)/V.
 */
#ifndef ADMM_ORACLE_H
#define ADMM_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OR_OK = 0,
  OR_NOT_CONVERGED = 1, /* ADMM hit max_iter, or a local Newton hit its cap */
  OR_EINVAL = -1,       /* bad argument */
  OR_EDOMAIN = -5       /* det F <= 0 or NaN met */
};

enum { OR_NEOHOOKE = 0, OR_LCE = 1 };

/* Material of one phase.
 *   OR_NEOHOOKE: W = mu/2 (|F|^2 - 3) - mu ln J + lambda/2 (ln J)^2
 *   OR_LCE:      W = mu/2 [ a^(1/3) (|F|^2 + (1/a - 1) |F^T n|^2) - 3 ]
 *                    + kappa/2 (J - 1)^2
 *                    + mu alpha/2 (|F^T n|^2 - (n0 . F^T n)^2)
 *                (neo-classical energy with step length tensor
 *                 L(n) = a^(-1/3) (I + (a-1) n n), a volumetric penalty, and
 *                 the non-ideality of Sec. 5.1 with the cross-link director
 *                 n0 of the voxel; a >= 1: the director elongates the
 *                 material). The Frank term and the dissipation of Sec. 5.1
 *                 enter the local problem through or_site (below) and
 *                 or_admm_run. */
typedef struct {
  int model;
  double mu, lambda; /* neo-Hookean */
  double a, kappa;   /* LCE */
  double alpha;      /* LCE non-ideality strength (0: ideal) */
  double frank;      /* LCE Frank constant kappa_F, energy density x voxel^2 */
  double nu_F, nu_n; /* LCE dissipation coefficients of F and of the director */
} or_material;

/* What the full LCE model adds at one voxel: the cross-link director n0 of
 * the non-ideality, and a constant symmetric form Sc (row-major 3x3) with
 * W += n . Sc n, which carries the Frank term with the neighbours' directors
 * lagged and the director's dissipation (or_admm_run builds it). A NULL site
 * means alpha = 0 and Sc = 0. */
typedef struct {
  double n0[3];
  double Sc[9];
} or_site;

/* Options of the per-voxel Newton solve of the local problem. */
typedef struct {
  int max_iter;     /* Newton iteration cap (100) */
  double gtol;      /* stop when |grad| <= gtol * scale before a step (1e-15) */
  double step_tol;  /* stop after a full PD Newton step with |d| <= step_tol*max(1,|F|) */
} or_newton;

/* ADMM parameters. */
typedef struct {
  double rho_min, rho_max; /* clamp of the adaptive penalty */
  double kappa_rho, tau;   /* adaptive-penalty factor and ratio threshold */
  int adapt_rho;           /* 0: fixed rho, 1: adaptive rule after each test */
  double tol_p, tol_d;     /* primal / dual tolerances */
  double mu_ref;           /* representative modulus in r_d */
  int max_iter;            /* iteration cap */
  int fixed_iters;         /* 1: run exactly max_iter iterations, no test */
  or_newton newton;
  /* Inexact local step (the two strategies of Sec. 2.1 and Sec. 4): Step 1
   * runs in passes of at most local_chunk Newton iterations per voxel, each
   * pass continuing from the previous iterate (F and, for the LCE, the
   * director), until the pass's stopping test holds or local_passes passes
   * have run.
   *   local_ratio > 0 (the strategy the paper adopts): every iteration but
   *     the first of a load step; the test is r_l <= local_ratio r_d, where
   *     r_l = |P(F) - Lambda - rho (grad u - F)| / mu_ref (RMS over voxels)
   *     and r_d is the previous iteration's dual residual.
   *   local_fraction > 0: every iteration; the test is that the local Newton
   *     solve has converged (its own stopping rule) at no fewer than
   *     local_fraction V voxels.
   * Both zero: exact local solves. At most one of them is nonzero. With an
   * inexact Step 1 the convergence test also requires r_l <= tol_d. */
  double local_ratio;
  int local_chunk;
  int local_passes;
  int local_start_iter;    /* index of this call's first iteration in the load step */
  double local_rd_prev;    /* r_d of the iteration before it (when local_start_iter > 0) */
  double local_fraction;
  /* Mixed boundary conditions (Sec. 2.3: some components of <F> prescribed,
   * the complementary components of the average stress zero; the UNI, PE and
   * EB protocols of Sec. 5): bit k (k = 3i + j) of free_mask leaves <F>_ij
   * free. Step 2 then minimises the augmented Lagrangian over it as well as
   * over u, which sets <F>_ij = <F_{i+1} - Lambda_i / rho>_ij, and Step 3
   * then leaves <Lambda>_ij = 0, so <P>_ij = 0 at convergence. */
  unsigned free_mask;
  /* Time step of the load step (Sec. 5.1's implicit discretisation), read
   * where a material has nu_F or nu_n > 0: Step 1 then adds
   * nu_F/(2 dt) |F - F^n|^2 and nu_n/(2 dt) (1 - (n . n^n)^2), with F^n, n^n
   * the fields at the start of the call. */
  double dt;
} or_params;

/* ---- small pieces, exposed so that tests can pin each one ---- */

/* 3D DFT of a complex field (re, im: V doubles each), separable direct sums.
 * inverse = 0: forward unnormalised; inverse = 1: conjugate kernel and 1/V. */
int or_dft3(int n1, int n2, int n3, const double *re, const double *im,
            double *out_re, double *out_im, int inverse);

/* Gradient of the displacement: G_iJ = Fbar_iJ + (u_i(x+e_J) - u_i(x-e_J))/2. */
int or_gradient(int n1, int n2, int n3, const double *u, const double Fbar[9],
                double *G);

/* Step 2 (Helmholtz projection): u = argmin_u sum_x |D_h u - H|^2 with zero
 * mean and no null-mode content. H: 9*V, u: 3*V. max_imag (may be NULL)
 * receives max |Im| of the inverse transform relative to max |Re|. */
int or_project(int n1, int n2, int n3, const double *H, double *u,
               double *max_imag);

/* Energy, first Piola stress and tangent dP_iJ/dF_kL (81 doubles, row
 * (3i+J), column (3k+L)) of one material point; n and site (may be NULL) are
 * read by OR_LCE only. */
double or_energy(const or_material *m, const double F[9], const double n[3],
                 const or_site *site);
int or_stress(const or_material *m, const double F[9], const double n[3],
              const or_site *site, double P[9]);
int or_tangent(const or_material *m, const double F[9], const double n[3],
               const or_site *site, double C[81]);

/* Top eigenvector of F F^T with the sign / tie rules of the director update.
 * n_prev: previous director (unit). Writes unit n. */
int or_director(const double F[9], const double n_prev[3], double n[3]);

/* LCE with the director eliminated: W_r(F) = min over unit n of W(F, n).
 * The director terms form a quadratic n . M(F) n; the minimiser is the
 * eigenvector of the smallest eigenvalue of M (for the ideal model the top
 * eigenvector of F F^T), with the rules of or_director for signs and ties.
 * Writes n, the stress P = dW_r/dF (= P(F, n)) and the tangent
 * K = d2W_r/dF2 (81 doubles, or NULL), which adds to the fixed-director
 * tangent the eigenvector's sensitivity to F. */
int or_relaxed(const or_material *m, const double F[9], const or_site *site,
               const double n_prev[3], double n[3], double P[9], double K[81]);

/* Step 1 (local problem) at one point: F = argmin W(F,n) + rho/2 |F - A|^2,
 * for the LCE jointly over F and the unit director n (Newton on the relaxed
 * objective W_r(F) + rho/2 |F - A|^2). F holds the warm start on entry and
 * the minimiser on exit; n (LCE) holds the previous director on entry and the
 * minimising one on exit. iters (may be NULL) receives the Newton iteration
 * count. */
int or_prox(const or_material *m, double rho, const double A[9], const or_site *site,
            const or_newton *opt, double F[9], double n[3], int *iters);

/* Adaptive penalty rule applied after the convergence test. */
double or_rho_update(double rho, double r_p, double r_d, const or_params *p);

/* ---- the whole iteration ---- */

/* Runs ADMM iterations on one periodic cell.
 *   phase: V bytes indexing mats; Fbar: macroscopic gradient (row-major; its
 *   free components, see free_mask, are updated in place);
 *   u (3V), F (9V), Lambda (9V): state, updated in place; director (3V) or NULL;
 *   director0 (3V): cross-link directors of the non-ideality, or NULL (then
 *   no material may have alpha != 0);
 *   rho: in/out penalty; hist_* (max_iter doubles each, may be NULL) receive
 *   r_p, r_d and the rho used at each iteration; iters: iterations done.
 * Returns OR_OK (converged or fixed count done), OR_NOT_CONVERGED, or an error. */
int or_admm_run(int n1, int n2, int n3, const unsigned char *phase,
                const or_material *mats, int n_mat, double Fbar[9],
                const or_params *p, double *u, double *F, double *Lambda,
                double *director, const double *director0, double *rho, double *hist_rp,
                double *hist_rd, double *hist_rho, int *iters,
                int *newton_fail);

/* Homogenised first Piola stress <P> = (1/V) sum_x P(F(x)) (plain summation in
 * voxel order), and the mean multiplier <Lambda>. Either output may be NULL.
 * director0 as in or_admm_run. */
int or_mean_stress(int n1, int n2, int n3, const unsigned char *phase,
                   const or_material *mats, int n_mat, const double *F,
                   const double *director, const double *director0,
                   const double *Lambda, double P_mean[9], double Lambda_mean[9]);

/* Orientation tensor of Sec. 5 (polydomain order parameter):
 * S = 3/2 (<n (x) n> - I/3) over the voxels whose phase is an LCE. */
int or_orientation(int n1, int n2, int n3, const unsigned char *phase,
                   const or_material *mats, int n_mat, const double *director,
                   double S[9]);

/* Stability modulus of Sec. 2.5 (quadratic functionals and Bloch waves):
 *   beta = min over unit Bloch waves v = p(x) exp(i omega . x), p periodic,
 *          <p, p> = 1, of <grad v, L grad v>
 * (averages over the unit-volume cell; L(x) = d2W/dF2 at the equilibrium
 * state F, director; the LCE with its director eliminated). On the grid the
 * gradient of v is exp(i omega . x) D_w p with the shifted central
 * difference (D_w p)_ij(x) = (p_i(x+e_j) e^{i w_j} - p_i(x-e_j) e^{-i w_j})/2,
 * omega in radians per voxel (2 pi/(k n_j) for a k-cell super-lattice along
 * x_j). ADMM of Steps 1'-4' with penalty rho:
 *   1' G = (L + rho I)^{-1} (g + rho D_w p)        (needs L + rho I > 0)
 *   2' p = argmin over <p, p> = 1 of |D_w p - (G - g/rho)|^2: in Fourier
 *      space p^ = b^ / (|K|^2 - sigma), b = D_w^H (G - g/rho),
 *      |K|^2 = sum_j sin^2(xi_j + w_j), sigma < min |K|^2 the root of
 *      sum |b^|^2/(|K|^2 - sigma)^2 = V^2 (bisection)
 *   3' g += rho (D_w p - G)
 *   4' r_p = |D_w p - G|, r_d = rho |D_w p - D_w p_prev| (RMS), both <= tol.
 * p_re, p_im (3V each): start in (normalised first), mode out. beta: the
 * Rayleigh quotient <D_w p, L D_w p> of the last p; sigma_rho (may be NULL):
 * rho sigma of the last Step 2', which equals beta at the fixed point.
 * Returns OR_OK, OR_NOT_CONVERGED, OR_EDOMAIN (L + rho I not positive
 * definite) or OR_EINVAL. */
int or_bloch(int n1, int n2, int n3, const unsigned char *phase, const or_material *mats,
             int n_mat, const double *F, const double *director, const double omega[3],
             double rho, double tol, int max_iter, double *p_re, double *p_im, double *beta,
             double *sigma_rho, int *iters);

/* Number of OpenMP threads the oracle uses (1 without OpenMP), and setting
 * it (n > 0). */
int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
