/*
 * admm_oracle.c -- plain double-precision CPU oracle for one ADMM iteration of
 * Zhou & Bhattacharya, "Accelerated computational micromechanics"
 * (arXiv 2010.06697).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library; the product path never does. It is
 * deliberately slow and literal: direct (not fast) Fourier sums, a scalar
 * Newton solve per voxel, plain loops in voxel order. Nothing here is shared
 * with the HIP library.
 *
 * What each function follows in the paper:
 *   or_dft3        - the discrete Fourier transform of the periodic setting,
 *                    Sec. 2.3, written as its defining sum along each axis.
 *   or_gradient    - the central difference of Sec. 2.3 (the first-derivative
 *                    symbol i sin(h xi)/h) plus the prescribed mean <F>.
 *   or_project     - Step 2 of Sec. 2.1 (Helmholtz projection), solved in
 *                    Fourier space as in Sec. 2.3 with central-difference
 *                    symbols; the Laplacian is taken as D_h^T D_h (the sum of
 *                    the squared first-difference symbols), which makes Step 2
 *                    the exact minimiser over u of the discrete augmented
 *                    Lagrangian and keeps the multiplier divergence-free.
 *   or_prox        - Step 1 of Sec. 2.1 (local problem): the point-wise
 *                    stationarity condition W_F(F) - Lambda - rho(grad u - F) = 0,
 *                    solved as the minimiser of W + rho/2 |F - A|^2.
 *   or_admm_run    - Steps 1-4 of Sec. 2.1 in order, the multiplier update
 *                    of Step 3, the primal/dual residuals of Step 4, and the
 *                    adaptive penalty rule of Sec. 2.1 ("Penalty parameter").
 *   or_mean_stress - the homogenised (average) stress of Sec. 2.3.
 */
#include "admm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

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

/* ------------------------------------------------------------------------ */
/* 3x3 helpers (row-major, A[3*i+j])                                        */
/* ------------------------------------------------------------------------ */

static double det3(const double *A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* cofactor matrix: C_ij = (-1)^(i+j) minor_ij, so that A^{-T} = C / det A */
static void cof3(const double *A, double *C) {
  C[0] = A[4] * A[8] - A[5] * A[7];
  C[1] = A[5] * A[6] - A[3] * A[8];
  C[2] = A[3] * A[7] - A[4] * A[6];
  C[3] = A[2] * A[7] - A[1] * A[8];
  C[4] = A[0] * A[8] - A[2] * A[6];
  C[5] = A[1] * A[6] - A[0] * A[7];
  C[6] = A[1] * A[5] - A[2] * A[4];
  C[7] = A[2] * A[3] - A[0] * A[5];
  C[8] = A[0] * A[4] - A[1] * A[3];
}

static double dot9(const double *a, const double *b) {
  double s = 0.0;
  for (int k = 0; k < 9; ++k) s += a[k] * b[k];
  return s;
}

static double norm9(const double *a) { return sqrt(dot9(a, a)); }

/* ------------------------------------------------------------------------ */
/* Constitutive models                                                      */
/* ------------------------------------------------------------------------ */

/* |F^T n|^2 */
static double ftn2(const double *F, const double *n, double *Ftn) {
  double s = 0.0;
  for (int L = 0; L < 3; ++L) {
    double v = 0.0;
    for (int k = 0; k < 3; ++k) v += F[3 * k + L] * n[k];
    if (Ftn) Ftn[L] = v;
    s += v * v;
  }
  return s;
}

double or_energy(const or_material *m, const double F[9], const double n[3],
                 const or_site *site) {
  double J = det3(F);
  if (!(J > 0.0)) return INFINITY;
  double f2 = dot9(F, F);
  if (m->model == OR_NEOHOOKE) {
    double lj = log(J);
    return 0.5 * m->mu * (f2 - 3.0) - m->mu * lj + 0.5 * m->lambda * lj * lj;
  }
  /* OR_LCE */
  double a13 = cbrt(m->a), Ftn[3];
  double t = ftn2(F, n, Ftn);
  double W = 0.5 * m->mu * (a13 * (f2 + (1.0 / m->a - 1.0) * t) - 3.0) +
             0.5 * m->kappa * (J - 1.0) * (J - 1.0);
  if (site) {
    /* non-ideality mu alpha/2 (|F^T n|^2 - (n0 . F^T n)^2), then n . Sc n */
    double q = site->n0[0] * Ftn[0] + site->n0[1] * Ftn[1] + site->n0[2] * Ftn[2];
    W += 0.5 * m->mu * m->alpha * (t - q * q);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) W += n[i] * site->Sc[3 * i + j] * n[j];
  }
  return W;
}

int or_stress(const or_material *m, const double F[9], const double n[3],
              const or_site *site, double P[9]) {
  double J = det3(F);
  if (!(J > 0.0)) return OR_EDOMAIN;
  double C[9], G[9];
  cof3(F, C);
  for (int k = 0; k < 9; ++k) G[k] = C[k] / J; /* F^{-T} */
  if (m->model == OR_NEOHOOKE) {
    /* P = mu (F - F^{-T}) + lambda ln J F^{-T} */
    double lj = log(J);
    for (int k = 0; k < 9; ++k)
      P[k] = m->mu * (F[k] - G[k]) + m->lambda * lj * G[k];
    return OR_OK;
  }
  /* P = mu a^{1/3} (F + (1/a - 1) n (F^T n)) + kappa (J - 1) J F^{-T} */
  double a13 = cbrt(m->a), Ftn[3];
  ftn2(F, n, Ftn);
  for (int i = 0; i < 3; ++i)
    for (int L = 0; L < 3; ++L)
      P[3 * i + L] = m->mu * a13 * (F[3 * i + L] + (1.0 / m->a - 1.0) * n[i] * Ftn[L]) +
                     m->kappa * (J - 1.0) * J * G[3 * i + L];
  if (site && m->alpha != 0.0) {
    /* + mu alpha n (x) (F^T n - (n0 . F^T n) n0) */
    double q = site->n0[0] * Ftn[0] + site->n0[1] * Ftn[1] + site->n0[2] * Ftn[2];
    for (int i = 0; i < 3; ++i)
      for (int L = 0; L < 3; ++L)
        P[3 * i + L] += m->mu * m->alpha * n[i] * (Ftn[L] - q * site->n0[L]);
  }
  return OR_OK;
}

int or_tangent(const or_material *m, const double F[9], const double n[3],
               const or_site *site, double Cm[81]) {
  double J = det3(F);
  if (!(J > 0.0)) return OR_EDOMAIN;
  double C[9], Fi[9]; /* Fi[3*J+k] = (F^{-1})_Jk = C_kJ / det */
  cof3(F, C);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Fi[3 * a + b] = C[3 * b + a] / J;
  for (int i = 0; i < 3; ++i)
    for (int Jx = 0; Jx < 3; ++Jx)
      for (int k = 0; k < 3; ++k)
        for (int L = 0; L < 3; ++L) {
          double d_ik = (i == k), d_JL = (Jx == L);
          double v;
          if (m->model == OR_NEOHOOKE) {
            /* mu d_ik d_JL + (mu - lambda ln J) Fi_Jk Fi_Li + lambda Fi_Ji Fi_Lk */
            double lj = log(J);
            v = m->mu * d_ik * d_JL +
                (m->mu - m->lambda * lj) * Fi[3 * Jx + k] * Fi[3 * L + i] +
                m->lambda * Fi[3 * Jx + i] * Fi[3 * L + k];
          } else {
            /* mu a^{1/3} (d_ik + (1/a - 1) n_i n_k) d_JL
               + kappa [(2J - 1) J Fi_Ji Fi_Lk - (J - 1) J Fi_Jk Fi_Li] */
            double a13 = cbrt(m->a);
            v = m->mu * a13 * (d_ik + (1.0 / m->a - 1.0) * n[i] * n[k]) * d_JL +
                m->kappa * ((2.0 * J - 1.0) * J * Fi[3 * Jx + i] * Fi[3 * L + k] -
                            (J - 1.0) * J * Fi[3 * Jx + k] * Fi[3 * L + i]);
            /* non-ideality: mu alpha n_i n_k (d_JL - n0_J n0_L) */
            if (site && m->alpha != 0.0)
              v += m->mu * m->alpha * n[i] * n[k] * (d_JL - site->n0[Jx] * site->n0[L]);
          }
          Cm[(3 * i + Jx) * 9 + (3 * k + L)] = v;
        }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Director: top eigenvector of F F^T (cyclic Jacobi on a 3x3 matrix)       */
/* ------------------------------------------------------------------------ */

static void jacobi3(double B[9], double Vv[9], double w[3]) {
  for (int k = 0; k < 9; ++k) Vv[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = B[1] * B[1] + B[2] * B[2] + B[5] * B[5];
    double dia = B[0] * B[0] + B[4] * B[4] + B[8] * B[8];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double bpq = B[3 * p + q];
        if (bpq == 0.0) continue;
        /* rotation that zeroes B_pq */
        double theta = (B[3 * q + q] - B[3 * p + p]) / (2.0 * bpq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* B <- R^T B R with R = I + (c-1)(e_p e_p + e_q e_q) + s(e_p e_q - e_q e_p) */
        for (int k = 0; k < 3; ++k) { /* columns p, q */
          double bkp = B[3 * k + p], bkq = B[3 * k + q];
          B[3 * k + p] = c * bkp - s * bkq;
          B[3 * k + q] = s * bkp + c * bkq;
        }
        for (int k = 0; k < 3; ++k) { /* rows p, q */
          double bpk = B[3 * p + k], bqk = B[3 * q + k];
          B[3 * p + k] = c * bpk - s * bqk;
          B[3 * q + k] = s * bpk + c * bqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = Vv[3 * k + p], vkq = Vv[3 * k + q];
          Vv[3 * k + p] = c * vkp - s * vkq;
          Vv[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  w[0] = B[0];
  w[1] = B[4];
  w[2] = B[8];
}

/* Coefficient of the non-ideality relative to the director term of the
   neo-classical energy, and of Sc: with c = mu a^(1/3) (1 - 1/a) / 2 the
   director terms are n . M n, M = -c F F^T + (mu alpha/2) F P0 F^T + Sc,
   P0 = I - n0 n0, and the minimising director maximises n . S n with
   S = -M / c = F F^T - gamma F P0 F^T - Sc / c, gamma = alpha / (a^(1/3)(1 - 1/a)).
   Returns 0 (S = F F^T) for the ideal model or without a site. */
static int director_form(const or_material *m, const or_site *site, double *gamma,
                         double *inv_c) {
  if (!m || !site || m->model != OR_LCE || !(m->a > 1.0)) return 0;
  double a13 = cbrt(m->a), c = 0.5 * m->mu * a13 * (1.0 - 1.0 / m->a);
  *gamma = m->alpha / (a13 * (1.0 - 1.0 / m->a));
  *inv_c = 1.0 / c;
  return 1;
}

/* Eigen-decomposition of S (F F^T for the ideal model, see director_form)
   sorted by decreasing eigenvalue (w[0] >= w[1] >= w[2], eigenvectors in the
   columns of V), and the minimising director: the top eigenvector, its sign
   chosen so that n . n_prev >= 0. When the top eigenvalue is degenerate (the
   leading ncl eigenvalues within 1e-12 relative) every unit vector of that
   eigenspace is a minimiser and the previous director's projection onto it
   is kept. Returns ncl. */
static int director_eig(const or_material *m, const or_site *site, const double F[9],
                        const double n_prev[3], double n[3], double w[3], double V[9]) {
  double B[9], Vv[9], wu[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[3 * i + k] * F[3 * j + k];
      B[3 * i + j] = s;
    }
  double gamma = 0.0, inv_c = 0.0;
  if (director_form(m, site, &gamma, &inv_c)) {
    double Fn0[3];
    for (int i = 0; i < 3; ++i)
      Fn0[i] = F[3 * i] * site->n0[0] + F[3 * i + 1] * site->n0[1] + F[3 * i + 2] * site->n0[2];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        B[3 * i + j] = B[3 * i + j] - gamma * (B[3 * i + j] - Fn0[i] * Fn0[j]) -
                       inv_c * site->Sc[3 * i + j];
  }
  jacobi3(B, Vv, wu);
  int order[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a) /* sort eigenvalues descending */
    for (int b = a + 1; b < 3; ++b)
      if (wu[order[b]] > wu[order[a]]) {
        int t = order[a];
        order[a] = order[b];
        order[b] = t;
      }
  for (int e = 0; e < 3; ++e) {
    w[e] = wu[order[e]];
    for (int k = 0; k < 3; ++k) V[3 * k + e] = Vv[3 * k + order[e]];
  }
  double tie = 1e-12 * fmax(fabs(w[0]), fabs(w[2]));
  double out[3];
  int ncl = 1;
  while (ncl < 3 && w[0] - w[ncl] <= tie) ++ncl;
  if (ncl == 1) {
    for (int k = 0; k < 3; ++k) out[k] = V[3 * k];
  } else {
    for (int k = 0; k < 3; ++k) out[k] = 0.0;
    for (int e = 0; e < ncl; ++e) {
      double c = 0.0;
      for (int k = 0; k < 3; ++k) c += V[3 * k + e] * n_prev[k];
      for (int k = 0; k < 3; ++k) out[k] += c * V[3 * k + e];
    }
    double nn = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
    if (nn < 1e-8)
      for (int k = 0; k < 3; ++k) out[k] = V[3 * k];
  }
  double s = out[0] * n_prev[0] + out[1] * n_prev[1] + out[2] * n_prev[2];
  if (s < 0.0)
    for (int k = 0; k < 3; ++k) out[k] = -out[k];
  double nn = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
  for (int k = 0; k < 3; ++k) n[k] = out[k] / nn;
  return ncl;
}

int or_director(const double F[9], const double n_prev[3], double n[3]) {
  double w[3], V[9];
  director_eig(NULL, NULL, F, n_prev, n, w, V);
  return OR_OK;
}

/* The LCE energy with the director eliminated, W_r(F) = min_n W(F, n): for
   a >= 1 the director term (mu a^(1/3)/2)(1/a - 1)|F^T n|^2 is smallest at
   the top eigenvector of B = F F^T, so W_r(F) = W(F, n(F)) and, by the
   envelope theorem, dW_r/dF = P(F, n(F)). Its second derivative adds to the
   fixed-director tangent the eigenvector sensitivity of the top eigenvalue:
       d2 lambda_1 = 2 |dF^T n|^2 + 2 sum_k (t_k . dB n)^2 / (lambda_1 - lambda_k)
   over the other eigenvectors t_k, with t_k . dB n = w_k : dF,
       (w_k)_iJ = (t_k)_i (F^T n)_J + n_i (F^T t_k)_J.
   The first part is already in the fixed-director tangent; the second, times
   mu a^(1/3)(1/a - 1)/2, is negative semidefinite. Eigenvectors in the top
   eigenspace of n (ties, see director_eig) contribute nothing. K += that
   term. With the non-ideality, S = F F^T - gamma F P0 F^T (director_form;
   Sc does not depend on F) and t_k . dS n = w_k : dF with
       w_k = t_k (x) F^T n + n (x) F^T t_k - gamma (t_k (x) P0 F^T n + n (x) P0 F^T t_k). */
static void lce_rotation_term(const or_material *m, const or_site *site, const double F[9],
                              const double n[3], const double w[3], const double V[9], int ncl,
                              double *K) {
  double c2 = m->mu * cbrt(m->a) * (1.0 / m->a - 1.0); /* 2 c */
  double gamma = 0.0, inv_c = 0.0;
  int ext = director_form(m, site, &gamma, &inv_c);
  double ftn[3], pftn[3];
  for (int J = 0; J < 3; ++J) ftn[J] = F[J] * n[0] + F[3 + J] * n[1] + F[6 + J] * n[2];
  if (ext) {
    double q = site->n0[0] * ftn[0] + site->n0[1] * ftn[1] + site->n0[2] * ftn[2];
    for (int J = 0; J < 3; ++J) pftn[J] = ftn[J] - q * site->n0[J];
  }
  for (int e = ncl; e < 3; ++e) {
    double t[3] = {V[e], V[3 + e], V[6 + e]};
    double ftt[3], wk[9];
    for (int J = 0; J < 3; ++J) ftt[J] = F[J] * t[0] + F[3 + J] * t[1] + F[6 + J] * t[2];
    for (int i = 0; i < 3; ++i)
      for (int J = 0; J < 3; ++J) wk[3 * i + J] = t[i] * ftn[J] + n[i] * ftt[J];
    if (ext) {
      double q = site->n0[0] * ftt[0] + site->n0[1] * ftt[1] + site->n0[2] * ftt[2];
      for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J)
          wk[3 * i + J] -= gamma * (t[i] * pftn[J] + n[i] * (ftt[J] - q * site->n0[J]));
    }
    double f = c2 / (w[0] - w[e]);
    for (int a = 0; a < 9; ++a)
      for (int b = 0; b < 9; ++b) K[9 * a + b] += f * wk[a] * wk[b];
  }
}

/* LCE options valid for the director elimination: a >= 1, and a > 1 where
   the non-ideality or Sc is used (at a = 1 the neo-classical director term
   vanishes and S above is not defined) */
static int lce_site_ok(const or_material *m, const or_site *site) {
  if (!(m->a >= 1.0) || !(m->alpha >= 0.0)) return 0;
  if (site && !(m->a > 1.0)) {
    if (m->alpha != 0.0) return 0;
    for (int k = 0; k < 9; ++k)
      if (site->Sc[k] != 0.0) return 0;
  }
  return 1;
}

int or_relaxed(const or_material *m, const double F[9], const or_site *site,
               const double n_prev[3], double n[3], double P[9], double K[81]) {
  if (!m || !F || !n_prev || !n || m->model != OR_LCE || !lce_site_ok(m, site)) return OR_EINVAL;
  double w[3], V[9];
  int ncl = director_eig(m, site, F, n_prev, n, w, V);
  if (P && or_stress(m, F, n, site, P) != OR_OK) return OR_EDOMAIN;
  if (K) {
    if (or_tangent(m, F, n, site, K) != OR_OK) return OR_EDOMAIN;
    lce_rotation_term(m, site, F, n, w, V, ncl, K);
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 1: the local problem at one point                                   */
/* ------------------------------------------------------------------------ */

/* Cholesky factorisation of a 9x9 symmetric matrix in place (lower part);
   returns 0 when a pivot is not positive. */
static int chol9(double *K) {
  for (int j = 0; j < 9; ++j) {
    double d = K[9 * j + j];
    for (int k = 0; k < j; ++k) d -= K[9 * j + k] * K[9 * j + k];
    if (!(d > 0.0)) return 0;
    d = sqrt(d);
    K[9 * j + j] = d;
    for (int i = j + 1; i < 9; ++i) {
      double v = K[9 * i + j];
      for (int k = 0; k < j; ++k) v -= K[9 * i + k] * K[9 * j + k];
      K[9 * i + j] = v / d;
    }
  }
  return 1;
}

static void chol9_solve(const double *L, const double *b, double *x) {
  double y[9];
  for (int i = 0; i < 9; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[9 * i + k] * y[k];
    y[i] = v / L[9 * i + i];
  }
  for (int i = 8; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 9; ++k) v -= L[9 * k + i] * x[k];
    x[i] = v / L[9 * i + i];
  }
}

static double prox_objective(const or_material *m, double rho, const double *A,
                             const double *F, const double *n, const or_site *site) {
  double W = or_energy(m, F, n, site);
  double d2 = 0.0;
  for (int k = 0; k < 9; ++k) d2 += (F[k] - A[k]) * (F[k] - A[k]);
  return W + 0.5 * rho * d2;
}

static double moduli_sum(const or_material *m) {
  return m->model == OR_NEOHOOKE ? m->mu + m->lambda : m->mu * cbrt(m->a) + m->kappa;
}

/* Newton's method with Armijo backtracking on phi(F) = W(F,n) + rho/2|F-A|^2
   at fixed n. Returns OR_OK, OR_NOT_CONVERGED or OR_EDOMAIN; *it = iterations. */
static int newton_fixed_n(const or_material *m, double rho, const double *A,
                          const or_newton *opt, double *F, const double *n,
                          const or_site *site, int *it) {
  double P[9], g[9], K[81], d[9], Ft[9];
  double scale_mod = moduli_sum(m) + rho;
  for (int iter = 0; iter < opt->max_iter; ++iter) {
    if (or_stress(m, F, n, site, P) != OR_OK) {
      *it = iter;
      return OR_EDOMAIN;
    }
    for (int k = 0; k < 9; ++k) g[k] = P[k] + rho * (F[k] - A[k]);
    double scale = scale_mod * (1.0 + norm9(F) + norm9(A));
    if (norm9(g) <= opt->gtol * scale) {
      *it = iter;
      return OR_OK;
    }
    or_tangent(m, F, n, site, K);
    for (int k = 0; k < 9; ++k) K[10 * k] += rho;
    int pd = chol9(K);
    if (pd) {
      double mg[9];
      for (int k = 0; k < 9; ++k) mg[k] = -g[k];
      chol9_solve(K, mg, d);
    } else {
      for (int k = 0; k < 9; ++k) d[k] = -g[k];
    }
    double slope = dot9(g, d);
    double phi0 = prox_objective(m, rho, A, F, n, site);
    /* Armijo backtracking on phi. Once the predicted decrease falls below the
       rounding floor of phi itself, the energy test is noise; the step is then
       accepted on a decrease of the gradient norm instead. */
    double fn0 = norm9(F);
    double floor_phi = 1e-12 * scale_mod * (1.0 + fn0 * fn0);
    int small = -slope <= floor_phi;
    double gn = norm9(g);
    double t = 1.0;
    int accepted = 0;
    for (int ls = 0; ls < 60; ++ls) {
      for (int k = 0; k < 9; ++k) Ft[k] = F[k] + t * d[k];
      if (det3(Ft) > 0.0) {
        if (!small) {
          double phit = prox_objective(m, rho, A, Ft, n, site);
          if (phit <= phi0 + 1e-4 * t * slope) {
            accepted = 1;
            break;
          }
        } else {
          double Pt[9], gt[9];
          or_stress(m, Ft, n, site, Pt);
          for (int k = 0; k < 9; ++k) gt[k] = Pt[k] + rho * (Ft[k] - A[k]);
          if (norm9(gt) <= (1.0 - 1e-4 * t) * gn) {
            accepted = 1;
            break;
          }
        }
      }
      t *= 0.5;
    }
    if (!accepted) {
      *it = iter + 1;
      return OR_NOT_CONVERGED;
    }
    memcpy(F, Ft, sizeof(Ft));
    double fn = norm9(F);
    if (pd && t == 1.0 && norm9(d) <= opt->step_tol * (fn > 1.0 ? fn : 1.0)) {
      *it = iter + 1;
      return OR_OK;
    }
  }
  *it = opt->max_iter;
  return OR_NOT_CONVERGED;
}

/* LCE: Newton's method on the relaxed objective phi_r(F) = W_r(F) +
   rho/2 |F - A|^2, i.e. on F and the director jointly with the director
   eliminated (W_r above). At each iterate n = n(F) (continuity with the
   director of the previous iterate); backtracking as in newton_fixed_n, on
   phi_r with the director recomputed at every trial point, so the iterates
   descend monotonically. phi_r need not be convex: near states of uniaxial
   symmetry its curvature along the director-rotation mode goes like
   -1/(lambda_1 - lambda_2). The Newton matrix is therefore the relaxed
   tangent plus (rho + tau) I with the smallest tau of the sequence
   0, rho/16, rho/8, rho/4, ... for which the relaxed tangent plus
   (rho + tau - rho/16) I has a Cholesky factorisation (Newton's method with
   a multiple of the identity added to the Hessian, Nocedal & Wright,
   Numerical Optimization, Sec. 3.4): a pure Newton step where phi_r is
   convex with modulus rho/16, a descent direction of a positive-definite
   model elsewhere. The solve stops at a stationary point of phi_r, which
   with n = n(F) is a stationary point of the joint problem in (F, n). */
static int newton_relaxed(const or_material *m, double rho, const double A[9],
                          const or_newton *opt, double F[9], double n[3],
                          const or_site *site, int *it) {
  double P[9], g[9], Kr[81], d[9], Ft[9], nt[3], w[3], V[9], ncur[3];
  double scale_mod = moduli_sum(m) + rho;
  int ncl = director_eig(m, site, F, n, ncur, w, V);
  for (int iter = 0; iter < opt->max_iter; ++iter) {
    if (or_stress(m, F, ncur, site, P) != OR_OK) {
      *it = iter;
      memcpy(n, ncur, sizeof(ncur));
      return OR_EDOMAIN;
    }
    for (int k = 0; k < 9; ++k) g[k] = P[k] + rho * (F[k] - A[k]);
    double scale = scale_mod * (1.0 + norm9(F) + norm9(A));
    double gn = norm9(g);
    if (gn <= opt->gtol * scale) {
      *it = iter;
      memcpy(n, ncur, sizeof(ncur));
      return OR_OK;
    }
    or_tangent(m, F, ncur, site, Kr);
    for (int k = 0; k < 9; ++k) Kr[10 * k] += rho;
    lce_rotation_term(m, site, F, ncur, w, V, ncl, Kr);
    /* smallest tau of 0, rho/16, rho/8, ... with Kr + (tau - rho/16) I
       positive definite; the step uses Kr + tau I */
    double tau = 0.0, Ks[81];
    int found = 0;
    for (int tries = 0; tries < 64 && !found; ++tries) {
      memcpy(Ks, Kr, sizeof(Ks));
      for (int k = 0; k < 9; ++k) Ks[10 * k] += tau - rho / 16.0;
      if (chol9(Ks)) found = 1;
      else tau = tau == 0.0 ? rho / 16.0 : 2.0 * tau;
    }
    for (int k = 0; k < 9; ++k) Kr[10 * k] += tau;
    if (!found || !chol9(Kr)) {
      *it = iter + 1;
      memcpy(n, ncur, sizeof(ncur));
      return OR_NOT_CONVERGED;
    }
    double mg[9];
    for (int k = 0; k < 9; ++k) mg[k] = -g[k];
    chol9_solve(Kr, mg, d);
    double slope = dot9(g, d);
    double phi0 = prox_objective(m, rho, A, F, ncur, site);
    double fn0 = norm9(F);
    double floor_phi = 1e-12 * scale_mod * (1.0 + fn0 * fn0);
    int small = -slope <= floor_phi;
    double t = 1.0;
    int accepted = 0, nclt = 1;
    double wt[3], Vt[9];
    for (int ls = 0; ls < 60; ++ls) {
      for (int k = 0; k < 9; ++k) Ft[k] = F[k] + t * d[k];
      if (det3(Ft) > 0.0) {
        nclt = director_eig(m, site, Ft, ncur, nt, wt, Vt);
        if (!small) {
          if (prox_objective(m, rho, A, Ft, nt, site) <= phi0 + 1e-4 * t * slope) {
            accepted = 1;
            break;
          }
        } else {
          double Pt[9], gt[9];
          or_stress(m, Ft, nt, site, Pt);
          for (int k = 0; k < 9; ++k) gt[k] = Pt[k] + rho * (Ft[k] - A[k]);
          if (norm9(gt) <= (1.0 - 1e-4 * t) * gn) {
            accepted = 1;
            break;
          }
        }
      }
      t *= 0.5;
    }
    if (!accepted) {
      *it = iter + 1;
      memcpy(n, ncur, sizeof(ncur));
      return OR_NOT_CONVERGED;
    }
    memcpy(F, Ft, sizeof(Ft));
    memcpy(ncur, nt, sizeof(nt));
    memcpy(w, wt, sizeof(wt));
    memcpy(V, Vt, sizeof(Vt));
    ncl = nclt;
    double fn = norm9(F);
    if (t == 1.0 && norm9(d) <= opt->step_tol * (fn > 1.0 ? fn : 1.0)) {
      *it = iter + 1;
      memcpy(n, ncur, sizeof(ncur));
      return OR_OK;
    }
  }
  *it = opt->max_iter;
  memcpy(n, ncur, sizeof(ncur));
  return OR_NOT_CONVERGED;
}

/* Ideal LCE (no site terms): with the director eliminated the energy depends
   on F only through its singular values f1 >= f2 >= f3 > 0 (the director is
   the top left singular vector, |F^T n|^2 = f1^2):
       W_r(f) = mu a^(1/3)/2 (f1^2 + f2^2 + f3^2 + (1/a - 1) f1^2) - 3 mu/2
                + kappa/2 (f1 f2 f3 - 1)^2.
   For an energy of the singular values alone the local problem shares A's
   singular vectors. Write A = sum_i a_i u_i v_i^T with {u_i}, {v_i}
   right-handed orthonormal, a1 >= a2 >= |a3| and a3 of the sign of det A.
   For every F with det F > 0, tr(F^T A) <= sum_i f_i a_i (von Neumann's trace
   inequality in its form for proper rotations), with equality at
   F = sum_i f_i u_i v_i^T; |F|^2 and W_r depend on f alone. Hence
       min_F W_r(F) + rho/2 |F - A|^2 = min_f W_r(f) + rho/2 |f - a|^2,
   a problem in three unknowns whose minimiser is ordered like a (exchanging
   two unordered entries lowers both the coupling to a and, for the first
   entry, the director term). The singular basis comes from the eigenvectors
   of A A^T; where the top singular value is tied, u1 follows the previous
   director as in director_eig (every such u1 gives a minimiser). Newton's
   method on the three unknowns with the same stopping rules and the same
   backtracking as newton_relaxed; the 9-component gradient at
   F = sum f_i u_i v_i^T is sum_i (dh/df_i) u_i v_i^T, so its norm is that of
   the 3-component gradient and the gradient test means the same. The start
   is the current F's diagonal in the singular basis, or a (with entries
   below a1/16 raised to a1/16) where that has the lower objective. The
   solve runs to its stopping rules within max(max_iter, 100) iterations,
   also in the passes of the inexact step, whose chunk cap it does not
   take: a truncated solve would cost more passes than it saves. */
static double spec_h(double mua, double beta, double mu, double kap, double rho,
                     const double *f, const double *a) {
  double J = f[0] * f[1] * f[2];
  if (!(J > 0.0)) return INFINITY;
  double s = 0.0, d = 0.0;
  for (int i = 0; i < 3; ++i) {
    s += f[i] * f[i];
    d += (f[i] - a[i]) * (f[i] - a[i]);
  }
  return 0.5 * mua * (s + beta * f[0] * f[0]) - 1.5 * mu + 0.5 * kap * (J - 1.0) * (J - 1.0) +
         0.5 * rho * d;
}

static void spec_grad(double mua, double beta, double kap, double rho, const double *f,
                      const double *a, double *g) {
  double J = f[0] * f[1] * f[2];
  double p[3] = {f[1] * f[2], f[0] * f[2], f[0] * f[1]};
  for (int i = 0; i < 3; ++i) g[i] = mua * f[i] + rho * (f[i] - a[i]) + kap * (J - 1.0) * p[i];
  g[0] += mua * beta * f[0];
}

static int prox_spectral(const or_material *m, double rho, const double A[9],
                         const or_newton *opt, double F[9], double n[3], int *it) {
  const double mua = m->mu * cbrt(m->a), beta = 1.0 / m->a - 1.0, kap = m->kappa;
  double w[3], V[9], u[3][3], v[3][3], a[3];
  director_eig(NULL, NULL, A, n, u[0], w, V);
  /* u2: the eigenvector (of the top two) least aligned with u1, made
     orthogonal to it; u3 = u1 x u2 */
  double r[2][3], rn[2];
  for (int e = 0; e < 2; ++e) {
    double c = V[e] * u[0][0] + V[3 + e] * u[0][1] + V[6 + e] * u[0][2];
    for (int k = 0; k < 3; ++k) r[e][k] = V[3 * k + e] - c * u[0][k];
    rn[e] = r[e][0] * r[e][0] + r[e][1] * r[e][1] + r[e][2] * r[e][2];
  }
  int e2 = rn[0] > rn[1] ? 0 : 1;
  for (int k = 0; k < 3; ++k) u[1][k] = r[e2][k] / sqrt(rn[e2]);
  u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
  u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
  u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  /* v_i = A^T u_i / a_i for i = 1, 2 (orthogonalised); v3 = v1 x v2 and
     a3 = u3 . A v3, signed */
  for (int i = 0; i < 2; ++i) {
    for (int J = 0; J < 3; ++J) v[i][J] = A[J] * u[i][0] + A[3 + J] * u[i][1] + A[6 + J] * u[i][2];
    if (i == 1) {
      double c = v[1][0] * v[0][0] + v[1][1] * v[0][1] + v[1][2] * v[0][2];
      for (int J = 0; J < 3; ++J) v[1][J] -= c * v[0][J];
    }
    a[i] = sqrt(v[i][0] * v[i][0] + v[i][1] * v[i][1] + v[i][2] * v[i][2]);
    if (!(a[i] > 0.0)) {
      *it = 0;
      return OR_EDOMAIN;
    }
    for (int J = 0; J < 3; ++J) v[i][J] /= a[i];
  }
  v[2][0] = v[0][1] * v[1][2] - v[0][2] * v[1][1];
  v[2][1] = v[0][2] * v[1][0] - v[0][0] * v[1][2];
  v[2][2] = v[0][0] * v[1][1] - v[0][1] * v[1][0];
  a[2] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int J = 0; J < 3; ++J) a[2] += u[2][i] * A[3 * i + J] * v[2][J];
  /* start */
  double f[3], fa[3];
  for (int i = 0; i < 3; ++i) {
    f[i] = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int J = 0; J < 3; ++J) f[i] += u[i][k] * F[3 * k + J] * v[i][J];
    fa[i] = a[i] > a[0] / 16.0 ? a[i] : a[0] / 16.0;
  }
  if (!(spec_h(mua, beta, m->mu, kap, rho, f, a) <= spec_h(mua, beta, m->mu, kap, rho, fa, a)))
    memcpy(f, fa, sizeof(f));
  const double scale_mod = moduli_sum(m) + rho;
  const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  int rc = OR_NOT_CONVERGED, iter;
  const int cap = opt->max_iter > 100 ? opt->max_iter : 100;
  for (iter = 0; iter < cap; ++iter) {
    double g[3];
    spec_grad(mua, beta, kap, rho, f, a, g);
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (gn <= opt->gtol * scale_mod * (1.0 + nf + na)) {
      rc = OR_OK;
      break;
    }
    /* Hessian of h, plus the smallest tau of 0, rho/16, rho/8, ... that
       makes it positive definite */
    double J = f[0] * f[1] * f[2], p[3] = {f[1] * f[2], f[0] * f[2], f[0] * f[1]};
    double H[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        H[3 * i + j] = kap * p[i] * p[j] + (i == j ? mua + rho : kap * (J - 1.0) * f[3 - i - j]);
    H[0] += mua * beta;
    double L[9], tau = 0.0;
    int pd = 0;
    for (int tries = 0; tries < 64 && !pd; ++tries) {
      memcpy(L, H, sizeof(L));
      for (int i = 0; i < 3; ++i) L[4 * i] += tau;
      pd = 1;
      for (int j = 0; j < 3 && pd; ++j) {
        double d = L[4 * j];
        for (int k = 0; k < j; ++k) d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 0.0)) pd = 0;
        else {
          L[4 * j] = sqrt(d);
          for (int i = j + 1; i < 3; ++i) {
            double x = L[3 * i + j];
            for (int k = 0; k < j; ++k) x -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = x / L[4 * j];
          }
        }
      }
      if (!pd) tau = tau == 0.0 ? rho / 16.0 : 2.0 * tau;
    }
    if (!pd) break;
    double y[3], d[3];
    for (int i = 0; i < 3; ++i) {
      double x = -g[i];
      for (int k = 0; k < i; ++k) x -= L[3 * i + k] * y[k];
      y[i] = x / L[4 * i];
    }
    for (int i = 2; i >= 0; --i) {
      double x = y[i];
      for (int k = i + 1; k < 3; ++k) x -= L[3 * k + i] * d[k];
      d[i] = x / L[4 * i];
    }
    double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
    int small = -slope <= 1e-12 * scale_mod * (1.0 + nf * nf);
    double h0 = spec_h(mua, beta, m->mu, kap, rho, f, a), t = 1.0, ft[3];
    int acc = 0;
    for (int ls = 0; ls < 60 && !acc; ++ls) {
      for (int i = 0; i < 3; ++i) ft[i] = f[i] + t * d[i];
      if (ft[0] * ft[1] * ft[2] > 0.0) {
        if (!small) {
          acc = spec_h(mua, beta, m->mu, kap, rho, ft, a) <= h0 + 1e-4 * t * slope;
        } else {
          double gt[3];
          spec_grad(mua, beta, kap, rho, ft, a, gt);
          acc = sqrt(gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2]) <= (1.0 - 1e-4 * t) * gn;
        }
      }
      if (!acc) t *= 0.5;
    }
    if (!acc) {
      ++iter;
      break;
    }
    memcpy(f, ft, sizeof(f));
    double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (t == 1.0 && nd <= opt->step_tol * (nf > 1.0 ? nf : 1.0)) {
      ++iter;
      rc = OR_OK;
      break;
    }
  }
  *it = iter;
  for (int k = 0; k < 3; ++k)
    for (int J = 0; J < 3; ++J)
      F[3 * k + J] = f[0] * u[0][k] * v[0][J] + f[1] * u[1][k] * v[1][J] + f[2] * u[2][k] * v[2][J];
  for (int k = 0; k < 3; ++k) n[k] = u[0][k];
  return rc;
}

int or_prox(const or_material *m, double rho, const double A[9], const or_site *site,
            const or_newton *opt, double F[9], double n[3], int *iters) {
  if (!m || !A || !opt || !F || !(rho > 0.0)) return OR_EINVAL;
  int it = 0, rc;
  if (m->model == OR_NEOHOOKE) {
    rc = newton_fixed_n(m, rho, A, opt, F, n, NULL, &it);
  } else {
    if (!n || !lce_site_ok(m, site)) return OR_EINVAL;
    if (!site)
      rc = prox_spectral(m, rho, A, opt, F, n, &it);
    else
      rc = newton_relaxed(m, rho, A, opt, F, n, site, &it);
  }
  if (iters) *iters = it;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Periodic grid: DFT, gradient, Step 2                                     */
/* ------------------------------------------------------------------------ */

static int valid_dims(int n1, int n2, int n3) { return n1 >= 1 && n2 >= 1 && n3 >= 1; }

/* direct DFT of every line along one axis, in place on (re, im) */
static void dft_axis(int n1, int n2, int n3, int axis, double *re, double *im, int inverse) {
  int N = axis == 0 ? n1 : (axis == 1 ? n2 : n3);
  if (N == 1) return;
  size_t V = (size_t)n1 * n2 * n3;
  size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)n1 : (size_t)n1 * n2);
  size_t nlines = V / (size_t)N;
  double *c = (double *)malloc(sizeof(double) * N * N);
  double *s = (double *)malloc(sizeof(double) * N * N);
  double sg = inverse ? 1.0 : -1.0;
  for (int m = 0; m < N; ++m)
    for (int k = 0; k < N; ++k) {
      long t = ((long)m * k) % N;
      double ang = TWO_PI * (double)t / (double)N;
      c[m * N + k] = cos(ang);
      s[m * N + k] = sg * sin(ang);
    }
#pragma omp parallel
  {
    double *lr = (double *)malloc(sizeof(double) * N);
    double *li = (double *)malloc(sizeof(double) * N);
#pragma omp for schedule(static)
    for (size_t line = 0; line < nlines; ++line) {
      size_t base;
      if (axis == 0)
        base = line * (size_t)n1;
      else if (axis == 1)
        base = (line / n1) * (size_t)n1 * n2 + (line % n1);
      else
        base = line;
      for (int k = 0; k < N; ++k) {
        lr[k] = re[base + k * stride];
        li[k] = im[base + k * stride];
      }
      for (int m = 0; m < N; ++m) {
        const double *cm = c + (size_t)m * N, *sm = s + (size_t)m * N;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < N; ++k) {
          sr += lr[k] * cm[k] - li[k] * sm[k];
          si += lr[k] * sm[k] + li[k] * cm[k];
        }
        re[base + m * stride] = sr;
        im[base + m * stride] = si;
      }
    }
    free(lr);
    free(li);
  }
  free(c);
  free(s);
}

int or_dft3(int n1, int n2, int n3, const double *re, const double *im,
            double *out_re, double *out_im, int inverse) {
  if (!valid_dims(n1, n2, n3) || !re || !out_re || !out_im) return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  memcpy(out_re, re, V * sizeof(double));
  if (im)
    memcpy(out_im, im, V * sizeof(double));
  else
    memset(out_im, 0, V * sizeof(double));
  dft_axis(n1, n2, n3, 0, out_re, out_im, inverse);
  dft_axis(n1, n2, n3, 1, out_re, out_im, inverse);
  dft_axis(n1, n2, n3, 2, out_re, out_im, inverse);
  if (inverse) {
    double sc = 1.0 / (double)V;
    for (size_t x = 0; x < V; ++x) {
      out_re[x] *= sc;
      out_im[x] *= sc;
    }
  }
  return OR_OK;
}

int or_gradient(int n1, int n2, int n3, const double *u, const double Fbar[9], double *G) {
  if (!valid_dims(n1, n2, n3) || !u || !Fbar || !G) return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  int nn[3] = {n1, n2, n3};
#pragma omp parallel for schedule(static)
  for (long k3 = 0; k3 < n3; ++k3)
    for (int k2 = 0; k2 < n2; ++k2)
      for (int k1 = 0; k1 < n1; ++k1) {
        int kk[3] = {k1, k2, (int)k3};
        size_t x = ((size_t)k3 * n2 + k2) * n1 + k1;
        for (int j = 0; j < 3; ++j) {
          int kp[3] = {kk[0], kk[1], kk[2]}, km[3] = {kk[0], kk[1], kk[2]};
          kp[j] = (kk[j] + 1) % nn[j];
          km[j] = (kk[j] - 1 + nn[j]) % nn[j];
          size_t xp = ((size_t)kp[2] * n2 + kp[1]) * n1 + kp[0];
          size_t xm = ((size_t)km[2] * n2 + km[1]) * n1 + km[0];
          for (int i = 0; i < 3; ++i)
            G[(size_t)(3 * i + j) * V + x] =
                Fbar[3 * i + j] + 0.5 * (u[(size_t)i * V + xp] - u[(size_t)i * V + xm]);
        }
      }
  return OR_OK;
}

/* modified wavenumber sin(2 pi m / N) of the central difference, exactly zero
   at m = 0 and m = N/2 */
static double kmod(int m, int N) {
  int t = ((m % N) + N) % N;
  if (t == 0 || 2 * t == N) return 0.0;
  return sin(TWO_PI * (double)t / (double)N);
}

static int null_mode(int m, int N) {
  int t = ((m % N) + N) % N;
  return t == 0 || 2 * t == N;
}

int or_project(int n1, int n2, int n3, const double *H, double *u, double *max_imag) {
  if (!valid_dims(n1, n2, n3) || !H || !u) return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  double *ur = (double *)calloc(3 * V, sizeof(double)); /* 3 accumulators, Re */
  double *ui = (double *)calloc(3 * V, sizeof(double)); /* Im */
  double *hr = (double *)malloc(V * sizeof(double));
  double *hi = (double *)malloc(V * sizeof(double));
  double *tr = (double *)malloc(V * sizeof(double));
  double *ti = (double *)malloc(V * sizeof(double));
  if (!ur || !ui || !hr || !hi || !tr || !ti) {
    free(ur); free(ui); free(hr); free(hi); free(tr); free(ti);
    return OR_EINVAL;
  }
  /* u_hat_i = -i sum_j K_j H_hat_ij / |K|^2, accumulated one component at a time */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      or_dft3(n1, n2, n3, H + (size_t)(3 * i + j) * V, NULL, hr, hi, 0);
      for (int m3 = 0; m3 < n3; ++m3)
        for (int m2 = 0; m2 < n2; ++m2)
          for (int m1 = 0; m1 < n1; ++m1) {
            size_t x = ((size_t)m3 * n2 + m2) * n1 + m1;
            if (null_mode(m1, n1) && null_mode(m2, n2) && null_mode(m3, n3)) continue;
            double K[3] = {kmod(m1, n1), kmod(m2, n2), kmod(m3, n3)};
            double k2 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
            double w = K[j] / k2;
            /* -i * w * (hr + i hi) = w*hi - i*w*hr */
            ur[(size_t)i * V + x] += w * hi[x];
            ui[(size_t)i * V + x] -= w * hr[x];
          }
    }
  double mi = 0.0, mr = 0.0;
  for (int i = 0; i < 3; ++i) {
    or_dft3(n1, n2, n3, ur + (size_t)i * V, ui + (size_t)i * V, tr, ti, 1);
    for (size_t x = 0; x < V; ++x) {
      u[(size_t)i * V + x] = tr[x];
      if (fabs(tr[x]) > mr) mr = fabs(tr[x]);
      if (fabs(ti[x]) > mi) mi = fabs(ti[x]);
    }
  }
  if (max_imag) *max_imag = mr > 0.0 ? mi / mr : mi;
  free(ur); free(ui); free(hr); free(hi); free(tr); free(ti);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Steps 1-4                                                                */
/* ------------------------------------------------------------------------ */

double or_rho_update(double rho, double r_p, double r_d, const or_params *p) {
  /* rho <- kappa rho           if r_p / r_d > tau
     rho <- max(rho/kappa, min) if r_d / r_p > tau
     then clamped to rho_max */
  double out = rho;
  if (r_p > p->tau * r_d)
    out = p->kappa_rho * rho;
  else if (r_d > p->tau * r_p)
    out = fmax(rho / p->kappa_rho, p->rho_min);
  if (out > p->rho_max) out = p->rho_max;
  return out;
}

/* The data of Step 1 beyond A and rho for the full LCE model (Sec. 5.1). */
typedef struct {
  int n1, n2, n3;
  size_t V;
  const unsigned char *phase;
  const or_material *mats;
  const double *director0; /* cross-link directors (non-ideality) */
  const double *lag;       /* directors at the start of the iteration (Frank) */
  const double *dir_n;     /* directors at the start of the call (dissipation) */
  const double *F_n;       /* F at the start of the call (dissipation) */
  double dt;
} step1_data;

/* Local problem of voxel x. Returns its site (NULL for the ideal model) and,
   where F is dissipative, turns (rho, A) into the equivalent
   (rho + nu_F/dt, (rho A + nu_F/dt F^n) / (rho + nu_F/dt)). The site's Sc:
   the Frank energy kappa_F/2 sum over bonds |Q(x+e) - Q(x)|^2, Q = n (x) n,
   equals const - kappa_F sum over bonds (n(x) . n(y))^2 for unit directors,
   so with the neighbours lagged (the second approach of Sec. 2.1 for
   gradients of internal variables) voxel x sees -kappa_F sum_y n~(y) n~(y)^T
   over its six neighbours of an LCE phase; the director's dissipation
   nu_n/(2 dt)|n - n^n|^2 is taken in the sign-blind form
   nu_n/(2 dt)(1 - (n . n^n)^2) (equal to first order), i.e.
   -(nu_n/(2 dt)) n^n n^n^T. */
static const or_site *step1_site(const step1_data *c, size_t x, double *rho, double A[9],
                                 double Fn_buf[9], or_site *s) {
  const or_material *m = &c->mats[c->phase[x]];
  if (m->nu_F > 0.0) {
    double nu = m->nu_F / c->dt, r2 = *rho + nu;
    for (int k = 0; k < 9; ++k) {
      Fn_buf[k] = c->F_n[k * c->V + x];
      A[k] = (*rho * A[k] + nu * Fn_buf[k]) / r2;
    }
    *rho = r2;
  }
  if (m->model != OR_LCE || (m->alpha == 0.0 && m->frank == 0.0 && m->nu_n == 0.0)) return NULL;
  for (int k = 0; k < 3; ++k) s->n0[k] = c->director0 ? c->director0[k * c->V + x] : 0.0;
  for (int k = 0; k < 9; ++k) s->Sc[k] = 0.0;
  if (m->frank > 0.0) {
    int k1 = (int)(x % (size_t)c->n1), k2 = (int)((x / (size_t)c->n1) % (size_t)c->n2),
        k3 = (int)(x / ((size_t)c->n1 * c->n2));
    for (int d = 0; d < 6; ++d) {
      int j1 = k1, j2 = k2, j3 = k3, sg = (d & 1) ? -1 : 1;
      if (d < 2) j1 = (k1 + sg + c->n1) % c->n1;
      else if (d < 4) j2 = (k2 + sg + c->n2) % c->n2;
      else j3 = (k3 + sg + c->n3) % c->n3;
      size_t y = ((size_t)j3 * c->n2 + j2) * c->n1 + j1;
      if (c->mats[c->phase[y]].model != OR_LCE) continue;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          s->Sc[3 * i + j] -= m->frank * c->lag[i * c->V + y] * c->lag[j * c->V + y];
    }
  }
  if (m->nu_n > 0.0) {
    double w = 0.5 * m->nu_n / c->dt;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        s->Sc[3 * i + j] -= w * c->dir_n[i * c->V + x] * c->dir_n[j * c->V + x];
  }
  return s;
}

int or_admm_run(int n1, int n2, int n3, const unsigned char *phase,
                const or_material *mats, int n_mat, double Fbar[9],
                const or_params *p, double *u, double *F, double *Lambda,
                double *director, const double *director0, double *rho, double *hist_rp,
                double *hist_rd, double *hist_rho, int *iters, int *newton_fail) {
  if (!valid_dims(n1, n2, n3) || !phase || !mats || n_mat < 1 || !Fbar || !p || !u ||
      !F || !Lambda || !rho || !(*rho > 0.0) || p->max_iter < 0)
    return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  for (size_t x = 0; x < V; ++x)
    if (phase[x] >= n_mat) return OR_EINVAL;
  int need_lag = 0, need_dirn = 0, need_Fn = 0;
  for (int q = 0; q < n_mat; ++q) {
    const or_material *m = &mats[q];
    if (!(m->nu_F >= 0.0) || (m->nu_F > 0.0 && !(p->dt > 0.0))) return OR_EINVAL;
    need_Fn |= m->nu_F > 0.0;
    if (m->model != OR_LCE) continue;
    if (!director || !(m->alpha >= 0.0) || !(m->frank >= 0.0) || !(m->nu_n >= 0.0) ||
        !(m->a >= 1.0))
      return OR_EINVAL;
    if ((m->alpha > 0.0 || m->frank > 0.0 || m->nu_n > 0.0) && !(m->a > 1.0)) return OR_EINVAL;
    if (m->alpha > 0.0 && !director0) return OR_EINVAL;
    if (m->nu_n > 0.0 && !(p->dt > 0.0)) return OR_EINVAL;
    need_lag |= m->frank > 0.0;
    need_dirn |= m->nu_n > 0.0;
  }
  double *lag = need_lag ? (double *)malloc(3 * V * sizeof(double)) : NULL;
  double *dir_n = need_dirn ? (double *)malloc(3 * V * sizeof(double)) : NULL;
  double *F_n = need_Fn ? (double *)malloc(9 * V * sizeof(double)) : NULL;
  if ((need_lag && !lag) || (need_dirn && !dir_n) || (need_Fn && !F_n)) {
    free(lag); free(dir_n); free(F_n);
    return OR_EINVAL;
  }
  if (dir_n) memcpy(dir_n, director, 3 * V * sizeof(double));
  if (F_n) memcpy(F_n, F, 9 * V * sizeof(double));
  step1_data s1 = {n1, n2, n3, V, phase, mats, director0, lag, dir_n, F_n, p->dt};

  double *Gold = (double *)malloc(9 * V * sizeof(double));
  double *Gnew = (double *)malloc(9 * V * sizeof(double));
  double *H = (double *)malloc(9 * V * sizeof(double));
  if (!Gold || !Gnew || !H) {
    free(Gold); free(Gnew); free(H); free(lag); free(dir_n); free(F_n);
    return OR_EINVAL;
  }
  or_gradient(n1, n2, n3, u, Fbar, Gold); /* grad u_0 = Fbar + D_h u_0 */

  int rc = p->fixed_iters ? OR_OK : OR_NOT_CONVERGED;
  int done = 0, fails = 0, dom = 0;
  double rd_prev = p->local_rd_prev;
  double *g2 = (double *)malloc(V * sizeof(double));
  if (!g2) {
    free(Gold); free(Gnew); free(H); free(lag); free(dir_n); free(F_n);
    return OR_EINVAL;
  }
  if (p->local_ratio < 0.0 || p->local_fraction < 0.0 || p->local_fraction > 1.0 ||
      p->free_mask >= 512u ||
      (p->local_ratio > 0.0 && p->local_fraction > 0.0) ||
      ((p->local_ratio > 0.0 || p->local_fraction > 0.0) &&
       (p->local_chunk < 1 || p->local_passes < 1))) {
    free(Gold); free(Gnew); free(H); free(g2); free(lag); free(dir_n); free(F_n);
    return OR_EINVAL;
  }
  for (int it = 0; it < p->max_iter; ++it) {
    double r = *rho;
    if (lag) memcpy(lag, director, 3 * V * sizeof(double));
    double rl = 0.0; /* r_l after Step 1 (0 when solved exactly) */
    const int inexact = p->local_fraction > 0.0 ||
                        (p->local_ratio > 0.0 && p->local_start_iter + it > 0);
    if (inexact) {
      /* Step 1 solved inexactly: passes of at most local_chunk Newton
         iterations per voxel until r_l <= local_ratio * r_d (previous), or
         until the local solves have converged at local_fraction of the voxels */
      or_newton chunk = p->newton;
      chunk.max_iter = p->local_chunk;
      for (int pass = 0; pass < p->local_passes; ++pass) {
        long conv = 0;
#pragma omp parallel for schedule(static) reduction(+ : dom, conv)
        for (long xl = 0; xl < (long)V; ++xl) {
          size_t x = (size_t)xl;
          double A[9], Fx[9], nx[3] = {0.0, 0.0, 1.0}, P[9];
          for (int c = 0; c < 9; ++c) {
            A[c] = Gold[c * V + x] + Lambda[c * V + x] / r;
            Fx[c] = F[c * V + x];
          }
          if (director)
            for (int c = 0; c < 3; ++c) nx[c] = director[c * V + x];
          const or_material *m = &mats[phase[x]];
          int its = 0;
          double rx = r, Fn[9];
          or_site sb;
          const or_site *site = step1_site(&s1, x, &rx, A, Fn, &sb);
          int pr = or_prox(m, rx, A, site, &chunk, Fx, nx, &its);
          if (pr == OR_OK) conv += 1;
          if (pr == OR_EDOMAIN || or_stress(m, Fx, nx, site, P) != OR_OK) {
            dom += 1;
            g2[x] = 0.0;
          } else {
            double s2 = 0.0;
            for (int c = 0; c < 9; ++c) {
              double gc = P[c] + rx * (Fx[c] - A[c]);
              s2 += gc * gc;
            }
            g2[x] = s2;
          }
          for (int c = 0; c < 9; ++c) F[c * V + x] = Fx[c];
          if (director)
            for (int c = 0; c < 3; ++c) director[c * V + x] = nx[c];
        }
        if (dom) break;
        double sl = 0.0;
        for (size_t x = 0; x < V; ++x) sl += g2[x];
        rl = sqrt(sl / (double)V) / p->mu_ref;
        if (p->local_fraction > 0.0) {
          if ((double)conv >= p->local_fraction * (double)V) break;
        } else {
          if (rl <= p->local_ratio * rd_prev) break;
        }
      }
      if (dom) {
        rc = OR_EDOMAIN;
        done = it;
        break;
      }
    } else {
      /* Step 1: F_{i+1} = argmin W(F) + rho/2 |F - (grad u_i + Lambda_i / rho)|^2 */
#pragma omp parallel for schedule(static) reduction(+ : fails, dom)
      for (long xl = 0; xl < (long)V; ++xl) {
        size_t x = (size_t)xl;
        double A[9], Fx[9], nx[3] = {0.0, 0.0, 1.0};
        for (int c = 0; c < 9; ++c) {
          A[c] = Gold[c * V + x] + Lambda[c * V + x] / r;
          Fx[c] = F[c * V + x];
        }
        if (director)
          for (int c = 0; c < 3; ++c) nx[c] = director[c * V + x];
        int its = 0;
        double rx = r, Fn[9];
        or_site sb;
        const or_site *site = step1_site(&s1, x, &rx, A, Fn, &sb);
        int pr = or_prox(&mats[phase[x]], rx, A, site, &p->newton, Fx, nx, &its);
        if (pr == OR_NOT_CONVERGED) fails += 1;
        if (pr == OR_EDOMAIN) dom += 1;
        for (int c = 0; c < 9; ++c) F[c * V + x] = Fx[c];
        if (director)
          for (int c = 0; c < 3; ++c) director[c * V + x] = nx[c];
      }
      if (dom) {
        rc = OR_EDOMAIN;
        done = it;
        break;
      }
    }
    /* Step 2: -Lap u_{i+1} = div(-F_{i+1} + Lambda_i / rho); a free
       component of <F> minimises |<F> + D_h u - H|^2 too: the mean of H */
    for (size_t k = 0; k < 9 * V; ++k) H[k] = F[k] - Lambda[k] / r;
    or_project(n1, n2, n3, H, u, NULL);
    for (int c = 0; c < 9; ++c)
      if (p->free_mask & (1u << c)) {
        double sm = 0.0;
        for (size_t x = 0; x < V; ++x) sm += H[c * V + x];
        Fbar[c] = sm / (double)V;
      }
    /* Step 3: Lambda_{i+1} = Lambda_i + rho (grad u_{i+1} - F_{i+1}) */
    or_gradient(n1, n2, n3, u, Fbar, Gnew);
    for (size_t k = 0; k < 9 * V; ++k) Lambda[k] += r * (Gnew[k] - F[k]);
    /* Step 4: r_p = |grad u_{i+1} - F_{i+1}|, r_d = rho/mu |grad u_{i+1} - grad u_i| */
    double sp = 0.0, sd = 0.0;
    for (size_t x = 0; x < V; ++x)
      for (int c = 0; c < 9; ++c) {
        double e = Gnew[c * V + x] - F[c * V + x];
        double dd = Gnew[c * V + x] - Gold[c * V + x];
        sp += e * e;
        sd += dd * dd;
      }
    double rp = sqrt(sp / (double)V);
    double rd = r / p->mu_ref * sqrt(sd / (double)V);
    if (hist_rp) hist_rp[it] = rp;
    if (hist_rd) hist_rd[it] = rd;
    if (hist_rho) hist_rho[it] = r;
    rd_prev = rd;
    double *t = Gold;
    Gold = Gnew;
    Gnew = t;
    done = it + 1;
    if (!(rp == rp) || !(rd == rd)) {
      rc = OR_EDOMAIN;
      break;
    }
    /* with an inexact Step 1, equilibrium also needs a small local residual
       (the appendix bounds it by the dual and local residuals together) */
    if (!p->fixed_iters && rp <= p->tol_p && rd <= p->tol_d && rl <= p->tol_d) {
      rc = OR_OK;
      break;
    }
    if (p->adapt_rho) *rho = or_rho_update(r, rp, rd, p);
  }
  if (iters) *iters = done;
  if (newton_fail) *newton_fail = fails;
  free(Gold);
  free(Gnew);
  free(H);
  free(g2);
  free(lag);
  free(dir_n);
  free(F_n);
  return rc;
}

int or_mean_stress(int n1, int n2, int n3, const unsigned char *phase,
                   const or_material *mats, int n_mat, const double *F,
                   const double *director, const double *director0, const double *Lambda,
                   double P_mean[9], double Lambda_mean[9]) {
  if (!valid_dims(n1, n2, n3) || !phase || !mats || !F) return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  double sP[9] = {0}, sL[9] = {0};
  for (size_t x = 0; x < V; ++x) {
    if (phase[x] >= n_mat) return OR_EINVAL;
    double Fx[9], P[9], nx[3] = {0.0, 0.0, 1.0};
    for (int c = 0; c < 9; ++c) Fx[c] = F[c * V + x];
    if (director)
      for (int c = 0; c < 3; ++c) nx[c] = director[c * V + x];
    or_site sb, *site = NULL;
    if (director0 && mats[phase[x]].model == OR_LCE && mats[phase[x]].alpha != 0.0) {
      for (int c = 0; c < 3; ++c) sb.n0[c] = director0[c * V + x];
      for (int c = 0; c < 9; ++c) sb.Sc[c] = 0.0;
      site = &sb;
    }
    if (or_stress(&mats[phase[x]], Fx, nx, site, P) != OR_OK) return OR_EDOMAIN;
    for (int c = 0; c < 9; ++c) sP[c] += P[c];
    if (Lambda)
      for (int c = 0; c < 9; ++c) sL[c] += Lambda[c * V + x];
  }
  for (int c = 0; c < 9; ++c) {
    if (P_mean) P_mean[c] = sP[c] / (double)V;
    if (Lambda_mean) Lambda_mean[c] = sL[c] / (double)V;
  }
  return OR_OK;
}

int or_orientation(int n1, int n2, int n3, const unsigned char *phase,
                   const or_material *mats, int n_mat, const double *director,
                   double S[9]) {
  if (!valid_dims(n1, n2, n3) || !phase || !mats || !director || !S) return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3, cnt = 0;
  double Q[9] = {0};
  for (size_t x = 0; x < V; ++x) {
    if (phase[x] >= n_mat) return OR_EINVAL;
    if (mats[phase[x]].model != OR_LCE) continue;
    double n[3] = {director[x], director[V + x], director[2 * V + x]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q[3 * i + j] += n[i] * n[j];
    cnt += 1;
  }
  for (int k = 0; k < 9; ++k)
    S[k] = cnt ? 1.5 * (Q[k] / (double)cnt - ((k % 4 == 0) ? 1.0 / 3.0 : 0.0)) : 0.0;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Bloch-wave stability modulus (Sec. 2.5)                                  */
/* ------------------------------------------------------------------------ */

/* (D_w p)(x) for the complex field p (re, im: 3V each): 9 complex values */
static void bloch_grad(int n1, int n2, int n3, const double *pr, const double *pi,
                       const double w[3], size_t x, double gr[9], double gi[9]) {
  size_t V = (size_t)n1 * n2 * n3;
  int nn[3] = {n1, n2, n3};
  int k[3] = {(int)(x % (size_t)n1), (int)((x / (size_t)n1) % (size_t)n2),
              (int)(x / ((size_t)n1 * n2))};
  for (int j = 0; j < 3; ++j) {
    int kp[3] = {k[0], k[1], k[2]}, km[3] = {k[0], k[1], k[2]};
    kp[j] = (k[j] + 1) % nn[j];
    km[j] = (k[j] - 1 + nn[j]) % nn[j];
    size_t xp = ((size_t)kp[2] * n2 + kp[1]) * n1 + kp[0];
    size_t xm = ((size_t)km[2] * n2 + km[1]) * n1 + km[0];
    double c = cos(w[j]), s = sin(w[j]);
    for (int i = 0; i < 3; ++i) {
      /* (p(x+e) e^{iw} - p(x-e) e^{-iw}) / 2 */
      double ar = pr[i * V + xp], ai = pi[i * V + xp];
      double br = pr[i * V + xm], bi = pi[i * V + xm];
      gr[3 * i + j] = 0.5 * ((ar * c - ai * s) - (br * c + bi * s));
      gi[3 * i + j] = 0.5 * ((ar * s + ai * c) - (bi * c - br * s));
    }
  }
}

/* tangent L + rho I at voxel x, Cholesky factorised; 0 when not positive definite */
static int bloch_factor(const or_material *m, const double *F, const double *director, size_t V,
                        size_t x, double rho, double K[81]) {
  double Fx[9], n[3] = {0.0, 0.0, 1.0}, nn[3];
  for (int c = 0; c < 9; ++c) Fx[c] = F[c * V + x];
  if (director)
    for (int c = 0; c < 3; ++c) n[c] = director[c * V + x];
  if (m->model == OR_LCE) {
    double P[9];
    if (or_relaxed(m, Fx, NULL, n, nn, P, K) != OR_OK) return 0;
  } else if (or_tangent(m, Fx, n, NULL, K) != OR_OK) {
    return 0;
  }
  for (int k = 0; k < 9; ++k) K[10 * k] += rho;
  return chol9(K);
}

int or_bloch(int n1, int n2, int n3, const unsigned char *phase, const or_material *mats,
             int n_mat, const double *F, const double *director, const double omega[3],
             double rho, double tol, int max_iter, double *p_re, double *p_im, double *beta,
             double *sigma_rho, int *iters) {
  if (!valid_dims(n1, n2, n3) || !phase || !mats || n_mat < 1 || !F || !omega || !(rho > 0.0) ||
      !(tol >= 0.0) || max_iter < 1 || !p_re || !p_im || !beta)
    return OR_EINVAL;
  size_t V = (size_t)n1 * n2 * n3;
  for (size_t x = 0; x < V; ++x)
    if (phase[x] >= n_mat || (mats[phase[x]].model == OR_LCE && !director)) return OR_EINVAL;
  double *Lf = (double *)malloc(81 * V * sizeof(double));      /* factors */
  double *Gr = (double *)calloc(9 * V, sizeof(double)), *Gi = (double *)calloc(9 * V, sizeof(double));
  double *gr = (double *)calloc(9 * V, sizeof(double)), *gi = (double *)calloc(9 * V, sizeof(double));
  double *Hr = (double *)malloc(9 * V * sizeof(double)), *Hi = (double *)malloc(9 * V * sizeof(double));
  double *br = (double *)malloc(3 * V * sizeof(double)), *bi = (double *)malloc(3 * V * sizeof(double));
  double *sr = (double *)malloc(3 * V * sizeof(double)), *si = (double *)malloc(3 * V * sizeof(double));
  double *K2 = (double *)malloc(V * sizeof(double)), *B2 = (double *)malloc(V * sizeof(double));
  double *Dor = (double *)malloc(9 * V * sizeof(double)), *Doi = (double *)malloc(9 * V * sizeof(double));
  int rc = OR_EINVAL;
  if (!Lf || !Gr || !Gi || !gr || !gi || !Hr || !Hi || !br || !bi || !sr || !si || !K2 || !B2 ||
      !Dor || !Doi)
    goto done;
  rc = OR_OK;
  for (size_t x = 0; x < V && rc == OR_OK; ++x)
    if (!bloch_factor(&mats[phase[x]], F, director, V, x, rho, Lf + 81 * x)) rc = OR_EDOMAIN;
  if (rc != OR_OK) goto done;
  {
    /* start: p normalised, G = g = 0 */
    double s2 = 0.0;
    for (size_t k = 0; k < 3 * V; ++k) s2 += p_re[k] * p_re[k] + p_im[k] * p_im[k];
    if (!(s2 > 0.0)) {
      rc = OR_EINVAL;
      goto done;
    }
    double sc = sqrt((double)V / s2);
    for (size_t k = 0; k < 3 * V; ++k) {
      p_re[k] *= sc;
      p_im[k] *= sc;
    }
    /* |K(xi + w)|^2 with xi_j = 2 pi m_j / n_j */
    int nn[3] = {n1, n2, n3};
    double K2min = INFINITY;
    for (size_t x = 0; x < V; ++x) {
      int m[3] = {(int)(x % (size_t)n1), (int)((x / (size_t)n1) % (size_t)n2),
                  (int)(x / ((size_t)n1 * n2))};
      double k2 = 0.0;
      for (int j = 0; j < 3; ++j) {
        double sj = sin(TWO_PI * m[j] / nn[j] + omega[j]);
        k2 += sj * sj;
      }
      K2[x] = k2;
      if (k2 < K2min) K2min = k2;
    }
    rc = OR_NOT_CONVERGED;
    int done_it = 0;
    double sig = 0.0;
    for (int it = 0; it < max_iter; ++it) {
      /* Step 1': G = (L + rho I)^{-1} (g + rho D_w p); keep D_w p for r_d */
      for (size_t x = 0; x < V; ++x) {
        double dr[9], di[9], rr[9], ri[9], xr[9], xi[9];
        bloch_grad(n1, n2, n3, p_re, p_im, omega, x, dr, di);
        for (int c = 0; c < 9; ++c) {
          Dor[c * V + x] = dr[c];
          Doi[c * V + x] = di[c];
          rr[c] = gr[c * V + x] + rho * dr[c];
          ri[c] = gi[c * V + x] + rho * di[c];
        }
        chol9_solve(Lf + 81 * x, rr, xr);
        chol9_solve(Lf + 81 * x, ri, xi);
        for (int c = 0; c < 9; ++c) {
          Gr[c * V + x] = xr[c];
          Gi[c * V + x] = xi[c];
          Hr[c * V + x] = xr[c] - gr[c * V + x] / rho;
          Hi[c * V + x] = xi[c] - gi[c * V + x] / rho;
        }
      }
      /* Step 2': b = D_w^H H, (D_w^H H)_i(x) = sum_j (e^{-iw_j} H_ij(x-e_j) - e^{iw_j} H_ij(x+e_j))/2 */
      for (size_t x = 0; x < V; ++x) {
        int k[3] = {(int)(x % (size_t)n1), (int)((x / (size_t)n1) % (size_t)n2),
                    (int)(x / ((size_t)n1 * n2))};
        for (int i = 0; i < 3; ++i) {
          double ar = 0.0, ai = 0.0;
          for (int j = 0; j < 3; ++j) {
            int kp[3] = {k[0], k[1], k[2]}, km[3] = {k[0], k[1], k[2]};
            kp[j] = (k[j] + 1) % nn[j];
            km[j] = (k[j] - 1 + nn[j]) % nn[j];
            size_t xp = ((size_t)kp[2] * n2 + kp[1]) * n1 + kp[0];
            size_t xm = ((size_t)km[2] * n2 + km[1]) * n1 + km[0];
            double c = cos(omega[j]), s = sin(omega[j]);
            double hmr = Hr[(3 * i + j) * V + xm], hmi = Hi[(3 * i + j) * V + xm];
            double hpr = Hr[(3 * i + j) * V + xp], hpi = Hi[(3 * i + j) * V + xp];
            /* e^{-iw} hm - e^{iw} hp */
            ar += 0.5 * ((hmr * c + hmi * s) - (hpr * c - hpi * s));
            ai += 0.5 * ((hmi * c - hmr * s) - (hpi * c + hpr * s));
          }
          br[i * V + x] = ar;
          bi[i * V + x] = ai;
        }
      }
      for (int i = 0; i < 3; ++i)
        or_dft3(n1, n2, n3, br + i * V, bi + i * V, sr + i * V, si + i * V, 0);
      double bb = 0.0;
      for (size_t x = 0; x < V; ++x) {
        double v = 0.0;
        for (int i = 0; i < 3; ++i)
          v += sr[i * V + x] * sr[i * V + x] + si[i * V + x] * si[i * V + x];
        B2[x] = v;
        bb += v;
      }
      if (!(bb > 0.0)) {
        rc = OR_EINVAL;
        break;
      }
      /* sum B2/(K2 - sigma)^2 = V^2 on (K2min - sqrt(bb)/V, K2min) by bisection */
      double lo = K2min - sqrt(bb) / (double)V, hi = K2min;
      for (int b = 0; b < 200; ++b) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double f = 0.0;
        for (size_t x = 0; x < V; ++x) {
          double d = K2[x] - mid;
          f += B2[x] / (d * d);
        }
        if (f > (double)V * (double)V)
          hi = mid;
        else
          lo = mid;
      }
      sig = lo;
      for (size_t x = 0; x < V; ++x) {
        double d = 1.0 / (K2[x] - sig);
        for (int i = 0; i < 3; ++i) {
          sr[i * V + x] *= d;
          si[i * V + x] *= d;
        }
      }
      for (int i = 0; i < 3; ++i)
        or_dft3(n1, n2, n3, sr + i * V, si + i * V, p_re + i * V, p_im + i * V, 1);
      /* Step 3' and 4' */
      double sp = 0.0, sd = 0.0;
      for (size_t x = 0; x < V; ++x) {
        double dr[9], di[9];
        bloch_grad(n1, n2, n3, p_re, p_im, omega, x, dr, di);
        for (int c = 0; c < 9; ++c) {
          double er = dr[c] - Gr[c * V + x], ei = di[c] - Gi[c * V + x];
          gr[c * V + x] += rho * er;
          gi[c * V + x] += rho * ei;
          sp += er * er + ei * ei;
          double fr = dr[c] - Dor[c * V + x], fi = di[c] - Doi[c * V + x];
          sd += fr * fr + fi * fi;
        }
      }
      double rp = sqrt(sp / (double)V), rd = rho * sqrt(sd / (double)V);
      done_it = it + 1;
      if (rp <= tol && rd <= tol) {
        rc = OR_OK;
        break;
      }
    }
    /* Rayleigh quotient of the last p: <D_w p, L D_w p> with L = (L + rho I) - rho I */
    double q = 0.0;
    for (size_t x = 0; x < V; ++x) {
      double dr[9], di[9];
      bloch_grad(n1, n2, n3, p_re, p_im, omega, x, dr, di);
      const double *L = Lf + 81 * x;
      /* |L^T d|^2 - rho |d|^2 for real and imaginary parts */
      for (int part = 0; part < 2; ++part) {
        const double *d = part ? di : dr;
        for (int j = 0; j < 9; ++j) {
          double t = 0.0;
          for (int i = j; i < 9; ++i) t += L[9 * i + j] * d[i];
          q += t * t;
        }
        for (int j = 0; j < 9; ++j) q -= rho * d[j] * d[j];
      }
    }
    *beta = q / (double)V;
    if (sigma_rho) *sigma_rho = rho * sig;
    if (iters) *iters = done_it;
  }
done:
  free(Lf); free(Gr); free(Gi); free(gr); free(gi); free(Hr); free(Hi); free(br); free(bi);
  free(sr); free(si); free(K2); free(B2); free(Dor); free(Doi);
  return rc;
}
