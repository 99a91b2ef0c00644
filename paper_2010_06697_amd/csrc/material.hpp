// material.hpp -- per-voxel local problem (Step 1 of Sec. 2.1): minimise
//     phi(F) = W(F) + rho/2 |F - A|^2,   A = grad u + Lambda/rho,
// for two stored energies, written in the displacement gradient E = F - I so
// that nothing cancels at small strain:
//   neo-Hookean      W = mu/2 (|F|^2 - 3) - mu ln J + lambda/2 (ln J)^2
//   neo-classical    W = mu/2 [a^(1/3) (|F|^2 + (1/a - 1) |F^T n|^2) - 3]
//   (LCE, Sec. 5.1)      + kappa/2 (J - 1)^2,  at a fixed unit director n
// with
//     J - 1 = tr E + s2(E) + det E          (s2: sum of principal 2x2 minors)
//     cof F = J F^-T = (1 + tr E) I - E^T + cof E
//     J (F - F^-T) = (s2 + det E) I + J E + E^T - cof E.
// Newton's method on the 9-vector E with the analytic tangent plus rho I:
//     neo-Hookean   mu d_ik d_JL + (mu - lambda ln J) Fi_Jk Fi_Li
//                   + lambda Fi_Ji Fi_Lk
//     LCE           mu a^(1/3) (d_ik + (1/a - 1) n_i n_k) d_JL
//                   - kappa (J - 1) J Fi_Jk Fi_Li + kappa (2J - 1) J Fi_Ji Fi_Lk
// (Fi = F^-1), a Cholesky factorisation (steepest descent when it is not
// positive definite) and backtracking (Armijo on phi, or on |grad phi| once
// the predicted decrease is below phi's rounding floor), rejecting det F <= 0.
// The float form's exact step solves the neo-Hookean problem in closed form
// up to one scalar instead (neo_closed), the LCE's ideal model in A's
// singular basis (lce_spectral).
//
// Precision: J - 1, ln J and phi are double in both modes. The iterate, the
// stress and the gradient are TG, the tangent, its factorisation and the
// solve TH: double/double in the FP64 mode, float/float in the reduced mode.
#pragma once

#include "common.hpp"

namespace admm {

// ln(1 + x) by the series ln((1+s)/(1-s)) = 2 (s + s^3/3 + s^5/5 + ...),
// s = x / (2 + x): for J = 1 + x in [0.8, 1.25], |s| <= 1/9 and ten terms
// leave a truncation below 1e-18 relative. The library log1p elsewhere.
__device__ __forceinline__ double log1p_near1(double x) {
  if (x > -0.2 && x < 0.25) {
    const double s = x / (2.0 + x);
    const double z = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    return 2.0 * s * p;
  }
  return log1p(x);
}

// state of the local problem at one iterate
template <typename TG> struct Point {
  double jm1;   // J - 1
  double lnJ;   // ln J (neo-Hookean only)
  TG gn2;       // |grad phi|^2
  TG G[9];      // F^-T
  TG g[9];      // grad phi = P + rho (E - A)
};

// J - 1 in double from the (exactly converted) components of E, and the
// cofactor of E in TG. False when det F <= 0.
template <typename TG>
__device__ __forceinline__ bool kinematics(const TG *E, TG *cE, double &jm1, double &tr,
                                           double &q) {
  double e[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) e[k] = (double)E[k];
  const double c0 = e[4] * e[8] - e[5] * e[7];
  const double c1 = e[5] * e[6] - e[3] * e[8];
  const double c2 = e[3] * e[7] - e[4] * e[6];
  const double c4 = e[0] * e[8] - e[2] * e[6];
  const double c8 = e[0] * e[4] - e[1] * e[3];
  tr = e[0] + e[4] + e[8];
  const double s2 = c0 + c4 + c8;
  const double dE = e[0] * c0 + e[1] * c1 + e[2] * c2;
  q = s2 + dE;
  jm1 = tr + q;
  cE[0] = (TG)c0;
  cE[1] = (TG)c1;
  cE[2] = (TG)c2;
  cE[3] = E[2] * E[7] - E[1] * E[8];
  cE[4] = (TG)c4;
  cE[5] = E[1] * E[6] - E[0] * E[7];
  cE[6] = E[1] * E[5] - E[2] * E[4];
  cE[7] = E[2] * E[3] - E[0] * E[5];
  cE[8] = (TG)c8;
  return 1.0 + jm1 > 0.0;
}

template <typename TG> struct NeoHooke {
  TG mu, lam;

  __device__ double smod() const { return (double)mu + (double)lam; }

  __device__ __forceinline__ bool point(const TG *E, const TG *A, TG rho, Point<TG> &s) const {
    TG cE[9];
    double tr, q;
    if (!kinematics(E, cE, s.jm1, tr, q)) return false;
    s.lnJ = log1p_near1(s.jm1);
    const TG Jt = (TG)(1.0 + s.jm1), iJ = (TG)1 / Jt, qt = (TG)q, trt = (TG)tr;
    const TG lnJt = (TG)s.lnJ;
    TG gn2 = (TG)0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int a = 3 * i + j;
        const TG Et = E[3 * j + i];
        const TG dia = (i == j) ? (TG)1 : (TG)0;
        const TG G = (cE[a] - Et + dia * ((TG)1 + trt)) * iJ;
        const TG P = mu * iJ * (dia * qt + Jt * E[a] + Et - cE[a]) + lam * lnJt * G;
        const TG g = P + rho * (E[a] - A[a]);
        s.G[a] = G;
        s.g[a] = g;
        gn2 += g * g;
      }
    s.gn2 = gn2;
    return true;
  }

  __device__ __forceinline__ double phi(const TG *E, const TG *A, double rho,
                                        const Point<TG> &s) const {
    double tr = (double)E[0] + (double)E[4] + (double)E[8], e2 = 0.0, d2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double ek = (double)E[k], dk = ek - (double)A[k];
      e2 += ek * ek;
      d2 += dk * dk;
    }
    const double m = (double)mu, l = (double)lam;
    return 0.5 * m * (2.0 * tr + e2) - m * s.lnJ + 0.5 * l * s.lnJ * s.lnJ + 0.5 * rho * d2;
  }

  // coefficients of the tangent: dia d_ik d_JL + c1 Fi_Jk Fi_Li + c2 Fi_Ji Fi_Lk
  template <typename TH>
  __device__ __forceinline__ void coeffs(const Point<TG> &s, TG rho, TH &dia, TH &c1,
                                         TH &c2) const {
    dia = (TH)(mu + rho);
    c1 = (TH)((double)mu - (double)lam * s.lnJ);
    c2 = (TH)lam;
  }
  template <typename TH> __device__ __forceinline__ TH director_term(int, int) const {
    return (TH)0;
  }
};

// What the full LCE model (Sec. 5.1) adds at one voxel. The director terms
// of the energy are n . M n with M = -c F F^T + (mu alpha/2) F P0 F^T + Sc,
// c = mu a^(1/3)(1 - 1/a)/2, P0 = I - n0 n0 (non-ideality, cross-link
// director n0) and Sc constant (the Frank term with the neighbours'
// directors lagged, the director's dissipation). The minimising director
// is the top eigenvector of S = -M/c = F F^T - gamma (F F^T - (F n0)(F n0)^T)
// - inv_c Sc, gamma = alpha / (a^(1/3)(1 - 1/a)), inv_c = 1/c.
struct DirForm {
  double n0[3];
  double sc[6];  // Sc packed: xx, xy, xz, yy, yz, zz
  double gamma, inv_c;
};

__device__ __forceinline__ double sc_at(const double *sc, int i, int j) {
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  return sc[lo == 0 ? hi : (lo == 1 ? 2 + hi : 5)];
}

template <typename TG> struct Lce {
  TG mua;    // mu a^(1/3)
  TG beta;   // 1/a - 1
  TG kappa;
  TG mu;
  TG n[3];       // unit director, in the arithmetic of the iterate
  double nd[3];  // the same director in double: the objective phi uses it,
                 // since a float-rounded director is not unit to 1e-8 and
                 // W depends on |n| at that level
  TG mual = (TG)0;                 // mu alpha (non-ideality)
  const DirForm *form = nullptr;   // null: the ideal model

  __device__ double smod() const { return (double)mua + (double)kappa; }

  __device__ __forceinline__ bool point(const TG *E, const TG *A, TG rho, Point<TG> &s) const {
    TG cE[9];
    double tr, q;
    if (!kinematics(E, cE, s.jm1, tr, q)) return false;
    s.lnJ = 0.0;
    const TG Jt = (TG)(1.0 + s.jm1), iJ = (TG)1 / Jt, trt = (TG)tr;
    const TG kv = kappa * (TG)s.jm1;  // kappa (J - 1)
    // F^T n = n + E^T n
    TG ftn[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) ftn[l] = n[l] + E[l] * n[0] + E[3 + l] * n[1] + E[6 + l] * n[2];
    TG gn2 = (TG)0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int a = 3 * i + j;
        const TG dia = (i == j) ? (TG)1 : (TG)0;
        const TG cof = cE[a] - E[3 * j + i] + dia * ((TG)1 + trt);  // J F^-T
        TG P = mua * (dia + E[a] + beta * n[i] * ftn[j]) + kv * cof;
        if (form) {
          // non-ideality: mu alpha n (x) (F^T n - (n0 . F^T n) n0)
          const TG q = (TG)form->n0[0] * ftn[0] + (TG)form->n0[1] * ftn[1] + (TG)form->n0[2] * ftn[2];
          P += mual * n[i] * (ftn[j] - q * (TG)form->n0[j]);
        }
        const TG g = P + rho * (E[a] - A[a]);
        s.G[a] = cof * iJ;
        s.g[a] = g;
        gn2 += g * g;
      }
    s.gn2 = gn2;
    return true;
  }

  __device__ __forceinline__ double phi(const TG *E, const TG *A, double rho,
                                        const Point<TG> &s) const {
    double tr = (double)E[0] + (double)E[4] + (double)E[8], e2 = 0.0, d2 = 0.0, t2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double ek = (double)E[k], dk = ek - (double)A[k];
      e2 += ek * ek;
      d2 += dk * dk;
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double v = nd[l] + (double)E[l] * nd[0] + (double)E[3 + l] * nd[1] +
                       (double)E[6 + l] * nd[2];
      t2 += v * v;
    }
    const double f2 = 3.0 + 2.0 * tr + e2;
    double W = 0.5 * (double)mua * (f2 + (double)beta * t2) - 1.5 * (double)mu +
               0.5 * (double)kappa * s.jm1 * s.jm1 + 0.5 * rho * d2;
    if (form) {
      double ft[3], q = 0.0, sn = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        ft[l] = nd[l] + (double)E[l] * nd[0] + (double)E[3 + l] * nd[1] + (double)E[6 + l] * nd[2];
        q += form->n0[l] * ft[l];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) sn += nd[i] * sc_at(form->sc, i, j) * nd[j];
      W += 0.5 * (double)mual * (t2 - q * q) + sn;
    }
    return W;
  }

  template <typename TH>
  __device__ __forceinline__ void coeffs(const Point<TG> &s, TG rho, TH &dia, TH &c1,
                                         TH &c2) const {
    const double J = 1.0 + s.jm1;
    dia = (TH)(mua + rho);
    c1 = (TH)(-(double)kappa * s.jm1 * J);
    c2 = (TH)((double)kappa * (2.0 * J - 1.0) * J);
  }
  // mu a^(1/3) (1/a - 1) n_i n_k d_JL for the entry ((iJ), (kL))
  template <typename TH> __device__ __forceinline__ TH director_term(int a, int b) const {
    const int i = a / 3, J = a % 3, k = b / 3, L = b % 3;
    TH v = J == L ? (TH)(mua * beta * n[i] * n[k]) : (TH)0;
    if (form)  // mu alpha n_i n_k (d_JL - n0_J n0_L)
      v += (TH)(mual * n[i] * n[k]) *
           ((TH)(J == L ? 1.0 : 0.0) - (TH)(form->n0[J] * form->n0[L]));
    return v;
  }
};

// |I + X|_F^2 from X
template <typename TG> __device__ __forceinline__ TG norm2_ipx(const TG *X) {
  TG tr = X[0] + X[4] + X[8], x2 = (TG)0;
#pragma unroll
  for (int k = 0; k < 9; ++k) x2 += X[k] * X[k];
  return fmax((TG)3 + (TG)2 * tr + x2, (TG)0);
}

__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }

constexpr __host__ __device__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// det(I + E) > 0, decided exactly as the point evaluations decide it
template <typename TG> __device__ __forceinline__ bool admissible(const TG *E) {
  TG cE[9];
  double jm1, tr, q;
  return kinematics(E, cE, jm1, tr, q);
}

// The iterations of newton() from the point s at E; on exit s is the point
// of the returned iterate when KEEP is set (otherwise it may be stale). ONE:
// a single full Newton step, no stopping test and no line search (returns 1,
// or -1 with E unchanged where the tangent is not positive definite).
template <typename TG, typename TH, bool KEEP, typename M, bool ONE = false>
__device__ int newton_loop(TG *E, const TG *A, const M &m, TG rho, int maxit, double gtol,
                           double step_tol, Point<TG> &s) {
  const double smod = m.smod() + (double)rho;
  const double nA = sqrt((double)norm2_ipx(A));
  const double tol_step2 = step_tol * step_tol;
  // phi at the current iterate when the line search evaluated it there (the
  // accepted trial point), so that the next iteration does not evaluate it again
  double phi_cur = 0.0;
  bool have_phi = false;
  for (int it = 0; it < maxit; ++it) {
    const double nF2 = (double)norm2_ipx(E);
    const double thr = gtol * smod * (1.0 + sqrt(nF2) + nA);
    if (!ONE && (double)s.gn2 <= thr * thr) return it;

    // prox tangent, lower triangle packed, assembled in TH
    TH L[45], Gh[9], id[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Gh[k] = (TH)s.G[k];
    TH dia, c1, c2;
    m.coeffs(s, rho, dia, c1, c2);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        const int i = a / 3, J = a % 3, k = b / 3, l = b % 3;
        TH v = c1 * Gh[3 * k + J] * Gh[3 * i + l] + c2 * Gh[a] * Gh[b] +
               m.template director_term<TH>(a, b);
        if (a == b) v += dia;
        L[tri(a, b)] = v;
      }
    bool pd = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      TH d = L[tri(j, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
      pd = pd && (d > (TH)0);
      id[j] = rsqrt_t(d);
#pragma unroll
      for (int i = j + 1; i < 9; ++i) {
        TH v = L[tri(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
        L[tri(i, j)] = v * id[j];
      }
    }
    TG d[9];
    if (pd) {
      TH y[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        TH v = (TH)(-s.g[i]);
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
        y[i] = v * id[i];
      }
#pragma unroll
      for (int i = 8; i >= 0; --i) {
        TH v = y[i];
#pragma unroll
        for (int k = i + 1; k < 9; ++k) v -= L[tri(k, i)] * y[k];
        y[i] = v * id[i];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = (TG)y[i];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = -s.g[i];
    }
    if (ONE) {
      if (!pd) return -1;
#pragma unroll
      for (int k = 0; k < 9; ++k) E[k] += d[k];
      return 1;
    }

    TG slope_t = (TG)0, nd2_t = (TG)0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      slope_t += s.g[k] * d[k];
      nd2_t += d[k] * d[k];
    }
    const double slope = (double)slope_t, nd2 = (double)nd2_t;
    const bool small = -slope <= 1e-12 * smod * (1.0 + nF2);
    // float iterate: a full Newton step already below the step tolerance is
    // taken as it is; the float gradient is at its rounding floor there and
    // no longer decides a line search
    const bool tiny = sizeof(TG) == 4 && pd && nd2 <= tol_step2 * fmax(1.0, nF2);
    if (!KEEP && tiny) {
      // the full step ends the solve when det F > 0 there and it is also
      // below the tolerance at the new iterate: the point evaluation at
      // E + d (stress and gradient) has no use then
      TG En[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) En[k] = E[k] + d[k];
      if (admissible(En) && nd2 <= tol_step2 * fmax(1.0, (double)norm2_ipx(En))) {
#pragma unroll
        for (int k = 0; k < 9; ++k) E[k] = En[k];
        return it + 1;
      }
    }
    const double phi0 = small ? 0.0 : (have_phi ? phi_cur : m.phi(E, A, rho, s));
    have_phi = false;
    double t = 1.0;
    bool acc = false;
    Point<TG> st;
    TG Et[9];
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Et[k] = E[k] + (TG)t * d[k];
      if (m.point(Et, A, rho, st)) {
        if (tiny) {
          acc = true;
          break;
        }
        if (!small) {
          const double ph = m.phi(Et, A, rho, st);
          if (ph <= phi0 + 1e-4 * t * slope) {
            acc = true;
            phi_cur = ph;
            have_phi = true;
            break;
          }
        } else {
          const double f = 1.0 - 1e-4 * t;
          if ((double)st.gn2 <= f * f * (double)s.gn2) {
            acc = true;
            break;
          }
        }
      }
      t *= 0.5;
    }
    if (!acc) return -1;
#pragma unroll
    for (int k = 0; k < 9; ++k) E[k] = Et[k];
    s = st;
    if (pd && t == 1.0 && nd2 <= tol_step2 * fmax(1.0, (double)norm2_ipx(E))) return it + 1;
  }
  return -1;
}

// Newton solve of the local problem at fixed material data M. E: warm start
// in, minimiser out. Stops when |grad phi| <= gtol (moduli + rho)(1 + |F| + |A|)
// before a step, or after a full positive-definite Newton step with
// |dE| <= step_tol max(1, |F|) (which leaves an error of order |dE|^2).
// Returns the iteration count (>= 0), -1 when the cap or the line search gave
// up (E keeps the last accepted iterate; a second call with the remaining
// budget continues the same iterates), -2 when det F <= 0 at the start.
// g2 (optional) receives |grad phi|^2 at the returned iterate.
// One full Newton step from E, for a point inside the region of quadratic
// convergence (the closed form's): no line search. False (E unchanged) when
// det F <= 0 at E or the tangent is not positive definite there.
template <typename TG, typename TH, typename M>
__device__ bool newton_polish(TG *E, const TG *A, const M &m, TG rho) {
  Point<TG> s;
  if (!m.point(E, A, rho, s)) return false;
  return newton_loop<TG, TH, false, M, true>(E, A, m, rho, 1, 0.0, 0.0, s) == 1;
}

template <typename TG, typename TH, typename M>
__device__ int newton(TG *E, const TG *A, const M &m, TG rho, int maxit, double gtol,
                      double step_tol, double *g2 = nullptr) {
  Point<TG> s;
  if (!m.point(E, A, rho, s)) return -2;
  if (!g2) return newton_loop<TG, TH, false>(E, A, m, rho, maxit, gtol, step_tol, s);
  int ret = newton_loop<TG, TH, true>(E, A, m, rho, maxit, gtol, step_tol, s);
  *g2 = (double)s.gn2;
  return ret;
}

// ---------------------------------------------------------------------------
// neo-Hookean local problem up to one scalar (exact mode). phi is isotropic,
// so its minimiser is coaxial with A: with A = U diag(a) V^T (U, V rotations,
// det A > 0), F = U diag(f) V^T, and the stationarity
//     m F + c F^-T = rho A,   m = mu + rho,  c = lambda ln J - mu,
// splits into m f_i^2 - rho a_i f_i + c = 0 with the root
//     f_i = a_i h(x_i),  h(x) = (rho + S(x)) / (2m),  S(x) = sqrt(rho^2 - 4 m c / x),
// at the eigenvalues x_i = a_i^2 of B = A A^T (the other root sends ln J to
// -infinity as c -> 0). gamma = c + mu = lambda ln J then solves
//     g(gamma) = gamma - lambda (ln det A + sum_i ln h(x_i)) = 0,
// g' = 1 + lambda sum_i 1 / (x_i S_i h_i) > 0, by Newton's method kept inside
// a bracket (the upper end where S(x_min) stays real). F = P A with P = h(B),
// evaluated as the quadratic that interpolates h at x_1 >= x_2 >= x_3
// (Newton's divided differences, written in forms free of cancellation), so
// only B's eigenvalues are needed (closed form for a symmetric 3x3 matrix).
// Everything in double, in the displacement-gradient form: B - I, h - 1 and
// P - I are formed without subtracting numbers near one. Returns the Newton
// count; -2 when the warm start has det F <= 0 (as newton()); -3 where the
// form does not apply (det A <= 0, no root below the bracket's upper end, no
// convergence), for the caller to run the nine-component Newton instead.
// ---------------------------------------------------------------------------
// reciprocal and square root in double from the hardware approximations
// (v_rcp_f64, v_rsq_f64), each refined by Newton's method: two steps for
// the reciprocal (the relative error e becomes e^2 each), one for 1/sqrt and
// one for sqrt itself. For x > 0, finite.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double sqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  const double q = x * r;
  return fma(0.5 * r, fma(-q, q, x), q);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r * fma(-0.5 * x * r, r, 1.5);
}

// log1p_near1 with the division on the refined reciprocal
__device__ __forceinline__ double log1p_near1_nr(double x) {
  if (x > -0.2 && x < 0.25) {
    const double s = x * rcp_nr(2.0 + x);
    const double z = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    return 2.0 * s * p;
  }
  return log1p(x);
}

// det(I + E) - 1 of the warm start F = I + E, by kinematics()'s formulas
// (admissibility decided as the point evaluations decide it), without the
// cofactor
template <typename TG>
__device__ __forceinline__ double warm_jm1(const TG *E) {
  double e[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) e[k] = (double)E[k];
  const double c0 = e[4] * e[8] - e[5] * e[7];
  const double c1 = e[5] * e[6] - e[3] * e[8];
  const double c2 = e[3] * e[7] - e[4] * e[6];
  const double c4 = e[0] * e[8] - e[2] * e[6];
  const double c8 = e[0] * e[4] - e[1] * e[3];
  const double tr = e[0] + e[4] + e[8];
  return tr + ((c0 + c4 + c8) + (e[0] * c0 + e[1] * c1 + e[2] * c2));
}

// warm_jm1 as one float that keeps both of its uses: NaN where the warm
// start is inadmissible, else the nearest float above -1 (the closed form
// tests 1 + j > 0 and starts its scalar iteration from the float value)
__device__ __forceinline__ float warm_code(double jm1) {
  if (!(1.0 + jm1 > 0.0)) return __builtin_nanf("");
  const float f = (float)jm1;
  return f > -1.0f ? f : -0x1.fffffep-1f;
}

// E: out (written only when the return value is >= 0); jw: warm_code of
// det(I + E) - 1 of the warm start
template <typename TG>
__device__ int neo_closed(TG *E, const TG *At, float jw, double mu, double lam, double rho,
                          int maxit, double tol) {
  if (!(1.0 + (double)jw > 0.0)) return -2;
  double a[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) a[k] = (double)At[k];
  // det A - 1 = tr a + s2(a) + det a
  const double m0 = a[4] * a[8] - a[5] * a[7];
  const double m1 = a[5] * a[6] - a[3] * a[8];
  const double m2 = a[3] * a[7] - a[4] * a[6];
  const double jA = (a[0] + a[4] + a[8]) + (m0 + (a[0] * a[8] - a[2] * a[6]) +
                                            (a[0] * a[4] - a[1] * a[3])) +
                    (a[0] * m0 + a[1] * m1 + a[2] * m2);
  if (!(jA > -1.0)) return -3;
  const double lnA = log1p_near1_nr(jA);
  // B - I = a + a^T + a a^T
  double b[6];  // 00 11 22 01 02 12
  {
    const int I[6] = {0, 1, 2, 0, 0, 1}, J[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int i = I[k], j = J[k];
      b[k] = a[3 * i + j] + a[3 * j + i] + a[3 * i] * a[3 * j] + a[3 * i + 1] * a[3 * j + 1] +
             a[3 * i + 2] * a[3 * j + 2];
    }
  }
  // eigenvalues e_1 >= e_2 >= e_3 of B - I: the roots t = 2 p cos(angle) of
  // the deviator's characteristic cubic t^3 - 3 p2 t - det = 0 from the
  // angle in float, then one Newton step each in double (the error goes
  // from float's to double's; at a double root the step is skipped, and
  // there an error in the nodes moves g and P only at second order); their
  // sum is exact by construction
  const double qm = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
  const double c00 = b[0] - qm, c11 = b[1] - qm, c22 = b[2] - qm;
  const double p2 = (c00 * c00 + c11 * c11 + c22 * c22 +
                     2.0 * (b[3] * b[3] + b[4] * b[4] + b[5] * b[5])) * (1.0 / 6.0);
  double e1 = qm, e2 = qm, e3 = qm;
  if (p2 > 1e-60) {
    const double dC = c00 * (c11 * c22 - b[5] * b[5]) - b[3] * (b[3] * c22 - b[5] * b[4]) +
                      b[4] * (b[3] * b[5] - c11 * b[4]);
    const float p2f = (float)p2, pf = __builtin_amdgcn_sqrtf(p2f);
    const float r = fminf(1.0f, fmaxf(-1.0f, (float)dC * __builtin_amdgcn_rcpf(2.0f * p2f * pf)));
    const float cpf = __cosf(acosf(r) * (1.0f / 3.0f));  // angle in [0, pi/3]
    const float spf = __builtin_amdgcn_sqrtf(fmaxf(0.0f, 1.0f - cpf * cpf));
    double t1 = (double)(2.0f * pf * cpf);
    double t3 = (double)(2.0f * pf * (-0.5f * cpf - 0.8660254f * spf));  // angle + 2 pi/3
    auto refine = [&](double &t) {
      const double dp = 3.0 * (t * t - p2);
      if (fabs(dp) > 1e-3 * p2) t -= (t * (t * t - 3.0 * p2) - dC) * rcp_nr(dp);
    };
    refine(t1);
    refine(t3);
    e1 = qm + t1;
    e3 = qm + t3;
    e2 = 3.0 * qm - e1 - e3;
  }
  const double x1 = 1.0 + e1, x2 = 1.0 + e2, x3 = 1.0 + e3;
  if (!(x3 > 0.0)) return -3;
  const double m = mu + rho, r2 = rho * rho;
  const double es[3] = {e1, e2, e3};
  const double ixd[3] = {rcp_nr(x1), rcp_nr(x2), rcp_nr(x3)};
  const double ghi = mu + r2 * x3 / (4.0 * m);  // S(x_3) real up to here
  // gamma to float accuracy by Newton's method in float (hardware
  // reciprocal, square root and logarithm: the step in double below removes
  // their error too), kept inside the bracket [lo, hi] of g's sign change
  const float lamf = (float)lam, muf = (float)mu;
  const float r2f = (float)r2, m4f = (float)(4.0 * m), lnAf = (float)lnA;
  const float c2f = (float)(rho + 2.0 * mu);
  float ix[3], ef[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ix[i] = (float)ixd[i];
    ef[i] = (float)es[i];
  }
  constexpr float kLn2 = 0.69314718f;
  float lo = -INFINITY, hi = (float)ghi;
  float gam = fminf(lamf * kLn2 * __builtin_amdgcn_logf(1.0f + jw), 0.5f * hi);
  int it = 0;
  bool done = false;
  for (; it < maxit; ++it) {
    float Sf[3], df[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Sf[i] = __builtin_amdgcn_sqrtf(fmaxf(0.0f, r2f - m4f * (gam - muf) * ix[i]));
      df[i] = -2.0f * (gam + muf * ef[i]) * ix[i] * __builtin_amdgcn_rcpf(Sf[i] + c2f);
    }
    const float dp = df[0] + df[1] + df[2] + (df[0] * df[1] + df[0] * df[2] + df[1] * df[2]) +
                     df[0] * df[1] * df[2];
    const float g = gam - lamf * (lnAf + kLn2 * __builtin_amdgcn_logf(1.0f + dp));
    if (g > 0.0f) hi = gam; else lo = gam;
    const float gp = 1.0f + lamf * (ix[0] * __builtin_amdgcn_rcpf(Sf[0] * (1.0f + df[0])) +
                                    ix[1] * __builtin_amdgcn_rcpf(Sf[1] * (1.0f + df[1])) +
                                    ix[2] * __builtin_amdgcn_rcpf(Sf[2] * (1.0f + df[2])));
    const float step = g * __builtin_amdgcn_rcpf(gp);
    if (fabsf(step) <= (float)tol * (1.0f + fabsf(gam))) {
      gam -= step;
      done = true;
      ++it;
      break;
    }
    float nx = gam - step;
    if (!(nx > lo && nx < hi)) nx = lo == -INFINITY ? gam - 2.0f * fabsf(step) - 1.0f : 0.5f * (lo + hi);
    gam = nx;
  }
  if (!done) return -3;
  // one Newton step in double from there (the error goes from float's to
  // its square), with S_i and h_i - 1 carried to the new gamma to first
  // order (dS/dgamma = -2m / (x S), dh/dgamma = -1 / (x S))
  double G = (double)gam;
  double S[3], d[3], w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    S[i] = sqrt_nr(r2 - 4.0 * m * (G - mu) * ixd[i]);
    d[i] = -2.0 * (G + mu * es[i]) * ixd[i] * rcp_nr(S[i] + rho + 2.0 * mu);
    w[i] = ixd[i] * rcp_nr(S[i]);  // -dh_i/dgamma
  }
  {
    const double dp = d[0] + d[1] + d[2] + (d[0] * d[1] + d[0] * d[2] + d[1] * d[2]) +
                      d[0] * d[1] * d[2];
    const double g = G - lam * (lnA + log1p_near1_nr(dp));
    const double sw = w[0] * rcp_nr(1.0 + d[0]) + w[1] * rcp_nr(1.0 + d[1]) +
                      w[2] * rcp_nr(1.0 + d[2]);
    const double delta = -g * rcp_nr(1.0 + lam * sw);
    G += delta;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      S[i] -= 2.0 * m * w[i] * delta;
      d[i] -= w[i] * delta;
    }
  }
  if (!(G < ghi)) return -3;
  // P - I = (h_1 - 1) I + h[x1,x2] (B - x1 I) + h[x1,x2,x3] (B - x1 I)(B - x2 I)
  const double km = 2.0 * (G - mu);  // 4 m c / (2 m)
  const double i12 = ixd[0] * ixd[1] * rcp_nr(S[0] + S[1]);
  const double h12 = km * i12;
  const double h123 = -km * i12 * ixd[2] * rcp_nr(S[1] + S[2]) *
                      (S[1] + (r2 * (x1 + x3) - 2.0 * m * km) * rcp_nr(x3 * S[2] + x1 * S[0]));
  // C1 = B - x1 I, C2 = B - x2 I (symmetric, in the order of b)
  const double C1[6] = {b[0] - e1, b[1] - e1, b[2] - e1, b[3], b[4], b[5]};
  const double C2[6] = {b[0] - e2, b[1] - e2, b[2] - e2, b[3], b[4], b[5]};
  auto sym = [](const double *M, int i, int j) {
    return i == j ? M[i] : M[i + j + 2];  // (0,1) -> 3, (0,2) -> 4, (1,2) -> 5
  };
  double Pm[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double q = sym(C1, i, 0) * sym(C2, 0, j) + sym(C1, i, 1) * sym(C2, 1, j) +
                       sym(C1, i, 2) * sym(C2, 2, j);
      Pm[3 * i + j] = (i == j ? d[0] : 0.0) + h12 * sym(C1, i, j) + h123 * q;
    }
  // E = F - I = (P - I) + (P - I) a + a
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      E[3 * i + j] = (TG)(Pm[3 * i + j] + a[3 * i + j] +
                          (Pm[3 * i] * a[j] + Pm[3 * i + 1] * a[3 + j] + Pm[3 * i + 2] * a[6 + j]));
  return it;
}

// ---------------------------------------------------------------------------
// director: the unit top eigenvector of F F^T (double), cyclic Jacobi on the
// symmetric 3x3 matrix; sign chosen so that n . n_prev >= 0; when the top
// eigenvalue is degenerate (relative gap <= 1e-12) every unit vector of the
// top eigenspace minimises the energy and the projection of n_prev onto it is
// kept.
// ---------------------------------------------------------------------------

// Vv holds the starting basis on entry (B already expressed in it) and the
// eigenvectors on exit
__device__ __forceinline__ void jacobi3(double *B, double *Vv) {
  for (int sweep = 0; sweep < 30; ++sweep) {
    const double off = B[1] * B[1] + B[2] * B[2] + B[5] * B[5];
    const double dia = B[0] * B[0] + B[4] * B[4] + B[8] * B[8];
    if (off <= 1e-34 * dia || off == 0.0) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2, r = 3 - p - q;
      const double bpq = B[3 * p + q];
      // (a rotation by an angle below 1e-30 changes nothing in double)
      if (!(fabs(bpq) > 1e-30 * (fabs(B[3 * p + p]) + fabs(B[3 * q + q])))) continue;
      // the rotation's tangent t = sign(theta) / (|theta| + sqrt(theta^2 + 1))
      // (1 / (2 theta) where theta^2 would overflow), cosine and sine, on the
      // refined hardware reciprocal and square roots; B stays symmetric and
      // is updated in the form with tau = s / (1 + c) (B_pq becomes zero)
      const double theta = (B[3 * q + q] - B[3 * p + p]) * rcp_nr(2.0 * bpq);
      const double at = fabs(theta);
      const double t = at > 1e100 ? 0.5 * rcp_nr(theta)
                                  : (theta >= 0 ? 1.0 : -1.0) * rcp_nr(at + sqrt_nr(fma(theta, theta, 1.0)));
      const double c = rsqrt_nr(fma(t, t, 1.0)), sn = t * c;
      const double tau = sn * rcp_nr(1.0 + c);
      B[3 * p + p] -= t * bpq;
      B[3 * q + q] += t * bpq;
      B[3 * p + q] = B[3 * q + p] = 0.0;
      {
        const double g = B[3 * r + p], h = B[3 * r + q];
        B[3 * r + p] = B[3 * p + r] = g - sn * (h + g * tau);
        B[3 * r + q] = B[3 * q + r] = h + sn * (g - h * tau);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double g = Vv[3 * k + p], h = Vv[3 * k + q];
        Vv[3 * k + p] = g - sn * (h + g * tau);
        Vv[3 * k + q] = h + sn * (g - h * tau);
      }
    }
  }
}

// Eigen-decomposition of B = F F^T (double) sorted by decreasing eigenvalue,
// w[0] >= w[1] >= w[2] with the eigenvectors in the columns of V, and the
// minimising director n by the rules above. Returns the size of the top
// eigenvalue's cluster (1 when it is simple).
template <typename TG>
__device__ int director_eig(const TG *E, const double *np, double *n, double *w, double *V,
                            const double *V0 = nullptr, const DirForm *form = nullptr) {
  double F[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) F[k] = (double)E[k] + ((k % 4 == 0) ? 1.0 : 0.0);
  double B[9], Vv[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      B[3 * i + j] = F[3 * i] * F[3 * j] + F[3 * i + 1] * F[3 * j + 1] + F[3 * i + 2] * F[3 * j + 2];
  if (form) {
    // S = F F^T - gamma (F F^T - (F n0)(F n0)^T) - inv_c Sc
    double fn0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      fn0[i] = F[3 * i] * form->n0[0] + F[3 * i + 1] * form->n0[1] + F[3 * i + 2] * form->n0[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        B[3 * i + j] = B[3 * i + j] - form->gamma * (B[3 * i + j] - fn0[i] * fn0[j]) -
                       form->inv_c * sc_at(form->sc, i, j);
  }
  if (V0) {
    // start from a nearby eigenbasis (the current iterate's): B <- V0^T B V0
    // is then almost diagonal and the sweeps converge at once
    double T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        T[3 * i + j] = B[3 * i] * V0[j] + B[3 * i + 1] * V0[3 + j] + B[3 * i + 2] * V0[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        B[3 * i + j] = V0[i] * T[j] + V0[3 + i] * T[3 + j] + V0[6 + i] * T[6 + j];
#pragma unroll
    for (int k = 0; k < 9; ++k) Vv[k] = V0[k];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Vv[k] = (k % 4 == 0) ? 1.0 : 0.0;
  }
  jacobi3(B, Vv);
  const double wu[3] = {B[0], B[4], B[8]};
  int o0 = 0, o1 = 1, o2 = 2;  // descending order
  if (wu[o1] > wu[o0]) { int t = o0; o0 = o1; o1 = t; }
  if (wu[o2] > wu[o0]) { int t = o0; o0 = o2; o2 = t; }
  if (wu[o2] > wu[o1]) { int t = o1; o1 = o2; o2 = t; }
  const int ord[3] = {o0, o1, o2};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    w[e] = wu[ord[e]];
#pragma unroll
    for (int k = 0; k < 3; ++k) V[3 * k + e] = Vv[3 * k + ord[e]];
  }
  const double tie = 1e-12 * fmax(fabs(w[0]), fabs(w[2]));
  const int ncl = (w[0] - w[1] <= tie) ? ((w[0] - w[2] <= tie) ? 3 : 2) : 1;
  double out[3];
  if (ncl == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = V[3 * k];
  } else {
    out[0] = out[1] = out[2] = 0.0;
    for (int e = 0; e < ncl; ++e) {
      const double pr = V[e] * np[0] + V[3 + e] * np[1] + V[6 + e] * np[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) out[k] += pr * V[3 * k + e];
    }
    if (out[0] * out[0] + out[1] * out[1] + out[2] * out[2] < 1e-16)
#pragma unroll
      for (int k = 0; k < 3; ++k) out[k] = V[3 * k];
  }
  if (out[0] * np[0] + out[1] * np[1] + out[2] * np[2] < 0.0)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = -out[k];
  const double inv = 1.0 / sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = out[k] * inv;
  return ncl;
}

// Cholesky factorisation of a packed lower triangle in place, with the
// reciprocal square roots of the pivots in id. False when a pivot is not
// positive.
template <typename T> __device__ __forceinline__ bool chol_packed(T *L, T *id) {
  bool pd = true;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    T d = L[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
    pd = pd && (d > (T)0);
    id[j] = rsqrt_t(d);
#pragma unroll
    for (int i = j + 1; i < 9; ++i) {
      T v = L[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
      L[tri(i, j)] = v * id[j];
    }
  }
  return pd;
}

// Relaxed LCE tangent plus (rho - shift) I at E with director nc and the
// sorted eigen-decomposition (w, V, ncl) of F F^T, packed lower triangle.
template <typename T>
__device__ __forceinline__ void lce_relaxed_tangent(const T *E, const Lce<T> &M, const Point<T> &s,
                                                    T rho, double c2, const double *nc,
                                                    const double *w, const double *V, int ncl,
                                                    T shift, T *L) {
  T dia, k1, k2;
  M.coeffs(s, rho, dia, k1, k2);
  dia -= shift;
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int i = a / 3, J = a % 3, k = b / 3, l = b % 3;
      T v = k1 * s.G[3 * k + J] * s.G[3 * i + l] + k2 * s.G[a] * s.G[b] +
            M.template director_term<T>(a, b);
      if (a == b) v += dia;
      L[tri(a, b)] = v;
    }
  // eigenvector sensitivity of the top eigenvalue; with the non-ideality
  // w_e also carries -gamma (t (x) P0 F^T n + n (x) P0 F^T t)
  double F[9], ftn[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) F[k] = (double)E[k] + ((k % 4 == 0) ? 1.0 : 0.0);
#pragma unroll
  for (int J = 0; J < 3; ++J) ftn[J] = F[J] * nc[0] + F[3 + J] * nc[1] + F[6 + J] * nc[2];
  const DirForm *fm = M.form;
  double pftn[3] = {0.0, 0.0, 0.0};
  if (fm) {
    const double q = fm->n0[0] * ftn[0] + fm->n0[1] * ftn[1] + fm->n0[2] * ftn[2];
#pragma unroll
    for (int J = 0; J < 3; ++J) pftn[J] = ftn[J] - q * fm->n0[J];
  }
  for (int e = ncl; e < 3; ++e) {
    const double t0 = V[e], t1 = V[3 + e], t2 = V[6 + e];
    double wk[9], ftt[3];
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      ftt[J] = F[J] * t0 + F[3 + J] * t1 + F[6 + J] * t2;
      wk[J] = t0 * ftn[J] + nc[0] * ftt[J];
      wk[3 + J] = t1 * ftn[J] + nc[1] * ftt[J];
      wk[6 + J] = t2 * ftn[J] + nc[2] * ftt[J];
    }
    if (fm) {
      const double q = fm->n0[0] * ftt[0] + fm->n0[1] * ftt[1] + fm->n0[2] * ftt[2];
#pragma unroll
      for (int J = 0; J < 3; ++J) {
        const double pftt = ftt[J] - q * fm->n0[J];
        wk[J] -= fm->gamma * (t0 * pftn[J] + nc[0] * pftt);
        wk[3 + J] -= fm->gamma * (t1 * pftn[J] + nc[1] * pftt);
        wk[6 + J] -= fm->gamma * (t2 * pftn[J] + nc[2] * pftt);
      }
    }
    const double f = c2 / (w[0] - w[e]);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) L[tri(a, b)] += (T)(f * wk[a] * wk[b]);
  }
}

// ---------------------------------------------------------------------------
// LCE local problem jointly in F and the director. With a >= 1 the director
// part of the energy is smallest at the top eigenvector of B = F F^T, so the
// joint problem is Newton's method on the relaxed objective
//     phi_r(F) = W(F, n(F)) + rho/2 |F - A|^2,
// whose gradient is the fixed-director one at n(F) and whose Hessian adds to
// the fixed-director tangent the top eigenvector's sensitivity to F,
//     c2 / (w_0 - w_e) w_e w_e^T,  (w_e)_iJ = t_i (F^T n)_J + n_i (F^T t)_J,
// over the eigenvectors t = t_e outside the top cluster, c2 = mu a^(1/3)(1/a - 1)
// (negative semidefinite). phi_r need not be convex (near uniaxially
// symmetric states the curvature along the director-rotation mode goes like
// -1/(w_0 - w_1)); where the Newton matrix is not positive definite with a
// margin of rho/16 a multiple of the identity is added (above), and every
// trial point of the backtracking recomputes the director (continuity with
// the current one), so the iterates descend monotonically to a stationary
// point of phi_r, i.e. of the joint problem in (F, n).
// n: previous director in, minimising director out. Returns as newton().
// ---------------------------------------------------------------------------
template <typename T>
__device__ int lce_newton(T *E, const T *A, Lce<T> &M, double c2, T rho, double *n, int maxit,
                          double gtol, double step_tol) {
  double w[3], V[9], nc[3];
  int ncl = director_eig(E, n, nc, w, V, nullptr, M.form);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    M.n[k] = (T)nc[k];
    M.nd[k] = nc[k];
  }
  Point<T> s;
  if (!M.point(E, A, rho, s)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = nc[k];
    return -2;
  }
  const double smod = M.smod() + (double)rho;
  const double nA = sqrt((double)norm2_ipx(A));
  const double tol_step2 = step_tol * step_tol;
  double phi_cur = 0.0;  // phi at the accepted trial point (see newton_loop)
  bool have_phi = false;
  int ret = -1;
  for (int it = 0; it < maxit; ++it) {
    const double nF2 = (double)norm2_ipx(E);
    const double thr = gtol * smod * (1.0 + sqrt(nF2) + nA);
    if ((double)s.gn2 <= thr * thr) {
      ret = it;
      break;
    }
    // Newton matrix: the relaxed tangent plus (rho + tau) I, lower triangle
    // packed, with the smallest tau of 0, rho/16, rho/8, ... for which the
    // relaxed tangent plus (rho + tau - rho/16) I has a Cholesky
    // factorisation (Newton's method with a multiple of the identity added,
    // Nocedal & Wright, Sec. 3.4): a pure Newton step where phi_r is convex
    // with modulus rho/16, a descent direction of a positive-definite model
    // where it is not (near uniaxially symmetric states, or at A = I where
    // every director is a minimiser)
    T L[45], id[9];
    const T margin = (T)0.0625 * rho;
    T tau = (T)0;
    bool pd = false;
    for (int tries = 0; tries < 64 && !pd; ++tries) {
      lce_relaxed_tangent(E, M, s, rho, c2, nc, w, V, ncl, margin - tau, L);
      pd = chol_packed(L, id);
      if (!pd) tau = tau == (T)0 ? margin : (T)2 * tau;
    }
    if (pd) {
      lce_relaxed_tangent(E, M, s, rho, c2, nc, w, V, ncl, -tau, L);
      pd = chol_packed(L, id);
    }
    if (!pd) {
      ret = -1;
      break;
    }
    T d[9];
    {
      T y[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        T v = -s.g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
        y[i] = v * id[i];
      }
#pragma unroll
      for (int i = 8; i >= 0; --i) {
        T v = y[i];
#pragma unroll
        for (int k = i + 1; k < 9; ++k) v -= L[tri(k, i)] * y[k];
        y[i] = v * id[i];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = y[i];
    }
    T slope_t = (T)0, nd2_t = (T)0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      slope_t += s.g[k] * d[k];
      nd2_t += d[k] * d[k];
    }
    const double slope = (double)slope_t, nd2 = (double)nd2_t;
    const bool small = -slope <= 1e-12 * smod * (1.0 + nF2);
    const bool tiny = sizeof(T) == 4 && nd2 <= tol_step2 * fmax(1.0, nF2);
    const double phi0 = small ? 0.0 : (have_phi ? phi_cur : M.phi(E, A, rho, s));
    have_phi = false;
    double t = 1.0;
    bool acc = false;
    Point<T> st;
    T Et[9];
    double nt[3], wt[3], Vt[9];
    int nclt = 1;
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Et[k] = E[k] + (T)t * d[k];
      nclt = director_eig(Et, nc, nt, wt, Vt, V, M.form);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        M.n[k] = (T)nt[k];
        M.nd[k] = nt[k];
      }
      if (M.point(Et, A, rho, st)) {
        if (tiny) {
          acc = true;
          break;
        }
        if (!small) {
          const double ph = M.phi(Et, A, rho, st);
          if (ph <= phi0 + 1e-4 * t * slope) {
            acc = true;
            phi_cur = ph;
            have_phi = true;
            break;
          }
        } else {
          const double f = 1.0 - 1e-4 * t;
          if ((double)st.gn2 <= f * f * (double)s.gn2) {
            acc = true;
            break;
          }
        }
      }
      t *= 0.5;
    }
    if (!acc) {
      ret = -1;
      break;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) E[k] = Et[k];
    s = st;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      nc[k] = nt[k];
      w[k] = wt[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) V[k] = Vt[k];
    ncl = nclt;
    if (t == 1.0 && nd2 <= tol_step2 * fmax(1.0, (double)norm2_ipx(E))) {
      ret = it + 1;
      break;
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = nc[k];
  return ret;
}

// ---------------------------------------------------------------------------
// Ideal LCE (no non-ideality, Frank or director-dissipation term): with the
// director eliminated the energy is a function of the singular values
// f1 >= f2 >= f3 > 0 of F alone (the director is the top left singular
// vector), W_r = mua/2 (|f|^2 + beta f1^2) - 3 mu/2 + kappa/2 (f1 f2 f3 - 1)^2,
// mua = mu a^(1/3), beta = 1/a - 1. The minimiser of W_r(F) + rho/2 |F - A|^2
// then has A's singular vectors (von Neumann's trace inequality over proper
// rotations: tr(F^T A) <= sum f_i a_i when det F > 0, a3 carrying the sign of
// det A), and Step 1 reduces to the three unknowns f:
//     h(f) = W_r(f) + rho/2 |f - a|^2,
// minimised by Newton's method (Hessian shifted by the smallest of 0, rho/16,
// rho/8, ... that makes it positive definite; Armijo backtracking on h, or on
// |grad h| once the predicted decrease is below rounding). At
// F = sum f_i u_i v_i^T the 9-component gradient is sum_i (dh/df_i) u_i v_i^T,
// so the stopping test on |grad h| is the nine-component one. Everything in
// double, whatever T. The basis: eigenvectors of A A^T (director_eig, which
// resolves a tied top singular value towards the previous director), u2 the
// one of the top two eigenvectors least aligned with u1, made orthogonal to
// it, u3 = u1 x u2; v_i = A^T u_i / a_i (i = 1, 2), v3 = v1 x v2,
// a3 = u3 . A v3. The start is the current F's diagonal in that basis, or a
// with entries below a1/16 raised to it, whichever has the lower h.
// E: F - I in/out; Am: A - I; n: previous director in, new one out.
// Returns the Newton iterations, -1 when not converged, -2 for rank(A) < 2.
// ---------------------------------------------------------------------------
struct SpecH {
  double mua, beta, kap, rho, c0;  // c0 = -3 mu / 2
  double a[3];
  __device__ __forceinline__ double h(const double *f) const {
    const double J = f[0] * f[1] * f[2];
    if (!(J > 0.0)) return __builtin_huge_val();
    double s = 0.0, d = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      s += f[i] * f[i];
      d += (f[i] - a[i]) * (f[i] - a[i]);
    }
    return 0.5 * mua * (s + beta * f[0] * f[0]) + c0 + 0.5 * kap * (J - 1.0) * (J - 1.0) +
           0.5 * rho * d;
  }
  __device__ __forceinline__ void grad(const double *f, double *g) const {
    const double Jm1 = f[0] * f[1] * f[2] - 1.0;
    g[0] = mua * (1.0 + beta) * f[0] + rho * (f[0] - a[0]) + kap * Jm1 * (f[1] * f[2]);
    g[1] = mua * f[1] + rho * (f[1] - a[1]) + kap * Jm1 * (f[0] * f[2]);
    g[2] = mua * f[2] + rho * (f[2] - a[2]) + kap * Jm1 * (f[0] * f[1]);
  }
};

template <typename T>
__device__ int lce_spectral(T *E, const T *Am, double mua, double beta, double kap, double mu,
                            double rho, double *n, int maxit, double gtol, double step_tol) {
  double w[3], Ve[9], u[9], v[9];  // u, v: singular vectors in rows (u[3i + k])
  director_eig(Am, n, u, w, Ve);
  double Ad[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ad[k] = (double)Am[k] + ((k % 4 == 0) ? 1.0 : 0.0);
  {
    double r0[3], r1[3];
    const double c0 = Ve[0] * u[0] + Ve[3] * u[1] + Ve[6] * u[2];
    const double c1 = Ve[1] * u[0] + Ve[4] * u[1] + Ve[7] * u[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r0[k] = Ve[3 * k] - c0 * u[k];
      r1[k] = Ve[3 * k + 1] - c1 * u[k];
    }
    const double q0 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    const double q1 = r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2];
    const bool use0 = q0 > q1;
    const double inv = rsqrt_nr(use0 ? q0 : q1);
#pragma unroll
    for (int k = 0; k < 3; ++k) u[3 + k] = (use0 ? r0[k] : r1[k]) * inv;
  }
  u[6] = u[1] * u[5] - u[2] * u[4];
  u[7] = u[2] * u[3] - u[0] * u[5];
  u[8] = u[0] * u[4] - u[1] * u[3];
  SpecH H;
  H.mua = mua;
  H.beta = beta;
  H.kap = kap;
  H.rho = rho;
  H.c0 = -1.5 * mu;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int J = 0; J < 3; ++J)
      v[3 * i + J] = Ad[J] * u[3 * i] + Ad[3 + J] * u[3 * i + 1] + Ad[6 + J] * u[3 * i + 2];
    if (i == 1) {
      const double c = v[3] * v[0] + v[4] * v[1] + v[5] * v[2];
#pragma unroll
      for (int J = 0; J < 3; ++J) v[3 + J] -= c * v[J];
    }
    const double ai = sqrt_nr(v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                           v[3 * i + 2] * v[3 * i + 2]);
    if (!(ai > 0.0)) return -2;
    H.a[i] = ai;
    const double inv = rcp_nr(ai);
#pragma unroll
    for (int J = 0; J < 3; ++J) v[3 * i + J] *= inv;
  }
  v[6] = v[1] * v[5] - v[2] * v[4];
  v[7] = v[2] * v[3] - v[0] * v[5];
  v[8] = v[0] * v[4] - v[1] * v[3];
  {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int J = 0; J < 3; ++J) s += u[6 + i] * Ad[3 * i + J] * v[6 + J];
    H.a[2] = s;
  }
  // start
  double f[3], fa[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int J = 0; J < 3; ++J)
        s += u[3 * i + k] * ((double)E[3 * k + J] + (k == J ? 1.0 : 0.0)) * v[3 * i + J];
    f[i] = s;
    fa[i] = fmax(H.a[i], H.a[0] * 0.0625);
  }
  if (!(H.h(f) <= H.h(fa))) {
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = fa[i];
  }
  const double smod = mua + kap + rho;
  const double na = sqrt_nr(H.a[0] * H.a[0] + H.a[1] * H.a[1] + H.a[2] * H.a[2]);
  int ret = -1;
  for (int it = 0; it < maxit; ++it) {
    double g[3];
    H.grad(f, g);
    // norms, the Cholesky factor and the solves on the refined hardware
    // square roots and reciprocals
    const double gn = sqrt_nr(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double nf = sqrt_nr(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (gn <= gtol * smod * (1.0 + nf + na)) {
      ret = it;
      break;
    }
    const double Jm1 = f[0] * f[1] * f[2] - 1.0;
    const double p0 = f[1] * f[2], p1 = f[0] * f[2], p2 = f[0] * f[1];
    const double d00 = mua * (1.0 + beta) + rho + kap * p0 * p0;
    const double d11 = mua + rho + kap * p1 * p1, d22 = mua + rho + kap * p2 * p2;
    const double o10 = kap * (p1 * p0 + Jm1 * f[2]);
    const double o20 = kap * (p2 * p0 + Jm1 * f[1]);
    const double o21 = kap * (p2 * p1 + Jm1 * f[0]);
    // (i00, i11, i22: reciprocals of the factor's diagonal)
    double tau = 0.0, i00 = 0.0, l10 = 0.0, l20 = 0.0, i11 = 0.0, l21 = 0.0, i22 = 0.0;
    bool pd = false;
    for (int tries = 0; tries < 64 && !pd; ++tries) {
      const double e0 = d00 + tau;
      pd = e0 > 0.0;
      if (pd) {
        i00 = rsqrt_nr(e0);
        l10 = o10 * i00;
        l20 = o20 * i00;
        const double e1 = d11 + tau - l10 * l10;
        pd = e1 > 0.0;
        if (pd) {
          i11 = rsqrt_nr(e1);
          l21 = (o21 - l20 * l10) * i11;
          const double e2 = d22 + tau - l20 * l20 - l21 * l21;
          pd = e2 > 0.0;
          if (pd) i22 = rsqrt_nr(e2);
        }
      }
      if (!pd) tau = tau == 0.0 ? 0.0625 * rho : 2.0 * tau;
    }
    if (!pd) break;
    const double y0 = -g[0] * i00, y1 = (-g[1] - l10 * y0) * i11;
    const double y2 = (-g[2] - l20 * y0 - l21 * y1) * i22;
    double d[3];
    d[2] = y2 * i22;
    d[1] = (y1 - l21 * d[2]) * i11;
    d[0] = (y0 - l10 * d[1] - l20 * d[2]) * i00;
    const double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
    const bool small = -slope <= 1e-12 * smod * (1.0 + nf * nf);
    const double h0 = small ? 0.0 : H.h(f);
    double t = 1.0, ft[3];
    bool acc = false;
    for (int ls = 0; ls < 60 && !acc; ++ls) {
#pragma unroll
      for (int i = 0; i < 3; ++i) ft[i] = f[i] + t * d[i];
      if (ft[0] * ft[1] * ft[2] > 0.0) {
        if (!small) {
          acc = H.h(ft) <= h0 + 1e-4 * t * slope;
        } else {
          double gt[3];
          H.grad(ft, gt);
          acc = sqrt_nr(gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2]) <= (1.0 - 1e-4 * t) * gn;
        }
      }
      if (!acc) t *= 0.5;
    }
    if (!acc) break;
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = ft[i];
    const double nd = sqrt_nr(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    nf = sqrt_nr(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (t == 1.0 && nd <= step_tol * fmax(nf, 1.0)) {
      ret = it + 1;
      break;
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      E[3 * k + J] = (T)(f[0] * u[k] * v[J] + f[1] * u[3 + k] * v[3 + J] +
                         f[2] * u[6 + k] * v[6 + J] - (k == J ? 1.0 : 0.0));
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = u[k];
  return ret;
}

}  // namespace admm
