// material.hpp -- per-voxel local problem (Step 1 of Sec. 2.1) for the
// compressible neo-Hookean energy
//     W(F) = mu/2 (|F|^2 - 3) - mu ln J + lambda/2 (ln J)^2,
// written in the displacement gradient E = F - I so that nothing cancels at
// small strain:
//     J - 1 = tr E + s2(E) + det E          (s2: sum of principal 2x2 minors)
//     cof F = (1 + tr E) I - E^T + cof E
//     J (F - F^-T) = (s2 + det E) I + J E + E^T - cof E
//     P = mu (F - F^-T) + lambda ln J F^-T,   ln J = log1p(J - 1).
// The local problem minimises phi(E) = W(I + E) + rho/2 |E - A|^2 by Newton's
// method on the 9-vector E with the analytic tangent
//     dP_iJ/dF_kL = mu d_ik d_JL + (mu - lambda ln J) Fi_Jk Fi_Li
//                   + lambda Fi_Ji Fi_Lk        (Fi = F^-1)
// plus rho I, a Cholesky factorisation (steepest descent when it is not
// positive definite) and backtracking (Armijo on phi, or on |grad phi| once
// the predicted decrease is below phi's rounding floor), rejecting det F <= 0.
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

template <typename TG> struct NHPoint {
  double lnJ;   // ln J (double)
  TG gn2;       // |grad phi|^2
  TG G[9];      // F^-T
  TG g[9];      // grad phi = P + rho (E - A)
};

// state of the local problem at E; false when det F <= 0
template <typename TG>
__device__ __forceinline__ bool nh_point(const TG *E, const TG *A, TG rho, TG mu, TG lam,
                                         NHPoint<TG> &s) {
  // J - 1 in double from the (exactly converted) components of E
  double e[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) e[k] = (double)E[k];
  const double c0 = e[4] * e[8] - e[5] * e[7];
  const double c1 = e[5] * e[6] - e[3] * e[8];
  const double c2 = e[3] * e[7] - e[4] * e[6];
  const double c4 = e[0] * e[8] - e[2] * e[6];
  const double c8 = e[0] * e[4] - e[1] * e[3];
  const double tr = e[0] + e[4] + e[8];
  const double s2 = c0 + c4 + c8;
  const double dE = e[0] * c0 + e[1] * c1 + e[2] * c2;
  const double jm1 = tr + s2 + dE;
  const double J = 1.0 + jm1;
  if (!(J > 0.0)) return false;
  s.lnJ = log1p_near1(jm1);
  TG cE[9];
  cE[0] = (TG)c0;
  cE[1] = (TG)c1;
  cE[2] = (TG)c2;
  cE[3] = E[2] * E[7] - E[1] * E[8];
  cE[4] = (TG)c4;
  cE[5] = E[1] * E[6] - E[0] * E[7];
  cE[6] = E[1] * E[5] - E[2] * E[4];
  cE[7] = E[2] * E[3] - E[0] * E[5];
  cE[8] = (TG)c8;
  const TG Jt = (TG)J, iJ = (TG)1 / Jt, q = (TG)(s2 + dE), trt = (TG)tr;
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
      const TG P = mu * iJ * (dia * q + Jt * E[a] + Et - cE[a]) + lam * lnJt * G;
      const TG g = P + rho * (E[a] - A[a]);
      s.G[a] = G;
      s.g[a] = g;
      gn2 += g * g;
    }
  s.gn2 = gn2;
  return true;
}

template <typename TG>
__device__ __forceinline__ double nh_phi(const TG *E, const TG *A, double rho, double mu,
                                         double lam, double lnJ) {
  double tr = (double)E[0] + (double)E[4] + (double)E[8], e2 = 0.0, d2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double ek = (double)E[k], dk = ek - (double)A[k];
    e2 += ek * ek;
    d2 += dk * dk;
  }
  return 0.5 * mu * (2.0 * tr + e2) - mu * lnJ + 0.5 * lam * lnJ * lnJ + 0.5 * rho * d2;
}

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

// Newton solve of the local problem. E: warm start in, minimiser out.
// Stops when |grad phi| <= gtol (mu + lambda + rho)(1 + |F| + |A|) before a
// step, or after a full positive-definite Newton step with
// |dE| <= step_tol max(1, |F|) (which leaves an error of order |dE|^2).
// Returns the iteration count (>= 0), -1 when the cap or the line search gave
// up (E keeps the last accepted iterate), -2 when det F <= 0 at the start.
template <typename TG, typename TH>
__device__ int nh_newton(TG *E, const TG *A, TG rho, TG mu, TG lam, int maxit, double gtol,
                         double step_tol) {
  NHPoint<TG> s;
  if (!nh_point(E, A, rho, mu, lam, s)) return -2;
  const double smod = (double)mu + (double)lam + (double)rho;
  const double nA = sqrt((double)norm2_ipx(A));
  const double tol_step2 = step_tol * step_tol;
  for (int it = 0; it < maxit; ++it) {
    const double nF2 = (double)norm2_ipx(E);
    const double thr = gtol * smod * (1.0 + sqrt(nF2) + nA);
    if ((double)s.gn2 <= thr * thr) return it;

    // prox tangent, lower triangle packed, assembled in TH
    TH L[45], Gh[9], id[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Gh[k] = (TH)s.G[k];
    const TH c1 = (TH)((double)mu - (double)lam * s.lnJ), lh = (TH)lam, dia = (TH)(mu + rho);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        const int i = a / 3, J = a % 3, k = b / 3, l = b % 3;
        TH v = c1 * Gh[3 * k + J] * Gh[3 * i + l] + lh * Gh[a] * Gh[b];
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

    double slope = 0.0, nd2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      slope += (double)s.g[k] * (double)d[k];
      nd2 += (double)d[k] * (double)d[k];
    }
    const bool small = -slope <= 1e-12 * smod * (1.0 + nF2);
    // float iterate: a full Newton step already below the step tolerance is
    // taken as it is; the float gradient is at its rounding floor there and
    // no longer decides a line search
    const bool tiny = sizeof(TG) == 4 && pd && nd2 <= tol_step2 * fmax(1.0, nF2);
    const double phi0 = small ? 0.0 : nh_phi(E, A, rho, mu, lam, s.lnJ);
    double t = 1.0;
    bool acc = false;
    NHPoint<TG> st;
    TG Et[9];
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Et[k] = E[k] + (TG)t * d[k];
      if (nh_point(Et, A, rho, mu, lam, st)) {
        if (tiny) {
          acc = true;
          break;
        }
        if (!small) {
          if (nh_phi(Et, A, rho, mu, lam, st.lnJ) <= phi0 + 1e-4 * t * slope) {
            acc = true;
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

}  // namespace admm
