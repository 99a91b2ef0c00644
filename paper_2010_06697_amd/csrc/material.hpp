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
// J, ln J, the stress and the gradient are always double; the tangent, its
// factorisation and the solve are in HT (float in the reduced-precision mode).
#pragma once

#include "common.hpp"

namespace admm {

struct NHPoint {
  double J, lnJ, gn;
  double G[9];  // F^-T
  double g[9];  // grad phi = P + rho (E - A)
};

__device__ __forceinline__ bool nh_point(const double *E, const double *A, double rho, double mu,
                                         double lam, NHPoint &s) {
  double cE[9];
  cE[0] = E[4] * E[8] - E[5] * E[7];
  cE[1] = E[5] * E[6] - E[3] * E[8];
  cE[2] = E[3] * E[7] - E[4] * E[6];
  cE[3] = E[2] * E[7] - E[1] * E[8];
  cE[4] = E[0] * E[8] - E[2] * E[6];
  cE[5] = E[1] * E[6] - E[0] * E[7];
  cE[6] = E[1] * E[5] - E[2] * E[4];
  cE[7] = E[2] * E[3] - E[0] * E[5];
  cE[8] = E[0] * E[4] - E[1] * E[3];
  const double tr = E[0] + E[4] + E[8];
  const double s2 = cE[0] + cE[4] + cE[8];
  const double dE = E[0] * cE[0] + E[1] * cE[1] + E[2] * cE[2];
  const double jm1 = tr + s2 + dE;
  const double J = 1.0 + jm1;
  if (!(J > 0.0)) return false;
  const double lnJ = log1p(jm1);
  const double iJ = 1.0 / J;
  const double q = s2 + dE;
  double gn = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int a = 3 * i + j;
      const double Et = E[3 * j + i];
      const double dia = (i == j) ? 1.0 : 0.0;
      const double G = (cE[a] - Et + dia * (1.0 + tr)) * iJ;
      const double P = mu * iJ * (dia * q + J * E[a] + Et - cE[a]) + lam * lnJ * G;
      const double g = P + rho * (E[a] - A[a]);
      s.G[a] = G;
      s.g[a] = g;
      gn += g * g;
    }
  s.J = J;
  s.lnJ = lnJ;
  s.gn = sqrt(gn);
  return true;
}

__device__ __forceinline__ double nh_phi(const double *E, const double *A, double rho, double mu,
                                         double lam, const NHPoint &s) {
  double tr = E[0] + E[4] + E[8], e2 = 0.0, d2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    e2 += E[k] * E[k];
    d2 += (E[k] - A[k]) * (E[k] - A[k]);
  }
  return 0.5 * mu * (2.0 * tr + e2) - mu * s.lnJ + 0.5 * lam * s.lnJ * s.lnJ + 0.5 * rho * d2;
}

// |I + X|_F from X
__device__ __forceinline__ double norm_ipx(const double *X) {
  double tr = X[0] + X[4] + X[8], x2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) x2 += X[k] * X[k];
  return sqrt(fmax(3.0 + 2.0 * tr + x2, 0.0));
}

constexpr __host__ __device__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Newton solve of the local problem. E: warm start in, minimiser out.
// Returns the iteration count (>= 0), -1 when the iteration cap or the line
// search gave up (E keeps the last accepted iterate), -2 when det F <= 0 at
// the start.
template <typename HT>
__device__ int nh_newton(double *E, const double *A, double rho, double mu, double lam, int maxit,
                         double gtol, double step_tol) {
  NHPoint s;
  if (!nh_point(E, A, rho, mu, lam, s)) return -2;
  const double smod = mu + lam + rho;
  const double nA = norm_ipx(A);
  for (int it = 0; it < maxit; ++it) {
    const double nF = norm_ipx(E);
    if (s.gn <= gtol * smod * (1.0 + nF + nA)) return it;

    // prox tangent, lower triangle packed
    HT L[45];
    const double c1 = mu - lam * s.lnJ;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        const int i = a / 3, J = a % 3, k = b / 3, l = b % 3;
        double v = c1 * s.G[3 * k + J] * s.G[3 * i + l] + lam * s.G[a] * s.G[b];
        if (a == b) v += mu + rho;
        L[tri(a, b)] = (HT)v;
      }
    bool pd = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      HT d = L[tri(j, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
      pd = pd && (d > (HT)0);
      d = sqrt(d);
      L[tri(j, j)] = d;
      const HT id = (HT)1 / d;
#pragma unroll
      for (int i = j + 1; i < 9; ++i) {
        HT v = L[tri(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
        L[tri(i, j)] = v * id;
      }
    }
    double d[9];
    if (pd) {
      HT y[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        HT v = (HT)(-s.g[i]);
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
        y[i] = v / L[tri(i, i)];
      }
#pragma unroll
      for (int i = 8; i >= 0; --i) {
        HT v = y[i];
#pragma unroll
        for (int k = i + 1; k < 9; ++k) v -= L[tri(k, i)] * y[k];
        y[i] = v / L[tri(i, i)];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = (double)y[i];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) d[i] = -s.g[i];
    }

    double slope = 0.0, nd = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      slope += s.g[k] * d[k];
      nd += d[k] * d[k];
    }
    nd = sqrt(nd);
    const bool small = -slope <= 1e-12 * smod * (1.0 + nF * nF);
    const double phi0 = small ? 0.0 : nh_phi(E, A, rho, mu, lam, s);
    double t = 1.0;
    bool acc = false;
    NHPoint st;
    double Et[9];
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Et[k] = E[k] + t * d[k];
      if (nh_point(Et, A, rho, mu, lam, st)) {
        if (!small) {
          if (nh_phi(Et, A, rho, mu, lam, st) <= phi0 + 1e-4 * t * slope) {
            acc = true;
            break;
          }
        } else if (st.gn <= (1.0 - 1e-4 * t) * s.gn) {
          acc = true;
          break;
        }
      }
      t *= 0.5;
    }
    if (!acc) return -1;
#pragma unroll
    for (int k = 0; k < 9; ++k) E[k] = Et[k];
    s = st;
    if (pd && t == 1.0 && nd <= step_tol * fmax(1.0, norm_ipx(E))) return it + 1;
  }
  return -1;
}

}  // namespace admm
