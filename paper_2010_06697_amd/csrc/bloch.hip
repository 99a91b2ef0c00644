// bloch.hip -- stability modulus over Bloch waves (Sec. 2.5: quadratic
// functionals and Bloch waves, Steps 1'-4'), double precision, one cell.
//
//   beta = min over p periodic, <p, p> = 1, of <D_w p, L D_w p>
//
// with L the tangent d2W/dF2 of the cell's current state (the LCE with its
// director eliminated) and D_w the shifted central difference
// (D_w p)_ij(x) = (p_i(x+e_j) e^{i w_j} - p_i(x-e_j) e^{-i w_j}) / 2. ADMM:
//   1' G = (L + rho I)^{-1} (g + rho D_w p)     (L + rho I factorised once)
//   2' p = argmin over the unit sphere of |D_w p - (G - g/rho)|^2: with
//      b = D_w^H (G - g/rho), p^ = b^ / (|K|^2 - sigma), |K|^2 =
//      sum_j sin^2(xi_j + w_j), sigma < min |K|^2 the root of
//      sum |b^|^2 / (|K|^2 - sigma)^2 = V^2 (bisection, one workgroup)
//   3' g += rho (D_w p - G)
//   4' r_p = |D_w p - G|, r_d = rho |D_w p - D_w p_prev| (RMS over voxels).
// Complex fields are double2, component-major [c][x3][x2][x1].
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"
#include "material.hpp"

namespace admm {

namespace {

__device__ __forceinline__ double2 cexp_mul(double2 a, double c, double s) {
  return double2{a.x * c - a.y * s, a.x * s + a.y * c};
}

// deterministic workgroup sum (result in thread 0)
template <int NV>
__device__ __forceinline__ void bl_block_sum(double *v, double *red) {
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * nw + wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k * nw + w];
      v[k] = s;
    }
  __syncthreads();
}

struct BlochArgs {
  int n1, n2, n3, V;
  double c[3], s[3];  // cos, sin of w_j
  double rho;
  const double *E;    // F - I (9V)
  const double *dir;  // director (3V) or null
  const uint8_t *phase;
  const Material *mats;
  int n_mat;
  double *Lf;         // per voxel: 45 packed factor entries + 9 reciprocal pivots
  double2 *p, *G, *g, *Dold, *s2;  // p, s2: 3V; G, g, Dold: 9V
  double *part;       // per workgroup partial sums
  double *scal;       // [0] sigma, [1] r_p, [2] r_d, [3] beta, [4] error flag,
                      // [5] |p|^2 of the start, [6] zero-start flag, [7] stop
                      // (0 iterating, 1 converged, 2 error), [8] iterations run
  double tol;         // on r_p and r_d
  const double *k2t;  // sin^2(2 pi m/n_j + w_j): n1 + n2 + n3 entries
  double k2min;
};

// the iterations enqueued after the one that converged (or failed) do nothing
__device__ __forceinline__ bool bl_stopped(const BlochArgs &a) { return a.scal[7] != 0.0; }

__device__ __forceinline__ void neighbours(const BlochArgs &a, int x, int j, int &xp, int &xm) {
  const int x1 = x % a.n1, x2 = (x / a.n1) % a.n2, x3 = x / (a.n1 * a.n2);
  if (j == 0) {
    xp = x - x1 + (x1 + 1 == a.n1 ? 0 : x1 + 1);
    xm = x - x1 + (x1 == 0 ? a.n1 - 1 : x1 - 1);
  } else if (j == 1) {
    const int r = (x3 * a.n2) * a.n1 + x1;
    xp = r + (x2 + 1 == a.n2 ? 0 : x2 + 1) * a.n1;
    xm = r + (x2 == 0 ? a.n2 - 1 : x2 - 1) * a.n1;
  } else {
    const int r = x2 * a.n1 + x1;
    xp = r + (x3 + 1 == a.n3 ? 0 : x3 + 1) * a.n2 * a.n1;
    xm = r + (x3 == 0 ? a.n3 - 1 : x3 - 1) * a.n2 * a.n1;
  }
}

// (D_w p)(x): out[3i + j]
__device__ __forceinline__ void dgrad(const BlochArgs &a, const double2 *p, int x, double2 *out) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int xp, xm;
    neighbours(a, x, j, xp, xm);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 up = cexp_mul(p[i * a.V + xp], a.c[j], a.s[j]);
      const double2 um = cexp_mul(p[i * a.V + xm], a.c[j], -a.s[j]);
      out[3 * i + j] = double2{0.5 * (up.x - um.x), 0.5 * (up.y - um.y)};
    }
  }
}

// L^{-T} L^{-1} b for the packed factor
__device__ __forceinline__ void chol_solve(const double *L, const double *id, const double *b,
                                           double *x) {
  double y[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
    y[i] = v * id[i];
  }
#pragma unroll
  for (int i = 8; i >= 0; --i) {
    double v = y[i];
#pragma unroll
    for (int k = i + 1; k < 9; ++k) v -= L[tri(k, i)] * y[k];
    y[i] = v * id[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) x[i] = y[i];
}

// tangent + rho I at every voxel, factorised
__global__ __launch_bounds__(kThreads) void k_bl_factor(BlochArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  double E[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) E[c] = a.E[c * a.V + x];
  const int ph = a.phase[x];
  double L[45], id[9];
  bool ok = ph < a.n_mat;
  if (ok) {
    const Material m = a.mats[ph];
    Point<double> s;
    if (m.model == 1) {
      Lce<double> M;
      M.mua = m.mua;
      M.beta = m.beta;
      M.kappa = m.kappa;
      M.mu = m.mu;
      double np[3] = {a.dir[x], a.dir[a.V + x], a.dir[2 * a.V + x]};
      const double nn = 1.0 / sqrt(np[0] * np[0] + np[1] * np[1] + np[2] * np[2]);
#pragma unroll
      for (int k = 0; k < 3; ++k) np[k] *= nn;
      double w[3], Vv[9], nc[3];
      const int ncl = director_eig(E, np, nc, w, Vv);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        M.n[k] = nc[k];
        M.nd[k] = nc[k];
      }
      ok = M.point(E, E, 0.0, s);
      if (ok) lce_relaxed_tangent(E, M, s, a.rho, m.mua * m.beta, nc, w, Vv, ncl, 0.0, L);
    } else {
      NeoHooke<double> M;
      M.mu = m.mu;
      M.lam = m.lam;
      ok = M.point(E, E, 0.0, s);
      if (ok) {
        double dia, c1, c2;
        M.coeffs(s, a.rho, dia, c1, c2);
#pragma unroll
        for (int p = 0; p < 9; ++p)
#pragma unroll
          for (int q = 0; q <= p; ++q) {
            const int i = p / 3, J = p % 3, k = q / 3, l = q % 3;
            double v = c1 * s.G[3 * k + J] * s.G[3 * i + l] + c2 * s.G[p] * s.G[q];
            if (p == q) v += dia;
            L[tri(p, q)] = v;
          }
      }
    }
    if (ok) ok = chol_packed(L, id);
  }
  if (!ok) {
    a.scal[4] = 1.0;  // benign race: every writer stores the same value
    return;
  }
  double *o = a.Lf + (size_t)x * 54;
#pragma unroll
  for (int k = 0; k < 45; ++k) o[k] = L[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) o[45 + k] = id[k];
}

// Step 1': G = (L + rho I)^{-1} (g + rho D_w p); keeps D_w p for r_d
__global__ __launch_bounds__(kThreads) void k_bl_local(BlochArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V || bl_stopped(a)) return;
  double2 d[9];
  dgrad(a, a.p, x, d);
  double br[9], bi[9], xr[9], xi[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    a.Dold[c * a.V + x] = d[c];
    const double2 gv = a.g[c * a.V + x];
    br[c] = gv.x + a.rho * d[c].x;
    bi[c] = gv.y + a.rho * d[c].y;
  }
  const double *o = a.Lf + (size_t)x * 54;
  chol_solve(o, o + 45, br, xr);
  chol_solve(o, o + 45, bi, xi);
#pragma unroll
  for (int c = 0; c < 9; ++c) a.G[c * a.V + x] = double2{xr[c], xi[c]};
}

// Step 2' right-hand side: b = D_w^H (G - g/rho) into s2
__global__ __launch_bounds__(kThreads) void k_bl_div(BlochArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V || bl_stopped(a)) return;
  const double ir = 1.0 / a.rho;
  double2 b[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int xp, xm;
    neighbours(a, x, j, xp, xm);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int c = 3 * i + j;
      const double2 Gm = a.G[c * a.V + xm], gm = a.g[c * a.V + xm];
      const double2 Gp = a.G[c * a.V + xp], gp = a.g[c * a.V + xp];
      const double2 hm = cexp_mul(double2{Gm.x - gm.x * ir, Gm.y - gm.y * ir}, a.c[j], -a.s[j]);
      const double2 hp = cexp_mul(double2{Gp.x - gp.x * ir, Gp.y - gp.y * ir}, a.c[j], a.s[j]);
      b[i].x += 0.5 * (hm.x - hp.x);
      b[i].y += 0.5 * (hm.y - hp.y);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) a.s2[i * a.V + x] = b[i];
}

// One axis of the 3D transform of `ncomp` complex fields: each workgroup
// takes B lines (B * N <= 2048), consecutive in x1 for the x2 / x3 axes.
template <bool INV>
__global__ __launch_bounds__(kThreads) void k_bl_fft(double2 *data, int ncomp, int n1, int n2,
                                                    int n3, int axis, Plan1D pl,
                                                    const double2 *tw, int B, const double *stop) {
  extern __shared__ double2 lds[];
  if (*stop != 0.0) return;  // uniform over the workgroup
  const int N = pl.n;
  double2 *A = lds, *Bf = lds + B * N;
  const int nlines = ncomp * n1 * n2 * n3 / N;
  const int l0 = blockIdx.x * B;
  const int t = threadIdx.x, nt = blockDim.x;
  // element k of line l: global index
  auto gidx = [&](int l, int k) -> long long {
    if (axis == 0) return (long long)l * N + k;
    if (axis == 1) {
      // lines ordered (c, x3, x1)
      const int x1 = l % n1, r = l / n1;  // r = c * n3 + x3
      return ((long long)r * n2 + k) * n1 + x1;
    }
    const int x1 = l % n1, r = l / n1, x2 = r % n2, c = r / n2;  // lines (c, x2, x1)
    return (((long long)c * n3 + k) * n2 + x2) * n1 + x1;
  };
  for (int e = t; e < B * N; e += nt) {
    int l, k;
    if (axis == 0) {
      l = e / N;
      k = e % N;
    } else {
      l = e % B;
      k = e / B;
    }
    const int gl = l0 + l;
    A[l * N + k] = gl < nlines ? data[gidx(gl, k)] : double2{0.0, 0.0};
  }
  __syncthreads();
  double2 *res = fft_lines<INV>(A, Bf, pl, tw, B, N, 1, false, t, nt);
  for (int e = t; e < B * N; e += nt) {
    int l, k;
    if (axis == 0) {
      l = e / N;
      k = e % N;
    } else {
      l = e % B;
      k = e / B;
    }
    const int gl = l0 + l;
    if (gl < nlines) data[gidx(gl, k)] = res[l * N + k];
  }
}

__device__ __forceinline__ double k2_at(const BlochArgs &a, int x) {
  const int m1 = x % a.n1, m2 = (x / a.n1) % a.n2, m3 = x / (a.n1 * a.n2);
  return a.k2t[m1] + a.k2t[a.n1 + m2] + a.k2t[a.n1 + a.n2 + m3];
}

// the secular equation of Step 2' in one workgroup: sigma by bisection on
// (k2min - sqrt(sum |b^|^2)/V, k2min)
__global__ __launch_bounds__(1024) void k_bl_secular(BlochArgs a) {
  __shared__ double red[16];
  __shared__ double lohi[2];
  if (bl_stopped(a)) return;
  const double V = (double)a.V;
  double bb[1] = {0.0};
  for (int x = threadIdx.x; x < a.V; x += blockDim.x)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 v = a.s2[i * a.V + x];
      bb[0] += v.x * v.x + v.y * v.y;
    }
  bl_block_sum<1>(bb, red);
  if (threadIdx.x == 0) {
    lohi[0] = a.k2min - sqrt(bb[0]) / V;
    lohi[1] = a.k2min;
    // a zero right-hand side, or an iteration that diverged (penalty too
    // small for the tangent's negative part)
    if (!(bb[0] > 0.0) || !isfinite(bb[0])) a.scal[4] = 1.0;
  }
  __syncthreads();
  for (int it = 0; it < 200; ++it) {
    const double lo = lohi[0], hi = lohi[1], mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;  // uniform: every thread reads the same values
    double f[1] = {0.0};
    for (int x = threadIdx.x; x < a.V; x += blockDim.x) {
      double b2 = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 v = a.s2[i * a.V + x];
        b2 += v.x * v.x + v.y * v.y;
      }
      const double d = k2_at(a, x) - mid;
      f[0] += b2 / (d * d);
    }
    bl_block_sum<1>(f, red);
    if (threadIdx.x == 0) {
      if (f[0] > V * V)
        lohi[1] = mid;
      else
        lohi[0] = mid;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.scal[0] = lohi[0];
}

// p^ = b^ / (|K|^2 - sigma), with the 1/V of the inverse transform
__global__ __launch_bounds__(kThreads) void k_bl_scale(BlochArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V || bl_stopped(a)) return;
  const double f = 1.0 / ((k2_at(a, x) - a.scal[0]) * (double)a.V);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 v = a.s2[i * a.V + x];
    a.p[i * a.V + x] = double2{v.x * f, v.y * f};
  }
}

// Steps 3' and 4' (partial sums per workgroup)
__global__ __launch_bounds__(kThreads) void k_bl_update(BlochArgs a) {
  __shared__ double red[2 * (kThreads / 64)];
  if (bl_stopped(a)) return;  // uniform over the workgroup
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (x < a.V) {
    double2 d[9];
    dgrad(a, a.p, x, d);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double2 G = a.G[c * a.V + x], Do = a.Dold[c * a.V + x];
      const double er = d[c].x - G.x, ei = d[c].y - G.y;
      double2 gv = a.g[c * a.V + x];
      gv.x += a.rho * er;
      gv.y += a.rho * ei;
      a.g[c * a.V + x] = gv;
      v[0] += er * er + ei * ei;
      const double fr = d[c].x - Do.x, fi = d[c].y - Do.y;
      v[1] += fr * fr + fi * fi;
    }
  }
  bl_block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    a.part[2 * blockIdx.x] = v[0];
    a.part[2 * blockIdx.x + 1] = v[1];
  }
}

// Rayleigh quotient <D_w p, L D_w p> = |L_f^T d|^2 - rho |d|^2 (partials)
__global__ __launch_bounds__(kThreads) void k_bl_rayleigh(BlochArgs a) {
  __shared__ double red[kThreads / 64];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  double q[1] = {0.0};
  if (x < a.V) {
    double2 d[9];
    dgrad(a, a.p, x, d);
    const double *L = a.Lf + (size_t)x * 54, *id = L + 45;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        // column j of the factor: diagonal 1/id[j], below it L[tri(i, j)]
        double t = (part ? d[j].y : d[j].x) / id[j];
#pragma unroll
        for (int i = j + 1; i < 9; ++i) t += L[tri(i, j)] * (part ? d[i].y : d[i].x);
        q[0] += t * t;
      }
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const double dv = part ? d[j].y : d[j].x;
        q[0] -= a.rho * dv * dv;
      }
    }
  }
  bl_block_sum<1>(q, red);
  if (threadIdx.x == 0) a.part[2 * blockIdx.x] = q[0];
}

// fixed-order sum of the partials: NV values per workgroup -> scal[dst..];
// ITER: the end of an iteration, which also counts it and decides the stop
template <int NV, bool ITER = false>
__global__ __launch_bounds__(kThreads) void k_bl_reduce(BlochArgs a, int nblk, int dst) {
  __shared__ double red[NV * (kThreads / 64)];
  if (ITER && bl_stopped(a)) return;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += a.part[2 * b + k];
  bl_block_sum<NV>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) a.scal[dst + k] = v[k];
    if (ITER) {
      a.scal[8] += 1.0;
      const double rp = sqrt(a.scal[1] / (double)a.V);
      const double rd = a.rho * sqrt(a.scal[2] / (double)a.V);
      if (a.scal[4] != 0.0) a.scal[7] = 2.0;
      else if (rp <= a.tol && rd <= a.tol) a.scal[7] = 1.0;
    }
  }
}

// zero fill of n doubles (the multiplier and the scalars start at zero)
__global__ __launch_bounds__(kThreads) void k_bl_zero(double *q, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    q[k] = 0.0;
}

// partial sums of |p|^2 of the start vector
__global__ __launch_bounds__(kThreads) void k_bl_norm(BlochArgs a) {
  __shared__ double red[kThreads / 64];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  double q[1] = {0.0};
  if (x < a.V)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 v = a.p[i * a.V + x];
      q[0] += v.x * v.x + v.y * v.y;
    }
  bl_block_sum<1>(q, red);
  if (threadIdx.x == 0) a.part[2 * blockIdx.x] = q[0];
}

// <p, p> = 1 (sum |p|^2 = V) from the sum in scal[5]; a zero start is an
// error (flag in scal[6])
__global__ __launch_bounds__(kThreads) void k_bl_normalize(BlochArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const double s2 = a.scal[5];
  if (!(s2 > 0.0) || !isfinite(s2)) {
    if (x == 0) a.scal[6] = 1.0;
    return;
  }
  if (x >= a.V) return;
  const double sc = sqrt((double)a.V / s2);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 v = a.p[i * a.V + x];
    a.p[i * a.V + x] = double2{v.x * sc, v.y * sc};
  }
}

// Work buffers of the allocation-free entry point: one array per device,
// held until the process ends; its address is looked up once per device
// (hipGetSymbolAddress) and only that address is used on the host.
constexpr size_t kBlochScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kBlochScratchBytes];

}  // namespace

// bytes of the work buffers of one solve on this cell
size_t bloch_work_bytes(const RveDesc &D) {
  const size_t V = (size_t)D.V;
  const size_t nblk = (V + kThreads - 1) / kThreads;
  return V * 54 * 8 + (3 + 9 + 9 + 9 + 3) * V * 16 + 2 * nblk * 8 + 16 * 8 +
         (size_t)(D.n1 + D.n2 + D.n3) * 8;
}

size_t bloch_scratch_bytes() { return kBlochScratchBytes; }

// device address of this device's scratch array (looked up on first use)
int bloch_scratch(void **ptr) {
  static std::mutex mu;
  static void *addr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return -1;
    addr[dev] = q;
  }
  *ptr = addr[dev];
  return 0;
}

// host side: one solve (see include/admm.h, admm_bloch). work: device
// buffer of at least bloch_work_bytes(D) bytes, or null to allocate one for
// the call.
int bloch_solve(hipStream_t st, const RveDesc &D, const Material *mats_d, int n_mat,
                const void *tw, const double omega[3], double rho, double tol, int max_iter,
                double *p, void *work, double *beta, double *sigma_rho, int *iters,
                int *status) {
  BlochArgs a{};
  a.n1 = D.n1;
  a.n2 = D.n2;
  a.n3 = D.n3;
  a.V = (int)D.V;
  for (int j = 0; j < 3; ++j) {
    a.c[j] = std::cos(omega[j]);
    a.s[j] = std::sin(omega[j]);
  }
  a.rho = rho;
  a.tol = tol;
  a.E = static_cast<const double *>(D.E);
  a.dir = static_cast<const double *>(D.dir);
  a.phase = D.phase;
  a.mats = mats_d;
  a.n_mat = n_mat;
  const size_t V = (size_t)D.V;
  const int nblk = (int)((V + kThreads - 1) / kThreads);
  // |K|^2 per axis and its minimum (separable); at most 3 * kMaxN entries
  const int ns[3] = {D.n1, D.n2, D.n3};
  double k2h[3 * kMaxN];
  int nk = 0;
  double k2min = 0.0;
  for (int j = 0; j < 3; ++j) {
    double mn = 1e300;
    for (int m = 0; m < ns[j]; ++m) {
      const double v = std::sin(2.0 * M_PI * m / ns[j] + omega[j]);
      k2h[nk++] = v * v;
      mn = std::min(mn, v * v);
    }
    k2min += mn;
  }
  a.k2min = k2min;
  // work buffers
  void *buf = work;
  if (!buf && hipMalloc(&buf, bloch_work_bytes(D)) != hipSuccess) return -1;
  char *q = static_cast<char *>(buf);
  a.Lf = reinterpret_cast<double *>(q);
  q += V * 54 * 8;
  a.g = reinterpret_cast<double2 *>(q);
  q += 9 * V * 16;
  a.G = reinterpret_cast<double2 *>(q);
  q += 9 * V * 16;
  a.Dold = reinterpret_cast<double2 *>(q);
  q += 9 * V * 16;
  a.s2 = reinterpret_cast<double2 *>(q);
  q += 3 * V * 16;
  a.p = reinterpret_cast<double2 *>(q);  // p (interleaved complex)
  q += 3 * V * 16;
  a.part = reinterpret_cast<double *>(q);
  q += 2 * (size_t)nblk * 8;
  a.scal = reinterpret_cast<double *>(q);
  q += 16 * 8;
  a.k2t = reinterpret_cast<const double *>(q);
  int rc = 0;
  auto fail = [&](int code) {
    rc = code;
    return code;
  };
  const dim3 grid(nblk), blk(kThreads);
  do {
    // the multiplier and the scalars start at zero (a fill kernel: the
    // buffer may hold an earlier call's values)
    hipLaunchKernelGGL(k_bl_zero, dim3(std::min(nblk * 9, 4096)), blk, 0, st,
                       reinterpret_cast<double *>(a.g), 18 * V);
    hipLaunchKernelGGL(k_bl_zero, dim3(1), blk, 0, st, a.scal, (size_t)16);
    if (hipMemcpyAsync(const_cast<double *>(a.k2t), k2h, (size_t)nk * 8, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(a.p, p, 3 * V * 16, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      fail(-1);
      break;
    }
    hipLaunchKernelGGL(k_bl_factor, grid, blk, 0, st, a);
    // normalise the start on the device: <p, p> = 1
    hipLaunchKernelGGL(k_bl_norm, grid, blk, 0, st, a);
    hipLaunchKernelGGL((k_bl_reduce<1>), dim3(1), blk, 0, st, a, nblk, 5);
    hipLaunchKernelGGL(k_bl_normalize, grid, blk, 0, st, a);
    double scal[16];
    if (hipMemcpyAsync(scal, a.scal, sizeof(scal), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      fail(-1);
      break;
    }
    if (scal[6] != 0.0) {
      fail(-2);  // zero start
      break;
    }
    if (scal[4] != 0.0) {
      fail(-3);  // L + rho I not positive definite somewhere
      break;
    }
    const Plan1D pls[3] = {D.p1, D.p2, D.p3};
    const double2 *twd = static_cast<const double2 *>(tw);
    auto fft3 = [&](double2 *data, bool inv) {
      for (int ax = 0; ax < 3; ++ax) {
        const int N = pls[ax].n;
        const int B = std::max(1, std::min(64, 2048 / N));
        const int nl = 3 * (int)(V / N);
        const int g = (nl + B - 1) / B;
        const size_t lds = 2 * (size_t)B * N * sizeof(double2);
        if (inv)
          hipLaunchKernelGGL(k_bl_fft<true>, dim3(g), blk, lds, st, data, 3, a.n1, a.n2, a.n3, ax,
                             pls[ax], twd, B, a.scal + 7);
        else
          hipLaunchKernelGGL(k_bl_fft<false>, dim3(g), blk, lds, st, data, 3, a.n1, a.n2, a.n3,
                             ax, pls[ax], twd, B, a.scal + 7);
      }
    };
    // iterations enqueued in chunks, the host reading the stop word once per
    // chunk: an iteration after the one that converged (or failed) does
    // nothing, so the result and the count are those of checking every one
    constexpr int kChunk = 16;
    int queued = 0;
    *status = 1;
    while (queued < max_iter) {
      const int m = std::min(kChunk, max_iter - queued);
      for (int k = 0; k < m; ++k) {
        hipLaunchKernelGGL(k_bl_local, grid, blk, 0, st, a);
        hipLaunchKernelGGL(k_bl_div, grid, blk, 0, st, a);
        fft3(a.s2, false);
        hipLaunchKernelGGL(k_bl_secular, dim3(1), dim3(1024), 0, st, a);
        // p^ = b^ / (|K|^2 - sigma) in place, inverse transform there, and
        // the two buffers swap roles (p in the transformed one)
        {
          BlochArgs b = a;
          b.p = a.s2;
          hipLaunchKernelGGL(k_bl_scale, grid, blk, 0, st, b);
        }
        fft3(a.s2, true);
        std::swap(a.p, a.s2);
        hipLaunchKernelGGL(k_bl_update, grid, blk, 0, st, a);
        hipLaunchKernelGGL((k_bl_reduce<2, true>), dim3(1), blk, 0, st, a, nblk, 1);
      }
      queued += m;
      if (hipMemcpyAsync(scal, a.scal, sizeof(scal), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        fail(-1);
        break;
      }
      if (scal[7] != 0.0) break;
    }
    if (rc) break;
    // the buffers swapped once per enqueued iteration, p only once per run one
    const int it = (int)scal[8];
    if ((queued - it) % 2) std::swap(a.p, a.s2);
    if (scal[7] == 2.0) {
      fail(-2);
      break;
    }
    if (scal[7] == 1.0) *status = 0;
    if (rc) break;
    hipLaunchKernelGGL(k_bl_rayleigh, grid, blk, 0, st, a);
    hipLaunchKernelGGL((k_bl_reduce<1>), dim3(1), blk, 0, st, a, nblk, 3);
    if (hipMemcpyAsync(scal, a.scal, sizeof(scal), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(p, a.p, 3 * V * 16, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      fail(-1);
      break;
    }
    *beta = scal[3] / (double)V;
    if (sigma_rho) *sigma_rho = rho * scal[0];
    if (iters) *iters = it;
  } while (false);
  (void)hipStreamSynchronize(st);
  if (!work) (void)hipFree(buf);
  if (hipGetLastError() != hipSuccess && rc == 0) rc = -1;
  return rc;
}

}  // namespace admm
