// common.hpp -- device-side data structures shared by the ADMM kernels and the
// host launcher (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace admm {

constexpr int kThreads = 256;   // threads per workgroup of every kernel
constexpr int kMaxStages = 8;   // radix stages of one 1D transform
constexpr int kMaxN = 256;      // largest supported edge

// n / d by one high multiply, for 0 <= n < 2^32 / d: m = ceil(2^32 / d), and
// m = 0 for d = 1 (the quotient is n). The transforms' index arithmetic
// divides by lengths known only at run time, where the general division
// costs about twenty instructions per use.
struct FastDiv {
  unsigned d, m;
};
inline FastDiv make_fastdiv(unsigned d) {
  FastDiv f;
  f.d = d;
  f.m = d <= 1 ? 0u : (unsigned)(((1ull << 32) + d - 1) / d);
  return f;
}
__device__ __forceinline__ int fdiv(int n, FastDiv f) {
  return f.m ? (int)__umulhi((unsigned)n, f.m) : n;
}

// radix plan of one 1D transform of length n; tw: offset of its twiddle table
// exp(-2 pi i t / n), t = 0..n-1, in the twiddle pool. nb[s], ns[s]: the
// butterflies per line (n / rad[s]) and the span before stage s (the product
// of the earlier radices), as divisors.
struct Plan1D {
  int n;
  int nst;
  int rad[kMaxStages];
  int tw;
  FastDiv nb[kMaxStages];
  FastDiv ns[kMaxStages];
};

inline void plan_divisors(Plan1D &p) {
  unsigned span = 1;
  for (int s = 0; s < p.nst; ++s) {
    p.nb[s] = make_fastdiv((unsigned)(p.n / p.rad[s]));
    p.ns[s] = make_fastdiv(span);
    span *= (unsigned)p.rad[s];
  }
}

// one periodic cell, as the kernels see it
struct RveDesc {
  int n1, n2, n3, m1;       // m1 = n1/2 + 1 (half spectrum along x1)
  long long V;              // voxels
  long long S;              // complex entries of one spectral component
  int rows;                 // x1-lines per workgroup of the per-voxel kernels
  int rows_f;               // x1-lines per workgroup of the x1 transforms
  int m1s;                  // row stride of the half spectra (m1 rounded up to 32
                            // bytes, so that every column tile starts on a sector)
  FastDiv f_n1, f_n2, f_m1, f_rows_f;  // the same as divisors
  Plan1D p1, p2, p3;
  const uint8_t *phase;
  void *u[2];               // displacement fluctuation (double in both
                            // precisions), ping-pong
  void *du;                 // float form: the correction u_{i+1} - u_i of
                            // Step 2 (3V float, in the workspace), else null
  void *E;                  // F - I
  void *Lam;                // multiplier
  void *dir;                // director (LCE) or null
  const void *dir0;         // cross-link director (non-ideality) or null
  void *dir_lag;            // directors of the previous iteration (Frank) or null
  void *dir_step;           // directors at the start of the load step (nu_n) or null
  void *E_step;             // F - I at the start of the load step (nu_F) or null
  void *spec;               // 9 spectral components, layout [c][x3][x2][m1]
  void *At;                 // float form without LCE phases: Step 1's data
                            // A - I = grad u + Ebar + Lambda/rho of the next
                            // iteration as the update formed it (9V float),
                            // then the warm start's det F - 1 (V float, in
                            // warm_code's form), valid while RveState::at_rho
                            // is the penalty; else null
  void *Q;                  // float form without the full LCE model's terms:
                            // F - A of the last local pass (9V float), whose
                            // D_h^T is Step 2's defect; else null
};

// per-cell iteration state, updated on the device
struct RveState {
  double rho;        // penalty of the next iteration
  double rho_used;   // penalty of the last iteration
  double rp, rd;     // residuals of the last iteration
  int iter;          // iterations of the current load step
  int cur;           // which u buffer holds u_i
  int active;        // 1 while the cell iterates
  int status;        // 0 running, 1 iteration cap, 2 converged, -5 domain error
  int newton_fail;   // local solves that hit the Newton cap
  int domain_err;    // set when det F <= 0 or NaN met
  int local_done;    // inexact local step: r_l reached its target (or the pass cap)
  int pad1;
  unsigned long long newton_iters;  // Newton iterations summed over voxels and iterations
  double rl;         // local residual after the last inexact pass
  double Ebar[9];       // <F> - I of the current iterate (free components move)
  double Ebar_prev[9];  // <F> - I of the previous iterate (r_d)
  unsigned free_mask;   // bit k: component k of <F> free (mixed conditions)
  int ref_iter;         // divergence watch: iteration of the last halving
  int n_retry;          // voxels the exact local pass left to its retry pass
                        // (cleared by k_finalize)
  int q_cur;           // 1: RveDesc::Q holds F - A of the current fields
                        // and penalty (the local step of this iteration
                        // wrote it), which Step 2 then reads; cleared by
                        // k_finalize and by every state upload
  double best_merit;    // divergence watch: smallest merit of the load step
  double ref_merit;     // divergence watch: merit at ref_iter
  double at_rho;        // penalty RveDesc::At was formed with by the last
                        // update (0: not formed in this call; reset by every
                        // state upload, so fields the caller wrote in between
                        // are read afresh)
};

// Divergence / stagnation watch of admm_solve, applied after each
// iteration's convergence test. merit = max(r_p / tol_p, r_d / tol_d).
// Diverged when the merit exceeds growth x the smallest merit of the load
// step (growth > 0), or when it has not halved for `stall` iterations
// (stall > 0). best / ref / ref_iter start at +inf / +inf / 0 with each load
// step. Shared by the device (k_finalize) and the host replay
// (admm_divergence_check).
__host__ __device__ inline bool divergence_watch(double rp, double rd, double tol_p, double tol_d,
                                                 int it, double growth, int stall, double &best,
                                                 double &ref, int &ref_iter) {
  const double tp = tol_p > 0.0 ? tol_p : 1e-300, td = tol_d > 0.0 ? tol_d : 1e-300;
  const double m = rp / tp > rd / td ? rp / tp : rd / td;
  if (m < best) best = m;
  if (m <= 0.5 * ref) {
    ref = m;
    ref_iter = it;
  }
  if (growth > 0.0 && m > growth * best) return true;
  return stall > 0 && it - ref_iter >= stall;
}

constexpr int kZSeg = 16;  // planes per workgroup of the update tiling (k_update walks them)
// tile width that selects the register-resident x2 / x3 pass of length 256
// (16 columns per workgroup, 16 points per thread, one LDS exchange per
// transform); open to an axis when every cell's length along it is 256
constexpr int kTileCol16 = -16;
constexpr int kLocalPassGrid = 2048;  // workgroups of the later inexact local passes

struct Material {
  int model;  // 0 neo-Hookean, 1 LCE
  int ext;    // 1: some term of the full LCE model (or nu_F) is on
  double mu, lam, a, kappa;
  double mua;   // mu a^(1/3)
  double beta;  // 1/a - 1
  double mual;  // mu alpha (non-ideality)
  double frank, nu_F, nu_n;
};

// scalar parameters of one launch sequence (passed by value: kernel arguments
// live in the constant/scalar path of the hardware)
struct IterParams {
  double rho_min, rho_max, kappa_rho, tau;
  double tol_p, tol_d, mu_ref;
  double gtol, step_tol;
  int adapt;
  int max_iter;
  int newton_max;
  int test_conv;     // 1: convergence test and iteration cap (admm_solve)
  int hist_cap;
  int n_rve;
  int n_mat;
  double local_ratio;     // inexact local step, r_l <= ratio r_d (0: off)
  int local_chunk;
  int local_passes;
  double local_fraction;  // inexact local step, converged fraction (0: off)
  double dt;              // time step (dissipation)
  double div_growth;      // divergence watch (admm_solve): growth factor (0: off)
  int stall_iters;        // divergence watch: stagnation window (0: off)
};

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };

// Workgroups are handed to the 8 XCDs round-robin (workgroup i -> XCD i % 8).
// Remap so that each XCD receives a contiguous range of logical tiles: tiles
// that share halo rows then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int nx = 8;
  int x = bid % nx, k = bid / nx;
  int per = nblk / nx, rem = nblk % nx;
  return x * per + (x < rem ? x : rem) + k;
}

// cell owning logical workgroup `blk`, given the prefix table blk0[0..n]
__device__ __forceinline__ int find_rve(const int *__restrict__ blk0, int n, int blk) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (blk0[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace admm
