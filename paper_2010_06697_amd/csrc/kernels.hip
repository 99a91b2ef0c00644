// kernels.hip -- the HIP kernels of one ADMM iteration (gfx950) and their
// host launchers.
//
// Step 2 solves D_h^T D_h u = D_h^T H for H = F - Lambda/rho, D_h the central
// difference. In Fourier space this is |K|^2 u_hat = b_hat with b = D_h^T H,
// b_i = -sum_j (H_ij(x+e_j) - H_ij(x-e_j))/2, whose transform is
// -i sum_j K_j H_hat_ij, K_j = sin(2 pi m_j/n_j): the Fourier-space solve of
// Sec. 2.3 with central-difference symbols. Forming b in real space first
// leaves three components to transform instead of nine.
//
// Per iteration, over every active cell of the batch, in this order:
//   k_local        Step 1: the local solve per voxel (F; in the float form
//                  without the full LCE model's terms also F - A for Step 2)
//   k_div_fwdx     b = D_h^T (F - Lambda/rho) (float form: the defect
//                  D_h^T (F - A), whose solve is u_{i+1} - u_i) and its
//                  forward real-to-complex FFT along x1 (two real rows per
//                  complex transform)
//   k_fft_y        forward FFT along x2 of the three components
//   k_poisson_z    forward FFT along x3, u_hat = b_hat / (|K|^2 V) (zero on
//                  the eight modes where every K_j vanishes), inverse along x3
//   k_fft_y        inverse FFT along x2
//   k_inv_x        inverse complex-to-real FFT along x1 into u_{i+1}
//   k_update       Step 3 (Lambda += rho (grad u_{i+1} - F)) and the
//                  per-workgroup partial sums of Step 4
//   k_finalize     fixed-order reduction of the partials, r_p, r_d, the
//                  convergence test and the adaptive penalty (Sec. 2.1)
// All scalar iteration state (rho, residuals, which u buffer is current,
// activity) lives in device memory, so the host only launches.
#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"
#include "material.hpp"

namespace admm {

// ----------------------------------------------------------------------------
// helpers
// ----------------------------------------------------------------------------

// The float form solves Step 2 for the correction u_{i+1} - u_i (defect
// correction) and keeps u in double; the double form solves for u_{i+1}.
template <typename T> constexpr bool kDefect = sizeof(T) == 4;

// neighbour offsets of voxel (x1,x2,x3) along +-e1, +-e2, +-e3 (periodic)
struct Stencil {
  int o[6];
};

__device__ __forceinline__ Stencil stencil(int n1, int n2, int n3, int x1, int x2, int x3) {
  const int x1p = x1 + 1 == n1 ? 0 : x1 + 1, x1m = x1 == 0 ? n1 - 1 : x1 - 1;
  const int x2p = x2 + 1 == n2 ? 0 : x2 + 1, x2m = x2 == 0 ? n2 - 1 : x2 - 1;
  const int x3p = x3 + 1 == n3 ? 0 : x3 + 1, x3m = x3 == 0 ? n3 - 1 : x3 - 1;
  const int row = (x3 * n2 + x2) * n1;
  Stencil s;
  s.o[0] = row + x1p;
  s.o[1] = row + x1m;
  s.o[2] = (x3 * n2 + x2p) * n1 + x1;
  s.o[3] = (x3 * n2 + x2m) * n1 + x1;
  s.o[4] = (x3p * n2 + x2) * n1 + x1;
  s.o[5] = (x3m * n2 + x2) * n1 + x1;
  return s;
}

// Every field lives in global memory, but a pointer read from the descriptor
// tables carries no address space: inside an inlined helper the compiler
// cannot always prove it global and accesses it with flat instructions (the
// local kernel ran 8% slower that way). Kernels access fields through these
// global-address-space views.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> global_view(T *p) {
  return (gptr<T>)p;
}

// x + 2 and x - 2 modulo n, for n = 1 (plane strain along x3) or n >= 4
__device__ __forceinline__ int wrap_plus2(int x, int n) {
  return n == 1 ? 0 : (x + 2 >= n ? x + 2 - n : x + 2);
}
__device__ __forceinline__ int wrap_minus2(int x, int n) {
  return n == 1 ? 0 : (x - 2 < 0 ? x - 2 + n : x - 2);
}

// central differences (u_i(x+e_j) - u_i(x-e_j))/2 of a 3-vector field; out[3i+j]
template <typename P>
__device__ __forceinline__ void grad_u(P u, int V, const Stencil &s, double *out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const auto ui = u + i * V;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out[3 * i + j] = 0.5 * ((double)ui[s.o[2 * j]] - (double)ui[s.o[2 * j + 1]]);
  }
}

// the same of u + du (float form: u_{i+1} = u_i + du, each value formed as
// it is stored, so the gradient equals the one of the stored u_{i+1})
template <typename P, typename Q>
__device__ __forceinline__ void grad_u_sum(P u, Q du, int V, const Stencil &s, double *out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const auto ui = u + i * V;
    const auto di = du + i * V;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int p = s.o[2 * j], m = s.o[2 * j + 1];
      out[3 * i + j] = 0.5 * ((ui[p] + (double)di[p]) - (ui[m] + (double)di[m]));
    }
  }
}

// Order of the divergence kernel's workgroups over a cell's ny x2 positions
// and nz x3 blocks: chunks of kZChunk x3 blocks, within a chunk the x3 block
// fastest. A workgroup's +-x3 neighbour lines are then read by the
// workgroups just before and after it, its +-x2 neighbours kZChunk
// workgroups away, both within what an XCD's L2 still holds (x2 fastest put
// the x3 neighbours a whole plane of streamed fields apart). The hardware
// deals workgroups to the XCDs in turn and xcd_remap gives each XCD a
// contiguous run of this order.
constexpr int kZChunk = 16;
__device__ __forceinline__ void chunk_order(int b, int ny, int nz, int &yg, int &zb) {
  const int ch = b / (ny * kZChunk);
  const int rem = b - ch * ny * kZChunk;
  const int zl = min(kZChunk, nz - ch * kZChunk);
  yg = rem / zl;
  zb = ch * kZChunk + rem - yg * zl;
}

// (x2, first x3) of workgroup b of a cell in the update / mean-stress tiling:
// R x1-lines (one x2 group) on kZSeg consecutive planes, x2 group fastest
// (the workgroups of neighbouring x2 groups run side by side)
__device__ __forceinline__ void column_tile(const RveDesc &D, int b, int row, int &x2, int &z0) {
  const int ny = (D.n2 + D.rows - 1) / D.rows;
  const int zb = b / ny;
  x2 = (b - zb * ny) * D.rows + row;
  z0 = zb * kZSeg;
}

// deterministic sum of NV doubles over the workgroup; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double *v, double *red /* LDS NV*nwaves */) {
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
}

// ----------------------------------------------------------------------------
// Step 1: local problem per voxel
// ----------------------------------------------------------------------------

// Occupancy of the local kernel: the Newton state (about 200 live registers)
// bounds it; a value of 2 or more trades spills for waves per SIMD.
#ifndef ADMM_LOCAL_WAVES_PER_EU
#define ADMM_LOCAL_WAVES_PER_EU 1
#endif

// LCE: the joint (F, director) Newton solve of lce_newton. Adds the Newton
// iterations to its.
template <typename T>
__device__ int lce_local(T *E, const T *At, const Material &m, double rho, double *n,
                         const IterParams &ip, int cap, int &its, const DirForm *form) {
  Lce<T> M;
  M.mua = (T)m.mua;
  M.beta = (T)m.beta;
  M.kappa = (T)m.kappa;
  M.mu = (T)m.mu;
  M.mual = (T)m.mual;
  M.form = form;
  const int rc = lce_newton<T>(E, At, M, m.mua * m.beta, (T)rho, n, cap, ip.gtol, ip.step_tol);
  its += rc >= 0 ? rc : cap;
  return rc;
}

// inexact local step in force for this cell and iteration: the ratio
// strategy needs the previous iteration's r_d, so it starts at the second
// iteration of a load step
__device__ __forceinline__ bool local_inexact(const IterParams &ip, const RveState *st) {
  return ip.local_fraction > 0.0 || (ip.local_ratio > 0.0 && st->iter > 0);
}

// Step 1 on the voxels of logical workgroup `blk`. Exact: one pass, every
// local problem solved to the Newton tolerances. Inexact: each pass runs at
// most local_chunk Newton iterations per voxel from its current iterate (F
// and the director) and stores the workgroup's sum of |local residual|^2 and
// count of converged solves, which k_local_check reduces. Passes after the
// first do nothing once the cell is done.
// launch modes of the local step: every problem solved exactly (no inexact
// strategy configured), the first pass of an inexact step, a later pass, and
// the exact step's second pass over the problems its first pass left to the
// nine-component Newton method (float form without LCE phases: the first
// pass then compiles only the neo-Hookean closed form, at the registers
// that need). The double form finishes the closed form's point with one
// full Newton step and runs the Newton solve where the closed form fails.
enum LocalMode { kLocalExact = 0, kLocalFirst = 1, kLocalLater = 2, kLocalRetry = 3 };
static_assert(kThreads / 32 == 8, "the retry pass reads a workgroup's bits as two uint4");
template <typename T, int LK, int MODE>
constexpr bool kClosedOnly = MODE == kLocalExact && kDefect<T> && LK == 0;
// the passes over every voxel in the float form without the full LCE
// model's terms: their F - A (RveDesc::Q, written by every pass) is what
// Step 2 then reads; without LCE phases they read Step 1's data where the
// update formed it at this penalty (RveDesc::At)
template <typename T, int LK, int MODE>
constexpr bool kFullPass = kDefect<T> && LK <= 1 && (MODE == kLocalExact || MODE == kLocalFirst);

// LK: 0 no LCE phase, 1 the ideal LCE, 2 some term of the full LCE model
// (non-ideality, Frank, dissipation) or the dissipation of F
template <typename T, int LK, int MODE>
__device__ __forceinline__ void local_tile(KernelArgs a, IterParams ip, int pass, int blk) {
  const int r = find_rve(a.blk_x, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  RveState *st = a.state + r;
  if (!st->active) return;
  const bool inexact =
      MODE != kLocalExact && MODE != kLocalRetry && local_inexact(ip, st);
  if (MODE == kLocalLater && (!inexact || st->local_done)) return;
  const int b = blk - a.blk_x[r];
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows;
  const int nrows = n2 * n3;
  const int V = (int)D.V;
  const int t = threadIdx.x;
  const int row = t / n1, x1 = t - row * n1;
  const int grow = b * R + row;
  int n_fail = 0, n_its = 0;
  double lsum[2] = {0.0, 0.0};  // |local residual|^2, converged
  // the voxels the closed form did not take: one bit per thread and workgroup
  unsigned *retry = a.retry_mask + (size_t)blk * (kThreads / 32);
  const bool mine = MODE != kLocalRetry || ((retry[t >> 5] >> (t & 31)) & 1u);
  bool deferred = false;
  if (row < R && grow < nrows && mine) {
    const double rho0 = st->rho;
    const double irho = 1.0 / rho0;
    const int x2 = grow % n2, x3 = grow / n2;
    const int idx = grow * n1 + x1;
    const auto u = global_view(static_cast<const double *>(D.u[st->cur]));
    const auto Eg = global_view(static_cast<T *>(D.E));
    const auto Lg = global_view(static_cast<const T *>(D.Lam));
    const Stencil sn = stencil(n1, n2, n3, x1, x2, x3);
    T E[9], At[9];
    float jw = 0.0f;  // warm_code of the warm start's det F - 1 (closed form)
    if (kFullPass<T, LK, MODE> && LK == 0 && D.At && st->at_rho == rho0) {
      // the update formed this data at this penalty, from the same values,
      // and the warm start's det F - 1 beside it: the closed form does not
      // read F itself
      const auto Ag = global_view(static_cast<const T *>(D.At));
#pragma unroll
      for (int c = 0; c < 9; ++c) At[c] = Ag[c * V + idx];
      if (kClosedOnly<T, LK, MODE>) {
        jw = Ag[9 * V + idx];
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) E[c] = Eg[c * V + idx];
      }
    } else {
      double A[9];
      grad_u(u, V, sn, A);
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        E[c] = Eg[c * V + idx];
        At[c] = (T)(A[c] + st->Ebar[c] + (double)Lg[c * V + idx] * irho);
      }
      if (MODE == kLocalExact) jw = warm_code(warm_jm1(E));
    }
    const auto phg = global_view(D.phase);
    const int ph = phg[idx];
    if (ph < a.n_mat) {
      const Material m = a.mats[ph];
      const int cap = inexact ? ip.local_chunk : ip.newton_max;
      int rc;
      double rho = rho0;
      if (LK == 2 && m.nu_F > 0.0) {
        // dissipation of F: rho/2|F - A|^2 + nu/2|F - F^n|^2 is
        // (rho + nu)/2 |F - (rho A + nu F^n)/(rho + nu)|^2 + const
        const auto Es = global_view(static_cast<const T *>(D.E_step));
        const double nu = m.nu_F / ip.dt, r2 = rho + nu;
#pragma unroll
        for (int c = 0; c < 9; ++c)
          At[c] = (T)((rho * (double)At[c] + nu * (double)Es[c * V + idx]) / r2);
        rho = r2;
      }
      if (LK >= 1 && m.model == 1) {
        const auto dg = global_view(static_cast<T *>(D.dir));
        double n[3] = {(double)dg[idx], (double)dg[V + idx], (double)dg[2 * V + idx]};
        const double nn = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        n[0] *= nn;
        n[1] *= nn;
        n[2] *= nn;
        DirForm form;
        const DirForm *fp = nullptr;
        if (LK == 2 && (m.mual != 0.0 || m.frank != 0.0 || m.nu_n != 0.0)) {
          // the full model's director terms at this voxel
          form.gamma = m.mual / (-m.mua * m.beta);
          form.inv_c = -2.0 / (m.mua * m.beta);
          form.n0[0] = form.n0[1] = form.n0[2] = 0.0;
          if (m.mual != 0.0) {
            const auto d0 = global_view(static_cast<const T *>(D.dir0));
            double q[3] = {(double)d0[idx], (double)d0[V + idx], (double)d0[2 * V + idx]};
            const double qn = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) form.n0[k] = q[k] * qn;
          }
#pragma unroll
          for (int k = 0; k < 6; ++k) form.sc[k] = 0.0;
          if (m.frank != 0.0) {
            // Frank term, neighbours of an LCE phase lagged by one iteration:
            // Sc -= kappa_F sum_y n~(y) n~(y)^T
            const auto lg = global_view(static_cast<const T *>(D.dir_lag));
#pragma unroll
            for (int q = 0; q < 6; ++q) {
              const int y = sn.o[q];
              const int py = phg[y];
              if (py >= a.n_mat || a.mats[py].model != 1) continue;
              const double v0 = (double)lg[y], v1 = (double)lg[V + y], v2 = (double)lg[2 * V + y];
              form.sc[0] -= m.frank * v0 * v0;
              form.sc[1] -= m.frank * v0 * v1;
              form.sc[2] -= m.frank * v0 * v2;
              form.sc[3] -= m.frank * v1 * v1;
              form.sc[4] -= m.frank * v1 * v2;
              form.sc[5] -= m.frank * v2 * v2;
            }
          }
          if (m.nu_n != 0.0) {
            // director dissipation: Sc -= nu_n/(2 dt) n^n n^n^T
            const auto ds = global_view(static_cast<const T *>(D.dir_step));
            const double v0 = (double)ds[idx], v1 = (double)ds[V + idx], v2 = (double)ds[2 * V + idx];
            const double w = 0.5 * m.nu_n / ip.dt;
            form.sc[0] -= w * v0 * v0;
            form.sc[1] -= w * v0 * v1;
            form.sc[2] -= w * v0 * v2;
            form.sc[3] -= w * v1 * v1;
            form.sc[4] -= w * v1 * v2;
            form.sc[5] -= w * v2 * v2;
          }
          fp = &form;
        }
        if (fp) {
          rc = lce_local<T>(E, At, m, rho, n, ip, cap, n_its, fp);
        } else {
          // the ideal model: the local problem in A's singular basis, solved
          // in full also in an inexact pass (the chunk cap would only add
          // passes, each rebuilding the basis)
          const int scap = cap > 100 ? cap : 100;
          rc = lce_spectral<T>(E, At, m.mua, m.beta, m.kappa, m.mu, rho, n, scap, ip.gtol,
                               ip.step_tol);
          n_its += rc >= 0 ? rc : scap;
        }
        dg[idx] = (T)n[0];
        dg[V + idx] = (T)n[1];
        dg[2 * V + idx] = (T)n[2];
        if (inexact && rc != -2) {
          Lce<T> M;
          M.mua = (T)m.mua;
          M.beta = (T)m.beta;
          M.kappa = (T)m.kappa;
          M.mu = (T)m.mu;
          M.mual = (T)m.mual;
          M.form = fp;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            M.n[k] = (T)n[k];
            M.nd[k] = n[k];
          }
          Point<T> sp;
          if (M.point(E, At, (T)rho, sp)) lsum[0] = (double)sp.gn2;
        }
      } else {
        NeoHooke<T> M;
        M.mu = (T)m.mu;
        M.lam = (T)m.lam;
        // exact mode: the minimiser up to one scalar; the nine-component
        // Newton where that form does not apply (in the retry pass when the
        // closed form is compiled alone). In the double form the closed
        // form's point (about 1e-12 relative, least accurate along
        // rotations, where the objective is only rho-stiff and Newton's
        // stopping test would accept it) is finished by one full Newton step.
        rc = -3;
        if (MODE == kLocalExact)
          rc = neo_closed<T>(E, At, jw, m.mu, m.lam, rho, cap, 1e-5);
        if (kClosedOnly<T, LK, MODE>) {
          if (rc == -3) {
            atomicOr(&retry[t >> 5], 1u << (t & 31));
            atomicAdd(&st->n_retry, 1);
            deferred = true;
            rc = 0;
          }
        } else {
          if (!kDefect<T> && rc >= 0) rc = newton_polish<T, T>(E, At, M, (T)rho) ? rc + 1 : -3;
          if (rc == -3)
            rc = newton<T, T>(E, At, M, (T)rho, cap, ip.gtol, ip.step_tol,
                               MODE == kLocalExact || MODE == kLocalRetry ? nullptr : &lsum[0]);
        }
        n_its = rc >= 0 ? rc : cap;
      }
      lsum[1] = rc >= 0 ? 1.0 : 0.0;
      n_fail = rc == -1 && !inexact;  // a pass that ends at its cap is no failure
      if (rc == -2) atomicOr(&st->domain_err, 1);
      if (!deferred) {
        if (kClosedOnly<T, LK, MODE> && rc < 0) {
          // the closed form returned no point: F stays as it was
#pragma unroll
          for (int c = 0; c < 9; ++c) E[c] = Eg[c * V + idx];
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c) Eg[c * V + idx] = E[c];
        }
      }
    } else {
      atomicOr(&st->domain_err, 2);  // invalid phase index
#pragma unroll
      for (int c = 0; c < 9; ++c) E[c] = Eg[c * V + idx];
    }
    // Step 2's field F - A of every voxel this pass settled (the retry pass
    // writes those it takes over)
    if (kDefect<T> && LK <= 1 && D.Q && !deferred) {
      const auto Qg = global_view(static_cast<T *>(D.Q));
#pragma unroll
      for (int c = 0; c < 9; ++c) Qg[c * V + idx] = (T)((double)E[c] - (double)At[c]);
    }
  }
  // (every workgroup of the cell stores the same flag; Step 2 reads it)
  if (kFullPass<T, LK, MODE> && D.Q && t == 0) st->q_cur = 1;
  // local residual of the inexact passes: one sum per workgroup (a fence
  // and arrival counter per workgroup, to let the last one decide, cost
  // more than a separate one-workgroup-per-cell kernel: the agent-scope
  // release writes back the XCD's L2)
  if (inexact) {
    __shared__ double gred[2 * (kThreads / 64)];
    block_sum<2>(lsum, gred);
    if (t == 0) a.lpart[blk] = make_double2(lsum[0], lsum[1]);
    __syncthreads();
  }
  // Newton statistics: summed per workgroup and added to one slot of the
  // update kernel's tiling (atomics from every wave on one address per cell
  // serialised the kernel's tail)
  __shared__ int wsum[2 * (kThreads / 64)];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    n_fail += __shfl_xor(n_fail, off, 64);
    n_its += __shfl_xor(n_its, off, 64);
  }
  const int wave = t >> 6, nw = (blockDim.x + 63) >> 6;
  if ((t & 63) == 0) {
    wsum[wave] = n_fail;
    wsum[nw + wave] = n_its;
  }
  __syncthreads();
  if (t == 0) {
    int f = 0, s = 0;
    for (int w = 0; w < nw; ++w) {
      f += wsum[w];
      s += wsum[nw + w];
    }
    // the update workgroup whose tile holds this workgroup's first line
    // folds the counts into its residual partials (a few workgroups share a
    // slot, so these atomics do not contend)
    const int g = b * R, x2 = g % n2, x3 = g / n2;
    const int slot = a.blk_u[r] + (x3 / kZSeg) * ((n2 + R - 1) / R) + x2 / R;
    if (f) atomicAdd(&a.newton_part[slot].x, f);
    if (s) atomicAdd(&a.newton_part[slot].y, s);
  }
}

// Step 1. The first pass runs one logical workgroup per workgroup; later
// inexact passes, which often find the cell done, run a smaller grid over
// logical workgroups blockIdx.x, blockIdx.x + gridDim.x, ... (a multiple of
// 8 workgroups, so each logical workgroup keeps its XCD). The exact mode
// compiles without the inexact bookkeeping.
template <typename T, int LK, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(ADMM_LOCAL_WAVES_PER_EU)))
void k_local(KernelArgs a, IterParams ip, int pass, int nblk) {
  if (MODE != kLocalLater && MODE != kLocalRetry) {
    local_tile<T, LK, MODE>(a, ip, pass, xcd_remap(blockIdx.x, gridDim.x));
    return;
  }
  if (MODE == kLocalRetry) {
    // nothing left over in any cell (the usual case): one round trip
    __shared__ int any_cell;
    if (threadIdx.x == 0) any_cell = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < a.n_rve; r += blockDim.x)
      if (a.state[r].n_retry) any_cell = 1;
    __syncthreads();
    if (!any_cell) return;
    // this workgroup's logical workgroups are blockIdx.x, blockIdx.x +
    // gridDim.x, ... (as in a later inexact pass); each thread looks at one
    // of them, kThreads per round, and the marked ones are solved one after
    // the other, their bits cleared once every thread has read its own
    __shared__ int list[kThreads];
    __shared__ int cnt;
    for (int k0 = 0; blockIdx.x + k0 * gridDim.x < nblk; k0 += kThreads) {
      if (threadIdx.x == 0) cnt = 0;
      __syncthreads();
      const int lb = blockIdx.x + (k0 + (int)threadIdx.x) * gridDim.x;
      if (lb < nblk) {
        const int blk = xcd_remap(lb, nblk);
        const uint4 *w = reinterpret_cast<const uint4 *>(a.retry_mask + (size_t)blk * (kThreads / 32));
        const uint4 w0 = w[0], w1 = w[1];
        if (w0.x | w0.y | w0.z | w0.w | w1.x | w1.y | w1.z | w1.w) list[atomicAdd(&cnt, 1)] = blk;
      }
      __syncthreads();
      const int n = cnt;
      for (int q = 0; q < n; ++q) {
        const int blk = list[q];
        local_tile<T, LK, MODE>(a, ip, pass, blk);
        __syncthreads();
        if (threadIdx.x < kThreads / 32) a.retry_mask[(size_t)blk * (kThreads / 32) + threadIdx.x] = 0u;
        __syncthreads();
      }
      __syncthreads();  // every thread has read cnt before the next round resets it
    }
    return;
  }
  for (int lb = blockIdx.x; lb < nblk; lb += gridDim.x) {
    const int blk = xcd_remap(lb, nblk);
    local_tile<T, LK, MODE>(a, ip, pass, blk);
    __syncthreads();  // LDS of this tile read before the next one writes it
  }
}

// Frank term: the directors of the previous iteration, copied before Step 1
// so that every local problem sees its neighbours' lagged directors.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lag(KernelArgs a) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_x, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  if (!a.state[r].active || !D.dir_lag) return;
  const int b = blk - a.blk_x[r];
  const int n1 = D.n1, R = D.rows, nrows = D.n2 * D.n3, V = (int)D.V;
  const int row = threadIdx.x / n1, x1 = threadIdx.x - row * n1;
  const int grow = b * R + row;
  if (row >= R || grow >= nrows) return;
  const int idx = grow * n1 + x1;
  const auto src = global_view(static_cast<const T *>(D.dir));
  const auto dst = global_view(static_cast<T *>(D.dir_lag));
#pragma unroll
  for (int k = 0; k < 3; ++k) dst[k * V + idx] = src[k * V + idx];
}

// Orientation tensor: per local workgroup, the sums of n (x) n over its LCE
// voxels (xx xy xz yy yz zz) and their count, then one workgroup per cell
// writes <n (x) n> sums (9) and the count to mean_out.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_orient(KernelArgs a) {
  __shared__ double red[7 * (kThreads / 64)];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_x, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const int b = blk - a.blk_x[r];
  const int n1 = D.n1, R = D.rows, nrows = D.n2 * D.n3, V = (int)D.V;
  const int row = threadIdx.x / n1, x1 = threadIdx.x - row * n1;
  const int grow = b * R + row;
  double v[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = 0.0;
  if (row < R && grow < nrows && D.dir) {
    const int idx = grow * n1 + x1;
    const int ph = global_view(D.phase)[idx];
    if (ph < a.n_mat && a.mats[ph].model == 1) {
      const auto dg = global_view(static_cast<const T *>(D.dir));
      const double n0 = dg[idx], n1v = dg[V + idx], n2v = dg[2 * V + idx];
      v[0] = n0 * n0;
      v[1] = n0 * n1v;
      v[2] = n0 * n2v;
      v[3] = n1v * n1v;
      v[4] = n1v * n2v;
      v[5] = n2v * n2v;
      v[6] = 1.0;
    }
  }
  block_sum<7>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 7; ++k) a.fpart[(size_t)blk * 9 + k] = v[k];
}

__global__ __launch_bounds__(kThreads) void k_orient_final(KernelArgs a) {
  __shared__ double red[7 * (kThreads / 64)];
  const int r = blockIdx.x;
  const int x0 = a.blk_x[r], nx = a.blk_x[r + 1] - x0;
  double v[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = 0.0;
  for (int k = threadIdx.x; k < nx; k += blockDim.x)
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] += a.fpart[(size_t)(x0 + k) * 9 + c];
  block_sum<7>(v, red);
  if (threadIdx.x == 0) {
    double *o = a.mean_out + 18 * (size_t)r;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2];
    o[3] = v[1]; o[4] = v[3]; o[5] = v[4];
    o[6] = v[2]; o[7] = v[4]; o[8] = v[5];
    o[9] = v[6];
  }
}

// Mixed conditions: per local workgroup, the sums of F_{i+1} - I -
// Lambda_i/rho over its voxels (cells with free components of <F> only),
// for k_fbar. A pass of its own, so that the local kernel carries none of it.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fsum(KernelArgs a) {
  __shared__ double red[9 * (kThreads / 64)];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_x, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  if (!st->active || !st->free_mask) return;
  const int b = blk - a.blk_x[r];
  const int n1 = D.n1, R = D.rows, nrows = D.n2 * D.n3;
  const int V = (int)D.V;
  const int t = threadIdx.x;
  const int row = t / n1, x1 = t - row * n1;
  const int grow = b * R + row;
  double h[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) h[c] = 0.0;
  if (row < R && grow < nrows) {
    const auto Eg = global_view(static_cast<const T *>(D.E));
    const auto Lg = global_view(static_cast<const T *>(D.Lam));
    const int idx = grow * n1 + x1;
    const double irho = 1.0 / st->rho;
#pragma unroll
    for (int c = 0; c < 9; ++c) h[c] = (double)Eg[c * V + idx] - (double)Lg[c * V + idx] * irho;
  }
  block_sum<9>(h, red);
  if (t == 0)
#pragma unroll
    for (int c = 0; c < 9; ++c) a.fpart[(size_t)blk * 9 + c] = h[c];
}

// Mixed conditions (Sec. 2.3; the UNI/PE/EB protocols of Sec. 5): Step 2
// minimises over the free components of <F> as well as over u, which gives
// <F>_k = <F_{i+1} - Lambda_i/rho>_k; the multiplier update then keeps
// <Lambda>_k = 0 (zero average stress at convergence). One workgroup per
// cell sums the local workgroups' partials in a fixed order; the previous
// <F> is kept for r_d.
__global__ __launch_bounds__(kThreads) void k_fbar(KernelArgs a) {
  __shared__ double red[9 * (kThreads / 64)];
  const int r = blockIdx.x;
  RveState *st = a.state + r;
  if (!st->active) return;
  const unsigned m = st->free_mask;
  if (!m) return;
  const int x0 = a.blk_x[r], nx = a.blk_x[r + 1] - x0;
  double v[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) v[c] = 0.0;
  for (int k = threadIdx.x; k < nx; k += blockDim.x)
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] += a.fpart[(size_t)(x0 + k) * 9 + c];
  block_sum<9>(v, red);
  if (threadIdx.x == 0) {
    const double V = (double)a.desc[r].V;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      st->Ebar_prev[c] = st->Ebar[c];
      if ((m >> c) & 1u) st->Ebar[c] = v[c] / V;
    }
  }
}

// After inexact pass `pass`, from the workgroups' partial sums (fixed order):
// the ratio strategy takes r_l = RMS |local residual| / mu_ref over the cell
// and ends Step 1 once r_l <= local_ratio r_d (r_d of the previous
// iteration); the fraction strategy once the converged local solves number
// at least local_fraction V. The last pass always ends it. An exact local
// step marks the cell done with r_l = 0.
__global__ __launch_bounds__(kThreads) void k_local_check(KernelArgs a, IterParams ip, int pass) {
  __shared__ double red[2 * (kThreads / 64)];
  const int r = blockIdx.x;
  RveState *st = a.state + r;
  if (!st->active) return;
  if (!local_inexact(ip, st)) {
    if (threadIdx.x == 0) {
      st->local_done = 1;
      st->rl = 0.0;
    }
    return;
  }
  if (pass > 0 && st->local_done) return;
  const int x0 = a.blk_x[r], nx = a.blk_x[r + 1] - x0;
  double v[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < nx; k += blockDim.x) {
    const double2 q = a.lpart[x0 + k];
    v[0] += q.x;
    v[1] += q.y;
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const double Vc = (double)a.desc[r].V;
    const double rl = sqrt(v[0] / Vc) / ip.mu_ref;
    st->rl = rl;
    const bool met = ip.local_fraction > 0.0 ? v[1] >= ip.local_fraction * Vc
                                             : rl <= ip.local_ratio * st->rd;
    st->local_done = (met || pass + 1 >= ip.local_passes) ? 1 : 0;
  }
}

// ----------------------------------------------------------------------------
// b = D_h^T (F - Lambda/rho) and its forward FFT along x1
// ----------------------------------------------------------------------------


template <typename T>
// six waves per SIMD (what its LDS allows at 1024 x1-points): at that budget
// the compiler issues a voxel's 73 loads in two batches rather than four
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_div_fwdx(KernelArgs a) {
  using C = typename cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_f, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  if (!st->active) return;
  const int b = blk - a.blk_f[r];
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows_f, m1 = D.m1, m1s = D.m1s;
  const int nrows = n2 * n3;
  const int row0 = b * R;
  const int ncl = (3 * R + 1) / 2;
  const int V = (int)D.V;
  const long long S = D.S;
  C *za = reinterpret_cast<C *>(smem);
  C *zb = za + ncl * n1;
  const int t = threadIdx.x, nthr = blockDim.x;
  // line rw of this workgroup: its R lines are consecutive along x3 at one x2
  // (so the +-x3 neighbours of the divergence are mostly the workgroup's own
  // lines, the rest those of its neighbours in the chunked order) when R
  // divides n3, else consecutive rows
  const bool colmode = n3 % R == 0;
  int x2b = 0, zc = 0;
  if (colmode) chunk_order(b, n2, n3 / R, x2b, zc);
  auto row_of = [&](int rw) { return colmode ? (zc * R + rw) * n2 + x2b : b * R + rw; };

  for (int w = t; w < ncl * n1; w += nthr) za[w] = C{(T)0, (T)0};
  __syncthreads();
  const double irho = 1.0 / st->rho;
  for (int v = t; v < R * n1; v += nthr) {
    const int row = fdiv(v, D.f_n1), x1 = v - row * n1;
    if (row0 + row >= nrows) continue;
    const int grow = row_of(row);
    const int x3 = fdiv(grow, D.f_n2), x2 = grow - x3 * n2;
    const Stencil sn = stencil(n1, n2, n3, x1, x2, x3);
    const T *Eg = static_cast<const T *>(D.E);
    const T *Lg = static_cast<const T *>(D.Lam);
    // float form: the defect D_h^T (H - D_h u_i), in double, whose solve is
    // the correction u_{i+1} - u_i (the transforms' float rounding then
    // scales with the correction, not with u itself). With Step 1's data
    // A = I + D_h u_i + Ebar + Lambda/rho, H - D_h u_i = F - A + Ebar, and
    // D_h^T of the constant Ebar vanishes: where the local step of this
    // iteration left Q = F - A, the defect is D_h^T Q.
    if (kDefect<T> && D.Q && st->q_cur) {
      const T *Qg = static_cast<const T *>(D.Q);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double bi = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const int c = (3 * i + j) * V;
          bi -= 0.5 * ((double)Qg[c + sn.o[2 * j]] - (double)Qg[c + sn.o[2 * j + 1]]);
        }
        const int ell = i * R + row;
        T *z = reinterpret_cast<T *>(za + (ell >> 1) * n1 + x1) + (ell & 1);
        *z = (T)bi;
      }
      continue;
    }
    // else D_h^T D_h u_i = -sum_j (u_i(x + 2 e_j) - 2 u_i(x) + u_i(x - 2 e_j)) / 4
    int o2[6];
    if (kDefect<T>) {
      const int y2 = wrap_plus2(x2, n2), ym = wrap_minus2(x2, n2);
      const int z2 = wrap_plus2(x3, n3), zm = wrap_minus2(x3, n3);
      const int x1p = wrap_plus2(x1, n1), x1m = wrap_minus2(x1, n1);
      const int rw0 = (x3 * n2 + x2) * n1;
      o2[0] = rw0 + x1p;
      o2[1] = rw0 + x1m;
      o2[2] = (x3 * n2 + y2) * n1 + x1;
      o2[3] = (x3 * n2 + ym) * n1 + x1;
      o2[4] = (z2 * n2 + x2) * n1 + x1;
      o2[5] = (zm * n2 + x2) * n1 + x1;
    }
    const double *ug = static_cast<const double *>(D.u[st->cur]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double bi = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int c = (3 * i + j) * V;
        const double hp = (double)Eg[c + sn.o[2 * j]] - (double)Lg[c + sn.o[2 * j]] * irho;
        const double hm =
            (double)Eg[c + sn.o[2 * j + 1]] - (double)Lg[c + sn.o[2 * j + 1]] * irho;
        bi -= 0.5 * (hp - hm);
      }
      if (kDefect<T>) {
        const double *ui = ug + i * V;
        const double u0 = ui[grow * n1 + x1];
        double lap = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) lap += (ui[o2[2 * j]] - u0) + (ui[o2[2 * j + 1]] - u0);
        bi += 0.25 * lap;
      }
      // line ell packs into the real or imaginary part of complex line
      // ell / 2; the part is selected by address, not by a branch, so that
      // the three components' loads share one basic block and are issued
      // together
      const int ell = i * R + row;
      T *z = reinterpret_cast<T *>(za + (ell >> 1) * n1 + x1) + (ell & 1);
      *z = (T)bi;
    }
  }
  __syncthreads();
  const C *tw = static_cast<const C *>(a.tw);
  C *res = fft_lines<false>(za, zb, D.p1, tw, ncl, n1, 1, false, t, nthr);
  C *spec = static_cast<C *>(D.spec);
  for (int w = t; w < ncl * m1; w += nthr) {
    const int p = fdiv(w, D.f_m1), m = w - p * m1;
    const C Zm = res[p * n1 + m];
    const C Zn = res[p * n1 + (m == 0 ? 0 : n1 - m)];
    const C Av = C{(T)0.5 * (Zm.x + Zn.x), (T)0.5 * (Zm.y - Zn.y)};
    const C Bv = C{(T)0.5 * (Zm.y + Zn.y), (T)(-0.5) * (Zm.x - Zn.x)};
    const int la = 2 * p, lb = 2 * p + 1;
    {
      const int c = fdiv(la, D.f_rows_f), rw = la - c * R;
      if (row0 + rw < nrows) spec[c * S + (long long)row_of(rw) * m1s + m] = Av;
    }
    if (lb < 3 * R) {
      const int c = fdiv(lb, D.f_rows_f), rw = lb - c * R;
      if (row0 + rw < nrows) spec[c * S + (long long)row_of(rw) * m1s + m] = Bv;
    }
  }
}

// ----------------------------------------------------------------------------
// FFT along x2 of the three spectral components (blockIdx.y = component)
// ----------------------------------------------------------------------------

template <typename T, int B, bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_y(KernelArgs a) {
  using C = typename cplx<T>::type;
  constexpr int PMAX = (kMaxN * B) / kThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_y, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  if (!a.state[r].active) return;
  const int b = blk - a.blk_y[r];
  const int n2 = D.n2, m1 = D.m1, m1s = D.m1s;
  const int nty = (m1 + B - 1) / B;
  const int x3 = b / nty, m0 = (b - x3 * nty) * B;
  C *base = static_cast<C *>(D.spec) + blockIdx.y * D.S + (long long)x3 * n2 * m1s;
  C *za = reinterpret_cast<C *>(smem);
  C *zb = za + n2 * B;
  const int t = threadIdx.x, nthr = blockDim.x;
  const int npts = n2 * B;
  // every load of the tile in flight before the first LDS store
  C v[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    const int x2 = w / B, bb = w - x2 * B;
    v[k] = (w < npts && m0 + bb < m1) ? base[x2 * m1s + m0 + bb] : C{(T)0, (T)0};
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) za[w] = v[k];
  }
  __syncthreads();
  const C *tw = static_cast<const C *>(a.tw);
  C *res = fft_lines<INV>(za, zb, D.p2, tw, B, 1, B, true, t, nthr);
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) v[k] = res[w];
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    const int x2 = w / B, bb = w - x2 * B;
    if (w < npts && m0 + bb < m1) base[x2 * m1s + m0 + bb] = v[k];
  }
}

// ----------------------------------------------------------------------------
// FFT along x3, Poisson solve in Fourier space, inverse FFT along x3
// (blockIdx.y = component)
// ----------------------------------------------------------------------------

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_poisson_z(KernelArgs a) {
  using C = typename cplx<T>::type;
  constexpr int PMAX = (kMaxN * B) / kThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_z, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  if (!a.state[r].active) return;
  const int b = blk - a.blk_z[r];
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, m1 = D.m1, m1s = D.m1s;
  const int plane = n2 * m1s;  // stride between x3 planes (padding columns included)
  const int q0 = b * B;
  const int npts = n3 * B;
  C *base = static_cast<C *>(D.spec) + blockIdx.y * D.S + q0;
  const C *tw = static_cast<const C *>(a.tw);
  C *za = reinterpret_cast<C *>(smem);
  C *zb = za + n3 * B;
  const int t = threadIdx.x, nthr = blockDim.x;
  C v[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    const int x3 = w / B, bb = w - x3 * B;
    v[k] = (w < npts && q0 + bb < plane) ? base[x3 * plane + bb] : C{(T)0, (T)0};
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) za[w] = v[k];
  }
  __syncthreads();
  C *res = fft_lines<false>(za, zb, D.p3, tw, B, 1, B, true, t, nthr);
  // u_hat = b_hat / (|K|^2 V); zero where every K_j vanishes
  const double iV = 1.0 / (double)D.V;
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) {
      const int m3 = w / B, bb = w - m3 * B;
      int q = q0 + bb;
      if (q >= plane) q = 0;
      const int m2 = q / m1s, mm1 = q - m2 * m1s;
      const bool pad = mm1 >= m1;  // padding column: stays zero
      const double K1 = (double)tw[D.p1.tw + (pad ? 0 : mm1)].y;
      const double K2 = (double)tw[D.p2.tw + m2].y;
      const double K3 = (double)tw[D.p3.tw + m3].y;
      const bool null = pad || ((mm1 == 0 || 2 * mm1 == n1) && (m2 == 0 || 2 * m2 == n2) &&
                                (m3 == 0 || 2 * m3 == n3));
      const T s = null ? (T)0 : (T)(iV / (K1 * K1 + K2 * K2 + K3 * K3));
      const C h = res[w];
      v[k] = C{h.x * s, h.y * s};
    }
  }
  // res is one of the two buffers and every thread has read what it needs
  // from it; the scaled values go to the other one
  C *dst = (res == za) ? zb : za;
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) dst[w] = v[k];
  }
  __syncthreads();
  res = fft_lines<true>(dst, res, D.p3, tw, B, 1, B, true, t, nthr);
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    if (w < npts) v[k] = res[w];
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const int w = t + k * nthr;
    const int x3 = w / B, bb = w - x3 * B;
    if (w < npts && q0 + bb < plane) base[x3 * plane + bb] = v[k];
  }
}

// ----------------------------------------------------------------------------
// x2 and x3 passes of length 256 at the tile width kTileCol16, register
// resident (k_col16; where a float launch also holds shorter lengths it is
// k_colreg below, which covers 256 the same way): a workgroup takes 16 columns (flattened over the cell's (x3, m1)
// for x2, (m2, m1) for x3, padding columns excluded); thread (c, j) =
// (t % 16, t / 16) holds elements j + 16 r (r = 0..15) of column c. With
// n = j + 16 r and k = 16 k1 + k2,
//     X[16 k1 + k2] = sum_j w16^(j k1) w256^(j k2) sum_r x[j + 16 r] w16^(r k2):
// a length-16 DFT over r in registers, the twiddle w256^(j k2), one exchange
// through LDS (thread (c, j) then holds k2 = j for every j'), a length-16 DFT
// over j'. Thread (c, j) ends with X[j + 16 k1], k1 = 0..15: the layout it
// loaded, so results go back in place and an inverse transform can follow.
// ----------------------------------------------------------------------------

// LDS slab of one k2 (16 x 16 values) padded by 8 values in float, so that
// the 4 rows a wave reads in the exchange fall in different banks (64 KiB
// without padding in double)
template <typename C> constexpr int col16_slab() { return sizeof(C) == 8 ? 264 : 256; }
template <typename C> constexpr size_t col16_lds() { return 16 * col16_slab<C>() * sizeof(C); }

// The exchange buffer holds a slab of SL values per k2; within it the value of
// (line c, point j) sits at c * 16 + j when JFAST (consecutive lanes take
// consecutive points), else at j * 16 + c (consecutive lanes take
// consecutive lines).
template <bool INV, int SL, bool JFAST, typename C>
__device__ __forceinline__ void col256(C *v, C *X, const C *__restrict__ tw, int c, int j) {
  dft16<INV>(v);
#pragma unroll
  for (int k2 = 1; k2 < 16; ++k2) {
    const C w = tw[j * k2];  // j k2 <= 225
    v[k2] = INV ? cmulc(v[k2], w) : cmul(v[k2], w);
  }
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) X[k2 * SL + (JFAST ? c * 16 + j : j * 16 + c)] = v[k2];
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) v[jj] = X[j * SL + (JFAST ? c * 16 + jj : jj * 16 + c)];
  dft16<INV>(v);
}

// MODE 0: x2 forward, 1: x2 inverse, 2: x3 forward, u_hat = b_hat/(|K|^2 V),
// x3 inverse (blockIdx.y = component)
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_col16(KernelArgs a) {
  using C = typename cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C *X = reinterpret_cast<C *>(smem);
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int *tab = MODE == 2 ? a.blk_z : a.blk_y;
  const int r = find_rve(tab, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  if (!a.state[r].active) return;
  const int b = blk - tab[r];
  const int n2 = D.n2, m1 = D.m1, m1s = D.m1s;
  const int t = threadIdx.x, c = t & 15, j = t >> 4;
  const int ncol = (MODE == 2 ? n2 : D.n3) * m1;
  const int g = b * 16 + c;
  const bool ok = g < ncol;
  const int outer = ok ? g / m1 : 0, q = ok ? g - outer * m1 : 0;
  // x2: column (x3 = outer, m1 = q), elements m1s apart; x3: column
  // (m2 = outer, m1 = q), elements one plane (n2 m1s) apart
  const long long es = MODE == 2 ? (long long)n2 * m1s : (long long)m1s;
  C *col = static_cast<C *>(D.spec) + blockIdx.y * D.S +
           (MODE == 2 ? (long long)outer * m1s : (long long)outer * n2 * m1s) + q;
  const C *tw = static_cast<const C *>(a.tw);
  const C *tw256 = tw + (MODE == 2 ? D.p3.tw : D.p2.tw);
  C v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = ok ? col[(j + 16 * k) * es] : C{(T)0, (T)0};
  col256<MODE == 1, col16_slab<C>(), false>(v, X, tw256, c, j);
  if (MODE == 2) {
    // thread (c, j) holds m3 = j + 16 k1
    const double iV = 1.0 / (double)D.V;
    const double K1 = (double)tw[D.p1.tw + q].y;
    const double K2 = (double)tw[D.p2.tw + outer].y;
    const double K12 = K1 * K1 + K2 * K2;
    const bool null12 = (q == 0 || 2 * q == D.n1) && (outer == 0 || 2 * outer == n2);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int m3 = j + 16 * k;
      const double K3 = (double)tw256[m3].y;
      const bool null = !ok || (null12 && (m3 == 0 || 2 * m3 == 256));
      const T s = null ? (T)0 : (T)(iV / (K12 + K3 * K3));
      v[k] = C{v[k].x * s, v[k].y * s};
    }
    __syncthreads();  // every thread has read the exchange buffer
    col256<true, col16_slab<C>(), false>(v, X, tw256, c, j);
  }
  if (ok) {
#pragma unroll
    for (int k = 0; k < 16; ++k) col[(j + 16 * k) * es] = v[k];
  }
}

// ----------------------------------------------------------------------------
// inverse complex-to-real FFT along x1 into u_{i+1}
// ----------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_inv_x(KernelArgs a) {
  using C = typename cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_f, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  if (!st->active) return;
  const int b = blk - a.blk_f[r];
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows_f;
  const int nrows = n2 * n3;
  const int row0 = b * R;
  const int ncl = (3 * R + 1) / 2;
  const int V = (int)D.V;
  const long long S = D.S;
  const C *spec = static_cast<const C *>(D.spec);
  C *za = reinterpret_cast<C *>(smem);
  C *zb = za + ncl * n1;
  const int t = threadIdx.x, nthr = blockDim.x;
  const int h = n1 / 2;

  // Z[k] = A[k] + i B[k] over the full length from the half spectra of the
  // two real lines (A, B Hermitian; DC and Nyquist taken as real)
  for (int w = t; w < ncl * n1; w += nthr) {
    const int p = fdiv(w, D.f_n1), k = w - p * n1;
    const int kk = k <= h ? k : n1 - k;
    C Av = C{(T)0, (T)0}, Bv = C{(T)0, (T)0};
    const int la = 2 * p, lb = 2 * p + 1;
    {
      const int c = fdiv(la, D.f_rows_f), rw = la - c * R;
      if (row0 + rw < nrows) Av = spec[c * S + (long long)(row0 + rw) * D.m1s + kk];
    }
    if (lb < 3 * R) {
      const int c = fdiv(lb, D.f_rows_f), rw = lb - c * R;
      if (row0 + rw < nrows) Bv = spec[c * S + (long long)(row0 + rw) * D.m1s + kk];
    }
    if (kk == 0 || kk == h) {
      Av.y = (T)0;
      Bv.y = (T)0;
    }
    if (k > h) {
      Av.y = -Av.y;
      Bv.y = -Bv.y;
    }
    za[w] = C{Av.x - Bv.y, Av.y + Bv.x};
  }
  __syncthreads();
  const C *tw = static_cast<const C *>(a.tw);
  C *res = fft_lines<true>(za, zb, D.p1, tw, ncl, n1, 1, false, t, nthr);
  // double form: u_{i+1}; float form: the correction u_{i+1} - u_i
  T *un = kDefect<T> ? static_cast<T *>(D.du) : static_cast<T *>(D.u[1 - st->cur]);
  for (int w = t; w < 3 * R * n1; w += nthr) {
    const int ell = fdiv(w, D.f_n1), x1 = w - ell * n1;
    const int c = fdiv(ell, D.f_rows_f), rw = ell - c * R;
    const int grow = row0 + rw;
    if (grow < nrows) {
      const C v = res[(ell >> 1) * n1 + x1];
      un[c * V + grow * n1 + x1] = (ell & 1) ? v.y : v.x;
    }
  }
}

// Register-resident x2 / x3 passes in float for the lengths 32, 48, 64, 96,
// 128 and 256 (cells of different lengths in one launch, each workgroup in
// one cell): a length N = T P is taken by T threads per column, P points each;
// a workgroup takes 256 / T columns. Thread (c, j) loads points j + T r
// (r < P) of column c; with n = j + T r and k = k2 + P k1,
//     X[P k1 + k2] = sum_j w_T^(j k1) w_N^(j k2) sum_r x[j + T r] w_P^(r k2):
// a length-P DFT in registers, the twiddle w_N^(j k2), one exchange through
// LDS, and thread (c, j) then takes the k2 = j + T q (q < P / T), each a
// length-T DFT over the T threads' values. It ends with X[j + T r'],
// r' = q + (P / T) k1: the layout it loaded (T divides P), so results go
// back in place and the x3 pass's inverse transform follows in registers.
__host__ __device__ constexpr int colreg_points(int n) {
  return (n == 32 || n == 64 || n == 128 || n == 256) ? 16 : (n == 48 ? 12 : (n == 96 ? 24 : 0));
}
// LDS slab of one k2: T x (256 / T) = 256 values padded by 8 (the rows a wave
// reads in the exchange fall in different banks)
constexpr int kColSlab = 264;

template <bool INV, int TT, int P>
__device__ __forceinline__ void colreg(float2 *v, float2 *X, const float2 *__restrict__ tw,
                                       int c, int j) {
  constexpr int CW = kThreads / TT;
  dftR<P, INV>(v);
#pragma unroll
  for (int k2 = 1; k2 < P; ++k2) {
    const float2 w = tw[j * k2];  // j k2 < N
    v[k2] = INV ? cmulc(v[k2], w) : cmul(v[k2], w);
  }
#pragma unroll
  for (int k2 = 0; k2 < P; ++k2) X[k2 * kColSlab + j * CW + c] = v[k2];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < P / TT; ++q) {
    float2 z[TT];
#pragma unroll
    for (int jj = 0; jj < TT; ++jj) z[jj] = X[(j + TT * q) * kColSlab + jj * CW + c];
    dftR<TT, INV>(z);
#pragma unroll
    for (int k1 = 0; k1 < TT; ++k1) v[q + (P / TT) * k1] = z[k1];
  }
}

// one workgroup's columns of one cell; MODE as k_col16
template <int MODE, int TT, int P>
__device__ __forceinline__ void colreg_tile(const KernelArgs &a, const RveDesc &D, int b,
                                            float2 *X) {
  constexpr int CW = kThreads / TT, N = TT * P;
  const int t = threadIdx.x, c = t % CW, j = t / CW;
  const int n2 = D.n2, m1 = D.m1, m1s = D.m1s;
  const int ncol = (MODE == 2 ? n2 : D.n3) * m1;
  const int g = b * CW + c;
  const bool ok = g < ncol;
  const int outer = ok ? g / m1 : 0, q = ok ? g - outer * m1 : 0;
  const long long es = MODE == 2 ? (long long)n2 * m1s : (long long)m1s;
  float2 *col = static_cast<float2 *>(D.spec) + blockIdx.y * D.S +
                (MODE == 2 ? (long long)outer * m1s : (long long)outer * n2 * m1s) + q;
  const float2 *tw = static_cast<const float2 *>(a.tw);
  const float2 *twN = tw + (MODE == 2 ? D.p3.tw : D.p2.tw);
  float2 v[P];
#pragma unroll
  for (int r = 0; r < P; ++r) v[r] = ok ? col[(j + TT * r) * es] : float2{0.0f, 0.0f};
  colreg<MODE == 1, TT, P>(v, X, twN, c, j);
  if (MODE == 2) {
    // thread (c, j) holds m3 = j + TT r
    const double iV = 1.0 / (double)D.V;
    const double K1 = (double)tw[D.p1.tw + q].y;
    const double K2 = (double)tw[D.p2.tw + outer].y;
    const double K12 = K1 * K1 + K2 * K2;
    const bool null12 = (q == 0 || 2 * q == D.n1) && (outer == 0 || 2 * outer == n2);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int m3 = j + TT * r;
      const double K3 = (double)twN[m3].y;
      const bool null = !ok || (null12 && (m3 == 0 || 2 * m3 == N));
      const float s = null ? 0.0f : (float)(iV / (K12 + K3 * K3));
      v[r] = float2{v[r].x * s, v[r].y * s};
    }
    __syncthreads();  // every thread has read the exchange buffer
    colreg<true, TT, P>(v, X, twN, c, j);
  }
  if (ok) {
#pragma unroll
    for (int r = 0; r < P; ++r) col[(j + TT * r) * es] = v[r];
  }
}

// MODE 0: x2 forward, 1: x2 inverse, 2: x3 forward, u_hat = b_hat/(|K|^2 V),
// x3 inverse (blockIdx.y = component). PMAX: the most points per thread any
// cell of the launch needs; the length 96 (24 points) is compiled only into
// the PMAX = 24 kernel, so the others keep the registers of 16 points.
template <int MODE, int PMAX>
__global__ __launch_bounds__(kThreads) void k_colreg(KernelArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  float2 *X = reinterpret_cast<float2 *>(smem);
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int *tab = MODE == 2 ? a.blk_z : a.blk_y;
  const int r = find_rve(tab, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  if (!a.state[r].active) return;
  const int b = blk - tab[r];
  switch (MODE == 2 ? D.n3 : D.n2) {  // uniform over the workgroup
    case 32: colreg_tile<MODE, 2, 16>(a, D, b, X); break;
    case 48: colreg_tile<MODE, 4, 12>(a, D, b, X); break;
    case 64: colreg_tile<MODE, 4, 16>(a, D, b, X); break;
    case 96:
      if constexpr (PMAX == 24) colreg_tile<MODE, 4, 24>(a, D, b, X);
      break;
    case 128: colreg_tile<MODE, 8, 16>(a, D, b, X); break;
    default: colreg_tile<MODE, 16, 16>(a, D, b, X); break;  // 256
  }
}

// Inverse complex-to-real transforms along x1 of length 256 in float,
// register resident. The cell's 3 n2 n3 real output lines, ordered
// (component, row), go 32 to a workgroup as 16 complex lines (lines 2p and
// 2p + 1 as the real and imaginary parts, the same pairing as k_inv_x).
// Thread (p, j) = (t / 16, t % 16) loads points j + 16 r of complex line p
// from the two half spectra (completed by Hermitian symmetry; the 16 threads
// of a line read consecutive entries), runs the length-256 transform of the
// x2 / x3 passes (col256, one exchange through LDS) and stores x1 = j + 16 k1
// of both real lines (64 consecutive bytes per line and store).
// exchange slab stride 257: the lanes of a wave, 16 points of 4 lines, fall
// in different banks both when they write and when they read the exchange
constexpr int kInvSlab = 257;
constexpr size_t kInvLds = 16 * kInvSlab * sizeof(float2);

__global__ __launch_bounds__(kThreads) void k_inv_x256(KernelArgs a) {
  using C = float2;
  extern __shared__ __align__(16) unsigned char smem[];
  C *X = reinterpret_cast<C *>(smem);
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_i, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  if (!st->active) return;
  const int b = blk - a.blk_i[r];
  const int nrows = D.n2 * D.n3, nl = 3 * nrows, m1s = D.m1s;
  const int V = (int)D.V;
  const long long S = D.S;
  const int t = threadIdx.x, p = t >> 4, j = t & 15;
  const int LA = b * 32 + 2 * p, LB = LA + 1;
  const bool okA = LA < nl, okB = LB < nl;
  const int cA = LA >= 2 * nrows ? 2 : (LA >= nrows ? 1 : 0), rA = LA - cA * nrows;
  const int cB = LB >= 2 * nrows ? 2 : (LB >= nrows ? 1 : 0), rB = LB - cB * nrows;
  const C *spec = static_cast<const C *>(D.spec);
  const C *sA = spec + cA * S + (long long)rA * m1s;
  const C *sB = spec + cB * S + (long long)rB * m1s;
  C v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = j + 16 * q;
    const int kk = k <= 128 ? k : 256 - k;
    C Av = okA ? sA[kk] : C{0.0f, 0.0f}, Bv = okB ? sB[kk] : C{0.0f, 0.0f};
    if (kk == 0 || kk == 128) {
      Av.y = 0.0f;
      Bv.y = 0.0f;
    }
    if (k > 128) {
      Av.y = -Av.y;
      Bv.y = -Bv.y;
    }
    v[q] = C{Av.x - Bv.y, Av.y + Bv.x};
  }
  const C *tw = static_cast<const C *>(a.tw) + D.p1.tw;
  col256<true, kInvSlab, true>(v, X, tw, p, j);
  float *du = static_cast<float *>(D.du);
  float *oA = du + cA * V + rA * 256, *oB = du + cB * V + rB * 256;
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) {
    if (okA) oA[j + 16 * k1] = v[k1].x;
    if (okB) oB[j + 16 * k1] = v[k1].y;
  }
}

// The fluctuation's components that D_h does not see: the mean and the
// Nyquist checkerboards chi_s(x) = (-1)^(s1 k1 + s2 k2 + s3 k3), s in {0,1}^3
// (s3 = 0 only when n3 = 1). Step 2 in the double form returns u without
// them; the float form adds corrections to u_i and would keep whatever u_i
// holds, so each call of the float form first removes them from u:
// k_null_sums (per update workgroup, the 24 sums of u_i chi_s), k_null_final
// (per cell, fixed order, coefficients / V), k_null_sub.
__device__ __forceinline__ double chi(int s, int k1, int k2, int k3) {
  const int e = ((s & 1) ? k1 : 0) + ((s & 2) ? k2 : 0) + ((s & 4) ? k3 : 0);
  return (e & 1) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(kThreads) void k_null_sums(KernelArgs a) {
  __shared__ double red[24 * (kThreads / 64)];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_u, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  const int b = blk - a.blk_u[r];
  const int V = (int)D.V, n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows;
  const double *u = static_cast<const double *>(D.u[st->cur]);
  const int t = threadIdx.x, row = t / n1, x1 = t - row * n1;
  int x2, z0;
  column_tile(D, b, row, x2, z0);
  double v[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = 0.0;
  for (int k = 0; k < kZSeg; ++k) {
    const int x3 = z0 + k;
    if (row >= R || x2 >= n2 || x3 >= n3) continue;
    const int idx = (x3 * n2 + x2) * n1 + x1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ui = u[i * V + idx];
#pragma unroll
      for (int sgn = 0; sgn < 8; ++sgn) v[8 * i + sgn] += ui * chi(sgn, x1, x2, x3);
    }
  }
  block_sum<24>(v, red);
  if (t == 0)
#pragma unroll
    for (int k = 0; k < 24; ++k) a.nullpart[(size_t)blk * 24 + k] = v[k];
}

__global__ __launch_bounds__(kThreads) void k_null_final(KernelArgs a) {
  __shared__ double red[24 * (kThreads / 64)];
  const int r = blockIdx.x;
  const int p0 = a.blk_u[r], nb = a.blk_u[r + 1] - p0;
  double v[24];
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x)
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] += a.nullpart[(size_t)(p0 + q) * 24 + k];
  block_sum<24>(v, red);
  if (threadIdx.x == 0) {
    const RveDesc &D = a.desc[r];
    const double iV = 1.0 / (double)D.V;
#pragma unroll
    for (int k = 0; k < 24; ++k)  // with n3 = 1 the patterns with s3 = 1 repeat s3 = 0
      a.nullc[(size_t)r * 24 + k] = (D.n3 == 1 && (k & 4)) ? 0.0 : v[k] * iV;
  }
}

__global__ __launch_bounds__(kThreads) void k_null_sub(KernelArgs a) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_u, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  const int b = blk - a.blk_u[r];
  const int V = (int)D.V, n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows;
  double *u = static_cast<double *>(D.u[st->cur]);
  const double *c = a.nullc + (size_t)r * 24;
  const int t = threadIdx.x, row = t / n1, x1 = t - row * n1;
  int x2, z0;
  column_tile(D, b, row, x2, z0);
  for (int k = 0; k < kZSeg; ++k) {
    const int x3 = z0 + k;
    if (row >= R || x2 >= n2 || x3 >= n3) continue;
    const int idx = (x3 * n2 + x2) * n1 + x1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double w = 0.0;
#pragma unroll
      for (int sgn = 0; sgn < 8; ++sgn) w += c[8 * i + sgn] * chi(sgn, x1, x2, x3);
      u[i * V + idx] -= w;
    }
  }
}

// float form, single Step 2 call (admm_project_step): u_prev = u + du, so
// that the call leaves u_{i+1} where the double form leaves it
template <typename T>
__global__ __launch_bounds__(kThreads) void k_compose_u(KernelArgs a) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_x, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const RveState *st = a.state + r;
  if (!st->active || !D.du) return;
  const int b = blk - a.blk_x[r];
  const int n1 = D.n1, R = D.rows, nrows = D.n2 * D.n3, V = (int)D.V;
  const int row = threadIdx.x / n1, x1 = threadIdx.x - row * n1;
  const int grow = b * R + row;
  if (row >= R || grow >= nrows) return;
  const int idx = grow * n1 + x1;
  const double *uo = static_cast<const double *>(D.u[st->cur]);
  double *un = static_cast<double *>(D.u[1 - st->cur]);
  const T *du = static_cast<const T *>(D.du);
#pragma unroll
  for (int i = 0; i < 3; ++i) un[i * V + idx] = uo[i * V + idx] + (double)du[i * V + idx];
}

// ----------------------------------------------------------------------------
// Step 3 + partial sums of Step 4, walking x3. A workgroup owns R x1-lines
// (one x2 group, every x1) on kZSeg consecutive planes and takes the planes
// in x3 order. Step 3 needs the central-difference gradients of two 3-vector
// fields: double form, u_{i+1} and u_i; float form, u_{i+1} = u_i + du
// (formed in double as it is stored) and du. Each thread keeps both at its
// voxel on the planes x3 - 1, x3 and x3 + 1 in registers, so a plane is read
// once (and one more at either end of the segment) instead of once for each
// of its +-x3 neighbours; the +-x1 neighbours come from the plane's lines in
// LDS; the +-x2 neighbours are the lines the workgroups of the adjacent x2
// groups read for themselves at about the same time (the x2 group runs
// fastest in the workgroup order).
// ----------------------------------------------------------------------------

// both fields at one voxel: a (double) and b (the float form keeps du in T)
template <typename T> struct UPair {
  double a[3];
  T b[3];
};

template <typename T>
__device__ __forceinline__ void load_pair(const RveDesc &D, const RveState *st, int V, int idx,
                                          UPair<T> &p) {
  const auto uo = global_view(static_cast<const double *>(D.u[st->cur]));
  if (kDefect<T>) {
    const auto dug = global_view(static_cast<const T *>(D.du));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p.b[i] = dug[i * V + idx];
      p.a[i] = uo[i * V + idx] + (double)p.b[i];
    }
  } else {
    const auto un = global_view(static_cast<const double *>(D.u[1 - st->cur]));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p.a[i] = un[i * V + idx];
      p.b[i] = (T)uo[i * V + idx];
    }
  }
}

// the workgroup's residual partials and the Newton statistics the local
// step's workgroups left in its slot (plus `f`, `sm`)
__device__ __forceinline__ void store_partials(KernelArgs &a, int blk, double *v, int f, int sm) {
  __shared__ double red[2 * (kThreads / 64)];
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    const int2 q = a.newton_part[blk];
    a.newton_part[blk] = int2{0, 0};
    a.partials[blk] = double4{v[0], v[1], (double)(q.x + f), (double)(q.y + sm)};
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(KernelArgs a) {
  __shared__ double lineA[2][3][kThreads];
  __shared__ T lineB[2][3][kThreads];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_u, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  RveState *st = a.state + r;
  if (!st->active) return;
  const int b = blk - a.blk_u[r];
  const int V = (int)D.V;
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows;
  const auto Eg = global_view(static_cast<const T *>(D.E));
  const auto Lg = global_view(static_cast<T *>(D.Lam));
  const auto un = global_view(static_cast<double *>(D.u[1 - st->cur]));
  const auto Ag = D.At ? global_view(static_cast<T *>(D.At)) : nullptr;
  const int t = threadIdx.x;
  const int row = t / n1, x1 = t - row * n1;
  int x2, z0;
  column_tile(D, b, row, x2, z0);
  const int nz = min(kZSeg, n3 - z0);  // uniform over the workgroup
  const bool act = row < R && x2 < n2;
  const int x2p = x2 + 1 >= n2 ? 0 : x2 + 1, x2m = x2 == 0 ? n2 - 1 : x2 - 1;
  const int l1p = row * n1 + (x1 + 1 == n1 ? 0 : x1 + 1);
  const int l1m = row * n1 + (x1 == 0 ? n1 - 1 : x1 - 1);
  const double rho = st->rho, irho = 1.0 / rho;
  UPair<T> pm, pc, pp;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    pc.a[i] = 0.0;
    pc.b[i] = (T)0;
  }
  if (act) {
    load_pair<T>(D, st, V, ((z0 == 0 ? n3 - 1 : z0 - 1) * n2 + x2) * n1 + x1, pm);
    load_pair<T>(D, st, V, (z0 * n2 + x2) * n1 + x1, pc);
  }
  double v[2] = {0.0, 0.0};
  for (int k = 0; k < nz; ++k) {
    const int x3 = z0 + k, buf = k & 1;
    // plane x3's lines for the +-x1 neighbours (two buffers: the one
    // written here was last read two planes ago, before the barrier that
    // every thread has since passed)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lineA[buf][i][t] = pc.a[i];
      lineB[buf][i][t] = pc.b[i];
    }
    __syncthreads();
    if (!act) continue;
    const int idx = (x3 * n2 + x2) * n1 + x1;
    // every load of the plane before its first store (a store may alias a
    // later load as far as the compiler knows)
    load_pair<T>(D, st, V, ((x3 + 1 == n3 ? 0 : x3 + 1) * n2 + x2) * n1 + x1, pp);
    UPair<T> q2p, q2m;
    load_pair<T>(D, st, V, (x3 * n2 + x2p) * n1 + x1, q2p);
    load_pair<T>(D, st, V, (x3 * n2 + x2m) * n1 + x1, q2m);
    T E[9], L[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      E[c] = Eg[c * V + idx];
      L[c] = Lg[c * V + idx];
    }
    // component c = 3 i + j: Dn = grad u_{i+1}, Dd its change over the
    // iteration (float form: grad du; double form: grad u_{i+1} - grad u_i)
    T lam[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ap[3] = {lineA[buf][i][l1p], q2p.a[i], pp.a[i]};
      const double am[3] = {lineA[buf][i][l1m], q2m.a[i], pm.a[i]};
      const double bp[3] = {(double)lineB[buf][i][l1p], (double)q2p.b[i], (double)pp.b[i]};
      const double bm[3] = {(double)lineB[buf][i][l1m], (double)q2m.b[i], (double)pm.b[i]};
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int c = 3 * i + j;
        const double Dn = 0.5 * (ap[j] - am[j]);
        const double gb = 0.5 * (bp[j] - bm[j]);
        const double Dd = kDefect<T> ? gb : Dn - gb;
        const double e = st->Ebar[c] + Dn - (double)E[c];
        lam[c] = (T)((double)L[c] + rho * e);
        // Step 1's data of the next iteration at this penalty, formed as the
        // local step forms it (same operands, same order of operations)
        if (kDefect<T> && Ag) Ag[c * V + idx] = (T)(Dn + st->Ebar[c] + (double)lam[c] * irho);
        const double dd = Dd + (st->Ebar[c] - st->Ebar_prev[c]);
        v[0] += e * e;
        v[1] += dd * dd;
      }
    }
    if (kDefect<T>) {
#pragma unroll
      for (int i = 0; i < 3; ++i) un[i * V + idx] = pc.a[i];
      // and the warm start's det F - 1 for the closed form of that step
      if (Ag) Ag[9 * V + idx] = warm_code(warm_jm1(E));
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) Lg[c * V + idx] = lam[c];
    pm = pc;
    pc = pp;
  }
  store_partials(a, blk, v, 0, 0);
}

// ----------------------------------------------------------------------------
// Step 4: residuals, convergence test, adaptive penalty (one workgroup / cell)
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_finalize(KernelArgs a, IterParams ip) {
  __shared__ double red[4 * (kThreads / 64)];
  const int r = blockIdx.x;
  RveState *st = a.state + r;
  if (!st->active) return;
  const int p0 = a.blk_u[r], nb = a.blk_u[r + 1] - p0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  // eight loads in flight per thread, added in the order of k as one at a
  // time would (the sums keep their bits)
  const int step = blockDim.x;
  int k = threadIdx.x;
  for (; k + 7 * step < nb; k += 8 * step) {
    double4 q[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = a.partials[p0 + k + j * step];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      v[0] += q[j].x;
      v[1] += q[j].y;
      v[2] += q[j].z;
      v[3] += q[j].w;
    }
  }
  for (; k < nb; k += step) {
    const double4 q = a.partials[p0 + k];
    v[0] += q.x;
    v[1] += q.y;
    v[2] += q.z;
    v[3] += q.w;
  }
  block_sum<4>(v, red);
  if (threadIdx.x != 0) return;
  // Newton statistics (integers, summed exactly in double)
  st->newton_fail += (int)v[2];
  st->newton_iters += (unsigned long long)v[3];
  const double V = (double)a.desc[r].V;
  const double rho = st->rho;
  const double rp = sqrt(v[0] / V);
  const double rd = rho / ip.mu_ref * sqrt(v[1] / V);
  const int it = st->iter;
  if (it < ip.hist_cap) {
    double *h = a.hist + ((long long)r * ip.hist_cap + it) * 3;
    h[0] = rp;
    h[1] = rd;
    h[2] = rho;
  }
  st->rp = rp;
  st->rd = rd;
  st->rho_used = rho;
  st->at_rho = a.desc[r].At ? rho : 0.0;
  st->n_retry = 0;  // the local step's retry pass has run
  st->q_cur = 0;   // the next local step decides
  st->iter = it + 1;
  st->cur ^= 1;
  if (st->domain_err || !(rp == rp) || !(rd == rd)) {
    st->status = -5;
    st->active = 0;
    return;
  }
  // with an inexact local step, equilibrium also needs a small local
  // residual (bounded, with r_d, by the appendix's identity)
  const bool local_ok =
      !(ip.local_ratio > 0.0 || ip.local_fraction > 0.0) || st->rl <= ip.tol_d;
  if (ip.test_conv && rp <= ip.tol_p && rd <= ip.tol_d && local_ok) {
    st->status = 2;  // converged
    st->active = 0;
    return;
  }
  if (ip.test_conv && divergence_watch(rp, rd, ip.tol_p, ip.tol_d, it, ip.div_growth,
                                       ip.stall_iters, st->best_merit, st->ref_merit,
                                       st->ref_iter)) {
    st->status = -6;  // diverged or stagnated: the last iterate is kept
    st->active = 0;
    return;
  }
  if (ip.adapt) {
    double nr = rho;
    if (rp > ip.tau * rd) nr = ip.kappa_rho * rho;
    else if (rd > ip.tau * rp) nr = fmax(rho / ip.kappa_rho, ip.rho_min);
    if (nr > ip.rho_max) nr = ip.rho_max;
    st->rho = nr;
  }
  if (ip.test_conv && it + 1 >= ip.max_iter) {
    st->status = 1;
    st->active = 0;
  }
}

// ----------------------------------------------------------------------------
// homogenised stress: partial sums of P(F) and Lambda (double)
// ----------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_mean_stress(KernelArgs a) {
  __shared__ double red[18 * (kThreads / 64)];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int r = find_rve(a.blk_u, a.n_rve, blk);
  const RveDesc &D = a.desc[r];
  const int b = blk - a.blk_u[r];
  const int V = (int)D.V;
  const int n1 = D.n1, n2 = D.n2, n3 = D.n3, R = D.rows;
  const T *Eg = static_cast<const T *>(D.E);
  const T *Lg = static_cast<const T *>(D.Lam);
  const int t = threadIdx.x;
  const int row = t / n1, x1 = t - row * n1;
  int x2, z0;
  column_tile(D, b, row, x2, z0);
  double v[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) v[k] = 0.0;
  int bad = 0;
  for (int k = 0; k < kZSeg; ++k) {
    const int x3 = z0 + k;
    if (row >= R || x2 >= n2 || x3 >= n3) continue;
    const int idx = (x3 * n2 + x2) * n1 + x1;
    double E[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      E[c] = (double)Eg[c * V + idx];
      v[9 + c] += (double)Lg[c * V + idx];
    }
    const int ph = global_view(D.phase)[idx];
    Point<double> s;
    bool ok = false;
    // with rho = 0 the gradient of the prox objective is the stress P
    if (ph < a.n_mat) {
      const Material m = a.mats[ph];
      if (m.model == 1) {
        Lce<double> M;
        M.mua = m.mua;
        M.beta = m.beta;
        M.kappa = m.kappa;
        M.mu = m.mu;
        const T *dg = static_cast<const T *>(D.dir);
        const double n0 = dg[idx], n1v = dg[V + idx], n2v = dg[2 * V + idx];
        const double nn = 1.0 / sqrt(n0 * n0 + n1v * n1v + n2v * n2v);
        M.n[0] = n0 * nn;
        M.n[1] = n1v * nn;
        M.n[2] = n2v * nn;
        DirForm form;
        if (m.mual != 0.0) {
          // the non-ideality's stress needs the cross-link director
          const T *d0 = static_cast<const T *>(D.dir0);
          double q[3] = {(double)d0[idx], (double)d0[V + idx], (double)d0[2 * V + idx]};
          const double qn = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
#pragma unroll
          for (int k = 0; k < 3; ++k) form.n0[k] = q[k] * qn;
          M.mual = m.mual;
          M.form = &form;
        }
        ok = M.point(E, E, 0.0, s);
      } else {
        NeoHooke<double> M;
        M.mu = m.mu;
        M.lam = m.lam;
        ok = M.point(E, E, 0.0, s);
      }
    }
    if (ok) {
#pragma unroll
      for (int c = 0; c < 9; ++c) v[c] += s.g[c];
    } else {
      bad = 1;
    }
  }
  if (bad) atomicOr(&a.state[r].domain_err, 1);
  block_sum<18>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 18; ++k) a.partials18[(long long)blk * 18 + k] = v[k];
}

__global__ __launch_bounds__(kThreads) void k_mean_final(KernelArgs a) {
  __shared__ double red[18 * (kThreads / 64)];
  const int r = blockIdx.x;
  const int p0 = a.blk_u[r], nb = a.blk_u[r + 1] - p0;
  double v[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) v[k] = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x)
#pragma unroll
    for (int k = 0; k < 18; ++k) v[k] += a.partials18[(long long)(p0 + q) * 18 + k];
  block_sum<18>(v, red);
  if (threadIdx.x == 0) {
    const double iV = 1.0 / (double)a.desc[r].V;
#pragma unroll
    for (int k = 0; k < 18; ++k) a.mean_out[r * 18 + k] = v[k] * iV;
  }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

template <typename T> constexpr int tileB() { return 128 / (int)sizeof(typename cplx<T>::type); }

struct Timed {
  const LaunchCfg &L;
  int kid;
  Timed(const LaunchCfg &l, int k) : L(l), kid(k) {
    if (L.timer) L.timer->begin(kid);
  }
  ~Timed() {
    if (L.timer) L.timer->end(kid);
  }
};

// the x2 / x3 passes at a runtime tile width (one of four compiled widths)
template <typename T, bool INV>
static void launch_fft_y(const LaunchCfg &L, const KernelArgs &a) {
  using C = typename cplx<T>::type;
  constexpr int B = tileB<T>();
  const dim3 blk(kThreads), grid(L.nblk_y, 3);
  if (L.tile_y == kTileCol16) {
    if (sizeof(T) == 4 && !L.col256_y) {
      if (L.lds_coly > reg_lds(false, 16))
        hipLaunchKernelGGL((k_colreg<INV ? 1 : 0, 24>), grid, blk, L.lds_coly, L.stream, a);
      else
        hipLaunchKernelGGL((k_colreg<INV ? 1 : 0, 16>), grid, blk, L.lds_coly, L.stream, a);
    } else {
      hipLaunchKernelGGL((k_col16<T, INV ? 1 : 0>), grid, blk, col16_lds<C>(), L.stream, a);
    }
    return;
  }
  const size_t lds = 2 * (size_t)L.n2max * L.tile_y * sizeof(C);
  if (L.tile_y == B / 4)
    hipLaunchKernelGGL((k_fft_y<T, B / 4, INV>), grid, blk, lds, L.stream, a);
  else if (L.tile_y == B / 2)
    hipLaunchKernelGGL((k_fft_y<T, B / 2, INV>), grid, blk, lds, L.stream, a);
  else if (L.tile_y == 2 * B)
    hipLaunchKernelGGL((k_fft_y<T, 2 * B, INV>), grid, blk, lds, L.stream, a);
  else
    hipLaunchKernelGGL((k_fft_y<T, B, INV>), grid, blk, lds, L.stream, a);
}

template <typename T>
static void launch_poisson_z(const LaunchCfg &L, const KernelArgs &a) {
  using C = typename cplx<T>::type;
  constexpr int B = tileB<T>();
  const dim3 blk(kThreads), grid(L.nblk_z, 3);
  if (L.tile_z == kTileCol16) {
    if (sizeof(T) == 4 && !L.col256_z) {
      if (L.lds_colz > reg_lds(false, 16))
        hipLaunchKernelGGL((k_colreg<2, 24>), grid, blk, L.lds_colz, L.stream, a);
      else
        hipLaunchKernelGGL((k_colreg<2, 16>), grid, blk, L.lds_colz, L.stream, a);
    } else {
      hipLaunchKernelGGL((k_col16<T, 2>), grid, blk, col16_lds<C>(), L.stream, a);
    }
    return;
  }
  const size_t lds = 2 * (size_t)L.n3max * L.tile_z * sizeof(C);
  if (L.tile_z == B / 4)
    hipLaunchKernelGGL((k_poisson_z<T, B / 4>), grid, blk, lds, L.stream, a);
  else if (L.tile_z == B / 2)
    hipLaunchKernelGGL((k_poisson_z<T, B / 2>), grid, blk, lds, L.stream, a);
  else if (L.tile_z == 2 * B)
    hipLaunchKernelGGL((k_poisson_z<T, 2 * B>), grid, blk, lds, L.stream, a);
  else
    hipLaunchKernelGGL((k_poisson_z<T, B>), grid, blk, lds, L.stream, a);
}

// one pass of Step 1 in the kernel variant of the context's materials
template <typename T, int LK>
static void launch_local(const LaunchCfg &L, const KernelArgs &a, const IterParams &ip, int pass,
                         bool inexact) {
  const dim3 blk(kThreads);
  if (!inexact) {
    hipLaunchKernelGGL((k_local<T, LK, kLocalExact>), dim3(L.nblk_x), blk, 0, L.stream, a, ip, 0,
                       L.nblk_x);
    if (kClosedOnly<T, LK, kLocalExact>)
      hipLaunchKernelGGL((k_local<T, LK, kLocalRetry>), dim3(std::min(L.nblk_x, kLocalPassGrid)),
                         blk, 0, L.stream, a, ip, 0, L.nblk_x);
  }
  else if (pass == 0)
    hipLaunchKernelGGL((k_local<T, LK, kLocalFirst>), dim3(L.nblk_x), blk, 0, L.stream, a, ip, 0,
                       L.nblk_x);
  else
    hipLaunchKernelGGL((k_local<T, LK, kLocalLater>), dim3(std::min(L.nblk_x, kLocalPassGrid)),
                       blk, 0, L.stream, a, ip, pass, L.nblk_x);
}

template <typename T>
static hipError_t launch_iteration_part(const LaunchCfg &L, const KernelArgs &a,
                                        const IterParams &ip, Part part) {
  const dim3 blk(kThreads);
  switch (part) {
    case Part::Local: {
      Timed tm(L, K_LOCAL);
      const bool inexact = ip.local_ratio > 0.0 || ip.local_fraction > 0.0;
      const int passes = inexact ? ip.local_passes : 1;
      if (L.any_frank) hipLaunchKernelGGL((k_lag<T>), dim3(L.nblk_x), blk, 0, L.stream, a);
      for (int pass = 0; pass < passes; ++pass) {
        switch (L.lce_kind) {
          case 0: launch_local<T, 0>(L, a, ip, pass, inexact); break;
          case 1: launch_local<T, 1>(L, a, ip, pass, inexact); break;
          default: launch_local<T, 2>(L, a, ip, pass, inexact); break;
        }
        if (inexact)
          hipLaunchKernelGGL(k_local_check, dim3(a.n_rve), blk, 0, L.stream, a, ip, pass);
      }
      break;
    }
    case Part::Project: {
      {
        Timed tm(L, K_DIV_FWDX);
        if (L.any_free) {
          hipLaunchKernelGGL((k_fsum<T>), dim3(L.nblk_x), blk, 0, L.stream, a);
          hipLaunchKernelGGL(k_fbar, dim3(a.n_rve), blk, 0, L.stream, a);
        }
        hipLaunchKernelGGL((k_div_fwdx<T>), dim3(L.nblk_f), blk, L.lds_x, L.stream, a);
      }
      {
        Timed tm(L, K_FFT_Y_FWD);
        launch_fft_y<T, false>(L, a);
      }
      {
        Timed tm(L, K_POISSON_Z);
        launch_poisson_z<T>(L, a);
      }
      {
        Timed tm(L, K_FFT_Y_INV);
        launch_fft_y<T, true>(L, a);
      }
      {
        Timed tm(L, K_INV_X);
        if (sizeof(T) == 4 && L.inv256)
          hipLaunchKernelGGL(k_inv_x256, dim3(L.nblk_i), blk, kInvLds, L.stream, a);
        else
          hipLaunchKernelGGL((k_inv_x<T>), dim3(L.nblk_f), blk, L.lds_x, L.stream, a);
      }
      break;
    }
    case Part::Update: {
      {
        Timed tm(L, K_UPDATE);
        hipLaunchKernelGGL((k_update<T>), dim3(L.nblk_u), blk, 0, L.stream, a);
      }
      {
        Timed tm(L, K_FINALIZE);
        hipLaunchKernelGGL(k_finalize, dim3(a.n_rve), blk, 0, L.stream, a, ip);
      }
      break;
    }
    case Part::StripNull: {
      if (kDefect<T>) {
        hipLaunchKernelGGL(k_null_sums, dim3(L.nblk_u), blk, 0, L.stream, a);
        hipLaunchKernelGGL(k_null_final, dim3(a.n_rve), blk, 0, L.stream, a);
        hipLaunchKernelGGL(k_null_sub, dim3(L.nblk_u), blk, 0, L.stream, a);
      }
      break;
    }
    case Part::ComposeU: {
      if (kDefect<T>) hipLaunchKernelGGL((k_compose_u<T>), dim3(L.nblk_x), blk, 0, L.stream, a);
      break;
    }
    case Part::MeanStress: {
      Timed tm(L, K_MEAN);
      hipLaunchKernelGGL((k_mean_stress<T>), dim3(L.nblk_u), blk, 0, L.stream, a);
      hipLaunchKernelGGL(k_mean_final, dim3(a.n_rve), blk, 0, L.stream, a);
      break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_orientation(const LaunchCfg &L, const KernelArgs &a, bool fp64) {
  const dim3 blk(kThreads);
  if (fp64)
    hipLaunchKernelGGL((k_orient<double>), dim3(L.nblk_x), blk, 0, L.stream, a);
  else
    hipLaunchKernelGGL((k_orient<float>), dim3(L.nblk_x), blk, 0, L.stream, a);
  hipLaunchKernelGGL(k_orient_final, dim3(a.n_rve), blk, 0, L.stream, a);
  return hipGetLastError();
}

hipError_t launch_part(const LaunchCfg &L, const KernelArgs &a, const IterParams &ip, Part part,
                       bool fp64) {
  return fp64 ? launch_iteration_part<double>(L, a, ip, part)
              : launch_iteration_part<float>(L, a, ip, part);
}

int tile_b(bool fp64) { return fp64 ? tileB<double>() : tileB<float>(); }

// register-resident x2 / x3 pass: points per thread for a length (0: not
// supported), columns per workgroup, LDS bytes for points per thread P
int reg_points(bool fp64, int n) { return fp64 ? (n == 256 ? 16 : 0) : colreg_points(n); }
int reg_columns(bool fp64, int n) {
  const int P = reg_points(fp64, n);
  return P ? kThreads / (n / P) : 0;
}
size_t reg_lds(bool fp64, int pmax) {
  return fp64 ? col16_lds<double2>() : (size_t)pmax * kColSlab * sizeof(float2);
}

bool tile_compiled(bool fp64, int B) {
  const int d = tile_b(fp64);
  return B == d / 4 || B == d / 2 || B == d || B == 2 * d;
}

}  // namespace admm
