// launch.hpp -- interface between the host API (admm_api.cpp) and the kernel
// launchers (kernels.hip).
#pragma once

#include "common.hpp"

namespace admm {

// device pointers handed to every kernel
struct KernelArgs {
  const RveDesc *desc;
  RveState *state;
  const int *blk_x;  // prefix tables: first logical workgroup of each cell
  const int *blk_y;
  const int *blk_z;
  const int *blk_u;
  const int *blk_f;  // the x1-transform kernels (div_fwdx, inv_x)
  const int *blk_i;  // the register-resident inverse x1 pass (32 real lines each)
  const Material *mats;
  const void *tw;       // twiddle pool (float2 or double2)
  double4 *partials;    // per update workgroup: sum e^2, sum dd^2, and the failed
                        // solves and Newton iterations of its rows' local step
  double *partials18;   // per workgroup: sums of P and Lambda
  double *mean_out;     // per cell: <P>, <Lambda>
  double *hist;         // per cell, per iteration: r_p, r_d, rho
  double2 *lpart;       // per local workgroup, inexact passes: (sum of |local
                        // residual|^2, count of converged local solves)
  double *fpart;        // per local workgroup: sums of F - I - Lambda/rho (9), for
                        // the free components of <F>
  int2 *newton_part;    // per update workgroup: failed solves and Newton iterations
                        // of the local-step workgroups in its tile
  unsigned *retry_mask; // per local workgroup, kThreads bits: voxels the exact
                        // pass's closed form left to the retry pass (zero between
                        // steps)
  double *nullpart;     // per update workgroup: 24 sums of u_i chi_s (float form)
  double *nullc;        // per cell: 24 null-mode coefficients of u
  int n_rve;
  int n_mat;
};

// kernel ids of the profiling interface (same order as in include/admm.h)
enum KernelId {
  K_LOCAL = 0, K_DIV_FWDX, K_FFT_Y_FWD, K_POISSON_Z, K_FFT_Y_INV, K_INV_X, K_UPDATE, K_FINALIZE,
  K_MEAN, K_COUNT
};

// brackets kernel launches with events on the launch stream when profiling
struct KernelTimer {
  virtual void begin(int kid) = 0;
  virtual void end(int kid) = 0;
  virtual ~KernelTimer() {}
};

// grid sizes and LDS bytes of one context
struct LaunchCfg {
  KernelTimer *timer;  // null unless profiling
  hipStream_t stream;
  int nblk_x, nblk_y, nblk_z, nblk_u, nblk_f;
  // float cells all of x1 length 256: the inverse x1 pass runs register
  // resident (k_inv_x256), nblk_i workgroups
  bool inv256;
  int nblk_i;
  int tile_y, tile_z;  // columns per workgroup of the x2 and x3 passes,
                       // or kTileCol16 (the register-resident pass)
  size_t lds_coly, lds_colz;  // LDS bytes of the register-resident passes
  bool col256_y, col256_z;     // every length along x2 (x3) is 256: k_col16
  int n2max, n3max;
  size_t lds_x;  // LDS bytes of the x1-pass kernels
  bool any_lce;   // some phase uses the LCE energy
  int lce_kind;   // 0 no LCE, 1 the ideal LCE, 2 some term of the full model or nu_F
  bool any_frank; // the Frank term needs the previous iteration's directors
  bool any_free;  // some cell leaves components of <F> free
};

// ComposeU: after a single Step 2 call of the float form, u_prev = u + du.
// StripNull: the float form removes the mean and the Nyquist checkerboards
// of u (which D_h does not see) before it iterates.
enum class Part { Local, Project, Update, MeanStress, ComposeU, StripNull };

// Bloch-wave stability modulus of one cell (double precision; bloch.hip).
// p: 3V complex (interleaved) start in, unit mode out. Returns 0, -1 (HIP
// error), -2 (a zero start or right-hand side), -3 (L + rho I not positive
// definite); status 0 converged, 1 iteration cap.
// work: device buffer of bloch_work_bytes(D) bytes, or null to allocate one
// for the call.
int bloch_solve(hipStream_t st, const RveDesc &D, const Material *mats_d, int n_mat,
                const void *tw, const double omega[3], double rho, double tol, int max_iter,
                double *p, void *work, double *beta, double *sigma_rho, int *iters,
                int *status);
size_t bloch_work_bytes(const RveDesc &D);

// The allocation-free variant's work buffer: a fixed-size device array in
// the library's code object (one per device). bloch_scratch() gives this
// device's address (looked up on first use); -1 on a HIP error.
size_t bloch_scratch_bytes();
int bloch_scratch(void **ptr);

// Orientation tensor sums of every cell into a.mean_out (<n (x) n> sums in
// entries 0..8, the LCE voxel count in entry 9).
hipError_t launch_orientation(const LaunchCfg &L, const KernelArgs &a, bool fp64);

// Enqueues one part of the iteration on L.stream.
hipError_t launch_part(const LaunchCfg &L, const KernelArgs &a, const IterParams &ip, Part part,
                       bool fp64);

// columns per tile of the FFT passes along x2 and x3: the default (128 bytes
// of complex per row) and whether a width is one of the compiled ones (a
// quarter, half, default, double)
int tile_b(bool fp64);
bool tile_compiled(bool fp64, int B);
int reg_points(bool fp64, int n);
int reg_columns(bool fp64, int n);
size_t reg_lds(bool fp64, int pmax);

}  // namespace admm
