// admm_api.cpp -- host side of the C ABI declared in include/admm.h: argument
// validation, radix plans and twiddle tables, the per-cell descriptors, and
// the launch sequence of Algorithm 1 (inner loop on the device, convergence
// state read back once per check interval).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <new>
#include <vector>

#include "../../include/admm.h"
#include "common.hpp"
#include "launch.hpp"

using namespace admm;

namespace {

enum { ST_RUNNING = 0, ST_CAP = 1, ST_CONVERGED = 2, ST_DOMAIN = -5, ST_DIVERGED = -6 };

bool is_2a3b(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// radices for length n: 8s first, 4 4 instead of 8 2, then 2, then 3s
Plan1D make_plan(int n) {
  Plan1D p{};
  p.n = n;
  int m = n, twos = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++twos;
  }
  std::vector<int> r;
  int e8 = twos / 3, rest = twos % 3;
  if (rest == 1 && e8 > 0) {
    --e8;
    rest = 4;  // 2^4 = 4 * 4
  }
  for (int k = 0; k < e8; ++k) r.push_back(8);
  if (rest == 4) {
    r.push_back(4);
    r.push_back(4);
  } else if (rest == 2) {
    r.push_back(4);
  } else if (rest == 1) {
    r.push_back(2);
  }
  while (m % 3 == 0) {
    m /= 3;
    r.push_back(3);
  }
  p.nst = (int)r.size();
  for (int k = 0; k < p.nst; ++k) p.rad[k] = r[k];
  plan_divisors(p);
  return p;
}

// exp(-2 pi i t/n), t = 0..n-1: long double evaluation rounded once, exact at
// the quarter points, and exactly Hermitian (w[n-t] = conj w[t]).
void twiddles(int n, std::vector<double> &re, std::vector<double> &im) {
  re.assign(n, 0.0);
  im.assign(n, 0.0);
  const long double tp = 6.283185307179586476925286766559005768L;
  for (int t = 0; t <= n / 2; ++t) {
    double c, s;
    if ((4 * t) % n == 0) {
      const int q = (4 * t) / n;  // 0, 1, 2
      c = q == 0 ? 1.0 : (q == 1 ? 0.0 : -1.0);
      s = q == 1 ? 1.0 : 0.0;
    } else {
      const long double ang = tp * (long double)t / (long double)n;
      c = (double)cosl(ang);
      s = (double)sinl(ang);
    }
    re[t] = c;
    im[t] = -s;
    if (t > 0 && t < n - t) {
      re[n - t] = c;
      im[n - t] = s;
    }
  }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// three half-spectrum components (the divergence of F - Lambda/rho, then the
// displacement fluctuation) per cell
// row stride of the half spectra: m1 = n1/2 + 1 entries rounded up to 32
// bytes (the columns past m1 are zero)
int spec_stride(int n1, bool fp64) { return (int)align_up((size_t)(n1 / 2 + 1), fp64 ? 2 : 4); }

size_t spec_bytes(int n1, int n2, int n3, bool fp64) {
  const size_t S = (size_t)n3 * n2 * spec_stride(n1, fp64);
  return align_up(3 * S * (fp64 ? 16 : 8), 256);
}

// float form: the correction u_{i+1} - u_i of Step 2 (3V float) after the spectra
size_t du_bytes(int n1, int n2, int n3, bool fp64) {
  return fp64 ? 0 : align_up(3 * (size_t)n1 * n2 * n3 * sizeof(float), 256);
}

int rows_per_block(int n1) { return std::max(1, kThreads / n1); }

// x1-lines per workgroup of the x1 transforms, for about `points` points per
// workgroup (more lines keep more of the workgroup busy in every radix stage;
// fewer need less LDS); the autotuner picks `points`
int rows_per_fft_block(int n1, int points) { return std::max(1, points / n1); }
int default_fft_points(bool fp64) { return fp64 ? 256 : 1024; }

// Radix sequences for a length n = 2^a 3^b that the autotuner tries: the
// powers of two split into radix-8, -4 and at most one radix-2 stage, the
// threes into radix-3 stages, every distinct order of each split (at most
// kMaxStages stages, at most `cap` sequences, the default plan first).
std::vector<Plan1D> plan_candidates(int n, size_t cap = 24) {
  std::vector<Plan1D> out;
  out.push_back(make_plan(n));
  int m = n, twos = 0, threes = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++twos;
  }
  while (m % 3 == 0) {
    m /= 3;
    ++threes;
  }
  for (int e8 = twos / 3; e8 >= 0; --e8)
    for (int e2 = 0; e2 <= 1; ++e2) {
      const int left = twos - 3 * e8 - e2;
      if (left < 0 || left % 2) continue;
      std::vector<int> r;
      r.insert(r.end(), e8, 8);
      r.insert(r.end(), left / 2, 4);
      r.insert(r.end(), e2, 2);
      r.insert(r.end(), threes, 3);
      if ((int)r.size() > kMaxStages || r.empty()) continue;
      std::sort(r.begin(), r.end());
      do {
        Plan1D p{};
        p.n = n;
        p.nst = (int)r.size();
        for (int k = 0; k < p.nst; ++k) p.rad[k] = r[k];
        bool dup = false;
        for (const Plan1D &q : out)
          dup = dup || (q.nst == p.nst && std::equal(q.rad, q.rad + q.nst, p.rad));
        if (!dup) out.push_back(p);
      } while (out.size() < cap && std::next_permutation(r.begin(), r.end()));
    }
  if (out.size() > cap) out.resize(cap);
  return out;
}

}  // namespace

// hipEvent pairs around every launch on the context's stream; elapsed times
// are summed per kernel when read
class EventTimer : public KernelTimer {
 public:
  explicit EventTimer(hipStream_t s) : stream_(s) {}
  ~EventTimer() override {
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
  }
  void begin(int kid) override {
    pending_kid_ = kid;
    pending_ = take();
    if (pending_) (void)hipEventRecord(pending_, stream_);
  }
  void end(int kid) override {
    hipEvent_t e1 = take();
    if (pending_ && e1 && kid == pending_kid_) {
      (void)hipEventRecord(e1, stream_);
      recs_.push_back({kid, pending_, e1});
    }
    pending_ = nullptr;
  }
  // folds recorded pairs into the totals; the stream must be synchronised
  void collect() {
    for (const Rec &r : recs_) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
        total_ms_[r.kid] += ms;
        count_[r.kid] += 1;
      }
    }
    recs_.clear();
    used_ = 0;
  }
  void reset() {
    recs_.clear();
    used_ = 0;
    for (int k = 0; k < K_COUNT; ++k) {
      total_ms_[k] = 0.0;
      count_[k] = 0;
    }
  }
  double total_ms(int k) const { return total_ms_[k]; }
  int count(int k) const { return count_[k]; }

 private:
  struct Rec {
    int kid;
    hipEvent_t e0, e1;
  };
  hipEvent_t take() {
    if (used_ == pool_.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool_.push_back(e);
    }
    return pool_[used_++];
  }
  hipStream_t stream_;
  std::vector<hipEvent_t> pool_;
  size_t used_ = 0;
  std::vector<Rec> recs_;
  hipEvent_t pending_ = nullptr;
  int pending_kid_ = -1;
  double total_ms_[K_COUNT] = {};
  int count_[K_COUNT] = {};
};

struct admm_ctx {
  int n_rve = 0, n_mat = 0;
  bool fp64 = true;
  hipStream_t stream = nullptr;
  admm_params params{};
  std::vector<admm_rve> rves;
  std::vector<RveDesc> desc_h;
  std::vector<RveState> state_h;
  int hist_cap = 0;
  // device
  RveDesc *desc_d = nullptr;
  RveState *state_d = nullptr;
  int *blk_d = nullptr;
  Material *mats_d = nullptr;
  void *tw_d = nullptr;
  double4 *partials_d = nullptr;
  double *partials18_d = nullptr;
  double *mean_d = nullptr;
  double *hist_d = nullptr;
  double2 *lpart_d = nullptr;
  double *fpart_d = nullptr;
  int2 *newton_part_d = nullptr;
  unsigned *retry_d = nullptr;
  void *at_d = nullptr;  // RveDesc::At of every cell (float form, no LCE)
  double *nullpart_d = nullptr;
  double *nullc_d = nullptr;
  std::vector<void *> owned;  // start-of-step copies and lagged directors
  bool any_nuF = false, any_nun = false, any_frank = false;
  void *workspace = nullptr;
  bool own_workspace = false;
  LaunchCfg L{};
  KernelArgs A{};
  EventTimer *timer = nullptr;
  // captured iteration sequences, one per convergence-test mode: `iters`
  // iterations recorded on cap_stream, replayed on `stream`
  struct Graph {
    hipGraphExec_t exec = nullptr;
    int iters = 0;
  } graph[2];
  hipStream_t cap_stream = nullptr;
  // per-cell workgroup counts of the x2 / x3 passes depend on the tile widths
  std::vector<int> blk_h;
  int xpoints = 0;  // points per workgroup of the x1 transforms
};

namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return ADMM_EHIP;   \
  } while (0)

// the start of a load step for the dissipation terms: F^n and n^n
int snapshot_step(admm_ctx *c) {
  const size_t s = c->fp64 ? 8 : 4;
  for (int r = 0; r < c->n_rve; ++r) {
    const RveDesc &D = c->desc_h[r];
    const size_t V = (size_t)D.V;
    if (D.E_step)
      HIP_TRY(hipMemcpyAsync(D.E_step, D.E, 9 * V * s, hipMemcpyDeviceToDevice, c->stream));
    if (D.dir_step)
      HIP_TRY(hipMemcpyAsync(D.dir_step, D.dir, 3 * V * s, hipMemcpyDeviceToDevice, c->stream));
  }
  return ADMM_OK;
}

int upload_states(admm_ctx *c, int q_cur = 0) {
  for (auto &s : c->state_h) {
    s.at_rho = 0.0;  // Step 1 reads the caller's fields
    s.n_retry = 0;   // (no retry bit survives a retry pass)
    s.q_cur = q_cur;  // and Step 2 too, unless told otherwise
  }
  HIP_TRY(hipMemcpyAsync(c->state_d, c->state_h.data(), sizeof(RveState) * c->n_rve,
                         hipMemcpyHostToDevice, c->stream));
  return ADMM_OK;
}

int download_states(admm_ctx *c) {
  HIP_TRY(hipMemcpyAsync(c->state_h.data(), c->state_d, sizeof(RveState) * c->n_rve,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->timer) c->timer->collect();
  return ADMM_OK;
}

// after a launch sequence: read the state back and make `u` the current
// fluctuation buffer of every cell again
int settle(admm_ctx *c) {
  int rc = download_states(c);
  if (rc != ADMM_OK) return rc;
  bool moved = false;
  for (int r = 0; r < c->n_rve; ++r) {
    const RveDesc &D = c->desc_h[r];
    if (c->state_h[r].cur == 1) {
      HIP_TRY(hipMemcpyAsync(D.u[0], D.u[1], 3 * (size_t)D.V * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
      c->state_h[r].cur = 0;
      moved = true;
    }
  }
  if (moved) {
    rc = upload_states(c);
    if (rc != ADMM_OK) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return ADMM_OK;
}

IterParams iter_params(const admm_ctx *c, int test_conv) {
  const admm_params &p = c->params;
  IterParams ip{};
  ip.rho_min = p.rho_min;
  ip.rho_max = p.rho_max;
  ip.kappa_rho = p.kappa_rho;
  ip.tau = p.tau;
  ip.tol_p = p.tol_p;
  ip.tol_d = p.tol_d;
  ip.mu_ref = p.mu_ref;
  ip.gtol = p.newton_gtol;
  ip.step_tol = p.newton_step_tol;
  ip.adapt = p.adapt_rho;
  ip.max_iter = p.max_iter;
  ip.newton_max = p.newton_max;
  ip.test_conv = test_conv;
  ip.hist_cap = c->hist_cap;
  ip.n_rve = c->n_rve;
  ip.n_mat = c->n_mat;
  ip.local_ratio = p.local_ratio;
  ip.local_chunk = p.local_chunk;
  ip.local_passes = p.local_passes;
  ip.local_fraction = p.local_fraction;
  ip.dt = p.dt;
  ip.div_growth = p.div_growth;
  ip.stall_iters = p.stall_iters;
  return ip;
}

void drop_graphs(admm_ctx *c) {
  for (auto &g : c->graph) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.iters = 0;
  }
}

// the register-resident x2 / x3 pass (tile width kTileCol16: k_colreg in
// float, k_col16 in double) is open to an axis when every cell's length
// along it is supported (float: 32, 48, 64, 96, 128, 256; double: 256)
bool col16_ok(const admm_ctx *c, int axis) {
  for (const RveDesc &D : c->desc_h)
    if (!reg_points(c->fp64, axis == 2 ? D.n2 : D.n3)) return false;
  return true;
}

// a tile width of the x2 (axis 2) or x3 (axis 3) pass: a compiled width
// within 64 KiB of LDS, or kTileCol16 where every cell's length is 256
bool tile_ok(const admm_ctx *c, int axis, int B) {
  if (B == kTileCol16) return col16_ok(c, axis);
  const size_t csz = c->fp64 ? sizeof(double2) : sizeof(float2);
  const int nmax = axis == 2 ? c->L.n2max : c->L.n3max;
  return tile_compiled(c->fp64, B) && 2 * (size_t)nmax * B * csz <= 65536;
}

// tile widths of the x2 / x3 passes: workgroup prefix tables (blk_h holds
// the x, y, z, u, f and i tables, n_rve + 1 entries each), grid sizes, upload.
// Under kTileCol16 an axis's workgroups take 16 columns each of the
// flattened (x3, m1) or (m2, m1) set.
static_assert(kTileCol16 == ADMM_TILE_REG16, "tile width of the register-resident pass");

int set_tiles(admm_ctx *c, int ty, int tz) {
  const int n = c->n_rve;
  int *by = c->blk_h.data() + (n + 1), *bz = c->blk_h.data() + 2 * (n + 1);
  by[0] = bz[0] = 0;
  int py = 0, pz = 0;
  for (int r = 0; r < n; ++r) {
    const RveDesc &D = c->desc_h[r];
    if (ty == kTileCol16) {
      const int cw = reg_columns(c->fp64, D.n2);
      by[r + 1] = by[r] + (D.n3 * D.m1 + cw - 1) / cw;
      py = std::max(py, reg_points(c->fp64, D.n2));
    } else {
      by[r + 1] = by[r] + D.n3 * ((D.m1 + ty - 1) / ty);
    }
    if (tz == kTileCol16) {
      const int cw = reg_columns(c->fp64, D.n3);
      bz[r + 1] = bz[r] + (D.n2 * D.m1 + cw - 1) / cw;
      pz = std::max(pz, reg_points(c->fp64, D.n3));
    } else {
      bz[r + 1] = bz[r] + (D.n2 * D.m1s + tz - 1) / tz;
    }
  }
  c->L.col256_y = c->L.col256_z = true;
  for (const RveDesc &D : c->desc_h) {
    c->L.col256_y = c->L.col256_y && D.n2 == 256;
    c->L.col256_z = c->L.col256_z && D.n3 == 256;
  }
  c->L.lds_coly = reg_lds(c->fp64, py);
  c->L.lds_colz = reg_lds(c->fp64, pz);
  c->L.tile_y = ty;
  c->L.tile_z = tz;
  c->L.nblk_y = by[n];
  c->L.nblk_z = bz[n];
  HIP_TRY(hipMemcpyAsync(c->blk_d, c->blk_h.data(), sizeof(int) * c->blk_h.size(),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  return ADMM_OK;
}

// radix plan of every transform of length len (the twiddle table stays)
int set_plan(admm_ctx *c, const Plan1D &p) {
  for (auto &D : c->desc_h) {
    Plan1D *q[3] = {&D.p1, &D.p2, &D.p3};
    for (Plan1D *x : q)
      if (x->n == p.n) {
        const int tw = x->tw;
        *x = p;
        x->tw = tw;
        plan_divisors(*x);
      }
  }
  HIP_TRY(hipMemcpyAsync(c->desc_d, c->desc_h.data(), sizeof(RveDesc) * c->n_rve,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  return ADMM_OK;
}

// points per workgroup of the x1 transforms: lines per workgroup of every
// cell, prefix table, grid size and LDS
int set_xpoints(admm_ctx *c, int points) {
  const int n = c->n_rve;
  int *bf = c->blk_h.data() + 4 * (n + 1);
  bf[0] = 0;
  int lds = 0;
  for (int r = 0; r < n; ++r) {
    RveDesc &D = c->desc_h[r];
    D.rows_f = rows_per_fft_block(D.n1, points);
    D.f_rows_f = make_fastdiv((unsigned)D.rows_f);
    bf[r + 1] = bf[r] + (D.n2 * D.n3 + D.rows_f - 1) / D.rows_f;
    lds = std::max(lds, 2 * ((3 * D.rows_f + 1) / 2) * D.n1);
  }
  c->L.nblk_f = bf[n];
  c->L.lds_x = (size_t)lds * (c->fp64 ? sizeof(double2) : sizeof(float2));
  c->xpoints = points;
  HIP_TRY(hipMemcpyAsync(c->desc_d, c->desc_h.data(), sizeof(RveDesc) * n, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->blk_d, c->blk_h.data(), sizeof(int) * c->blk_h.size(),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  return ADMM_OK;
}

int launch(admm_ctx *c, Part part, const IterParams &ip) {
  hipError_t e = launch_part(c->L, c->A, ip, part, c->fp64);
  return e == hipSuccess ? ADMM_OK : ADMM_EHIP;
}

int one_iteration(admm_ctx *c, const IterParams &ip) {
  int rc = launch(c, Part::Local, ip);
  if (rc == ADMM_OK) rc = launch(c, Part::Project, ip);
  if (rc == ADMM_OK) rc = launch(c, Part::Update, ip);
  return rc;
}

// Records k iterations into a graph. Every launch argument (buffers, grids,
// iteration parameters) is fixed for the context's lifetime and all
// iteration state lives in device memory, so the graph stays valid across
// calls. Capture needs a stream of its own (the caller's may be the null
// stream); the graph is then launched on the caller's stream.
int build_graph(admm_ctx *c, const IterParams &ip, int k, admm_ctx::Graph &g) {
  if (g.exec) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.iters = 0;
  }
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const hipStream_t saved = c->L.stream;
  c->L.stream = c->cap_stream;
  hipGraph_t graph = nullptr;
  int rc = ADMM_OK;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = ADMM_EHIP;
  } else {
    for (int it = 0; it < k && rc == ADMM_OK; ++it) rc = one_iteration(c, ip);
    if (hipStreamEndCapture(c->cap_stream, &graph) != hipSuccess) rc = ADMM_EHIP;
  }
  c->L.stream = saved;
  if (rc == ADMM_OK && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    g.exec = nullptr;
    rc = ADMM_EHIP;
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (rc == ADMM_OK) g.iters = k;
  return rc;
}

// n iterations: whole graphs of check_every iterations, the rest launched
// kernel by kernel (also everything while profiling)
int run_iterations(admm_ctx *c, const IterParams &ip, int n) {
  const int k = c->params.check_every;
  int done = 0, rc = ADMM_OK;
  if (c->params.use_graph && !c->timer && k >= 2 && n >= k) {
    admm_ctx::Graph &g = c->graph[ip.test_conv ? 1 : 0];
    if (!g.exec || g.iters != k) rc = build_graph(c, ip, k, g);
    for (; rc == ADMM_OK && done + k <= n; done += k)
      if (hipGraphLaunch(g.exec, c->stream) != hipSuccess) rc = ADMM_EHIP;
  }
  for (; rc == ADMM_OK && done < n; ++done) rc = one_iteration(c, ip);
  return rc;
}

bool valid_fbar(const double *F) {
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(F[k])) return false;
  const double d = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                   F[2] * (F[3] * F[7] - F[4] * F[6]);
  return d > 0.0;
}

void free_ctx(admm_ctx *c) {
  if (!c) return;
  (void)hipFree(c->desc_d);
  (void)hipFree(c->state_d);
  (void)hipFree(c->blk_d);
  (void)hipFree(c->mats_d);
  (void)hipFree(c->tw_d);
  (void)hipFree(c->partials_d);
  (void)hipFree(c->partials18_d);
  (void)hipFree(c->mean_d);
  (void)hipFree(c->hist_d);
  (void)hipFree(c->newton_part_d);
  (void)hipFree(c->retry_d);
  (void)hipFree(c->at_d);
  (void)hipFree(c->nullpart_d);
  (void)hipFree(c->nullc_d);
  (void)hipFree(c->lpart_d);
  (void)hipFree(c->fpart_d);
  for (void *q : c->owned) (void)hipFree(q);
  if (c->own_workspace) (void)hipFree(c->workspace);
  for (auto &g : c->graph)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c->timer;
  delete c;
}

}  // namespace

namespace {

// Step 2 (all cells) per call, best of three runs of `reps` calls, on the
// context's stream
int time_project(admm_ctx *c, int reps, double *ms) {
  const IterParams ip = iter_params(c, 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return ADMM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ADMM_EHIP;
  }
  int rc = launch(c, Part::Project, ip);
  double best = 1e300;
  for (int trial = 0; trial < 3 && rc == ADMM_OK; ++trial) {
    if (hipEventRecord(e0, c->stream) != hipSuccess) rc = ADMM_EHIP;
    for (int k = 0; k < reps && rc == ADMM_OK; ++k) rc = launch(c, Part::Project, ip);
    if (rc == ADMM_OK && hipEventRecord(e1, c->stream) != hipSuccess) rc = ADMM_EHIP;
    if (rc == ADMM_OK && hipEventSynchronize(e1) != hipSuccess) rc = ADMM_EHIP;
    float t = 0.0f;
    if (rc == ADMM_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = ADMM_EHIP;
    if (rc == ADMM_OK) best = std::min(best, (double)t / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return rc;
}

std::vector<int> lengths_of(const admm_ctx *c) {
  std::vector<int> n;
  for (const auto &D : c->desc_h)
    for (int v : {D.n1, D.n2, D.n3})
      if (std::find(n.begin(), n.end(), v) == n.end()) n.push_back(v);
  std::sort(n.begin(), n.end());
  return n;
}

void report_tuning(const admm_ctx *c, admm_tuning *out) {
  out->tile_y = c->L.tile_y;
  out->tile_z = c->L.tile_z;
  out->x_points = c->xpoints;
  const std::vector<int> n = lengths_of(c);
  out->n_len = (int32_t)std::min<size_t>(n.size(), 24);
  for (int k = 0; k < out->n_len; ++k) {
    out->len[k] = n[k];
    for (int s = 0; s < 8; ++s) out->radix[k][s] = 0;
    for (const auto &D : c->desc_h) {
      const Plan1D *q = D.p1.n == n[k] ? &D.p1 : D.p2.n == n[k] ? &D.p2 : D.p3.n == n[k] ? &D.p3
                                                                                           : nullptr;
      if (q) {
        for (int s = 0; s < q->nst && s < 8; ++s) out->radix[k][s] = q->rad[s];
        break;
      }
    }
  }
}

int tune(admm_ctx *c, int reps, admm_tuning *out) {
  const size_t csz = c->fp64 ? sizeof(double2) : sizeof(float2);
  const int d = tile_b(c->fp64);
  double best = 0.0;
  int rc = time_project(c, reps, &best);
  if (rc != ADMM_OK) return rc;
  out->ms_default = best;
  const int cand[4] = {d / 4, d / 2, d, 2 * d};
  // points per workgroup of the x1 transforms (LDS <= 64 KiB)
  {
    int keep = c->xpoints;
    for (int pts : {256, 512, 1024}) {
      if (pts == keep || 2 * ((3 * (size_t)std::max(1, pts / 4) + 1) / 2) * 4 * csz > 65536)
        continue;
      rc = set_xpoints(c, pts);
      double t = 0.0;
      if (rc == ADMM_OK) rc = time_project(c, reps, &t);
      if (rc != ADMM_OK) return rc;
      if (t < best) {
        best = t;
        keep = pts;
      }
    }
    rc = set_xpoints(c, keep);
    if (rc != ADMM_OK) return rc;
  }
  // tile width of the x2 pass, then of the x3 pass (LDS <= 64 KiB), and the
  // register-resident pass where every cell's length along the axis is 256
  for (int pass = 0; pass < 2 && rc == ADMM_OK; ++pass) {
    int keep = pass == 0 ? c->L.tile_y : c->L.tile_z;
    std::vector<int> cands(cand, cand + 4);
    cands.push_back(kTileCol16);
    for (int B : cands) {
      if (B == keep || !tile_ok(c, pass == 0 ? 2 : 3, B)) continue;
      rc = pass == 0 ? set_tiles(c, B, c->L.tile_z) : set_tiles(c, c->L.tile_y, B);
      double t = 0.0;
      if (rc == ADMM_OK) rc = time_project(c, reps, &t);
      if (rc != ADMM_OK) break;
      if (t < best) {
        best = t;
        keep = B;
      }
    }
    if (rc == ADMM_OK)
      rc = pass == 0 ? set_tiles(c, keep, c->L.tile_z) : set_tiles(c, c->L.tile_y, keep);
  }
  // radix plan of each transform length in turn
  for (int n : lengths_of(c)) {
    if (rc != ADMM_OK) break;
    const std::vector<Plan1D> cands = plan_candidates(n);
    Plan1D keep{};
    for (const auto &D : c->desc_h) {
      if (D.p1.n == n) keep = D.p1;
      else if (D.p2.n == n) keep = D.p2;
      else if (D.p3.n == n) keep = D.p3;
      if (keep.n == n) break;
    }
    for (const Plan1D &p : cands) {
      if (p.nst == keep.nst && std::equal(p.rad, p.rad + p.nst, keep.rad)) continue;
      rc = set_plan(c, p);
      double t = 0.0;
      if (rc == ADMM_OK) rc = time_project(c, reps, &t);
      if (rc != ADMM_OK) break;
      if (t < best) {
        best = t;
        keep = p;
      }
    }
    if (rc == ADMM_OK) rc = set_plan(c, keep);
  }
  if (rc == ADMM_OK) rc = time_project(c, reps, &out->ms_tuned);
  return rc;
}

// Persisted autotuner results (environment variable ADMM_AUTOTUNE_CACHE: a
// text file, one line per key). The key names the precision and every
// cell's grid; a line holds the tile widths, x1 points and the radix plan
// of each length, then the two timings.
std::string tuning_key(const admm_ctx *c) {
  std::string k = c->fp64 ? "fp64" : "fp32";
  for (const auto &D : c->desc_h)
    k += "|" + std::to_string(D.n1) + "x" + std::to_string(D.n2) + "x" + std::to_string(D.n3);
  return k;
}

bool read_tuning(const char *path, const std::string &key, admm_tuning *t) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (!found && std::fgets(line, sizeof(line), f)) {
    char kbuf[2048];
    int off = 0;
    if (std::sscanf(line, "%2047s %d %d %d %d%n", kbuf, &t->tile_y, &t->tile_z, &t->x_points,
                    &t->n_len, &off) != 5 || key != kbuf || t->n_len < 0 || t->n_len > 24)
      continue;
    const char *p = line + off;
    bool ok = true;
    for (int k = 0; k < t->n_len && ok; ++k) {
      int n = 0, used = 0;
      ok = std::sscanf(p, " %d:%n", &n, &used) == 1;
      p += used;
      t->len[k] = n;
      for (int st = 0; st < 8; ++st) t->radix[k][st] = 0;
      for (int st = 0; ok && st < 8; ++st) {
        int r = 0;
        if (std::sscanf(p, "%d%n", &r, &used) != 1) break;
        p += used;
        t->radix[k][st] = r;
        if (*p != '.') break;
        ++p;
      }
    }
    found = ok && std::sscanf(p, " %lf %lf", &t->ms_default, &t->ms_tuned) == 2;
  }
  std::fclose(f);
  return found;
}

void write_tuning(const char *path, const std::string &key, const admm_tuning &t) {
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d", key.c_str(), t.tile_y, t.tile_z, t.x_points, t.n_len);
  for (int k = 0; k < t.n_len; ++k) {
    std::fprintf(f, " %d:", t.len[k]);
    for (int st = 0; st < 8 && t.radix[k][st]; ++st)
      std::fprintf(f, st ? ".%d" : "%d", t.radix[k][st]);
  }
  std::fprintf(f, " %.6f %.6f\n", t.ms_default, t.ms_tuned);
  std::fclose(f);
}

}  // namespace

extern "C" {

int admm_check_grid(int32_t n1, int32_t n2, int32_t n3) {
  const int n[3] = {n1, n2, n3};
  for (int k = 0; k < 3; ++k) {
    if (n[k] <= 0) return ADMM_EINVAL;
    if (k == 2 && n[k] == 1) continue;  // plane strain
    if (n[k] % 2 != 0 || n[k] < 4 || n[k] > kMaxN || !is_2a3b(n[k])) return ADMM_EUNSUPPORTED;
  }
  return ADMM_OK;
}

size_t admm_workspace_bytes(const admm_rve *rves, int32_t n_rve, int32_t precision) {
  if (!rves || n_rve <= 0 || (precision != ADMM_FP64 && precision != ADMM_FP32_FP64RED)) return 0;
  size_t total = 0;
  for (int r = 0; r < n_rve; ++r) {
    if (admm_check_grid(rves[r].n[0], rves[r].n[1], rves[r].n[2]) != ADMM_OK) return 0;
    total += spec_bytes(rves[r].n[0], rves[r].n[1], rves[r].n[2], precision == ADMM_FP64) +
             du_bytes(rves[r].n[0], rves[r].n[1], rves[r].n[2], precision == ADMM_FP64);
  }
  return total;
}

const char *admm_strerror(int code) {
  switch (code) {
    case ADMM_OK: return "ok";
    case ADMM_NOT_CONVERGED: return "not converged within the iteration cap";
    case ADMM_EINVAL: return "invalid argument";
    case ADMM_EUNSUPPORTED: return "unsupported grid size or model";
    case ADMM_EHIP: return "HIP runtime error";
    case ADMM_ENOMEM: return "workspace too small or allocation failed";
    case ADMM_EDOMAIN: return "det F <= 0 or NaN met";
    case ADMM_EDIVERGED: return "residuals diverged or stagnated";
    case ADMM_ENOGPU: return "no HIP device";
    default: return "unknown status";
  }
}

int admm_init(admm_ctx **out, const admm_rve *rves, int32_t n_rve, const admm_material *mats,
              int32_t n_mat, const admm_params *params, int32_t precision, void *workspace,
              size_t workspace_bytes, void *hip_stream) {
  if (!out) return ADMM_EINVAL;
  *out = nullptr;
  if (!rves || n_rve <= 0 || !mats || n_mat <= 0 || n_mat > 256 || !params) return ADMM_EINVAL;
  if (precision != ADMM_FP64 && precision != ADMM_FP32_FP64RED) return ADMM_EINVAL;
  bool any_lce = false, any_ext = false, any_alpha = false, any_frank = false, any_nun = false,
       any_nuF = false;
  for (int q = 0; q < n_mat; ++q) {
    const admm_material &m = mats[q];
    if (!(m.alpha >= 0.0) || !(m.frank >= 0.0) || !(m.nu_F >= 0.0) || !(m.nu_n >= 0.0))
      return ADMM_EINVAL;
    const bool lce_terms = m.alpha > 0.0 || m.frank > 0.0 || m.nu_n > 0.0;
    if (m.model == ADMM_LCE) {
      if (!(m.mu > 0.0) || !(m.a >= 1.0) || !(m.kappa >= 0.0)) return ADMM_EINVAL;
      if (lce_terms && !(m.a > 1.0)) return ADMM_EINVAL;
      any_lce = true;
    } else if (m.model == ADMM_NEOHOOKE) {
      if (!(m.mu > 0.0) || !(m.lambda >= 0.0) || lce_terms) return ADMM_EINVAL;
    } else {
      return ADMM_EINVAL;
    }
    any_ext = any_ext || lce_terms || m.nu_F > 0.0;
    any_alpha = any_alpha || m.alpha > 0.0;
    any_frank = any_frank || m.frank > 0.0;
    any_nun = any_nun || m.nu_n > 0.0;
    any_nuF = any_nuF || m.nu_F > 0.0;
  }
  const admm_params &p = *params;
  if ((any_nun || any_nuF) && !(p.dt > 0.0)) return ADMM_EINVAL;
  if (!(p.rho0 > 0.0) || !(p.rho_min > 0.0) || !(p.rho_max >= p.rho_min) || !(p.kappa_rho > 1.0) ||
      !(p.tau > 0.0) || !(p.mu_ref > 0.0) || !(p.tol_p >= 0.0) || !(p.tol_d >= 0.0) ||
      p.max_iter < 1 || p.newton_max < 1 || !(p.newton_gtol >= 0.0) || !(p.newton_step_tol >= 0.0) ||
      (p.use_graph != 0 && p.use_graph != 1) || !(p.local_ratio >= 0.0) ||
      !(p.local_fraction >= 0.0 && p.local_fraction <= 1.0) ||
      (p.local_ratio > 0.0 && p.local_fraction > 0.0) ||
      ((p.local_ratio > 0.0 || p.local_fraction > 0.0) &&
       (p.local_chunk < 1 || p.local_passes < 1)) ||
      !(p.div_growth >= 0.0) || p.stall_iters < 0)
    return ADMM_EINVAL;
  for (int r = 0; r < n_rve; ++r) {
    const admm_rve &R = rves[r];
    int g = admm_check_grid(R.n[0], R.n[1], R.n[2]);
    if (g != ADMM_OK) return g;
    if (!R.phase || !R.u || !R.u_prev || !R.F || !R.Lambda || R.u == R.u_prev) return ADMM_EINVAL;
    if (any_lce && !R.director) return ADMM_EINVAL;
    if (any_alpha && !R.director0) return ADMM_EINVAL;
    if (!valid_fbar(R.Fbar)) return ADMM_EINVAL;
  }
  const bool fp64 = precision == ADMM_FP64;
  const size_t need = admm_workspace_bytes(rves, n_rve, precision);
  if (workspace && workspace_bytes < need) return ADMM_ENOMEM;
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % 256) != 0) return ADMM_EINVAL;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ADMM_ENOGPU;

  admm_ctx *c = new (std::nothrow) admm_ctx();
  if (!c) return ADMM_ENOMEM;
  c->n_rve = n_rve;
  c->n_mat = n_mat;
  c->fp64 = fp64;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->params = p;
  c->params.check_every = p.check_every > 0 ? p.check_every : 10;
  c->rves.assign(rves, rves + n_rve);
  c->hist_cap = std::min(std::max(p.max_iter, 64), 1 << 16);

#define INIT_TRY(expr)        \
  do {                        \
    if ((expr) != hipSuccess) { \
      free_ctx(c);            \
      return ADMM_EHIP;       \
    }                         \
  } while (0)

  // workspace
  if (workspace) {
    c->workspace = workspace;
  } else {
    if (hipMalloc(&c->workspace, need) != hipSuccess) {
      free_ctx(c);
      return ADMM_ENOMEM;
    }
    c->own_workspace = true;
  }

  // twiddle pool: one table per distinct length
  std::map<int, int> tw_off;
  std::vector<double> pool_re, pool_im;
  for (int r = 0; r < n_rve; ++r)
    for (int k = 0; k < 3; ++k) {
      const int n = rves[r].n[k];
      if (tw_off.count(n)) continue;
      tw_off[n] = (int)pool_re.size();
      std::vector<double> re, im;
      twiddles(n, re, im);
      pool_re.insert(pool_re.end(), re.begin(), re.end());
      pool_im.insert(pool_im.end(), im.begin(), im.end());
    }
  const size_t ntw = pool_re.size();
  if (fp64) {
    std::vector<double2> h(ntw);
    for (size_t k = 0; k < ntw; ++k) h[k] = double2{pool_re[k], pool_im[k]};
    INIT_TRY(hipMalloc(&c->tw_d, ntw * sizeof(double2)));
    INIT_TRY(hipMemcpy(c->tw_d, h.data(), ntw * sizeof(double2), hipMemcpyHostToDevice));
  } else {
    std::vector<float2> h(ntw);
    for (size_t k = 0; k < ntw; ++k) h[k] = float2{(float)pool_re[k], (float)pool_im[k]};
    INIT_TRY(hipMalloc(&c->tw_d, ntw * sizeof(float2)));
    INIT_TRY(hipMemcpy(c->tw_d, h.data(), ntw * sizeof(float2), hipMemcpyHostToDevice));
  }

  // descriptors and workgroup prefix tables
  const int B = tile_b(fp64);
  c->desc_h.resize(n_rve);
  std::vector<int> bx(n_rve + 1), by(n_rve + 1), bz(n_rve + 1), bu(n_rve + 1), bf(n_rve + 1),
      bi(n_rve + 1);
  bx[0] = by[0] = bz[0] = bu[0] = bf[0] = 0;
  size_t spec_off = 0;
  int n2max = 0, n3max = 0, lds_x = 0;
  for (int r = 0; r < n_rve; ++r) {
    const admm_rve &R = rves[r];
    RveDesc &D = c->desc_h[r];
    std::memset(&D, 0, sizeof(D));
    D.n1 = R.n[0];
    D.n2 = R.n[1];
    D.n3 = R.n[2];
    D.m1 = D.n1 / 2 + 1;
    D.m1s = spec_stride(D.n1, fp64);
    D.V = (long long)D.n1 * D.n2 * D.n3;
    D.S = (long long)D.n3 * D.n2 * D.m1s;
    D.rows = rows_per_block(D.n1);
    D.rows_f = rows_per_fft_block(D.n1, default_fft_points(fp64));
    D.f_n1 = make_fastdiv((unsigned)D.n1);
    D.f_n2 = make_fastdiv((unsigned)D.n2);
    D.f_m1 = make_fastdiv((unsigned)D.m1);
    D.f_rows_f = make_fastdiv((unsigned)D.rows_f);
    D.p1 = make_plan(D.n1);
    D.p2 = make_plan(D.n2);
    D.p3 = make_plan(D.n3);
    D.p1.tw = tw_off[D.n1];
    D.p2.tw = tw_off[D.n2];
    D.p3.tw = tw_off[D.n3];
    D.phase = R.phase;
    D.u[0] = R.u;
    D.u[1] = R.u_prev;
    D.E = R.F;
    D.Lam = R.Lambda;
    D.dir = R.director;
    D.dir0 = R.director0;
    D.dir_lag = D.dir_step = D.E_step = nullptr;
    D.spec = static_cast<char *>(c->workspace) + spec_off;
    spec_off += spec_bytes(D.n1, D.n2, D.n3, fp64);
    D.du = fp64 ? nullptr : static_cast<char *>(c->workspace) + spec_off;
    spec_off += du_bytes(D.n1, D.n2, D.n3, fp64);
    const int nrows = D.n2 * D.n3;
    bx[r + 1] = bx[r] + (nrows + D.rows - 1) / D.rows;
    bf[r + 1] = bf[r] + (nrows + D.rows_f - 1) / D.rows_f;
    bi[r + 1] = bi[r] + (3 * nrows + 31) / 32;
    by[r + 1] = by[r] + D.n3 * ((D.m1 + B - 1) / B);
    bz[r + 1] = bz[r] + (D.n2 * D.m1s + B - 1) / B;
    bu[r + 1] = bu[r] + ((D.n2 + D.rows - 1) / D.rows) *
                            ((D.n3 + kZSeg - 1) / kZSeg);
    n2max = std::max(n2max, D.n2);
    n3max = std::max(n3max, D.n3);
    lds_x = std::max(lds_x, 2 * ((3 * D.rows_f + 1) / 2) * D.n1);
  }
  // the spectra's padding columns stay zero: no kernel writes them but the
  // x3 pass, which maps zero to zero there
  INIT_TRY(hipMemset(c->workspace, 0, spec_off));
  // float form without the full LCE model's terms or dissipation of F:
  // F - A as the local step leaves it (9 floats per voxel), read by Step 2
  // instead of F, Lambda and u; without LCE phases also Step 1's data as the
  // update forms it (9 floats) and det F - 1 of the local step's warm start
  // (one float), read by the next local step at the same penalty instead of
  // the stencil gradient of u, Lambda and F
  if (!fp64 && !any_ext) {
    const size_t per = any_lce ? 9 : 19;
    size_t tot = 0;
    for (const RveDesc &D : c->desc_h) tot += per * (size_t)D.V;
    INIT_TRY(hipMalloc(&c->at_d, tot * sizeof(float)));
    size_t off = 0;
    for (RveDesc &D : c->desc_h) {
      float *base = static_cast<float *>(c->at_d) + off;
      if (!any_lce) D.At = base;
      D.Q = base + (any_lce ? 0 : 10 * (size_t)D.V);
      off += per * (size_t)D.V;
    }
  }
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  c->L.timer = nullptr;
  c->L.any_lce = any_lce;
  c->L.lce_kind = any_ext ? 2 : (any_lce ? 1 : 0);
  c->L.any_frank = any_frank;
  c->L.any_free = false;
  c->L.stream = c->stream;
  c->L.nblk_x = bx[n_rve];
  c->L.nblk_y = by[n_rve];
  c->L.nblk_z = bz[n_rve];
  c->L.tile_y = c->L.tile_z = B;
  c->L.nblk_u = bu[n_rve];
  c->L.nblk_f = bf[n_rve];
  c->L.nblk_i = bi[n_rve];
  {
    // the register-resident inverse x1 pass: float cells, every x1 length 256
    bool all256 = !fp64;
    for (const RveDesc &D : c->desc_h) all256 = all256 && D.n1 == 256 && D.m1s >= 129;
    c->L.inv256 = all256;
  }
  c->xpoints = default_fft_points(fp64);
  c->L.n2max = n2max;
  c->L.n3max = n3max;
  c->L.lds_x = (size_t)lds_x * csz;

  // the full LCE model's copies: directors of the previous iteration (Frank
  // term), directors and F at the start of the load step (dissipation)
  c->any_frank = any_frank;
  c->any_nun = any_nun;
  c->any_nuF = any_nuF;
  {
    const size_t s = fp64 ? 8 : 4;
    for (int r = 0; r < n_rve; ++r) {
      RveDesc &D = c->desc_h[r];
      const size_t V = (size_t)D.V;
      void *q = nullptr;
      if (any_frank) {
        INIT_TRY(hipMalloc(&q, 3 * V * s));
        c->owned.push_back(q);
        D.dir_lag = q;
      }
      if (any_nun) {
        INIT_TRY(hipMalloc(&q, 3 * V * s));
        c->owned.push_back(q);
        D.dir_step = q;
      }
      if (any_nuF) {
        INIT_TRY(hipMalloc(&q, 9 * V * s));
        c->owned.push_back(q);
        D.E_step = q;
      }
    }
  }
  INIT_TRY(hipMalloc(&c->desc_d, sizeof(RveDesc) * n_rve));
  INIT_TRY(hipMemcpy(c->desc_d, c->desc_h.data(), sizeof(RveDesc) * n_rve, hipMemcpyHostToDevice));
  INIT_TRY(hipMalloc(&c->blk_d, sizeof(int) * 6 * (n_rve + 1)));
  std::vector<int> &blk_h = c->blk_h;
  blk_h.clear();
  blk_h.insert(blk_h.end(), bx.begin(), bx.end());
  blk_h.insert(blk_h.end(), by.begin(), by.end());
  blk_h.insert(blk_h.end(), bz.begin(), bz.end());
  blk_h.insert(blk_h.end(), bu.begin(), bu.end());
  blk_h.insert(blk_h.end(), bf.begin(), bf.end());
  blk_h.insert(blk_h.end(), bi.begin(), bi.end());
  INIT_TRY(hipMemcpy(c->blk_d, blk_h.data(), sizeof(int) * blk_h.size(), hipMemcpyHostToDevice));

  std::vector<Material> mh(n_mat);
  for (int q = 0; q < n_mat; ++q) {
    const admm_material &m = mats[q];
    const bool lce = m.model == ADMM_LCE;
    const int ext = (m.alpha > 0.0 || m.frank > 0.0 || m.nu_n > 0.0 || m.nu_F > 0.0) ? 1 : 0;
    mh[q] = Material{m.model, ext, m.mu, m.lambda, m.a, m.kappa,
                     lce ? m.mu * std::cbrt(m.a) : 0.0, lce ? 1.0 / m.a - 1.0 : 0.0,
                     m.mu * m.alpha, m.frank, m.nu_F, m.nu_n};
  }
  INIT_TRY(hipMalloc(&c->mats_d, sizeof(Material) * n_mat));
  INIT_TRY(hipMemcpy(c->mats_d, mh.data(), sizeof(Material) * n_mat, hipMemcpyHostToDevice));

  INIT_TRY(hipMalloc(&c->partials_d, sizeof(double4) * (size_t)c->L.nblk_x));
  INIT_TRY(hipMalloc(&c->partials18_d, sizeof(double) * 18 * (size_t)c->L.nblk_u));
  INIT_TRY(hipMalloc(&c->mean_d, sizeof(double) * 18 * n_rve));
  INIT_TRY(hipMalloc(&c->hist_d, sizeof(double) * 3 * (size_t)c->hist_cap * n_rve));
  INIT_TRY(hipMalloc(&c->lpart_d, sizeof(double2) * (size_t)c->L.nblk_x));
  INIT_TRY(hipMalloc(&c->fpart_d, sizeof(double) * 9 * (size_t)c->L.nblk_x));
  INIT_TRY(hipMalloc(&c->newton_part_d, sizeof(int2) * (size_t)c->L.nblk_x));
  INIT_TRY(hipMemset(c->newton_part_d, 0, sizeof(int2) * (size_t)c->L.nblk_x));
  INIT_TRY(hipMalloc(&c->retry_d, sizeof(unsigned) * (kThreads / 32) * (size_t)c->L.nblk_x));
  INIT_TRY(hipMemset(c->retry_d, 0, sizeof(unsigned) * (kThreads / 32) * (size_t)c->L.nblk_x));
  if (!fp64) {
    INIT_TRY(hipMalloc(&c->nullpart_d, sizeof(double) * 24 * (size_t)c->L.nblk_u));
    INIT_TRY(hipMalloc(&c->nullc_d, sizeof(double) * 24 * (size_t)n_rve));
  }

  c->state_h.assign(n_rve, RveState{});
  for (int r = 0; r < n_rve; ++r) {
    RveState &s = c->state_h[r];
    s.rho = p.rho0;
    s.rho_used = p.rho0;
    s.active = 1;
    s.status = ST_RUNNING;
    s.best_merit = s.ref_merit = HUGE_VAL;
    s.ref_iter = 0;
    for (int k = 0; k < 9; ++k) {
      s.Ebar[k] = rves[r].Fbar[k] - ((k % 4 == 0) ? 1.0 : 0.0);
      s.Ebar_prev[k] = s.Ebar[k];
    }
  }
  INIT_TRY(hipMalloc(&c->state_d, sizeof(RveState) * n_rve));
  INIT_TRY(hipMemcpy(c->state_d, c->state_h.data(), sizeof(RveState) * n_rve, hipMemcpyHostToDevice));

  KernelArgs &A = c->A;
  A.desc = c->desc_d;
  A.state = c->state_d;
  A.blk_x = c->blk_d;
  A.blk_y = c->blk_d + (n_rve + 1);
  A.blk_z = c->blk_d + 2 * (n_rve + 1);
  A.blk_u = c->blk_d + 3 * (n_rve + 1);
  A.blk_f = c->blk_d + 4 * (n_rve + 1);
  A.blk_i = c->blk_d + 5 * (n_rve + 1);
  A.mats = c->mats_d;
  A.tw = c->tw_d;
  A.partials = c->partials_d;
  A.partials18 = c->partials18_d;
  A.mean_out = c->mean_d;
  A.hist = c->hist_d;
  A.newton_part = c->newton_part_d;
  A.retry_mask = c->retry_d;
  A.nullpart = c->nullpart_d;
  A.nullc = c->nullc_d;
  A.lpart = c->lpart_d;
  A.fpart = c->fpart_d;
  A.n_rve = n_rve;
  A.n_mat = n_mat;
  if (snapshot_step(c) != ADMM_OK || hipStreamSynchronize(c->stream) != hipSuccess) {
    free_ctx(c);
    return ADMM_EHIP;
  }
#undef INIT_TRY
  *out = c;
  return ADMM_OK;
}

void admm_destroy(admm_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
}

int admm_set_load(admm_ctx *ctx, int32_t rve, const double Fbar[9]) {
  if (!ctx || !Fbar || rve < 0 || rve >= ctx->n_rve) return ADMM_EINVAL;
  if (!valid_fbar(Fbar)) return ADMM_EINVAL;
  RveState &s = ctx->state_h[rve];
  // prescribed components take the new load; free ones keep their iterate
  for (int k = 0; k < 9; ++k) {
    ctx->rves[rve].Fbar[k] = Fbar[k];
    if (!((s.free_mask >> k) & 1u)) s.Ebar[k] = Fbar[k] - ((k % 4 == 0) ? 1.0 : 0.0);
    s.Ebar_prev[k] = s.Ebar[k];
  }
  s.iter = 0;
  s.active = 1;
  s.status = ST_RUNNING;
  s.best_merit = s.ref_merit = HUGE_VAL;
  s.ref_iter = 0;
  s.newton_fail = 0;
  s.newton_iters = 0;
  s.domain_err = 0;
  int rc = upload_states(ctx);
  if (rc == ADMM_OK) rc = snapshot_step(ctx);  // a new time step starts here
  if (rc != ADMM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ADMM_OK;
}

int admm_set_free(admm_ctx *ctx, int32_t rve, uint32_t free_mask) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve || free_mask >= 512u) return ADMM_EINVAL;
  RveState &s = ctx->state_h[rve];
  s.free_mask = free_mask;
  for (int k = 0; k < 9; ++k) s.Ebar_prev[k] = s.Ebar[k];
  bool any = false;
  for (const auto &q : ctx->state_h) any = any || q.free_mask != 0;
  if (any != ctx->L.any_free) {
    drop_graphs(ctx);  // the launch sequence changes
    ctx->L.any_free = any;
  }
  int rc = upload_states(ctx);
  if (rc != ADMM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ADMM_OK;
}

int admm_get_fbar(admm_ctx *ctx, int32_t rve, double Fbar_out[9]) {
  if (!ctx || !Fbar_out || rve < 0 || rve >= ctx->n_rve) return ADMM_EINVAL;
  int rc = download_states(ctx);
  if (rc != ADMM_OK) return rc;
  for (int k = 0; k < 9; ++k)
    Fbar_out[k] = ctx->state_h[rve].Ebar[k] + ((k % 4 == 0) ? 1.0 : 0.0);
  return ADMM_OK;
}

// shared by admm_bloch and admm_bloch_static: work is null (allocate for
// the call) or the static scratch
static int bloch_call(admm_ctx *ctx, int32_t rve, const double omega[3], double rho, double tol,
                      int32_t max_iter, void *p, void *work, double *beta_out,
                      double *sigma_rho_out, int32_t *iters_out, int32_t *status_out) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve || !omega || !p || !beta_out || !(rho > 0.0) ||
      !(tol >= 0.0) || max_iter < 1)
    return ADMM_EINVAL;
  for (int j = 0; j < 3; ++j)
    if (!std::isfinite(omega[j])) return ADMM_EINVAL;
  if (!ctx->fp64 || ctx->L.lce_kind == 2) return ADMM_EUNSUPPORTED;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  // the state the context iterates on: u is the current buffer after every
  // call, and F, the director hold the last iterate
  double beta = 0.0, sr = 0.0;
  int it = 0, status = 1;
  const int rc = bloch_solve(ctx->stream, ctx->desc_h[rve], ctx->mats_d, ctx->n_mat, ctx->tw_d,
                             omega, rho, tol, max_iter, static_cast<double *>(p), work, &beta,
                             &sr, &it, &status);
  if (rc == -3) return ADMM_EDOMAIN;
  if (rc == -2) return ADMM_EINVAL;
  if (rc != 0) return ADMM_EHIP;
  *beta_out = beta;
  if (sigma_rho_out) *sigma_rho_out = sr;
  if (iters_out) *iters_out = it;
  if (status_out) *status_out = status == 0 ? ADMM_OK : ADMM_NOT_CONVERGED;
  return ADMM_OK;
}

int admm_bloch(admm_ctx *ctx, int32_t rve, const double omega[3], double rho, double tol,
               int32_t max_iter, void *p, double *beta_out, double *sigma_rho_out,
               int32_t *iters_out, int32_t *status_out) {
  return bloch_call(ctx, rve, omega, rho, tol, max_iter, p, nullptr, beta_out, sigma_rho_out,
                    iters_out, status_out);
}

size_t admm_bloch_static_max_bytes(void) { return bloch_scratch_bytes(); }

int admm_bloch_static(admm_ctx *ctx, int32_t rve, const double omega[3], double rho, double tol,
                      int32_t max_iter, void *p, double *beta_out, double *sigma_rho_out,
                      int32_t *iters_out, int32_t *status_out) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve) return ADMM_EINVAL;
  if (bloch_work_bytes(ctx->desc_h[rve]) > bloch_scratch_bytes()) return ADMM_ENOMEM;
  void *work = nullptr;
  if (bloch_scratch(&work) != 0) return ADMM_EHIP;
  return bloch_call(ctx, rve, omega, rho, tol, max_iter, p, work, beta_out, sigma_rho_out,
                    iters_out, status_out);
}

int admm_orientation(admm_ctx *ctx, int32_t rve, double S_out[9]) {
  if (!ctx || !S_out || rve < 0 || rve >= ctx->n_rve || !ctx->L.any_lce) return ADMM_EINVAL;
  HIP_TRY(launch_orientation(ctx->L, ctx->A, ctx->fp64));
  double q[18];
  HIP_TRY(hipMemcpyAsync(q, ctx->mean_d + 18 * (size_t)rve, sizeof(q), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const double cnt = q[9];
  if (!(cnt > 0.0)) return ADMM_EINVAL;
  for (int k = 0; k < 9; ++k) S_out[k] = 1.5 * (q[k] / cnt - ((k % 4 == 0) ? 1.0 / 3.0 : 0.0));
  return ADMM_OK;
}

int admm_set_rho(admm_ctx *ctx, int32_t rve, double rho) {
  if (!ctx || !(rho > 0.0) || rve >= ctx->n_rve) return ADMM_EINVAL;
  for (int r = 0; r < ctx->n_rve; ++r)
    if (rve < 0 || r == rve) ctx->state_h[r].rho = rho;
  int rc = upload_states(ctx);
  if (rc != ADMM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ADMM_OK;
}

// admm_step and the single-part entry points run every cell that has not
// failed, whatever its convergence state
static int activate_all(admm_ctx *ctx) {
  for (auto &s : ctx->state_h) {
    s.active = s.status == ST_DOMAIN ? 0 : 1;
    if (s.status != ST_DOMAIN) s.status = ST_RUNNING;
  }
  return upload_states(ctx);
}

static int any_domain(const admm_ctx *ctx) {
  for (const auto &s : ctx->state_h)
    if (s.status == ST_DOMAIN || s.domain_err) return 1;
  return 0;
}

int admm_step(admm_ctx *ctx, int32_t n_iter, double *r_p, double *r_d, double *rho) {
  if (!ctx || n_iter < 0) return ADMM_EINVAL;
  int rc = activate_all(ctx);
  if (rc != ADMM_OK) return rc;
  const IterParams ip = iter_params(ctx, 0);
  if (n_iter > 0) rc = launch(ctx, Part::StripNull, ip);
  if (rc == ADMM_OK) rc = run_iterations(ctx, ip, n_iter);
  if (rc != ADMM_OK) return rc;
  rc = settle(ctx);
  if (rc != ADMM_OK) return rc;
  for (int r = 0; r < ctx->n_rve; ++r) {
    if (r_p) r_p[r] = ctx->state_h[r].rp;
    if (r_d) r_d[r] = ctx->state_h[r].rd;
    if (rho) rho[r] = ctx->state_h[r].rho;
  }
  return any_domain(ctx) ? ADMM_EDOMAIN : ADMM_OK;
}

int admm_solve(admm_ctx *ctx, int32_t *iters_out, int32_t *status_out) {
  if (!ctx) return ADMM_EINVAL;
  for (auto &s : ctx->state_h) s.active = (s.status == ST_RUNNING) ? 1 : 0;
  int rc = upload_states(ctx);
  if (rc != ADMM_OK) return rc;
  const IterParams ip = iter_params(ctx, 1);
  const int every = ctx->params.check_every;
  rc = launch(ctx, Part::StripNull, ip);
  if (rc != ADMM_OK) return rc;
  for (;;) {
    bool any = false;
    for (const auto &s : ctx->state_h) any = any || s.active;
    if (!any) break;
    rc = run_iterations(ctx, ip, every);
    if (rc != ADMM_OK) return rc;
    rc = download_states(ctx);
    if (rc != ADMM_OK) return rc;
  }
  rc = settle(ctx);
  if (rc != ADMM_OK) return rc;
  int all = ADMM_OK;
  for (int r = 0; r < ctx->n_rve; ++r) {
    const RveState &s = ctx->state_h[r];
    int st = s.status == ST_CONVERGED  ? ADMM_OK
             : s.status == ST_DOMAIN   ? ADMM_EDOMAIN
             : s.status == ST_DIVERGED ? ADMM_EDIVERGED
                                       : ADMM_NOT_CONVERGED;
    if (iters_out) iters_out[r] = s.iter;
    if (status_out) status_out[r] = st;
    if (st == ADMM_EDOMAIN) all = ADMM_EDOMAIN;
    else if (st == ADMM_EDIVERGED && all != ADMM_EDOMAIN) all = ADMM_EDIVERGED;
    else if (st == ADMM_NOT_CONVERGED && all == ADMM_OK) all = ADMM_NOT_CONVERGED;
  }
  return all;
}

int admm_local_step(admm_ctx *ctx) {
  if (!ctx) return ADMM_EINVAL;
  int rc = activate_all(ctx);
  if (rc == ADMM_OK) rc = launch(ctx, Part::Local, iter_params(ctx, 0));
  if (rc == ADMM_OK) rc = download_states(ctx);
  if (rc != ADMM_OK) return rc;
  return any_domain(ctx) ? ADMM_EDOMAIN : ADMM_OK;
}

int admm_project_step(admm_ctx *ctx) {
  if (!ctx) return ADMM_EINVAL;
  int rc = activate_all(ctx);
  const IterParams ip = iter_params(ctx, 0);
  if (rc == ADMM_OK) rc = launch(ctx, Part::StripNull, ip);
  if (rc == ADMM_OK) rc = launch(ctx, Part::Project, ip);
  if (rc == ADMM_OK) rc = launch(ctx, Part::ComposeU, ip);
  if (rc == ADMM_OK) rc = download_states(ctx);
  return rc;
}

int admm_update_step(admm_ctx *ctx) {
  if (!ctx) return ADMM_EINVAL;
  int rc = activate_all(ctx);
  if (rc == ADMM_OK) rc = launch(ctx, Part::Update, iter_params(ctx, 0));
  if (rc == ADMM_OK) rc = settle(ctx);
  if (rc != ADMM_OK) return rc;
  return any_domain(ctx) ? ADMM_EDOMAIN : ADMM_OK;
}

int admm_homogenized_stress(admm_ctx *ctx, int32_t rve, double P_out[9], double Lambda_out[9]) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve || !P_out) return ADMM_EINVAL;
  int rc = launch(ctx, Part::MeanStress, iter_params(ctx, 0));
  if (rc != ADMM_OK) return rc;
  double h[18];
  HIP_TRY(hipMemcpyAsync(h, ctx->mean_d + 18 * rve, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  rc = download_states(ctx);
  if (rc != ADMM_OK) return rc;
  for (int k = 0; k < 9; ++k) {
    P_out[k] = h[k];
    if (Lambda_out) Lambda_out[k] = h[9 + k];
  }
  return ctx->state_h[rve].domain_err ? ADMM_EDOMAIN : ADMM_OK;
}

int admm_history(admm_ctx *ctx, int32_t rve, int32_t max_n, double *r_p, double *r_d, double *rho,
                 int32_t *n_out) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve || max_n < 0) return ADMM_EINVAL;
  const int n = std::min(std::min(ctx->state_h[rve].iter, ctx->hist_cap), (int)max_n);
  std::vector<double> h(3 * (size_t)std::max(n, 1));
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->hist_d + (size_t)rve * ctx->hist_cap * 3,
                           sizeof(double) * 3 * n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  for (int k = 0; k < n; ++k) {
    if (r_p) r_p[k] = h[3 * k];
    if (r_d) r_d[k] = h[3 * k + 1];
    if (rho) rho[k] = h[3 * k + 2];
  }
  if (n_out) *n_out = n;
  return ADMM_OK;
}

int admm_cell_info(admm_ctx *ctx, int32_t rve, int32_t *iters, int32_t *status,
                   int32_t *newton_fail, int64_t *newton_iters) {
  if (!ctx || rve < 0 || rve >= ctx->n_rve) return ADMM_EINVAL;
  const RveState &s = ctx->state_h[rve];
  if (iters) *iters = s.iter;
  if (status)
    *status = s.status == ST_CONVERGED  ? ADMM_OK
              : s.status == ST_DOMAIN   ? ADMM_EDOMAIN
              : s.status == ST_DIVERGED ? ADMM_EDIVERGED
              : s.status == ST_CAP      ? ADMM_NOT_CONVERGED
                                        : ADMM_OK;
  if (newton_fail) *newton_fail = s.newton_fail;
  if (newton_iters) *newton_iters = (int64_t)s.newton_iters;
  return ADMM_OK;
}

int admm_profile_enable(admm_ctx *ctx, int32_t on) {
  if (!ctx) return ADMM_EINVAL;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (on) {
    if (!ctx->timer) ctx->timer = new (std::nothrow) EventTimer(ctx->stream);
    if (!ctx->timer) return ADMM_ENOMEM;
    ctx->timer->reset();
    ctx->L.timer = ctx->timer;
  } else {
    ctx->L.timer = nullptr;
  }
  return ADMM_OK;
}

int admm_autotune(admm_ctx *ctx, int32_t reps, admm_tuning *out) {
  if (!ctx || !out || reps < 0) return ADMM_EINVAL;
  int rc = ADMM_OK;
  const char *cache = reps > 0 ? std::getenv("ADMM_AUTOTUNE_CACHE") : nullptr;
  const std::string key = tuning_key(ctx);
  if (cache && *cache) {
    admm_tuning t{};
    if (read_tuning(cache, key, &t) && admm_set_tuning(ctx, &t) == ADMM_OK) {
      report_tuning(ctx, out);
      out->ms_default = t.ms_default;
      out->ms_tuned = t.ms_tuned;
      return ADMM_OK;
    }
  }
  if (reps > 0) {
    KernelTimer *timer = ctx->L.timer;
    ctx->L.timer = nullptr;
    const std::vector<RveState> saved = ctx->state_h;
    for (auto &s : ctx->state_h) s.active = 1;  // Step 2 skips inactive cells
    // Step 2 timed in the form the iterations run it: reading the local
    // step's F - A where the context holds it (the spectra and correction
    // it computes are scratch, overwritten by the next iteration)
    rc = upload_states(ctx, ctx->at_d ? 1 : 0);
    if (rc == ADMM_OK) rc = tune(ctx, reps, out);
    ctx->state_h = saved;
    const int rc2 = upload_states(ctx);
    if (rc == ADMM_OK) rc = rc2;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == ADMM_OK) rc = ADMM_EHIP;
    ctx->L.timer = timer;
  } else {
    out->ms_default = out->ms_tuned = 0.0;
  }
  const double msd = out->ms_default, mst = out->ms_tuned;
  report_tuning(ctx, out);
  out->ms_default = msd;
  out->ms_tuned = mst;
  if (rc == ADMM_OK && cache && *cache) write_tuning(cache, key, *out);
  return rc;
}

int admm_set_tuning(admm_ctx *ctx, const admm_tuning *t) {
  if (!ctx || !t) return ADMM_EINVAL;
  const size_t csz = ctx->fp64 ? sizeof(double2) : sizeof(float2);
  if (!tile_ok(ctx, 2, t->tile_y) || !tile_ok(ctx, 3, t->tile_z)) return ADMM_EINVAL;
  if (t->x_points != 256 && t->x_points != 512 && t->x_points != 1024) return ADMM_EINVAL;
  for (const auto &D : ctx->desc_h)
    if (2 * (size_t)((3 * rows_per_fft_block(D.n1, t->x_points) + 1) / 2) * D.n1 * csz > 65536)
      return ADMM_EINVAL;
  if (t->n_len < 0 || t->n_len > 24) return ADMM_EINVAL;
  const std::vector<int> lens = lengths_of(ctx);
  std::vector<Plan1D> plans;
  for (int k = 0; k < t->n_len; ++k) {
    const int n = t->len[k];
    if (std::find(lens.begin(), lens.end(), n) == lens.end()) return ADMM_EINVAL;
    Plan1D p{};
    p.n = n;
    long prod = 1;
    for (int st = 0; st < 8 && t->radix[k][st]; ++st) {
      const int R = t->radix[k][st];
      if ((R != 2 && R != 3 && R != 4 && R != 8) || p.nst >= kMaxStages) return ADMM_EINVAL;
      p.rad[p.nst++] = R;
      prod *= R;
    }
    if (prod != n) return ADMM_EINVAL;
    plans.push_back(p);
  }
  int rc = ADMM_OK;
  for (const Plan1D &p : plans)
    if (rc == ADMM_OK) rc = set_plan(ctx, p);
  if (rc == ADMM_OK) rc = set_xpoints(ctx, t->x_points);
  if (rc == ADMM_OK) rc = set_tiles(ctx, t->tile_y, t->tile_z);
  return rc;
}

int admm_profile_read(admm_ctx *ctx, int32_t kernel, double *total_ms, int32_t *launches) {
  if (!ctx || kernel < 0 || kernel >= K_COUNT) return ADMM_EINVAL;
  if (!ctx->timer) {
    if (total_ms) *total_ms = 0.0;
    if (launches) *launches = 0;
    return ADMM_OK;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->timer->collect();
  if (total_ms) *total_ms = ctx->timer->total_ms(kernel);
  if (launches) *launches = ctx->timer->count(kernel);
  return ADMM_OK;
}

int admm_divergence_check(const admm_params *params, const double *r_p, const double *r_d,
                          int32_t n, int32_t *at) {
  if (!params || !at || n < 0 || (n > 0 && (!r_p || !r_d))) return ADMM_EINVAL;
  *at = -1;
  double best = HUGE_VAL, ref = HUGE_VAL;
  int ref_iter = 0;
  for (int it = 0; it < n; ++it) {
    if (r_p[it] <= params->tol_p && r_d[it] <= params->tol_d) return ADMM_OK;  // converged
    if (divergence_watch(r_p[it], r_d[it], params->tol_p, params->tol_d, it, params->div_growth,
                         params->stall_iters, best, ref, ref_iter)) {
      *at = it;
      return ADMM_OK;
    }
  }
  return ADMM_OK;
}

}  // extern "C"

namespace {

// checkpoint layout: header, then per cell its grid, radix plans, state,
// load, history and fields (see admm_get_state)
struct StateHeader {
  char magic[8];
  int32_t version, precision, n_rve, hist_cap, state_size, flags;
  int32_t tile_y, tile_z, xpoints, reserved;
};
struct CellHeader {
  int32_t n[3], nst[3], rad[3][kMaxStages];
};
constexpr char kStateMagic[8] = {'A', 'D', 'M', 'M', 'S', 'T', 'A', 'T'};
enum { SF_DIR = 1, SF_LAG = 2, SF_DSTEP = 4, SF_ESTEP = 8 };

int state_flags(const admm_ctx *c) {
  const RveDesc &D = c->desc_h[0];
  return (D.dir ? SF_DIR : 0) | (D.dir_lag ? SF_LAG : 0) | (D.dir_step ? SF_DSTEP : 0) |
         (D.E_step ? SF_ESTEP : 0);
}

// the device fields of one cell in blob order: pointer and bytes
std::vector<std::pair<void *, size_t>> state_fields(const admm_ctx *c, int r) {
  const RveDesc &D = c->desc_h[r];
  const size_t V = (size_t)D.V, s = c->fp64 ? 8 : 4;
  std::vector<std::pair<void *, size_t>> f;
  f.push_back({D.u[0], 3 * V * sizeof(double)});
  f.push_back({D.E, 9 * V * s});
  f.push_back({D.Lam, 9 * V * s});
  if (D.dir) f.push_back({D.dir, 3 * V * s});
  if (D.dir_lag) f.push_back({D.dir_lag, 3 * V * s});
  if (D.dir_step) f.push_back({D.dir_step, 3 * V * s});
  if (D.E_step) f.push_back({D.E_step, 9 * V * s});
  return f;
}

size_t state_bytes(const admm_ctx *c) {
  size_t b = sizeof(StateHeader);
  for (int r = 0; r < c->n_rve; ++r) {
    b += sizeof(CellHeader) + sizeof(RveState) + 9 * sizeof(double) +
         3 * (size_t)c->hist_cap * sizeof(double);
    for (const auto &f : state_fields(c, r)) b += f.second;
  }
  return b;
}

}  // namespace

extern "C" {

int admm_get_state(admm_ctx *ctx, void *blob, size_t *bytes) {
  if (!ctx || !bytes) return ADMM_EINVAL;
  const size_t need = state_bytes(ctx);
  if (!blob || *bytes < need) {
    const bool query = !blob;
    *bytes = need;
    return query ? ADMM_OK : ADMM_ENOMEM;
  }
  int rc = settle(ctx);  // u current in the first buffer, states read back
  if (rc != ADMM_OK) return rc;
  char *q = static_cast<char *>(blob);
  StateHeader h{};
  std::memcpy(h.magic, kStateMagic, 8);
  h.version = 1;
  h.precision = ctx->fp64 ? ADMM_FP64 : ADMM_FP32_FP64RED;
  h.n_rve = ctx->n_rve;
  h.hist_cap = ctx->hist_cap;
  h.state_size = (int32_t)sizeof(RveState);
  h.flags = state_flags(ctx);
  h.tile_y = ctx->L.tile_y;
  h.tile_z = ctx->L.tile_z;
  h.xpoints = ctx->xpoints;
  std::memcpy(q, &h, sizeof(h));
  q += sizeof(h);
  for (int r = 0; r < ctx->n_rve; ++r) {
    const RveDesc &D = ctx->desc_h[r];
    CellHeader ch{};
    const Plan1D *pl[3] = {&D.p1, &D.p2, &D.p3};
    for (int k = 0; k < 3; ++k) {
      ch.n[k] = pl[k]->n;
      ch.nst[k] = pl[k]->nst;
      for (int st = 0; st < kMaxStages; ++st) ch.rad[k][st] = st < pl[k]->nst ? pl[k]->rad[st] : 0;
    }
    std::memcpy(q, &ch, sizeof(ch));
    q += sizeof(ch);
    std::memcpy(q, &ctx->state_h[r], sizeof(RveState));
    q += sizeof(RveState);
    std::memcpy(q, ctx->rves[r].Fbar, 9 * sizeof(double));
    q += 9 * sizeof(double);
    const size_t hb = 3 * (size_t)ctx->hist_cap * sizeof(double);
    HIP_TRY(hipMemcpy(q, ctx->hist_d + (size_t)r * ctx->hist_cap * 3, hb, hipMemcpyDeviceToHost));
    q += hb;
    for (const auto &f : state_fields(ctx, r)) {
      HIP_TRY(hipMemcpy(q, f.first, f.second, hipMemcpyDeviceToHost));
      q += f.second;
    }
  }
  *bytes = need;
  return ADMM_OK;
}

int admm_set_state(admm_ctx *ctx, const void *blob, size_t bytes) {
  if (!ctx || !blob) return ADMM_EINVAL;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const size_t need = state_bytes(ctx);
  if (bytes != need) return ADMM_EINVAL;
  const char *q = static_cast<const char *>(blob);
  StateHeader h;
  std::memcpy(&h, q, sizeof(h));
  if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 1 ||
      h.precision != (ctx->fp64 ? ADMM_FP64 : ADMM_FP32_FP64RED) || h.n_rve != ctx->n_rve ||
      h.hist_cap != ctx->hist_cap || h.state_size != (int32_t)sizeof(RveState) ||
      h.flags != state_flags(ctx) || !tile_ok(ctx, 2, h.tile_y) || !tile_ok(ctx, 3, h.tile_z) ||
      (h.xpoints != 256 && h.xpoints != 512 && h.xpoints != 1024))
    return ADMM_EINVAL;
  // validate every cell before changing anything
  std::vector<CellHeader> cells(ctx->n_rve);
  {
    const char *p = q + sizeof(h);
    for (int r = 0; r < ctx->n_rve; ++r) {
      std::memcpy(&cells[r], p, sizeof(CellHeader));
      const RveDesc &D = ctx->desc_h[r];
      const int nn[3] = {D.n1, D.n2, D.n3};
      for (int k = 0; k < 3; ++k) {
        const CellHeader &c = cells[r];
        if (c.n[k] != nn[k] || c.nst[k] < 0 || c.nst[k] > kMaxStages) return ADMM_EINVAL;
        long prod = 1;
        for (int st = 0; st < c.nst[k]; ++st) {
          const int R = c.rad[k][st];
          if (R != 2 && R != 3 && R != 4 && R != 8) return ADMM_EINVAL;
          prod *= R;
        }
        if (prod != nn[k]) return ADMM_EINVAL;
      }
      p += sizeof(CellHeader) + sizeof(RveState) + 9 * sizeof(double) +
           3 * (size_t)ctx->hist_cap * sizeof(double);
      for (const auto &f : state_fields(ctx, r)) p += f.second;
    }
  }
  // launch configuration: radix plans, tiles, x1 points
  for (int r = 0; r < ctx->n_rve; ++r) {
    RveDesc &D = ctx->desc_h[r];
    Plan1D *pl[3] = {&D.p1, &D.p2, &D.p3};
    for (int k = 0; k < 3; ++k) {
      pl[k]->nst = cells[r].nst[k];
      for (int st = 0; st < kMaxStages; ++st) pl[k]->rad[st] = cells[r].rad[k][st];
      plan_divisors(*pl[k]);
    }
  }
  int rc = set_xpoints(ctx, h.xpoints);  // also uploads the descriptors
  if (rc == ADMM_OK) rc = set_tiles(ctx, h.tile_y, h.tile_z);
  if (rc != ADMM_OK) return rc;
  q += sizeof(h);
  bool any_free = false;
  for (int r = 0; r < ctx->n_rve; ++r) {
    q += sizeof(CellHeader);
    std::memcpy(&ctx->state_h[r], q, sizeof(RveState));
    ctx->state_h[r].cur = 0;
    any_free = any_free || ctx->state_h[r].free_mask != 0;
    q += sizeof(RveState);
    std::memcpy(ctx->rves[r].Fbar, q, 9 * sizeof(double));
    q += 9 * sizeof(double);
    const size_t hb = 3 * (size_t)ctx->hist_cap * sizeof(double);
    HIP_TRY(hipMemcpy(ctx->hist_d + (size_t)r * ctx->hist_cap * 3, q, hb, hipMemcpyHostToDevice));
    q += hb;
    for (const auto &f : state_fields(ctx, r)) {
      HIP_TRY(hipMemcpy(f.first, q, f.second, hipMemcpyHostToDevice));
      q += f.second;
    }
  }
  if (any_free != ctx->L.any_free) {
    drop_graphs(ctx);
    ctx->L.any_free = any_free;
  }
  rc = upload_states(ctx);
  if (rc != ADMM_OK) return rc;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ADMM_OK;
}

}  // extern "C"
