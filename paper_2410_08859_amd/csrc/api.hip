// Host driver and C ABI (include/dd_uot.h).
#include "../../include/dd_uot.h"
#include "dd_types.h"

#include <limits.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

namespace dduot {
hipError_t launch_cell_solve(const Dev& d, int cell_base, int ncells, int lcap, int tcap,
                             int precision, bool moved, bool balance, int nt, const GangLaunch& gl,
                             hipStream_t st);
hipError_t gang_occupancy(int precision, int minb, size_t lds, int* occ);
hipError_t launch_cell_prep(const Dev& d, int cell_base, int ncells, int precision, hipStream_t st);
hipError_t launch_bound_begin(unsigned long long* acc, long long* bound, hipStream_t st);
hipError_t launch_bound_step(const Dev& d, Box* tb, int cell_base, int ncell, int nbasic,
                             int precision, unsigned long long* acc, long long* bound,
                             hipStream_t st);
hipError_t set_cell_lds_limit(size_t bytes, size_t gang_bytes);
size_t gang_lds_bytes(int precision, int lcap);
size_t cell_lds_bytes(int lcap, int cap, int precision, bool moved, bool big);
hipError_t launch_fill(double* p, long n, double v, hipStream_t st);
hipError_t launch_scale_copy(double* dst, const double* src, long n, double a, hipStream_t st);
hipError_t launch_check_grids(const double* mu, const double* nu, const double* beta, long n,
                              double* flag, hipStream_t st);
hipError_t launch_aggregate(const Dev& d, double* P, int nbasic, long ngrid, hipStream_t st);
hipError_t launch_kl_chunks(const int* cp, const int* cs, const int* cl, const Prob* probs,
                            const double* P, const double* Pg, const double* nu, double* part,
                            int nchunk, hipStream_t st);
hipError_t launch_getweights(const Dev& d, int part, int blo, int bhi, int glo, int ghi, bool last,
                             int nprob, hipStream_t st);
hipError_t launch_aggregate_sel(const Dev& d, int part, int glo, int ghi, double* P, int nbasic,
                                long ngrid, hipStream_t st);
hipError_t launch_advance(long long* kstep, hipStream_t st);
hipError_t launch_line_search(const Dev& d, const int* chunk_prob, const int* chunk_start,
                              const int* chunk_len, int nchunk, int nprob, int rounds,
                              hipStream_t st);
hipError_t launch_mix(const Dev& d, int part, int glo, int ghi, int nbasic, hipStream_t st);
hipError_t launch_cell_theta(const Dev& d, int glo, int ghi, hipStream_t st);
hipError_t launch_opt_weights(const Dev& d, int part, int blo, int bhi, int glo, int ghi,
                              int nbasic, long ngrid, int nprob, const int* chunk_prob,
                              const int* chunk_start, const int* chunk_len, int nchunk,
                              int rounds, int line_rounds, double* Pt, double* Pd,
                              hipStream_t st);
hipError_t launch_certificate(const Prob& p, const double* alpha, const double* mu, const double* nu,
                              const double* px, const double* P, const double* ydel, double* bhat,
                              double* dmu, double* dnu, double* scratch, double* part, int nblk,
                              hipStream_t st);
hipError_t launch_grad_ypos(const Prob& p, const double* alpha, const double* mu, const double* nu,
                            const double* ydel, const double* bhat, double gout, double* scratch,
                            double* mom, double* out, hipStream_t st);
hipError_t set_rows_lds_limit(size_t bytes);
hipError_t launch_refine(const RefineArgs& A, int fnbasic, const double* px_c, const double* abar_c,
                         double* px_f, double* abar_f, int fn1, hipStream_t st);
hipError_t launch_interp(const double* ac, int n1c, int n2c, double* af, hipStream_t st);
size_t from_duals_lds(int s, int gcols, int hrows);
hipError_t launch_from_duals(const DualsArgs& A, int nbasic, hipStream_t st);
hipError_t gs_x_update(const Prob& p, const double* beta, const double* nu, double* alpha,
                       double* scratch, hipStream_t st);
hipError_t gs_iteration(const Prob& p, const double* alpha, const double* mu, const double* nu,
                        double* beta, double* scratch, double* part, int nblk, hipStream_t st);
hipError_t gs_alpha_from_s(const Prob& p, const double* scratch, double* alpha, hipStream_t st);
hipError_t launch_pair_terms(const Prob& p, const double* alpha, const double* beta,
                             const double* scratch, const double* mu, const double* nu,
                             double* part, int nblk, hipStream_t st);
hipError_t launch_count_nnz(const Dev& d, int b0, int nb, double thr, unsigned long long* count,
                            hipStream_t st);
}  // namespace dduot

using namespace dduot;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(DDUOT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

static const int kChunk = 16384;
static const int kLineRounds = 40;   // GetWeights line: f' evaluations per step, at most
static const int kOptRounds = 12;    // GetWeights opt: direction + search rounds per step
static const int kCertBlocks = 1024;
static const int kPoolCheck = 2;     // half-iterations between pool checks

struct dduot_handle {
  int nprob = 0;
  int precision = 32;
  int cap = 0;         // box side of the larger in-LDS cell layout
  int tcap = 0;        // fast launch tier: cells whose Y-box side fits tcap
  hipStream_t stream = nullptr;
  std::vector<Prob> probs;
  std::vector<Cell> cells;
  int ncell[2] = {0, 0};
  int boff[2][4] = {}, bn[2][4] = {};   // staggered batches: global cell ranges
  bool staggered = false;
  bool any_line = false;                 // some problem uses GetWeights line (or opt)
  bool any_opt = false;                  // some problem uses GetWeights opt
  double *d_cell_theta = nullptr, *d_cell_dir = nullptr, *d_cell_ddh = nullptr;
  double *d_Pt = nullptr, *d_Pd = nullptr;   // opt: P_theta and P_{theta + d}
  long long nrec = 0;                    // history records written (steps of batches)
  int nbasic = 0;
  long ngrid = 0;
  long maxgrid = 0;
  int nchunk = 0;
  long long k = 0;     // half-iterations done
  int hist_cap = 4096;
  // device memory
  std::vector<void*> allocs;
  Dev d{};
  Prob* d_probs = nullptr;
  Cell* d_cells = nullptr;
  int* d_basic_prob = nullptr;
  int2* d_basic_xy = nullptr;
  int* d_basic_cell[2] = {nullptr, nullptr};
  unsigned long long* d_fx = nullptr;   // fixed-point sums of the aggregation
  double *d_mu = nullptr, *d_nu = nullptr, *d_P = nullptr, *d_Pg = nullptr, *d_px = nullptr,
         *d_pxc = nullptr, *d_abar = nullptr;
  int* d_awarm = nullptr;     // per basic cell: d_abar holds a cell potential there
  double* d_abar_keep = nullptr;   // autotune: the stored potential and flags,
  int* d_awarm_keep = nullptr;     // restored before every timed solve
  Box *d_box = nullptr, *d_cbox = nullptr, *d_nbox = nullptr, *d_cellbox = nullptr;
  long *d_voff = nullptr, *d_coff = nullptr, *d_nsize = nullptr, *d_csize = nullptr,
       *d_wsize = nullptr, *d_use = nullptr;
  int2* d_nsub = nullptr;
  Box* d_tbox = nullptr;                 // pool bounds: simulated boxes
  unsigned long long* d_bacc = nullptr;  // ... their per-step sums
  long long* d_bound = nullptr;          // ... and the largest over the coming steps
  int* d_sp = nullptr;
  long long* d_need = nullptr;
  int* d_capfail = nullptr;
  // pools (grown between steps by ensure_pools; not in `allocs`)
  double *d_pool[2] = {nullptr, nullptr}, *d_cand = nullptr;
  unsigned char* d_ws = nullptr;
  long pool_cap = 0, cand_cap = 0, ws_cap = 0;
  double *d_hbar = nullptr, *d_htil = nullptr;
  int *d_iters = nullptr, *d_conv = nullptr;
  double* d_bytes = nullptr;
  double* d_terms = nullptr;
  double* d_fall = nullptr;
  double* d_ydel = nullptr;
  double *d_mom = nullptr, *d_dy = nullptr;   // Y-position gradient (allocated on first use)
  double* d_gtmp = nullptr;                   // scaled gradients for host destinations
  long long* d_kstep = nullptr;               // device copy of k
  // captured A+B step pair (hipGraph), replayed by dd_uot_iterate
  bool use_graph = false;
  int nt = 256;        // threads per cell workgroup (dd_uot_autotune)
  // gangs for the wide cells (plain separable problems): G workgroups per
  // cell, at most wpc workgroups of the gang kernel per CU
  int gang_g = 4, gang_wpc = 2;
  int gang_occ[2] = {0, 0}, n_cu = 0;   // occupancy of the variants minb = 1, 2
  GangLaunch gl{0, 0, 1, 0};
  int* d_gabort = nullptr;
  int max_tile = 0;    // largest composite tile (points)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool moved = false;
  bool balance = false;   // some problem takes the balancing step
  int *d_chunk_prob = nullptr, *d_chunk_start = nullptr, *d_chunk_len = nullptr;
  double* d_chunk_part = nullptr;
  double *d_theta = nullptr, *d_hist = nullptr;
  double *d_line = nullptr, *d_line_part = nullptr;   // GetWeights line search state
  int* d_force = nullptr;
  double *d_bhat = nullptr, *d_dmu = nullptr, *d_dnu = nullptr, *d_scratch = nullptr,
         *d_cpart = nullptr;
  bool have_cert_prob[1] = {false};
  std::vector<int> cert_done;   // per problem: certificate arrays valid
  // timing
  bool timing = false;
  bool slot_fail = false;   // some step ran out of pool space (reported by dd_uot_score)
  int polish = 0;           // global Sinkhorn iterations of the polished score bounds
  double *d_pa = nullptr, *d_pb = nullptr;   // their potentials (allocated on first use)
  unsigned long long* d_cnt = nullptr;       // per basic cell counts (allocated on first use)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<long long> timed_recs;
};

template <typename T>
static int dalloc(dduot_handle* h, T** p, size_t count) {
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, sizeof(T) * count);
  if (e != hipSuccess) return fail(DDUOT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return DDUOT_OK;
}

#define CHK(x)            \
  do {                    \
    int r_ = (x);         \
    if (r_ != DDUOT_OK) { \
      return r_;          \
    }                     \
  } while (0)

extern "C" void dd_uot_default_config(dduot_config* c) {
  memset(c, 0, sizeof(*c));
  c->h = 0.0;
  c->lambda = 1.0;
  c->eps = 0.0;
  c->cell = 4;
  c->precision = 32;
  c->getweights = DDUOT_GW_SWIFT;
  c->init = DDUOT_INIT_BLOCK;
  c->sinkhorn_err = 2e-5;
  c->sinkhorn_max_iter = 1000;
  c->fixed_inner_iters = 0;
  c->trunc = 1e-15;
  c->lenience = 0.005;
  c->box_margin = 2;
  c->box_cap = 64;
  c->translate = 1;
  c->support_only = 1;
}

extern "C" const char* dd_uot_last_error(void) { return g_err.c_str(); }

static int validate(const dduot_config* c, const double* mu, const double* nu, int idx) {
  const std::string pre = "problem " + std::to_string(idx) + ": ";
  if (!c || !mu || !nu) return fail(DDUOT_EINVAL, pre + "null config or marginal");
  if (c->n1 <= 0 || c->n2 <= 0) return fail(DDUOT_EINVAL, pre + "grid sides must be positive");
  if (c->cell < 1 || 2 * c->cell > kMaxTile)
    return fail(DDUOT_EINVAL, pre + "basic cell side must be in [1, 8]");
  if (c->n1 % (2 * c->cell) || c->n2 % (2 * c->cell))
    return fail(DDUOT_EINVAL, pre + "grid sides must be divisible by 2*cell");
  if (!(c->lambda > 0.0) || !isfinite(c->lambda)) return fail(DDUOT_EINVAL, pre + "lambda must be > 0");
  if (!(c->eps > 0.0) || !isfinite(c->eps)) return fail(DDUOT_EINVAL, pre + "eps must be > 0");
  if (!(c->h >= 0.0) || !isfinite(c->h)) return fail(DDUOT_EINVAL, pre + "h must be >= 0");
  if (c->precision != 32 && c->precision != 64)
    return fail(DDUOT_EINVAL, pre + "precision must be 32 or 64");
  if (c->getweights < 0 || c->getweights > 5) return fail(DDUOT_EINVAL, pre + "bad getweights");
  if (c->init != DDUOT_INIT_BLOCK && c->init != DDUOT_INIT_PRODUCT)
    return fail(DDUOT_EINVAL, pre + "bad init");
  if (!(c->sinkhorn_err >= 0.0)) return fail(DDUOT_EINVAL, pre + "sinkhorn_err must be >= 0");
  if (c->sinkhorn_max_iter < 1) return fail(DDUOT_EINVAL, pre + "sinkhorn_max_iter must be >= 1");
  if (c->fixed_inner_iters < 0) return fail(DDUOT_EINVAL, pre + "fixed_inner_iters must be >= 0");
  if (!(c->trunc >= 0.0)) return fail(DDUOT_EINVAL, pre + "trunc must be >= 0");
  if (!(c->lenience >= 0.0)) return fail(DDUOT_EINVAL, pre + "lenience must be >= 0");
  if (c->box_margin < 0) return fail(DDUOT_EINVAL, pre + "box_margin must be >= 0");
  if (c->translate != 0 && c->translate != 1) return fail(DDUOT_EINVAL, pre + "translate must be 0 or 1");
  if (c->balance != 0 && c->balance != 1) return fail(DDUOT_EINVAL, pre + "balance must be 0 or 1");
  if (c->support_only != 0 && c->support_only != 1)
    return fail(DDUOT_EINVAL, pre + "support_only must be 0 or 1");
  if (c->box_cap < 2 * c->cell || c->box_cap > 128)
    return fail(DDUOT_EINVAL, pre + "box_cap must be in [2*cell, 128]");
  if (c->fast_cap < 0 || c->fast_cap > 128) return fail(DDUOT_EINVAL, pre + "fast_cap must be in [0, 128]");
  const long n = (long)c->n1 * c->n2;
  double sm = 0.0, sn = 0.0;
  for (long i = 0; i < n; ++i) {
    if (!(mu[i] > 0.0) || !isfinite(mu[i]) || !(nu[i] > 0.0) || !isfinite(nu[i]))
      return fail(DDUOT_EINVAL, pre + "masses must be finite and > 0 (full support)");
    sm += mu[i];
    sn += nu[i];
  }
  // the fixed-point aggregation holds point sums below 2^13
  if (!(sm < 1024.0) || !(sn < 1024.0))
    return fail(DDUOT_EINVAL, pre + "total masses must be below 1024 (rescale the problem)");
  return DDUOT_OK;
}

// Candidate doubles and workspace bytes of one step over partition `part`
// with the basic boxes `box` (the rule of k_cell_prep).
static void step_need(const dduot_handle* h, const std::vector<Box>& box, int part, long* cand,
                      long* ws) {
  const int base = part == 0 ? 0 : h->ncell[0];
  long c = 0, w = 0;
  for (int j = 0; j < h->ncell[part]; ++j) {
    const Cell& C = h->cells[base + j];
    const Box yb = cell_ybox(C, h->probs[C.prob], box.data());
    const long ny = (long)yb.l1 * yb.l2;
    const int side = std::max(yb.l1, yb.l2);
    c += (long)C.nb * ny;
    w += (long)cell_ws_layout(h->precision == 64 ? 8 : 4, ny, side, h->moved, side > h->cap).total;
  }
  *cand = c;
  *ws = w;
}

// Grow the pools to hold at least the given sizes (doubles, doubles, bytes).
// The state pools keep their content: the current one is copied into the
// new first pool.  Any captured graph holds the old pointers and is dropped.
static int ensure_pools(dduot_handle* h, long state, long cand, long ws) {
  hipStream_t st = h->stream;
  const long floor_d = 4096;
  if (state > h->pool_cap) {
    const long cap = std::max(state, floor_d);
    double *n0 = nullptr, *n1 = nullptr;
    hipError_t e = hipMalloc((void**)&n0, sizeof(double) * cap);
    if (e == hipSuccess) e = hipMalloc((void**)&n1, sizeof(double) * cap);
    if (e != hipSuccess) {
      if (n0) (void)hipFree(n0);
      return fail(DDUOT_ENOMEM, std::string("state pool of ") + std::to_string(cap) +
                                    " doubles: " + hipGetErrorString(e));
    }
    if (h->pool_cap > 0) {
      int sp = 0;
      HIPCHK(hipMemcpyAsync(&sp, h->d_sp, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipMemcpyAsync(n0, h->d_pool[sp], sizeof(double) * h->pool_cap,
                            hipMemcpyDeviceToDevice, st));
      static const int zero = 0;
      HIPCHK(hipMemcpyAsync(h->d_sp, &zero, sizeof(int), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
      (void)hipFree(h->d_pool[0]);
      (void)hipFree(h->d_pool[1]);
    }
    h->d_pool[0] = n0;
    h->d_pool[1] = n1;
    h->pool_cap = cap;
    h->d.pool0 = n0;
    h->d.pool1 = n1;
    h->d.pool_cap = cap;
    if (h->gexec) {
      (void)hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
  }
  if (cand > h->cand_cap || ws > h->ws_cap) {
    HIPCHK(hipStreamSynchronize(st));
    if (cand > h->cand_cap) {
      const long cap = std::max(cand, floor_d);
      if (h->d_cand) (void)hipFree(h->d_cand);
      h->d_cand = nullptr;
      h->cand_cap = 0;
      hipError_t e = hipMalloc((void**)&h->d_cand, sizeof(double) * cap);
      if (e != hipSuccess)
        return fail(DDUOT_ENOMEM, std::string("candidate pool: ") + hipGetErrorString(e));
      h->cand_cap = cap;
    }
    if (ws > h->ws_cap) {
      const long cap = std::max(ws, 8 * floor_d);
      if (h->d_ws) (void)hipFree(h->d_ws);
      h->d_ws = nullptr;
      h->ws_cap = 0;
      hipError_t e = hipMalloc((void**)&h->d_ws, cap);
      if (e != hipSuccess)
        return fail(DDUOT_ENOMEM, std::string("cell workspace pool: ") + hipGetErrorString(e));
      h->ws_cap = cap;
    }
    h->d.cand = h->d_cand;
    h->d.cand_cap = h->cand_cap;
    h->d.ws = h->d_ws;
    h->d.ws_cap = h->ws_cap;
    if (h->gexec) {
      (void)hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
  }
  return DDUOT_OK;
}

// Before the next `nhalf` half-iterations: bound their pool needs on the
// device (k_bound_*: the Y-box rule replayed without truncation, step after
// step, from the current boxes), read the bounds and the failure flags, and
// grow every pool below its bound to 1.25 times the bound.  A step that
// found a pool too small (not expected under these bounds) left the cells
// that did not fit (or, for the state pool, the whole state) unchanged:
// DDUOT_ESLOT.
// Launch shape of the gangs from gang_g and gang_wpc (G = 0 when gangs are
// off or do not apply).
static void gang_shape(dduot_handle* h) {
  h->gl.G = 0;
  h->gl.nwg = 0;
  h->gl.minb = h->gang_wpc >= 2 ? 2 : 1;
  const int occ = h->gang_occ[h->gl.minb - 1];
  if (h->gang_g <= 0 || h->moved || h->balance || occ <= 0) return;
  const int per = 8 * h->gang_g;
  const int nwg = std::min(occ, h->gang_wpc) * h->n_cu / per * per;
  if (nwg < per) return;
  h->gl.G = h->gang_g;
  h->gl.nwg = nwg;
}

static int check_pools(dduot_handle* h, int nhalf) {
  hipStream_t st = h->stream;
  HIPCHK(launch_bound_begin(h->d_bacc, h->d_bound, st));
  HIPCHK(hipMemcpyAsync(h->d_tbox, h->d_box, sizeof(Box) * h->nbasic, hipMemcpyDeviceToDevice, st));
  for (int i = 0; i < nhalf; ++i) {
    const int part = (int)((h->k + i) % 2);
    if (h->staggered) {
      for (int bt = 0; bt < 4; ++bt)
        HIPCHK(launch_bound_step(h->d, h->d_tbox, h->boff[part][bt], h->bn[part][bt], h->nbasic,
                                 h->precision, h->d_bacc, h->d_bound, st));
    } else {
      HIPCHK(launch_bound_step(h->d, h->d_tbox, h->boff[part][0], h->ncell[part], h->nbasic,
                               h->precision, h->d_bacc, h->d_bound, st));
    }
  }
  long long bound[3] = {0, 0, 0};
  std::vector<int> fl(h->nprob, 0);
  HIPCHK(hipMemcpyAsync(bound, h->d_bound, sizeof(bound), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(fl.data(), h->d_capfail, sizeof(int) * h->nprob, hipMemcpyDeviceToHost, st));
  int gab = 0;
  if (h->d_gabort) HIPCHK(hipMemcpyAsync(&gab, h->d_gabort, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (gab) {
    HIPCHK(hipMemsetAsync(h->d_gabort, 0, sizeof(int), st));
    HIPCHK(hipStreamSynchronize(st));
    return fail(DDUOT_EHIP, "a gang kernel wait ran past its limit (workgroups not co-resident); "
                            "the wide cells of the steps since the last check were abandoned");
  }
  auto want = [](long long n, long cap) { return n > cap ? (long)(n + n / 4) : 0L; };
  CHK(ensure_pools(h, want(bound[0], h->pool_cap), want(bound[1], h->cand_cap),
                   want(bound[2], h->ws_cap)));
  bool failed = false;
  for (int v : fl) failed = failed || v != 0;
  if (failed) {
    std::vector<int> zeros(h->nprob, 0);
    HIPCHK(hipMemcpyAsync(h->d_capfail, zeros.data(), sizeof(int) * h->nprob, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    h->slot_fail = true;
    return fail(DDUOT_ESLOT, "a step found a pool too small (the cells that did not fit kept "
                             "their state); the pools have been grown");
  }
  return DDUOT_OK;
}

// After a kernel wrote new basic boxes into d_box: place them compactly in a
// state pool large enough for them (the first one, made current), sized with
// the candidate and workspace needs of the next steps.  Synchronises.
static int place_state(dduot_handle* h) {
  hipStream_t st = h->stream;
  std::vector<Box> box(h->nbasic);
  HIPCHK(hipMemcpyAsync(box.data(), h->d_box, sizeof(Box) * h->nbasic, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<long> off(h->nbasic, 0);
  long tot = 0;
  for (int b = 0; b < h->nbasic; ++b) {
    off[b] = tot;
    tot += (long)box[b].l1 * box[b].l2;
  }
  long cneed = 0, wneed = 0;
  for (int part = 0; part < 2; ++part) {
    long c = 0, w = 0;
    step_need(h, box, part, &c, &w);
    cneed = std::max(cneed, c);
    wneed = std::max(wneed, w);
  }
  CHK(ensure_pools(h, 2 * tot, 2 * cneed, 2 * wneed));
  HIPCHK(hipMemcpyAsync(h->d_voff, off.data(), sizeof(long) * h->nbasic, hipMemcpyHostToDevice, st));
  static const int zero = 0;
  HIPCHK(hipMemcpyAsync(h->d_sp, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return DDUOT_OK;
}

// groups of basic indices along one axis: pairs from 0 (A) or offset pairs (B)
static std::vector<std::vector<int>> axis_groups(int nb, bool offset) {
  std::vector<std::vector<int>> g;
  if (!offset) {
    for (int a = 0; a < nb / 2; ++a) g.push_back({2 * a, 2 * a + 1});
  } else {
    for (int c = 0; c < nb / 2 + 1; ++c) {
      std::vector<int> v;
      for (int b : {2 * c - 1, 2 * c})
        if (b >= 0 && b < nb) v.push_back(b);
      g.push_back(v);
    }
  }
  return g;
}

static int build(dduot_handle* h, int nprob, const dduot_config* cfgs, const double* const* mus,
                 const double* const* nus, const double* const* yps) {
  for (int k = 0; k < nprob; ++k) CHK(validate(&cfgs[k], mus[k], nus[k], k));
  // moved Y points: all problems of a handle or none (one kernel variant)
  h->moved = yps && yps[0];
  for (int k = 0; k < nprob; ++k) {
    const bool mk = yps && yps[k];
    if (mk != h->moved) return fail(DDUOT_EINVAL, "moved Y points: give them for all problems or none");
    if (!mk) continue;
    if (!(cfgs[k].h > 0.0)) return fail(DDUOT_EINVAL, "moved Y points need h > 0");
    if (cfgs[k].balance) return fail(DDUOT_EINVAL, "the balancing step needs regular Y points");
    const long n = 2L * cfgs[k].n1 * cfgs[k].n2;
    for (long i = 0; i < n; ++i)
      if (!isfinite(yps[k][i])) return fail(DDUOT_EINVAL, "moved Y points must be finite");
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int max_lds = 0;
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  h->nprob = nprob;
  h->precision = cfgs[0].precision;
  h->cap = 0;
  for (int k = 0; k < nprob; ++k) {
    if (cfgs[k].precision != h->precision)
      return fail(DDUOT_EINVAL, "all problems of a handle must share one precision");
    h->cap = std::max(h->cap, cfgs[k].box_cap);
  }
  h->staggered = cfgs[0].getweights == DDUOT_GW_STAGGERED;
  for (int k = 0; k < nprob; ++k) {
    h->any_line |= cfgs[k].getweights == DDUOT_GW_LINE || cfgs[k].getweights == DDUOT_GW_OPT;
    h->any_opt |= cfgs[k].getweights == DDUOT_GW_OPT;
  }
  for (int k = 0; k < nprob; ++k)
    if ((cfgs[k].getweights == DDUOT_GW_STAGGERED) != h->staggered)
      return fail(DDUOT_EINVAL, "staggered GetWeights: all problems of a handle or none");
  const size_t lds_cell = cell_lds_bytes(h->cap, h->cap, h->precision, h->moved, false);
  if ((long)lds_cell > max_lds)
    return fail(DDUOT_EINVAL, "box_cap too large for the LDS of one workgroup");
  // fast tier: by default the largest box side whose cell LDS lets three
  // workgroups share a CU; cells with larger boxes run in a second launch
  int lds_cu = 0;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
          hipSuccess ||
      lds_cu <= 0)
    lds_cu = max_lds;
  int fc = cfgs[0].fast_cap;
  if (fc <= 0)
    for (int c = h->cap; c >= 1; --c)
      if (3 * cell_lds_bytes(c, h->cap, h->precision, h->moved, false) <= (size_t)lds_cu) {
        fc = c;
        break;
      }
  h->tcap = (fc <= 0 || fc >= h->cap) ? h->cap : fc;
  HIPCHK(set_cell_lds_limit(lds_cell, gang_lds_bytes(h->precision, h->cap)));

  // problems, basic cells, composite cells
  std::vector<int> basic_prob;
  std::vector<int2> basic_xy;
  // cells by partition, staggered batch and problem, concatenated below
  std::vector<std::vector<std::vector<Cell>>> staged[2];
  for (int part = 0; part < 2; ++part) staged[part].assign(4, std::vector<std::vector<Cell>>(nprob));
  std::vector<int> chunk_prob, chunk_start, chunk_len;
  long goff = 0;
  for (int k = 0; k < nprob; ++k) {
    const dduot_config& c = cfgs[k];
    Prob p{};
    p.n1 = c.n1; p.n2 = c.n2; p.s = c.cell;
    p.nb1 = c.n1 / c.cell; p.nb2 = c.n2 / c.cell;
    p.h = c.h; p.eps = c.eps; p.lam = c.lambda;
    p.kappa = c.lambda / (c.lambda + c.eps);
    p.K = c.lambda / c.eps;
    p.ch = c.h * c.h / c.eps;
    p.err = c.sinkhorn_err; p.trunc = c.trunc; p.lenience = c.lenience;
    p.getweights = c.getweights; p.fixed_iters = c.fixed_inner_iters; p.max_iter = c.sinkhorn_max_iter;
    p.margin = c.box_margin; p.precision = c.precision;
    p.translate = c.translate;
    p.balance = c.balance;
    p.support = c.support_only;
    if (c.balance) h->balance = true;
    p.moved = h->moved ? 1 : 0;
    p.grid_off = (int)goff;
    p.basic_off = (int)basic_prob.size();
    p.nbasic = p.nb1 * p.nb2;
    const long n = (long)c.n1 * c.n2;
    double mm = 0.0, mn = 0.0;
    for (long i = 0; i < n; ++i) { mm += mus[k][i]; mn += nus[k][i]; }
    p.mass_mu = mm; p.mass_nu = mn;
    for (int b1 = 0; b1 < p.nb1; ++b1)
      for (int b2 = 0; b2 < p.nb2; ++b2) {
        basic_prob.push_back(k);
        basic_xy.push_back(make_int2(b1 * p.s, b2 * p.s));
      }
    for (int part = 0; part < 2; ++part) {
      auto g1 = axis_groups(p.nb1, part == 1), g2 = axis_groups(p.nb2, part == 1);
      for (int ri = 0; ri < (int)g1.size(); ++ri)
        for (int ci = 0; ci < (int)g2.size(); ++ci) {
          const auto& r = g1[ri];
          const auto& cc = g2[ci];
          Cell C{};
          C.prob = k;
          C.nb = 0;
          for (int b1 : r)
            for (int b2 : cc) C.basic[C.nb++] = p.basic_off + b1 * p.nb2 + b2;
          C.x1 = r[0] * p.s; C.x2 = cc[0] * p.s;
          C.lx1 = (int)r.size() * p.s; C.lx2 = (int)cc.size() * p.s;
          // staggered batch: parity of the cell position (no two neighbours)
          staged[part][(ri % 2) * 2 + (ci % 2)][k].push_back(C);
        }
    }
    p.chunk_off = (int)chunk_prob.size();
    for (long s0 = 0; s0 < n; s0 += kChunk) {
      chunk_prob.push_back(k);
      chunk_start.push_back((int)s0);
      chunk_len.push_back((int)std::min<long>(kChunk, n - s0));
    }
    p.nchunk = (int)chunk_prob.size() - p.chunk_off;
    h->probs.push_back(p);
    goff += n;
    h->maxgrid = std::max(h->maxgrid, n);
  }
  h->ngrid = goff;
  for (int k = 0; k < nprob; ++k) h->max_tile = std::max(h->max_tile, 4 * cfgs[k].cell * cfgs[k].cell);
  // global order: partition, batch, problem; each (partition, batch) is one
  // contiguous range of cells (one launch for all problems)
  h->cells.clear();
  for (int part = 0; part < 2; ++part) {
    const int part_start = (int)h->cells.size();
    for (int bt = 0; bt < 4; ++bt) {
      h->boff[part][bt] = (int)h->cells.size();
      for (int k = 0; k < nprob; ++k) {
        h->probs[k].cell_off[part][bt] = (int)h->cells.size();
        h->probs[k].ncell[part][bt] = (int)staged[part][bt][k].size();
        h->cells.insert(h->cells.end(), staged[part][bt][k].begin(), staged[part][bt][k].end());
      }
      h->bn[part][bt] = (int)h->cells.size() - h->boff[part][bt];
    }
    h->ncell[part] = (int)h->cells.size() - part_start;
  }
  h->nbasic = (int)basic_prob.size();
  h->nchunk = (int)chunk_prob.size();
  std::vector<int> bcell[2];
  for (int part = 0; part < 2; ++part) {
    bcell[part].assign(h->nbasic, -1);
    const int base = part == 0 ? 0 : h->ncell[0];
    for (int c = 0; c < h->ncell[part]; ++c) {
      const Cell& C = h->cells[base + c];
      for (int q = 0; q < C.nb; ++q) bcell[part][C.basic[q]] = base + c;
    }
  }

  // host start state (Sec. 4.2 product start, or the block start)
  std::vector<double> mu_all(h->ngrid), nu_all(h->ngrid), px(h->ngrid), hbar(h->nbasic);
  std::vector<double> ydel_all(h->moved ? 2 * (size_t)h->ngrid : 0);
  std::vector<Box> box(h->nbasic);
  for (int k = 0; k < nprob; ++k) {
    const Prob& p = h->probs[k];
    const long n = (long)p.n1 * p.n2;
    std::copy(mus[k], mus[k] + n, mu_all.begin() + p.grid_off);
    std::copy(nus[k], nus[k] + n, nu_all.begin() + p.grid_off);
    const double* mu = mus[k];
    const double* nu = nus[k];
    const double h2 = p.h * p.h;
    // Y coordinates in pixel units: the grid index, or y'/h for moved points
    const double* yp = h->moved ? yps[k] : nullptr;
    auto yc = [&](long g, int ax, int idx) -> double { return yp ? yp[2 * g + ax] / p.h : (double)idx; };
    // moments of nu over the whole grid (product start)
    double N0 = 0, N1a = 0, N1b = 0, N2 = 0;
    if (cfgs[k].init == DDUOT_INIT_PRODUCT) {
      for (int i1 = 0; i1 < p.n1; ++i1)
        for (int i2 = 0; i2 < p.n2; ++i2) {
          const long g = (long)i1 * p.n2 + i2;
          const double v = nu[g], u1 = yc(g, 0, i1), u2 = yc(g, 1, i2);
          N0 += v; N1a += v * u1; N1b += v * u2; N2 += v * (u1 * u1 + u2 * u2);
        }
    }
    for (int b = 0; b < p.nbasic; ++b) {
      const int gb = p.basic_off + b;
      const int x1 = basic_xy[gb].x, x2 = basic_xy[gb].y;
      // block moments (local coordinates) of mu and nu
      double m0 = 0, m1a = 0, m1b = 0, m2 = 0, v0 = 0, v1a = 0, v1b = 0, v2 = 0;
      double g1 = 0, g1b = 0, g2 = 0;   // global-coordinate moments of mu (product start)
      for (int i1 = 0; i1 < p.s; ++i1)
        for (int i2 = 0; i2 < p.s; ++i2) {
          const long g = (long)(x1 + i1) * p.n2 + (x2 + i2);
          const double m = mu[g], v = nu[g];
          const double u1 = yc(g, 0, x1 + i1) - x1, u2 = yc(g, 1, x2 + i2) - x2;
          m0 += m; m1a += m * i1; m1b += m * i2; m2 += m * ((double)i1 * i1 + (double)i2 * i2);
          v0 += v; v1a += v * u1; v1b += v * u2; v2 += v * (u1 * u1 + u2 * u2);
          const double a1 = x1 + i1, a2 = x2 + i2;
          g1 += m * a1; g1b += m * a2; g2 += m * (a1 * a1 + a2 * a2);
        }
      if (cfgs[k].init == DDUOT_INIT_BLOCK) {
        // pi_i = mu_i x (nu on X_i) / |mu_i|
        const double cost = h2 * (v0 * m2 + m0 * v2 - 2.0 * (m1a * v1a + m1b * v1b)) / m0;
        const double t = v0 / m0;
        hbar[gb] = cost + p.eps * (v0 * (-log(m0) - 1.0) + m0 * p.mass_nu) +
                   p.lam * m0 * (t * log(t) - t + 1.0);
        box[gb] = Box{x1, x2, p.s, p.s};
        for (int i1 = 0; i1 < p.s; ++i1)
          for (int i2 = 0; i2 < p.s; ++i2) {
            const long g = (long)(x1 + i1) * p.n2 + (x2 + i2);
            px[p.grid_off + g] = mu[g] * t;
          }
      } else {
        // pi = mu x nu: nu_i = |mu_i| nu, P_X = |nu| mu
        const double cost = h2 * (N0 * g2 + m0 * N2 - 2.0 * (g1 * N1a + g1b * N1b));
        const double t = p.mass_nu;
        hbar[gb] = cost + p.lam * m0 * (t * log(t) - t + 1.0);
        box[gb] = Box{0, 0, p.n1, p.n2};
        for (int i1 = 0; i1 < p.s; ++i1)
          for (int i2 = 0; i2 < p.s; ++i2) {
            const long g = (long)(x1 + i1) * p.n2 + (x2 + i2);
            px[p.grid_off + g] = mu[g] * t;
          }
      }
    }
  }

  // device buffers
  CHK(dalloc(h, &h->d_probs, nprob));
  CHK(dalloc(h, &h->d_cells, h->cells.size()));
  CHK(dalloc(h, &h->d_basic_prob, h->nbasic));
  CHK(dalloc(h, &h->d_basic_xy, h->nbasic));
  CHK(dalloc(h, &h->d_basic_cell[0], h->nbasic));
  CHK(dalloc(h, &h->d_basic_cell[1], h->nbasic));
  CHK(dalloc(h, &h->d_ydel, h->moved ? 2 * (size_t)h->ngrid : 1));
  CHK(dalloc(h, &h->d_mu, h->ngrid));
  CHK(dalloc(h, &h->d_nu, h->ngrid));
  CHK(dalloc(h, &h->d_P, h->ngrid));
  CHK(dalloc(h, &h->d_Pg, h->ngrid));
  CHK(dalloc(h, &h->d_fx, 2 * (size_t)h->ngrid));
  CHK(dalloc(h, &h->d_px, h->ngrid));
  CHK(dalloc(h, &h->d_pxc, h->ngrid));
  CHK(dalloc(h, &h->d_abar, h->ngrid));
  CHK(dalloc(h, &h->d_awarm, h->nbasic));
  CHK(dalloc(h, &h->d_box, h->nbasic));
  CHK(dalloc(h, &h->d_cbox, h->nbasic));
  CHK(dalloc(h, &h->d_nbox, h->nbasic));
  CHK(dalloc(h, &h->d_cellbox, h->cells.size()));
  CHK(dalloc(h, &h->d_voff, h->nbasic));
  CHK(dalloc(h, &h->d_coff, h->nbasic));
  CHK(dalloc(h, &h->d_nsize, h->nbasic));
  CHK(dalloc(h, &h->d_nsub, h->nbasic));
  CHK(dalloc(h, &h->d_csize, h->cells.size()));
  CHK(dalloc(h, &h->d_wsize, h->cells.size()));
  CHK(dalloc(h, &h->d_use, 4));
  CHK(dalloc(h, &h->d_sp, 1));
  CHK(dalloc(h, &h->d_need, 4));
  CHK(dalloc(h, &h->d_tbox, h->nbasic));
  CHK(dalloc(h, &h->d_bacc, 4));
  CHK(dalloc(h, &h->d_bound, 4));
  CHK(dalloc(h, &h->d_capfail, nprob));
  CHK(dalloc(h, &h->d_hbar, h->nbasic));
  CHK(dalloc(h, &h->d_htil, h->nbasic));
  CHK(dalloc(h, &h->d_iters, h->cells.size()));
  CHK(dalloc(h, &h->d_conv, h->cells.size()));
  CHK(dalloc(h, &h->d_bytes, h->cells.size()));
  CHK(dalloc(h, &h->d_terms, h->cells.size()));
  CHK(dalloc(h, &h->d_fall, h->cells.size()));
  CHK(dalloc(h, &h->d_chunk_prob, h->nchunk));
  CHK(dalloc(h, &h->d_chunk_start, h->nchunk));
  CHK(dalloc(h, &h->d_chunk_len, h->nchunk));
  CHK(dalloc(h, &h->d_chunk_part, 2 * (size_t)h->nchunk));
  CHK(dalloc(h, &h->d_line_part, 2 * (size_t)h->nchunk));
  CHK(dalloc(h, &h->d_theta, nprob));
  CHK(dalloc(h, &h->d_cell_theta, h->cells.size()));
  CHK(dalloc(h, &h->d_cell_dir, h->cells.size()));
  CHK(dalloc(h, &h->d_cell_ddh, h->cells.size()));
  if (h->any_opt) {
    CHK(dalloc(h, &h->d_Pt, h->ngrid));
    CHK(dalloc(h, &h->d_Pd, h->ngrid));
  }
  CHK(dalloc(h, &h->d_line, 8 * (size_t)nprob));
  CHK(dalloc(h, &h->d_hist, (size_t)nprob * h->hist_cap * kHistFields));
  CHK(dalloc(h, &h->d_force, nprob));
  CHK(dalloc(h, &h->d_kstep, 1));
  CHK(dalloc(h, &h->d_bhat, h->ngrid));
  CHK(dalloc(h, &h->d_dmu, h->ngrid));
  CHK(dalloc(h, &h->d_dnu, h->ngrid));
  // certificate scratch: 5 grids, then the per-block table of the dense sums
  CHK(dalloc(h, &h->d_scratch, 6 * (size_t)h->maxgrid + 4096));
  CHK(dalloc(h, &h->d_cpart, (size_t)kCertBlocks * 8));
  h->cert_done.assign(nprob, 0);

  hipStream_t st = h->stream;
  HIPCHK(hipMemcpyAsync(h->d_probs, h->probs.data(), sizeof(Prob) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_cells, h->cells.data(), sizeof(Cell) * h->cells.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_basic_prob, basic_prob.data(), sizeof(int) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_basic_xy, basic_xy.data(), sizeof(int2) * h->nbasic, hipMemcpyHostToDevice, st));
  for (int part = 0; part < 2; ++part)
    HIPCHK(hipMemcpyAsync(h->d_basic_cell[part], bcell[part].data(), sizeof(int) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_mu, mu_all.data(), sizeof(double) * h->ngrid, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_nu, nu_all.data(), sizeof(double) * h->ngrid, hipMemcpyHostToDevice, st));
  if (h->moved) {
    // displacement in pixel units, y'/h - j, per grid point
    for (int k = 0; k < nprob; ++k) {
      const Prob& p = h->probs[k];
      for (int i1 = 0; i1 < p.n1; ++i1)
        for (int i2 = 0; i2 < p.n2; ++i2) {
          const long g = (long)i1 * p.n2 + i2;
          ydel_all[2 * (p.grid_off + g)] = yps[k][2 * g] / p.h - i1;
          ydel_all[2 * (p.grid_off + g) + 1] = yps[k][2 * g + 1] / p.h - i2;
        }
    }
    HIPCHK(hipMemcpyAsync(h->d_ydel, ydel_all.data(), sizeof(double) * ydel_all.size(),
                          hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(h->d_px, px.data(), sizeof(double) * h->ngrid, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_hbar, hbar.data(), sizeof(double) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_box, box.data(), sizeof(Box) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_chunk_prob, chunk_prob.data(), sizeof(int) * h->nchunk, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_chunk_start, chunk_start.data(), sizeof(int) * h->nchunk, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_chunk_len, chunk_len.data(), sizeof(int) * h->nchunk, hipMemcpyHostToDevice, st));
  HIPCHK(launch_fill(h->d_abar, h->ngrid, 0.0, st));
  {
    std::vector<int> zw(h->nbasic, 0);
    HIPCHK(hipMemcpyAsync(h->d_awarm, zw.data(), sizeof(int) * h->nbasic, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  HIPCHK(launch_fill(h->d_hist, (long)nprob * h->hist_cap * kHistFields, 0.0, st));
  std::vector<int> zeros(nprob, 0);
  HIPCHK(hipMemcpyAsync(h->d_capfail, zeros.data(), sizeof(int) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_force, zeros.data(), sizeof(int) * nprob, hipMemcpyHostToDevice, st));
  static const long long kzeros[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(h->d_need, kzeros, sizeof(kzeros), hipMemcpyHostToDevice, st));
  static const int kzero_i = 0;
  HIPCHK(hipMemcpyAsync(h->d_sp, &kzero_i, sizeof(int), hipMemcpyHostToDevice, st));
  static const long long kzero = 0;
  HIPCHK(hipMemcpyAsync(h->d_kstep, &kzero, sizeof(long long), hipMemcpyHostToDevice, st));

  Dev& d = h->d;
  d.lcap = h->cap;
  // gangs: the wide cells' list, the gangs' slots and barrier counters, sized
  // for the most workgroups the gang kernel can keep resident
  {
    int rate_khz = 0;
    HIPCHK(hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    const size_t lds_g = gang_lds_bytes(h->precision, h->cap);
    HIPCHK(gang_occupancy(h->precision, 1, lds_g, &h->gang_occ[0]));
    HIPCHK(gang_occupancy(h->precision, 2, lds_g, &h->gang_occ[1]));
    h->gl.limit = (long long)std::max(rate_khz, 1000) * 2000;   // 2 s
    const size_t nwg = (size_t)std::max(1, std::max(h->gang_occ[0], h->gang_occ[1])) *
                       std::max(1, h->n_cu);
    CHK(dalloc(h, &d.glist, h->cells.size()));
    CHK(dalloc(h, &d.gcount, 3));
    CHK(dalloc(h, &d.gpart, 2 * nwg * 256));
    CHK(dalloc(h, &d.gxch, 2 * nwg * 16));
    CHK(dalloc(h, &d.gcnt, nwg * 64));
    CHK(dalloc(h, &h->d_gabort, 1));
    HIPCHK(hipMemsetAsync(h->d_gabort, 0, sizeof(int), st));
    HIPCHK(hipMemsetAsync(h->d_iters, 0, sizeof(int) * h->cells.size(), st));
    CHK(dalloc(h, &d.gxcd, 32));
    CHK(dalloc(h, &d.gsolo, nwg * (2 * 256 + 2 * 16)));
    d.gabort = h->d_gabort;
    gang_shape(h);
  }
  // start state: block start = nu on the block; product start = |mu_i| nu,
  // written compactly into the first state pool
  {
    std::vector<long> off(h->nbasic + 1, 0);
    for (int b = 0; b < h->nbasic; ++b) off[b + 1] = off[b] + (long)box[b].l1 * box[b].l2;
    std::vector<double> stage(off[h->nbasic]);
    for (int k = 0; k < nprob; ++k) {
      const Prob& p = h->probs[k];
      for (int b = 0; b < p.nbasic; ++b) {
        const int gb = p.basic_off + b;
        const Box& bx = box[gb];
        double m0 = 0.0;
        if (cfgs[k].init == DDUOT_INIT_PRODUCT)
          for (int i1 = 0; i1 < p.s; ++i1)
            for (int i2 = 0; i2 < p.s; ++i2)
              m0 += mus[k][(long)(basic_xy[gb].x + i1) * p.n2 + (basic_xy[gb].y + i2)];
        double* dst = stage.data() + off[gb];
        for (int a1 = 0; a1 < bx.l1; ++a1)
          for (int a2 = 0; a2 < bx.l2; ++a2) {
            const double v = nus[k][(long)(bx.o1 + a1) * p.n2 + (bx.o2 + a2)];
            dst[(size_t)a1 * bx.l2 + a2] = cfgs[k].init == DDUOT_INIT_PRODUCT ? m0 * v : v;
          }
      }
    }
    long cneed = 0, wneed = 0;
    for (int part = 0; part < 2; ++part) {
      long c = 0, w = 0;
      step_need(h, box, part, &c, &w);
      cneed = std::max(cneed, c);
      wneed = std::max(wneed, w);
    }
    CHK(ensure_pools(h, 2 * off[h->nbasic], 2 * cneed, 2 * wneed));
    HIPCHK(hipMemcpyAsync(h->d_pool[0], stage.data(), sizeof(double) * stage.size(),
                          hipMemcpyHostToDevice, st));
    off.pop_back();
    HIPCHK(hipMemcpyAsync(h->d_voff, off.data(), sizeof(long) * off.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }

  d.probs = h->d_probs;
  d.cells = h->d_cells;
  d.basic_prob = h->d_basic_prob;
  d.basic_xy = h->d_basic_xy;
  d.basic_cell[0] = h->d_basic_cell[0];
  d.basic_cell[1] = h->d_basic_cell[1];
  d.mu = h->d_mu;
  d.nu = h->d_nu;
  d.P = h->d_P;
  d.Pg = h->d_Pg;
  d.fxacc = h->d_fx;
  d.px = h->d_px;
  d.pxc = h->d_pxc;
  d.abar = h->d_abar;
  d.awarm = h->d_awarm;
  d.box = h->d_box;
  d.voff = h->d_voff;
  d.sp = h->d_sp;
  d.cbox = h->d_cbox;
  d.coff = h->d_coff;
  d.nbox = h->d_nbox;
  d.nsub = h->d_nsub;
  d.nsize = h->d_nsize;
  d.nuse = h->d_use + 2;
  d.cellbox = h->d_cellbox;
  d.csize = h->d_csize;
  d.wsize = h->d_wsize;
  d.cuse = h->d_use;
  d.need = h->d_need;
  d.cap_fail = h->d_capfail;
  d.hbar = h->d_hbar;
  d.htil = h->d_htil;
  d.cell_iters = h->d_iters;
  d.cell_conv = h->d_conv;
  d.cell_bytes = h->d_bytes;
  d.cell_terms = h->d_terms;
  d.cell_fall = h->d_fall;
  d.ydel = h->d_ydel;
  d.kstep = h->d_kstep;
  d.chunk_part = h->d_chunk_part;
  d.theta = h->d_theta;
  d.cell_theta = h->d_cell_theta;
  d.cell_dir = h->d_cell_dir;
  d.cell_ddh = h->d_cell_ddh;
  d.line = h->d_line;
  d.line_part = h->d_line_part;
  d.hist = h->d_hist;
  d.force_greedy = h->d_force;
  d.hist_cap = h->hist_cap;
  HIPCHK(hipStreamSynchronize(st));
  return DDUOT_OK;
}

static void release(dduot_handle* h) {
  if (!h) return;
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& e : h->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (void* p : h->allocs) (void)hipFree(p);
  for (void* p : {(void*)h->d_pool[0], (void*)h->d_pool[1], (void*)h->d_cand, (void*)h->d_ws})
    if (p) (void)hipFree(p);
  delete h;
}

// Does p point to device (or managed) memory?  Host memory, registered or
// not, gives false.
static bool on_device(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // plain host memory is not known to HIP
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Host copies of the inputs given in device memory (the set-up reads them on
// the host: validation, masses, start state); host inputs are used in place.
static int stage_inputs(int nprob, const dduot_config* cfgs, const double* const* in, int per_point,
                        hipStream_t st, std::vector<std::vector<double>>& keep,
                        std::vector<const double*>& out) {
  out.assign(in, in + nprob);
  keep.resize(nprob);
  bool any = false;
  for (int k = 0; k < nprob; ++k) {
    if (!on_device(in[k])) continue;
    const size_t n = (size_t)per_point * cfgs[k].n1 * cfgs[k].n2;
    keep[k].resize(n);
    HIPCHK(hipMemcpyAsync(keep[k].data(), in[k], sizeof(double) * n, hipMemcpyDeviceToHost, st));
    out[k] = keep[k].data();
    any = true;
  }
  if (any) HIPCHK(hipStreamSynchronize(st));
  return DDUOT_OK;
}

extern "C" int dd_uot_init_batch_moved(int32_t nprob, const dduot_config* cfgs,
                                       const double* const* mus, const double* const* nus,
                                       const double* const* ypos, void* hip_stream,
                                       dduot_handle** out) {
  if (!out) return fail(DDUOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (nprob < 1 || !cfgs || !mus || !nus) return fail(DDUOT_EINVAL, "need at least one problem");
  for (int k = 0; k < nprob; ++k)
    if (cfgs[k].n1 <= 0 || cfgs[k].n2 <= 0) return fail(DDUOT_EINVAL, "grid sides must be positive");
  std::vector<std::vector<double>> km, kn, ky;
  std::vector<const double*> hm, hn, hy;
  const hipStream_t st0 = static_cast<hipStream_t>(hip_stream);
  CHK(stage_inputs(nprob, cfgs, mus, 1, st0, km, hm));
  CHK(stage_inputs(nprob, cfgs, nus, 1, st0, kn, hn));
  if (ypos) CHK(stage_inputs(nprob, cfgs, ypos, 2, st0, ky, hy));
  dduot_handle* h = new dduot_handle();
  h->stream = st0;
  int r = build(h, nprob, cfgs, hm.data(), hn.data(), ypos ? hy.data() : nullptr);
  if (r != DDUOT_OK) {
    std::string keep = g_err;
    release(h);
    g_err = keep;
    return r;
  }
  *out = h;
  return DDUOT_OK;
}

extern "C" int dd_uot_init_batch(int32_t nprob, const dduot_config* cfgs, const double* const* mus,
                                 const double* const* nus, void* hip_stream, dduot_handle** out) {
  return dd_uot_init_batch_moved(nprob, cfgs, mus, nus, nullptr, hip_stream, out);
}

extern "C" int dd_uot_init(const dduot_config* cfg, const double* mu, const double* nu,
                           void* hip_stream, dduot_handle** out) {
  return dd_uot_init_batch_moved(1, cfg, &mu, &nu, nullptr, hip_stream, out);
}

extern "C" int dd_uot_init_moved(const dduot_config* cfg, const double* mu, const double* nu,
                                 const double* ypos, void* hip_stream, dduot_handle** out) {
  if (!ypos) return fail(DDUOT_EINVAL, "ypos is NULL");
  return dd_uot_init_batch_moved(1, cfg, &mu, &nu, &ypos, hip_stream, out);
}

extern "C" void dd_uot_destroy(dduot_handle* h) {
  if (h) (void)hipStreamSynchronize(h->stream);
  release(h);
}

extern "C" int32_t dd_uot_num_problems(const dduot_handle* h) { return h ? h->nprob : 0; }
extern "C" int dd_uot_launch_caps(const dduot_handle* h, int32_t* fast_cap, int32_t* box_cap) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  if (fast_cap) *fast_cap = h->tcap;
  if (box_cap) *box_cap = h->cap;
  return DDUOT_OK;
}

extern "C" int dd_uot_synchronize(dduot_handle* h) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_set_eps(dduot_handle* h, int32_t prob, double eps) {
  if (!h || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad handle or problem");
  if (!(eps > 0.0) || !isfinite(eps)) return fail(DDUOT_EINVAL, "eps must be > 0");
  Prob& p = h->probs[prob];
  p.eps = eps;
  p.kappa = p.lam / (p.lam + eps);
  p.K = p.lam / eps;
  p.ch = p.h * p.h / eps;
  HIPCHK(hipMemcpyAsync(h->d_probs + prob, &p, sizeof(Prob), hipMemcpyHostToDevice, h->stream));
  static const int one = 1;
  HIPCHK(hipMemcpyAsync(h->d_force + prob, &one, sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->cert_done[prob] = 0;
  return DDUOT_OK;
}

extern "C" int dd_uot_set_err(dduot_handle* h, int32_t prob, double err) {
  if (!h || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad handle or problem");
  if (!(err >= 0.0) || !isfinite(err)) return fail(DDUOT_EINVAL, "err must be >= 0");
  Prob& p = h->probs[prob];
  p.err = err;
  HIPCHK(hipMemcpyAsync(h->d_probs + prob, &p, sizeof(Prob), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

// One parallel DomDecIter (Algorithm 4) over the cells [lo, lo + n) of
// partition `part` (all problems), GetWeights over batches [blo, bhi).
static int dd_step(dduot_handle* h, int part, int lo, int n, int blo, int bhi) {
  hipStream_t st = h->stream;
  const Dev& d = h->d;
  HIPCHK(launch_aggregate(d, h->d_P, h->nbasic, h->ngrid, st));
  HIPCHK(launch_cell_prep(d, lo, n, h->precision, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, st));
  }
  HIPCHK(launch_cell_solve(d, lo, n, h->cap, h->tcap, h->precision, h->moved, h->balance, h->nt, h->gl,
                           st));
  if (h->timing) {
    HIPCHK(hipEventRecord(e1, st));
    h->events.push_back({e0, e1});
    h->timed_recs.push_back(h->nrec);
  }
  // greedy candidate Y-marginal: candidates of the step's basic cells, the
  // state elsewhere
  HIPCHK(launch_aggregate_sel(d, part, lo, lo + n, h->d_Pg, h->nbasic, h->ngrid, st));
  HIPCHK(launch_kl_chunks(h->d_chunk_prob, h->d_chunk_start, h->d_chunk_len, h->d_probs, h->d_P,
                          h->d_Pg, h->d_nu, h->d_chunk_part, h->nchunk, st));
  HIPCHK(launch_getweights(d, part, blo, bhi, lo, lo + n, bhi == 4, h->nprob, st));
  if (h->any_line)
    HIPCHK(launch_line_search(d, h->d_chunk_prob, h->d_chunk_start, h->d_chunk_len, h->nchunk,
                              h->nprob, kLineRounds, st));
  HIPCHK(launch_cell_theta(d, lo, lo + n, st));
  if (h->any_opt)
    HIPCHK(launch_opt_weights(d, part, blo, bhi, lo, lo + n, h->nbasic, h->ngrid, h->nprob,
                              h->d_chunk_prob, h->d_chunk_start, h->d_chunk_len, h->nchunk,
                              kOptRounds, kLineRounds, h->d_Pt, h->d_Pd, st));
  HIPCHK(launch_mix(d, part, lo, lo + n, h->nbasic, st));
  HIPCHK(launch_advance(h->d_kstep, st));
  h->nrec += 1;
  return DDUOT_OK;
}

// One half-iteration over partition `part` for all problems: one step over
// all its cells, or (staggered) one step per batch in turn.
static int half_iteration(dduot_handle* h, int part) {
  if (h->staggered) {
    for (int bt = 0; bt < 4; ++bt) CHK(dd_step(h, part, h->boff[part][bt], h->bn[part][bt], bt, bt + 1));
  } else {
    CHK(dd_step(h, part, h->boff[part][0], h->ncell[part], 0, 4));
  }
  h->k += 1;
  return DDUOT_OK;
}

static int read_records(dduot_handle* h, int prob, long long from, long long to, std::vector<double>& out) {
  out.clear();
  if (to <= from) return DDUOT_OK;
  std::vector<double> all((size_t)h->hist_cap * kHistFields);
  HIPCHK(hipMemcpy(all.data(), h->d_hist + (size_t)prob * h->hist_cap * kHistFields,
                   sizeof(double) * all.size(), hipMemcpyDeviceToHost));
  for (long long r = std::max(from, to - h->hist_cap); r < to; ++r) {
    const double* rec = all.data() + (size_t)(r % h->hist_cap) * kHistFields;
    out.insert(out.end(), rec, rec + kHistFields);
  }
  return DDUOT_OK;
}

// Capture one A half-iteration followed by one B half-iteration into a graph
// (kernels only: fills are kernels, the record index is read on the device).
static int capture_pair(dduot_handle* h) {
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t keep = h->stream;
  const long long k0 = h->k, n0 = h->nrec;
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  h->stream = h->cap_stream;
  int r = half_iteration(h, 0);
  if (r == DDUOT_OK) r = half_iteration(h, 1);
  h->stream = keep;
  h->k = k0;
  h->nrec = n0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (r != DDUOT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(DDUOT_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->gexec = nullptr;
    return fail(DDUOT_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return DDUOT_OK;
}

// Threads per cell workgroup: time the cell solve of the next partition on
// the current state for every admissible size (at least the largest tile's
// point count) and keep the fastest.  The timed solves write only candidate
// buffers and the stitched potentials; the potentials and their flags are
// restored, so the state is unchanged.
// Times the cell solves of the next partition on the current state once per
// candidate launch (threads per cell nts[c], gang shape gls[c]; nts[c] = 0:
// not admissible, ms[c] = -1) with HIP events, every time from the same
// stored potentials (their warm start); the state is left as it was.
// *pick receives the fastest candidate.
static int time_cell_solves(dduot_handle* h, int n, const int* nts, const GangLaunch* gls,
                            double* ms, int* pick) {
  hipStream_t st = h->stream;
  const int part = (int)(h->k % 2);
  const int base = h->boff[part][0];
  CHK(check_pools(h, 1));
  HIPCHK(launch_aggregate(h->d, h->d_P, h->nbasic, h->ngrid, st));
  HIPCHK(launch_cell_prep(h->d, base, h->ncell[part], h->precision, st));
  if (!h->d_abar_keep) CHK(dalloc(h, &h->d_abar_keep, h->ngrid));
  if (!h->d_awarm_keep) CHK(dalloc(h, &h->d_awarm_keep, h->nbasic));
  HIPCHK(hipMemcpyAsync(h->d_abar_keep, h->d_abar, sizeof(double) * h->ngrid, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_awarm_keep, h->d_awarm, sizeof(int) * h->nbasic, hipMemcpyDeviceToDevice, st));
  auto restore = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(h->d_abar, h->d_abar_keep, sizeof(double) * h->ngrid,
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->d_awarm, h->d_awarm_keep, sizeof(int) * h->nbasic, hipMemcpyDeviceToDevice, st);
    return e;
  };
  double best = 1e300;
  *pick = -1;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int c = 0; c < n; ++c) {
    if (nts[c] <= 0) {
      ms[c] = -1.0;
      continue;
    }
    float t = 0.0f;
    hipError_t e = restore();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess)
      e = launch_cell_solve(h->d, base, h->ncell[part], h->cap, h->tcap, h->precision, h->moved,
                            h->balance, nts[c], gls[c], st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(DDUOT_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    }
    ms[c] = t;
    if (t < best) {
      best = t;
      *pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(restore());
  HIPCHK(hipStreamSynchronize(st));
  int gab = 0;   // a gang wait that ran past its limit (not expected)
  HIPCHK(hipMemcpy(&gab, h->d_gabort, sizeof(int), hipMemcpyDeviceToHost));
  if (gab) {
    HIPCHK(hipMemset(h->d_gabort, 0, sizeof(int)));
    return fail(DDUOT_EHIP, "autotune: a gang kernel wait ran past its limit");
  }
  if (h->gexec) {   // a captured step keeps the old launch shape
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  return DDUOT_OK;
}

extern "C" int dd_uot_autotune(dduot_handle* h, int32_t* chosen, double* ms) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  const int cand[3] = {64, 128, 256};
  int nts[3];
  GangLaunch gls[3];
  for (int c = 0; c < 3; ++c) {
    nts[c] = cand[c] >= h->max_tile ? cand[c] : 0;
    gls[c] = h->gl;
  }
  double t[3];
  int pick = -1;
  CHK(time_cell_solves(h, 3, nts, gls, t, &pick));
  if (pick >= 0) h->nt = nts[pick];
  if (ms)
    for (int c = 0; c < 3; ++c) ms[c] = t[c];
  if (chosen) *chosen = h->nt;
  return DDUOT_OK;
}

extern "C" int dd_uot_autotune_gang(dduot_handle* h, int32_t* G, int32_t* wgs_per_cu, double* ms) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  const int cg[7] = {0, 2, 4, 4, 8, 8, 16}, cw[7] = {2, 2, 1, 2, 1, 2, 2};
  const int keep_g = h->gang_g, keep_w = h->gang_wpc;
  int nts[7];
  GangLaunch gls[7];
  for (int c = 0; c < 7; ++c) {
    h->gang_g = cg[c];
    h->gang_wpc = cw[c];
    gang_shape(h);
    gls[c] = h->gl;
    // a shape that does not apply (moved Y, balancing, too few workgroups)
    // falls back to one workgroup per wide cell: timed once, as candidate 0
    nts[c] = (c == 0 || h->gl.G == cg[c]) ? h->nt : 0;
  }
  h->gang_g = keep_g;
  h->gang_wpc = keep_w;
  gang_shape(h);
  double t[7];
  int pick = -1;
  CHK(time_cell_solves(h, 7, nts, gls, t, &pick));
  if (pick >= 0) {
    h->gang_g = cg[pick];
    h->gang_wpc = cw[pick];
    gang_shape(h);
  }
  if (ms)
    for (int c = 0; c < 7; ++c) ms[c] = t[c];
  if (G) *G = h->gl.G;
  if (wgs_per_cu) *wgs_per_cu = h->gl.G > 0 ? h->gang_wpc : 0;
  return DDUOT_OK;
}

extern "C" int dd_uot_set_gang(dduot_handle* h, int32_t G, int32_t wgs_per_cu, int32_t* nwg) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  if (G < 0 || G > 64 || wgs_per_cu < 1) return fail(DDUOT_EINVAL, "need 0 <= G <= 64, wgs_per_cu >= 1");
  h->gang_g = G;
  h->gang_wpc = wgs_per_cu;
  gang_shape(h);
  if (h->gexec) {   // the captured step used the old launch shape
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (nwg) *nwg = h->gl.nwg;
  return h->gl.G;
}

extern "C" int dd_uot_set_graph(dduot_handle* h, int32_t enable) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  h->use_graph = enable != 0;
  return DDUOT_OK;
}

extern "C" int dd_uot_iterate(dduot_handle* h, int32_t n_half_iters, dduot_iter_stats* stats) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  if (n_half_iters < 0) return fail(DDUOT_EINVAL, "n_half_iters must be >= 0");
  const long long r0 = h->nrec;
  // the pools are checked (and grown) before every kPoolCheck half-iterations;
  // with a graph, A+B pairs are replayed (a B step first runs alone)
  const bool graph = h->use_graph && !h->timing;
  for (int i = 0; i < n_half_iters;) {
    int chunk = std::min(n_half_iters - i, kPoolCheck);
    if (graph && h->k % 2 == 1) chunk = 1;
    CHK(check_pools(h, chunk));
    if (graph && chunk == 2) {
      if (!h->gexec) CHK(capture_pair(h));
      HIPCHK(hipGraphLaunch(h->gexec, h->stream));
      h->k += 2;
      h->nrec += h->staggered ? 8 : 2;
    } else {
      for (int j = 0; j < chunk; ++j) CHK(half_iteration(h, (int)(h->k % 2)));
    }
    i += chunk;
  }
  for (int p = 0; p < h->nprob; ++p) h->cert_done[p] = 0;
  if (stats) {
    CHK(check_pools(h, 0));
    memset(stats, 0, sizeof(*stats));
    stats->half_iters = n_half_iters;
    std::vector<double> rec;
    for (int p = 0; p < h->nprob; ++p) {
      CHK(read_records(h, p, r0, h->nrec, rec));
      for (size_t r = 0; r + kHistFields <= rec.size(); r += kHistFields) {
        const double* x = rec.data() + r;
        if (x[0] < 1.0) stats->n_safe += 1;
        stats->n_cells += (int32_t)x[3];
        stats->point_iters += (int64_t)x[4];
        stats->max_inner = std::max(stats->max_inner, (int32_t)x[5]);
        stats->n_unconverged += (int32_t)x[6];
        stats->n_overflow += (int32_t)x[7];
        stats->inner_iters += (int64_t)x[8];
      }
    }
  }
  return DDUOT_OK;
}

extern "C" int dd_uot_history(dduot_handle* h, int32_t prob, int32_t max, double* out) {
  if (!h || prob < 0 || prob >= h->nprob || max < 0 || (!out && max > 0))
    return fail(DDUOT_EINVAL, "bad arguments");
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<double> rec;
  CHK(read_records(h, prob, 0, h->nrec, rec));
  const int n = (int)(rec.size() / kHistFields);
  const int m = std::min(n, (int)max);
  std::copy(rec.begin(), rec.begin() + (size_t)m * kHistFields, out);
  return m;
}

// Re-aggregate the current state into d_P (the state Y-marginal).
static int refresh_state_marginal(dduot_handle* h) {
  HIPCHK(launch_aggregate(h->d, h->d_P, h->nbasic, h->ngrid, h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_score(dduot_handle* h, int32_t prob, dduot_score* out) {
  if (!h || !out || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  const Prob& p = h->probs[prob];
  hipStream_t st = h->stream;
  CHK(refresh_state_marginal(h));
  HIPCHK(launch_kl_chunks(h->d_chunk_prob, h->d_chunk_start, h->d_chunk_len, h->d_probs, h->d_P,
                          h->d_P, h->d_nu, h->d_chunk_part, h->nchunk, st));
  const long g = p.grid_off;
  const long n = (long)p.n1 * p.n2;
  const size_t rows = sizeof(double) * std::max(p.n1, p.n2);
  HIPCHK(set_rows_lds_limit(std::max<size_t>(rows, 1024)));
  HIPCHK(launch_certificate(p, h->d_abar + g, h->d_mu + g, h->d_nu + g, h->d_px + g, h->d_P + g,
                            h->moved ? h->d_ydel + 2 * g : nullptr, h->d_bhat + g, h->d_dmu + g,
                            h->d_dnu + g, h->d_scratch, h->d_cpart, kCertBlocks, st));
  std::vector<double> part((size_t)kCertBlocks * 8), chunks(2 * (size_t)h->nchunk), hb(p.nbasic);
  HIPCHK(hipMemcpyAsync(part.data(), h->d_cpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(chunks.data(), h->d_chunk_part, sizeof(double) * chunks.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hb.data(), h->d_hbar + p.basic_off, sizeof(double) * p.nbasic, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < kCertBlocks; ++b)
    for (int k = 0; k < 8; ++k) s[k] += part[(size_t)b * 8 + k];
  double klp = 0.0;
  for (int c = 0; c < p.nchunk; ++c) klp += chunks[2 * (size_t)(p.chunk_off + c)];
  double hs = 0.0;
  for (double v : hb) hs += v;
  const double pd = p.lam * s[0];
  const double dual = p.eps * (p.mass_mu * p.mass_nu - s[1]) - s[2] - s[3];
  out->tracked = hs + p.lam * klp;
  out->pd_gap = pd;
  out->dual = dual;
  out->primal = dual + pd;
  out->rel_pd_gap = pd / fabs(dual);
  out->l1_err_x = s[4];
  out->l1_err_y = s[5];
  out->mass_x = s[6];
  out->mass_y = s[7];
  out->half_iters = h->k;
  out->overflow = h->slot_fail ? 1 : 0;
  h->cert_done[prob] = 1;
  // sparsity (Sec. 4.2: entries above 1e-14) and the weights / convergence of
  // the recorded steps
  if (!h->d_cnt) CHK(dalloc(h, &h->d_cnt, h->nbasic));
  HIPCHK(launch_count_nnz(h->d, p.basic_off, p.nbasic, 1e-14, h->d_cnt, st));
  std::vector<unsigned long long> cnt(p.nbasic);
  HIPCHK(hipMemcpyAsync(cnt.data(), h->d_cnt, sizeof(unsigned long long) * p.nbasic,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out->nnz = 0;
  for (unsigned long long c : cnt) out->nnz += (int64_t)c;
  std::vector<double> rec;
  CHK(read_records(h, prob, 0, h->nrec, rec));
  out->n_safe = 0;
  out->n_unconverged = 0;
  for (size_t r = 0; r + kHistFields <= rec.size(); r += kHistFields) {
    if (rec[r] < 1.0) out->n_safe += 1;
    out->n_unconverged += (int64_t)rec[r + 6];
  }
  // polished bounds: pairs (alpha_k, beta_k) of global Sinkhorn iterations
  // from alpha_0 = alpha_bar (k = 0 is the certificate's pair)
  out->polish_iters = 0;
  out->dual_polished = dual;
  out->primal_polished = std::min(out->tracked, out->primal);
  if (h->polish > 0 && !h->moved) {
    if (!h->d_pa) CHK(dalloc(h, &h->d_pa, h->maxgrid));
    if (!h->d_pb) CHK(dalloc(h, &h->d_pb, h->maxgrid));
    HIPCHK(hipMemcpyAsync(h->d_pa, h->d_abar + g, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(set_rows_lds_limit(std::max<size_t>(rows, 1024)));
    std::vector<double> pt((size_t)kCertBlocks * 4);
    for (int k = 1; k <= h->polish; ++k) {
      // alpha_k = X-update(beta_{k-1}), i.e. -eps kappa S of the previous pair
      if (k == 1) {
        HIPCHK(gs_x_update(p, h->d_bhat + g, h->d_nu + g, h->d_pa, h->d_scratch, st));
      } else {
        HIPCHK(gs_alpha_from_s(p, h->d_scratch, h->d_pa, st));
      }
      HIPCHK(gs_iteration(p, h->d_pa, h->d_mu + g, h->d_nu + g, h->d_pb, h->d_scratch,
                          h->d_cpart + 4 * kCertBlocks, kCertBlocks, st));
      HIPCHK(launch_pair_terms(p, h->d_pa, h->d_pb, h->d_scratch, h->d_mu + g, h->d_nu + g,
                               h->d_cpart, kCertBlocks, st));
      HIPCHK(hipMemcpyAsync(pt.data(), h->d_cpart, sizeof(double) * pt.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      double q[4] = {0, 0, 0, 0};
      for (int b = 0; b < kCertBlocks; ++b)
        for (int j = 0; j < 4; ++j) q[j] += pt[(size_t)b * 4 + j];
      const double dk = p.eps * (p.mass_mu * p.mass_nu - q[1]) - q[2] - q[3];
      const double ek = dk + p.lam * q[0];
      out->dual_polished = std::max(out->dual_polished, dk);
      out->primal_polished = std::min(out->primal_polished, ek);
      out->polish_iters = k;
    }
  }
  out->rel_gap_polished = (out->primal_polished - out->dual_polished) / fabs(out->dual_polished);
  (void)n;
  return DDUOT_OK;
}

extern "C" int dd_uot_set_polish(dduot_handle* h, int32_t n_iters) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  if (n_iters < 0 || n_iters > 10000) return fail(DDUOT_EINVAL, "n_iters must be in [0, 10000]");
  h->polish = n_iters;
  return DDUOT_OK;
}

extern "C" int dd_uot_marginals(dduot_handle* h, int32_t prob, double* px, double* py) {
  if (!h || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  const Prob& p = h->probs[prob];
  const long n = (long)p.n1 * p.n2;
  CHK(refresh_state_marginal(h));
  if (px) HIPCHK(hipMemcpyAsync(px, h->d_px + p.grid_off, sizeof(double) * n, hipMemcpyDefault, h->stream));
  if (py) HIPCHK(hipMemcpyAsync(py, h->d_P + p.grid_off, sizeof(double) * n, hipMemcpyDefault, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_basic_marginal(dduot_handle* h, int32_t prob, int32_t basic, int32_t box[4],
                                     double* values, int64_t cap) {
  if (!h || !box || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  const Prob& p = h->probs[prob];
  if (basic < 0 || basic >= p.nbasic) return fail(DDUOT_EINVAL, "basic cell out of range");
  const int gb = p.basic_off + basic;
  Box b;
  long off = 0;
  int sp = 0;
  HIPCHK(hipMemcpyAsync(&b, h->d_box + gb, sizeof(Box), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&off, h->d_voff + gb, sizeof(long), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&sp, h->d_sp, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  box[0] = b.o1; box[1] = b.o2; box[2] = b.l1; box[3] = b.l2;
  const int64_t n = (int64_t)b.l1 * b.l2;
  if (values && n > cap) return fail(DDUOT_EINVAL, "values buffer too small");
  if (n > 0 && values) {
    HIPCHK(hipMemcpyAsync(values, h->d_pool[sp] + off, sizeof(double) * n,
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return DDUOT_OK;
}

extern "C" int dd_uot_get_state(dduot_handle* h, int32_t* boxes, double* values, int64_t cap,
                                int64_t* n_values, double* px, double* hbar, double* abar,
                                int32_t* warm, int64_t* k) {
  if (!h || h->nprob != 1) return fail(DDUOT_EINVAL, "state access needs a single-problem handle");
  hipStream_t st = h->stream;
  const long n = (long)h->probs[0].n1 * h->probs[0].n2;
  std::vector<Box> bx(h->nbasic);
  std::vector<long> off(h->nbasic);
  int sp = 0;
  HIPCHK(hipMemcpyAsync(bx.data(), h->d_box, sizeof(Box) * h->nbasic, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(off.data(), h->d_voff, sizeof(long) * h->nbasic, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&sp, h->d_sp, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // the pool is compact in basic order: its first `tot` entries are the values
  long tot = 0;
  for (int b = 0; b < h->nbasic; ++b) {
    if (off[b] != tot) return fail(DDUOT_EHIP, "state pool not compact");
    tot += (long)bx[b].l1 * bx[b].l2;
  }
  if (n_values) *n_values = tot;
  if (values && cap < tot) return fail(DDUOT_EINVAL, "values buffer too small");
  if (boxes)
    for (int b = 0; b < h->nbasic; ++b) {
      boxes[4 * b] = bx[b].o1; boxes[4 * b + 1] = bx[b].o2;
      boxes[4 * b + 2] = bx[b].l1; boxes[4 * b + 3] = bx[b].l2;
    }
  if (values && tot > 0)
    HIPCHK(hipMemcpyAsync(values, h->d_pool[sp], sizeof(double) * tot, hipMemcpyDeviceToHost, st));
  if (px) HIPCHK(hipMemcpyAsync(px, h->d_px, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (hbar) HIPCHK(hipMemcpyAsync(hbar, h->d_hbar, sizeof(double) * h->nbasic, hipMemcpyDeviceToHost, st));
  if (abar) HIPCHK(hipMemcpyAsync(abar, h->d_abar, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (warm) HIPCHK(hipMemcpyAsync(warm, h->d_awarm, sizeof(int) * h->nbasic, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (k) *k = h->k;
  return DDUOT_OK;
}

extern "C" int dd_uot_set_state(dduot_handle* h, const int32_t* boxes, const double* values,
                                int64_t n_values, const double* px, const double* hbar,
                                const double* abar, const int32_t* warm, int64_t k,
                                int32_t force_greedy) {
  if (!h || h->nprob != 1) return fail(DDUOT_EINVAL, "state access needs a single-problem handle");
  if (!boxes || !values || !px || !hbar || !abar || !warm || k < 0)
    return fail(DDUOT_EINVAL, "null state array or negative k");
  const Prob& p = h->probs[0];
  const long n = (long)p.n1 * p.n2;
  std::vector<Box> bx(h->nbasic);
  long tot = 0;
  for (int b = 0; b < h->nbasic; ++b) {
    Box q{boxes[4 * b], boxes[4 * b + 1], boxes[4 * b + 2], boxes[4 * b + 3]};
    if (q.l1 < 0 || q.l2 < 0 || q.o1 < 0 || q.o2 < 0 || q.o1 + q.l1 > p.n1 || q.o2 + q.l2 > p.n2)
      return fail(DDUOT_EINVAL, "box outside the grid");
    bx[b] = q;
    tot += (long)q.l1 * q.l2;
  }
  if (tot != n_values) return fail(DDUOT_EINVAL, "n_values differs from the boxes' total area");
  for (long i = 0; i < tot; ++i)
    if (!(values[i] >= 0.0) || !isfinite(values[i])) return fail(DDUOT_EINVAL, "values must be finite and >= 0");
  hipStream_t st = h->stream;
  HIPCHK(hipMemcpyAsync(h->d_box, bx.data(), sizeof(Box) * h->nbasic, hipMemcpyHostToDevice, st));
  CHK(place_state(h));   // offsets, pools sized for the boxes, first pool current
  if (tot > 0)
    HIPCHK(hipMemcpyAsync(h->d_pool[0], values, sizeof(double) * tot, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_px, px, sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_hbar, hbar, sizeof(double) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_abar, abar, sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_awarm, warm, sizeof(int) * h->nbasic, hipMemcpyHostToDevice, st));
  const int fg = force_greedy ? 1 : 0;
  HIPCHK(hipMemcpyAsync(h->d_force, &fg, sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  h->k = k;
  h->cert_done[0] = 0;
  return DDUOT_OK;
}

extern "C" int dd_uot_potentials(dduot_handle* h, int32_t prob, double* alpha, double* beta_hat) {
  if (!h || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  const Prob& p = h->probs[prob];
  const long n = (long)p.n1 * p.n2;
  if (beta_hat && !h->cert_done[prob]) return fail(DDUOT_ESTATE, "beta_hat needs dd_uot_score first");
  if (alpha) HIPCHK(hipMemcpyAsync(alpha, h->d_abar + p.grid_off, sizeof(double) * n, hipMemcpyDefault, h->stream));
  if (beta_hat) HIPCHK(hipMemcpyAsync(beta_hat, h->d_bhat + p.grid_off, sizeof(double) * n, hipMemcpyDefault, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_backward(dduot_handle* h, int32_t prob, double gout, double* dmu, double* dnu) {
  if (!h || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  if (!h->cert_done[prob]) return fail(DDUOT_ESTATE, "call dd_uot_score before dd_uot_backward");
  const Prob& p = h->probs[prob];
  const long n = (long)p.n1 * p.n2;
  // gout * gradient on the device: into a device destination directly, else
  // into a device buffer copied out
  if ((dmu && !on_device(dmu)) || (dnu && !on_device(dnu)))
    if (!h->d_gtmp) CHK(dalloc(h, &h->d_gtmp, 2 * (size_t)h->maxgrid));
  double* outs[2] = {dmu, dnu};
  const double* src[2] = {h->d_dmu + p.grid_off, h->d_dnu + p.grid_off};
  for (int q = 0; q < 2; ++q) {
    if (!outs[q]) continue;
    const bool dev = on_device(outs[q]);
    double* dst = dev ? outs[q] : h->d_gtmp + (size_t)q * h->maxgrid;
    HIPCHK(launch_scale_copy(dst, src[q], n, gout, h->stream));
    if (!dev)
      HIPCHK(hipMemcpyAsync(outs[q], dst, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_backward_ypos(dduot_handle* h, int32_t prob, double gout, double* dypos) {
  if (!h || !dypos || prob < 0 || prob >= h->nprob) return fail(DDUOT_EINVAL, "bad arguments");
  if (!h->cert_done[prob]) return fail(DDUOT_ESTATE, "call dd_uot_score before dd_uot_backward_ypos");
  const Prob& p = h->probs[prob];
  if (!(p.h > 0.0)) return fail(DDUOT_EINVAL, "the Y-position gradient needs h > 0");
  const long n = (long)p.n1 * p.n2;
  const long g = p.grid_off;
  if (!h->d_mom) CHK(dalloc(h, &h->d_mom, 2 * (size_t)h->maxgrid));
  if (!h->d_dy) CHK(dalloc(h, &h->d_dy, 2 * (size_t)h->maxgrid));
  HIPCHK(launch_grad_ypos(p, h->d_abar + g, h->d_mu + g, h->d_nu + g,
                          h->moved ? h->d_ydel + 2 * g : nullptr, h->d_bhat + g, gout, h->d_scratch,
                          h->d_mom, h->d_dy, h->stream));
  HIPCHK(hipMemcpyAsync(dypos, h->d_dy, sizeof(double) * 2 * n, hipMemcpyDefault, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDUOT_OK;
}

extern "C" int dd_uot_set_timing(dduot_handle* h, int32_t enable) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  for (auto& e : h->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  h->events.clear();
  h->timed_recs.clear();
  h->timing = enable != 0;
  return DDUOT_OK;
}

extern "C" int dd_uot_kernel_time(dduot_handle* h, int64_t* launches, double* total_ms, double* algo_bytes) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  double ms = 0.0;
  for (auto& e : h->events) {
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
    ms += t;
  }
  double bytes = 0.0;
  for (int p = 0; p < h->nprob; ++p) {
    std::vector<double> all((size_t)h->hist_cap * kHistFields);
    HIPCHK(hipMemcpy(all.data(), h->d_hist + (size_t)p * h->hist_cap * kHistFields,
                     sizeof(double) * all.size(), hipMemcpyDeviceToHost));
    for (long long r : h->timed_recs) bytes += all[(size_t)(r % h->hist_cap) * kHistFields + 9];
  }
  if (launches) *launches = (int64_t)h->events.size();
  if (total_ms) *total_ms = ms;
  if (algo_bytes) *algo_bytes = bytes;
  return DDUOT_OK;
}

extern "C" int dd_uot_cell_stats(dduot_handle* h, int32_t part, int32_t max, int32_t* boxes,
                                 int32_t* iters, double* terms) {
  if (!h) return fail(DDUOT_EINVAL, "null handle");
  if (part != 0 && part != 1) return fail(DDUOT_EINVAL, "part must be 0 (A) or 1 (B)");
  const int base = h->boff[part][0], n = h->ncell[part];
  if (max < n) return fail(DDUOT_EINVAL, "max smaller than the partition's cell count");
  HIPCHK(hipStreamSynchronize(h->stream));
  if (boxes) {
    std::vector<Box> b(n);
    HIPCHK(hipMemcpy(b.data(), h->d_cellbox + base, sizeof(Box) * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
      boxes[4 * i] = b[i].o1;
      boxes[4 * i + 1] = b[i].o2;
      boxes[4 * i + 2] = b[i].l1;
      boxes[4 * i + 3] = b[i].l2;
    }
  }
  if (iters) HIPCHK(hipMemcpy(iters, h->d_iters + base, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (terms) HIPCHK(hipMemcpy(terms, h->d_terms + base, sizeof(double) * n, hipMemcpyDeviceToHost));
  return n;
}

// ---------------------------------------------------------------------------
// Multiscale: refinement of a state to the next finer grid, and the driver
// ---------------------------------------------------------------------------
extern "C" int dd_uot_refine(dduot_handle* coarse, const dduot_config* cfg, const double* mu,
                             const double* nu, void* hip_stream, dduot_handle** out) {
  if (!out) return fail(DDUOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!coarse || !cfg) return fail(DDUOT_EINVAL, "null handle or config");
  if (coarse->nprob != 1) return fail(DDUOT_EINVAL, "refinement needs a single-problem handle");
  if (coarse->moved) return fail(DDUOT_EINVAL, "refinement of moved Y points is not supported");
  const Prob& pc = coarse->probs[0];
  if (cfg->n1 != 2 * pc.n1 || cfg->n2 != 2 * pc.n2)
    return fail(DDUOT_EINVAL, "the fine grid must have twice the coarse points per axis");
  // every fine basic cell (cell fine points = cell/2 coarse points) must lie
  // inside one coarse basic cell
  if (cfg->cell > 2 * pc.s || (cfg->cell % 2 == 0 && (2 * pc.s) % cfg->cell) ||
      (cfg->cell % 2 == 1 && cfg->cell != 1))
    return fail(DDUOT_EINVAL, "each fine basic cell must lie inside one coarse basic cell");
  if (cfg->precision != coarse->precision)
    return fail(DDUOT_EINVAL, "coarse and fine precision differ");
  dduot_config c = *cfg;
  c.init = DDUOT_INIT_BLOCK;   // placeholder state, overwritten below
  dduot_handle* h = nullptr;
  CHK(dd_uot_init(&c, mu, nu, hip_stream, &h));
  // the coarse work must be complete before the fine stream reads its state
  if (coarse->stream != h->stream) {
    hipError_t e = hipStreamSynchronize(coarse->stream);
    if (e != hipSuccess) {
      dd_uot_destroy(h);
      return fail(DDUOT_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
  }
  auto body = [&]() -> int {
    hipStream_t st = h->stream;
    const Prob& pf = h->probs[0];
    int csp = 0;
    HIPCHK(hipMemcpyAsync(&csp, coarse->d_sp, sizeof(int), hipMemcpyDeviceToHost, coarse->stream));
    HIPCHK(hipStreamSynchronize(coarse->stream));
    RefineArgs A{};
    A.cbox = coarse->d_box;
    A.cvals = coarse->d_pool[csp];
    A.cvoff = coarse->d_voff;
    A.mu_c = coarse->d_mu;
    A.nu_c = coarse->d_nu;
    A.chbar = coarse->d_hbar;
    A.cn2 = pc.n2;
    A.cs = pc.s;
    A.cnb2 = pc.nb2;
    A.fxy = h->d_basic_xy;
    A.mu_f = h->d_mu;
    A.nu_f = h->d_nu;
    A.fn2 = pf.n2;
    A.fs = pf.s;
    A.trunc = pf.trunc;
    A.fbox = h->d_box;
    A.fwarm = h->d_awarm;
    A.cwarm = coarse->d_awarm;
    A.fvoff = h->d_voff;
    A.fhbar = h->d_hbar;
    A.phase = 0;
    HIPCHK(launch_refine(A, pf.nbasic, coarse->d_px, coarse->d_abar, h->d_px, h->d_abar, pf.n1, st));
    CHK(place_state(h));
    A.fvals = h->d_pool[0];
    A.phase = 1;
    HIPCHK(launch_refine(A, pf.nbasic, coarse->d_px, coarse->d_abar, h->d_px, h->d_abar, pf.n1, st));
    // the tracked pieces of the refined state are only estimates: the next
    // half-iteration is greedy, which recomputes them
    static const int one = 1;
    HIPCHK(hipMemcpyAsync(h->d_force, &one, sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return DDUOT_OK;
  };
  int r = body();
  if (r != DDUOT_OK) {
    std::string keep = g_err;
    dd_uot_destroy(h);
    g_err = keep;
    return r;
  }
  *out = h;
  return DDUOT_OK;
}


// ---- global Sinkhorn warm start (Sec. 4.4) and potential-based refinement ----
static const int kGsBlocks = 256;

static Prob grid_prob(const dduot_config* c) {
  Prob p{};
  p.n1 = c->n1; p.n2 = c->n2; p.s = c->cell;
  p.h = c->h; p.eps = c->eps; p.lam = c->lambda;
  p.kappa = c->lambda / (c->lambda + c->eps);
  p.K = c->lambda / c->eps;
  p.ch = c->h * c->h / c->eps;
  return p;
}

// Global Sinkhorn on device grids, the iteration of the oracle's uot.sinkhorn:
// alpha = X-update(beta); then per iteration the Y-update, the gap
// KL(P_X pi | e^{-alpha/lam} mu) of the pair (alpha, beta), stop if <= tol,
// else the X-update.  scratch: 5 grids; part: kGsBlocks doubles.
static int gs_solve(const Prob& p, const double* mu, const double* nu, double* alpha, double* beta,
                    double* scratch, double* part, int max_iter, double tol, hipStream_t st,
                    int* iters, double* pd_out) {
  HIPCHK(set_rows_lds_limit(std::max<size_t>(sizeof(double) * std::max(p.n1, p.n2), 1024)));
  HIPCHK(gs_x_update(p, beta, nu, alpha, scratch, st));
  double hp[kGsBlocks];
  double pd = INFINITY;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    HIPCHK(gs_iteration(p, alpha, mu, nu, beta, scratch, part, kGsBlocks, st));
    HIPCHK(hipMemcpyAsync(hp, part, sizeof(double) * kGsBlocks, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pd = 0.0;
    for (double v : hp) pd += v;
    if (pd <= tol) break;
    HIPCHK(gs_alpha_from_s(p, scratch, alpha, st));
  }
  if (iters) *iters = std::min(it, max_iter);
  if (pd_out) *pd_out = pd;
  return DDUOT_OK;
}

extern "C" int dd_uot_global_sinkhorn(const dduot_config* cfg, const double* mu, const double* nu,
                                      double* alpha, double* beta, int32_t max_iter, double tol,
                                      void* hip_stream, int32_t* iters, double* pd) {
  if (!cfg || !mu || !nu || !alpha || !beta) return fail(DDUOT_EINVAL, "null argument");
  if (cfg->n1 <= 0 || cfg->n2 <= 0) return fail(DDUOT_EINVAL, "grid sides must be positive");
  if (!(cfg->lambda > 0.0) || !isfinite(cfg->lambda) || !(cfg->eps > 0.0) || !isfinite(cfg->eps) ||
      !(cfg->h >= 0.0) || !isfinite(cfg->h))
    return fail(DDUOT_EINVAL, "lambda, eps must be > 0 and h >= 0");
  if (max_iter < 1) return fail(DDUOT_EINVAL, "max_iter must be >= 1");
  if (!(tol >= 0.0)) return fail(DDUOT_EINVAL, "tol must be >= 0");
  const long n = (long)cfg->n1 * cfg->n2;
  for (long i = 0; i < n; ++i)
    if (!(mu[i] > 0.0) || !isfinite(mu[i]) || !(nu[i] > 0.0) || !isfinite(nu[i]) || !isfinite(beta[i]))
      return fail(DDUOT_EINVAL, "masses must be finite and > 0, beta finite");
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<void*> mem;
  auto grab = [&](double** p, long count) -> int {
    HIPCHK(hipMalloc((void**)p, sizeof(double) * count));
    mem.push_back(*p);
    return DDUOT_OK;
  };
  auto body = [&]() -> int {
    double *d_mu, *d_nu, *d_a, *d_b, *d_s, *d_part;
    CHK(grab(&d_mu, n));
    CHK(grab(&d_nu, n));
    CHK(grab(&d_a, n));
    CHK(grab(&d_b, n));
    CHK(grab(&d_s, 5 * n));
    CHK(grab(&d_part, kGsBlocks));
    HIPCHK(hipMemcpyAsync(d_mu, mu, sizeof(double) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_nu, nu, sizeof(double) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_b, beta, sizeof(double) * n, hipMemcpyHostToDevice, st));
    const Prob p = grid_prob(cfg);
    CHK(gs_solve(p, d_mu, d_nu, d_a, d_b, d_s, d_part, max_iter, tol, st, iters, pd));
    HIPCHK(hipMemcpyAsync(alpha, d_a, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(beta, d_b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return DDUOT_OK;
  };
  const int r = body();
  for (void* p : mem) (void)hipFree(p);
  return r;
}

// ---- the global Sinkhorn without allocations ---------------------------------
// Its device scratch (the five grid buffers of the iteration and the
// per-block partial sums, for grids of at most kNoAllocPoints points) is a
// file-scope array: one copy per GPU, held until the process ends.  In host
// code `scratch` only names the symbol; its device address on the current
// GPU comes from hipGetSymbolAddress, once per device, and only that address
// is used.
static constexpr long kNoAllocPoints = 256L * 256L;
static constexpr long kNoAllocDoubles = 5 * kNoAllocPoints + kGsBlocks + 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];
static constexpr int kMaxDevices = 64;
static double* g_noalloc_ptr[kMaxDevices] = {};
static std::mutex g_noalloc_mu;

static int noalloc_scratch(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DDUOT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return DDUOT_OK;
}

extern "C" int dd_uot_global_sinkhorn_noalloc(const dduot_config* cfg, const double* mu,
                                              const double* nu, double* alpha, double* beta,
                                              int32_t max_iter, double tol, void* hip_stream,
                                              int32_t* iters, double* pd) {
  if (!cfg || !mu || !nu || !alpha || !beta) return fail(DDUOT_EINVAL, "null argument");
  if (cfg->n1 <= 0 || cfg->n2 <= 0) return fail(DDUOT_EINVAL, "grid sides must be positive");
  if (!(cfg->lambda > 0.0) || !isfinite(cfg->lambda) || !(cfg->eps > 0.0) || !isfinite(cfg->eps) ||
      !(cfg->h >= 0.0) || !isfinite(cfg->h))
    return fail(DDUOT_EINVAL, "lambda, eps must be > 0 and h >= 0");
  if (max_iter < 1) return fail(DDUOT_EINVAL, "max_iter must be >= 1");
  if (!(tol >= 0.0)) return fail(DDUOT_EINVAL, "tol must be >= 0");
  const long n = (long)cfg->n1 * cfg->n2;
  if (n > kNoAllocPoints)
    return fail(DDUOT_EINVAL, "grid larger than the scratch of the no-allocation entry point (" +
                                  std::to_string(kNoAllocPoints) + " points)");
  if (!on_device(mu) || !on_device(nu) || !on_device(alpha) || !on_device(beta))
    return fail(DDUOT_EINVAL, "mu, nu, alpha, beta must be device memory");
  hipStream_t st = (hipStream_t)hip_stream;
  double* sc = nullptr;
  CHK(noalloc_scratch(&sc));
  double* part = sc + 5 * n;
  double* flag = part + kGsBlocks;
  // the masses finite and > 0, beta finite, checked on the device
  HIPCHK(launch_fill(flag, 1, 0.0, st));
  HIPCHK(launch_check_grids(mu, nu, beta, n, flag, st));
  double bad = 0.0;
  HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad != 0.0) return fail(DDUOT_EINVAL, "masses must be finite and > 0, beta finite");
  const Prob p = grid_prob(cfg);
  CHK(gs_solve(p, mu, nu, alpha, beta, sc, part, max_iter, tol, st, iters, pd));
  HIPCHK(hipStreamSynchronize(st));
  return DDUOT_OK;
}

extern "C" int dd_uot_interpolate_potential(const double* coarse, int32_t n1c, int32_t n2c,
                                            double* fine, void* hip_stream) {
  if (!coarse || !fine || n1c <= 0 || n2c <= 0) return fail(DDUOT_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)hip_stream;
  const long nc = (long)n1c * n2c;
  double *dc = nullptr, *df = nullptr;
  auto body = [&]() -> int {
    HIPCHK(hipMalloc((void**)&dc, sizeof(double) * nc));
    HIPCHK(hipMalloc((void**)&df, sizeof(double) * 4 * nc));
    HIPCHK(hipMemcpyAsync(dc, coarse, sizeof(double) * nc, hipMemcpyHostToDevice, st));
    HIPCHK(launch_interp(dc, n1c, n2c, df, st));
    HIPCHK(hipMemcpyAsync(fine, df, sizeof(double) * 4 * nc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return DDUOT_OK;
  };
  const int r = body();
  if (dc) (void)hipFree(dc);
  if (df) (void)hipFree(df);
  return r;
}

// State of the single problem of h from device potentials (cost units) with
// per-basic-cell scan windows; the next half-iteration is greedy.
static int state_from_duals(dduot_handle* h, const double* d_alpha, const double* d_beta,
                            const std::vector<Box>& win) {
  const Prob& p = h->probs[0];
  hipStream_t st = h->stream;
  int gcols = 1, hrows = 1;
  for (const Box& b : win) {
    gcols = std::max(gcols, b.l2);
    hrows = std::max(hrows, b.l1);
  }
  int dev = 0, max_lds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((long)from_duals_lds(p.s, gcols, hrows) + 4096 > max_lds)
    return fail(DDUOT_EINVAL, "scan window too wide for the LDS of one workgroup");
  Box* d_win = nullptr;
  CHK(dalloc(h, &d_win, win.size()));
  HIPCHK(hipMemcpyAsync(d_win, win.data(), sizeof(Box) * win.size(), hipMemcpyHostToDevice, st));
  static const int one = 1;
  DualsArgs A{};
  A.alpha = d_alpha;
  A.beta = d_beta;
  A.mu = h->d_mu;
  A.nu = h->d_nu;
  A.bxy = h->d_basic_xy;
  A.win = d_win;
  A.n1 = p.n1;
  A.n2 = p.n2;
  A.s = p.s;
  A.gcols = gcols;
  A.hrows = hrows;
  A.eps = p.eps;
  A.lam = p.lam;
  A.ch = p.ch;
  A.trunc = p.trunc;
  A.mass_nu = p.mass_nu;
  A.box = h->d_box;
  A.voff = h->d_voff;
  A.px = h->d_px;
  A.hbar = h->d_hbar;
  A.phase = 0;
  HIPCHK(launch_from_duals(A, p.nbasic, st));
  CHK(place_state(h));
  A.vals = h->d_pool[0];
  A.phase = 1;
  HIPCHK(launch_from_duals(A, p.nbasic, st));
  HIPCHK(hipMemcpyAsync(h->d_abar, d_alpha, sizeof(double) * p.n1 * p.n2, hipMemcpyDeviceToDevice, st));
  std::vector<int> ones(h->nbasic, 1);
  HIPCHK(hipMemcpyAsync(h->d_awarm, ones.data(), sizeof(int) * h->nbasic, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_force, &one, sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return DDUOT_OK;
}

// New single-problem handle with a placeholder state (block start).
static int placeholder_handle(const dduot_config* cfg, const double* mu, const double* nu,
                              void* hip_stream, dduot_handle** out) {
  dduot_config c = *cfg;
  c.init = DDUOT_INIT_BLOCK;
  return dd_uot_init(&c, mu, nu, hip_stream, out);
}

static void destroy_keep_error(dduot_handle* h) {
  std::string keep = g_err;
  dd_uot_destroy(h);
  g_err = keep;
}

extern "C" int dd_uot_init_duals(const dduot_config* cfg, const double* mu, const double* nu,
                                 const double* alpha, const double* beta, void* hip_stream,
                                 dduot_handle** out) {
  if (!out) return fail(DDUOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!alpha || !beta) return fail(DDUOT_EINVAL, "null potential");
  if (!cfg) return fail(DDUOT_EINVAL, "null config");
  const long n = (long)cfg->n1 * cfg->n2;
  for (long i = 0; i < n; ++i)
    if (!isfinite(alpha[i]) || !isfinite(beta[i])) return fail(DDUOT_EINVAL, "potentials must be finite");
  dduot_handle* h = nullptr;
  CHK(placeholder_handle(cfg, mu, nu, hip_stream, &h));
  double *da = nullptr, *db = nullptr;
  auto body = [&]() -> int {
    CHK(dalloc(h, &da, n));
    CHK(dalloc(h, &db, n));
    HIPCHK(hipMemcpyAsync(da, alpha, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(db, beta, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    std::vector<Box> win(h->probs[0].nbasic, Box{0, 0, cfg->n1, cfg->n2});
    return state_from_duals(h, da, db, win);
  };
  const int r = body();
  if (r != DDUOT_OK) {
    destroy_keep_error(h);
    return r;
  }
  *out = h;
  return DDUOT_OK;
}

extern "C" void dd_uot_default_multiscale(dduot_multiscale* m) {
  memset(m, 0, sizeof(*m));
  m->levels = 7;
  m->coarse_cell = 4;
  m->eps_start_h2 = 2.0;
  m->eps_end_h2 = 0.5;
  m->halves_per_stage = 4;
  m->stage_max_halves = 16;
  m->stage_gap = 1e-3;
  m->coarse_max_iter = 1000;
  m->final_max_halves = 200;
  m->check_every = 4;
  m->target_rel_gap = 1e-6;
  m->dd_from = 256;
  m->global_max_iter = 2000;
  m->global_tol = 5e-6;
  m->coarse_box_cap = 80;
  m->coarse_lenience = 0.0;
  m->verbose = 0;
  m->polish_iters = 0;
  m->final_err_ratio = 0.0;
  m->final_err_min = 0.0;
}

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

extern "C" int dd_uot_solve_multiscale(const dduot_config* cfg, const dduot_multiscale* ms,
                                       const double* mu, const double* nu, void* hip_stream,
                                       dduot_handle** out, double* trace, int32_t trace_cap,
                                       int32_t* trace_len) {
  if (!out) return fail(DDUOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (trace_len) *trace_len = 0;
  if (!cfg || !ms || !mu || !nu) return fail(DDUOT_EINVAL, "null argument");
  if (trace_cap < 0 || (trace_cap > 0 && !trace)) return fail(DDUOT_EINVAL, "bad trace buffer");
  const int L = ms->levels;
  if (L < 1 || L > 12) return fail(DDUOT_EINVAL, "levels must be in [1, 12]");
  if (!(ms->eps_start_h2 > 0.0) || !(ms->eps_end_h2 > 0.0) || ms->eps_end_h2 > ms->eps_start_h2)
    return fail(DDUOT_EINVAL, "need 0 < eps_end_h2 <= eps_start_h2");
  if (ms->halves_per_stage < 1 || ms->final_max_halves < 0 || ms->check_every < 1 ||
      ms->stage_max_halves < ms->halves_per_stage || ms->coarse_max_iter < 1 ||
      ms->coarse_cell < 1 || 2 * ms->coarse_cell > kMaxTile)
    return fail(DDUOT_EINVAL, "bad iteration counts or coarse cell");
  if (!(ms->final_err_ratio >= 0.0) || !(ms->final_err_min >= 0.0) || ms->polish_iters < 0 ||
      ms->polish_iters > 10000)
    return fail(DDUOT_EINVAL, "final_err_ratio, final_err_min >= 0, polish_iters in [0, 10000]");
  if (ms->dd_from < 0 || ms->global_max_iter < 1 || !(ms->global_tol >= 0.0))
    return fail(DDUOT_EINVAL, "bad global Sinkhorn settings");
  if (ms->coarse_box_cap < 0 || ms->coarse_box_cap > 128 || !(ms->coarse_lenience >= 0.0))
    return fail(DDUOT_EINVAL, "coarse_box_cap must be in [0, 128], coarse_lenience >= 0");
  if (cfg->n1 % (1 << (L - 1)) || cfg->n2 % (1 << (L - 1)))
    return fail(DDUOT_EINVAL, "grid sides must be divisible by 2^(levels-1)");
  const double t0 = now_ms();
  // marginals of every layer: 2 x 2 sums of the next finer one
  std::vector<std::vector<double>> mus(L), nus(L);
  std::vector<int> n1s(L), n2s(L);
  mus[L - 1].assign(mu, mu + (size_t)cfg->n1 * cfg->n2);
  nus[L - 1].assign(nu, nu + (size_t)cfg->n1 * cfg->n2);
  n1s[L - 1] = cfg->n1;
  n2s[L - 1] = cfg->n2;
  for (int l = L - 2; l >= 0; --l) {
    const int a1 = n1s[l + 1] / 2, a2 = n2s[l + 1] / 2, f2 = n2s[l + 1];
    n1s[l] = a1;
    n2s[l] = a2;
    mus[l].assign((size_t)a1 * a2, 0.0);
    nus[l].assign((size_t)a1 * a2, 0.0);
    for (int i1 = 0; i1 < a1; ++i1)
      for (int i2 = 0; i2 < a2; ++i2)
        for (int q = 0; q < 4; ++q) {
          const size_t g = (size_t)(2 * i1 + q / 2) * f2 + (2 * i2 + q % 2);
          mus[l][(size_t)i1 * a2 + i2] += mus[l + 1][g];
          nus[l][(size_t)i1 * a2 + i2] += nus[l + 1][g];
        }
  }
  int tl = 0;
  long long halves_before = 0;   // half-iterations of the coarser layers
  auto record = [&](dduot_handle* h, const dduot_score& sc) {
    if (tl < trace_cap) {
      trace[5 * tl + 0] = (double)(halves_before + h->k);
      trace[5 * tl + 1] = now_ms() - t0;
      trace[5 * tl + 2] = sc.rel_pd_gap;
      trace[5 * tl + 3] = (sc.tracked - sc.dual) / fabs(sc.dual);
      trace[5 * tl + 4] = sc.rel_gap_polished;
      ++tl;
    }
  };
  // layers coarser than dd_from (never the finest) run the global Sinkhorn
  // (Sec. 4.4 "Sinkhorn warm start"); the plan of the last one's potentials,
  // split by basic cells, is refined to the first DD layer
  int first_dd = 0;
  if (ms->dd_from > 0)
    while (first_dd < L - 1 && std::max(n1s[first_dd], n2s[first_dd]) < ms->dd_from) ++first_dd;
  struct DevBufs {
    std::vector<void*> p;
    ~DevBufs() {
      for (void* q : p) (void)hipFree(q);
    }
  } gbufs;
  auto galloc = [&](double** p, long count) -> int {
    HIPCHK(hipMalloc((void**)p, sizeof(double) * count));
    gbufs.p.push_back(*p);
    return DDUOT_OK;
  };
  double *g_a = nullptr, *g_b = nullptr, *g_fb = nullptr;
  if (first_dd > 0) {
    hipStream_t st = (hipStream_t)hip_stream;
    const long nmax = (long)n1s[first_dd - 1] * n2s[first_dd - 1];
    double *g_mu, *g_nu, *g_s, *g_part;
    CHK(galloc(&g_a, nmax));
    CHK(galloc(&g_b, nmax));
    CHK(galloc(&g_mu, nmax));
    CHK(galloc(&g_nu, nmax));
    CHK(galloc(&g_s, 5 * nmax));
    CHK(galloc(&g_part, kGsBlocks));
    CHK(galloc(&g_fb, nmax));
    double mass = 0.0;
    for (double v : mus[0]) mass += v;
    for (int l = 0; l < first_dd; ++l) {
      dduot_config c = *cfg;
      c.n1 = n1s[l];
      c.n2 = n2s[l];
      c.h = cfg->h * (double)(1 << (L - 1 - l));
      const long n = (long)c.n1 * c.n2;
      HIPCHK(hipMemcpyAsync(g_mu, mus[l].data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(g_nu, nus[l].data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
      if (l == 0) {
        HIPCHK(launch_fill(g_b, n, 0.0, st));
      } else {
        // beta of the coarser layer, interpolated (alpha follows from it)
        HIPCHK(launch_interp(g_b, n1s[l - 1], n2s[l - 1], g_fb, st));
        HIPCHK(hipMemcpyAsync(g_b, g_fb, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      }
      const double h2 = c.h * c.h;
      double e = ms->eps_start_h2 * h2;
      const double e_end = ms->eps_end_h2 * h2;
      for (;;) {
        c.eps = e;
        const Prob p = grid_prob(&c);
        int it = 0;
        double pd = 0.0;
        CHK(gs_solve(p, g_mu, g_nu, g_a, g_b, g_s, g_part, ms->global_max_iter, ms->global_tol * mass,
                     st, &it, &pd));
        if (ms->verbose)
          fprintf(stderr, "[multiscale] global %dx%d eps %.3g h^2: %d iterations, KL/|mu| %.3g, %.0f ms\n",
                  c.n1, c.n2, e / h2, it, pd / mass, now_ms() - t0);
        if (e <= e_end * (1.0 + 1e-12)) break;
        e = std::max(e * 0.5, e_end);
      }
    }
  }
  dduot_handle* h = nullptr;
  if (first_dd > 0) {
    // DD state of the last global layer: its own potentials' plan split by
    // basic cells; the next layer refines it like any DD layer
    const int l = first_dd - 1;
    dduot_config c = *cfg;
    c.n1 = n1s[l];
    c.n2 = n2s[l];
    c.h = cfg->h * (double)(1 << (L - 1 - l));
    c.cell = std::min(cfg->cell, ms->coarse_cell);
    c.box_cap = std::max(c.box_cap, ms->coarse_box_cap);
    c.lenience = ms->coarse_lenience;
    if (std::max(c.n1, c.n2) <= 64) c.box_cap = std::max(c.box_cap, std::max(c.n1, c.n2));
    c.eps = ms->eps_end_h2 * c.h * c.h;
    CHK(placeholder_handle(&c, mus[l].data(), nus[l].data(), hip_stream, &h));
    std::vector<Box> win(h->probs[0].nbasic, Box{0, 0, c.n1, c.n2});
    const int r = state_from_duals(h, g_a, g_b, win);
    if (r != DDUOT_OK) {
      destroy_keep_error(h);
      return r;
    }
  }
  for (int l = first_dd; l < L; ++l) {
    const double scale = (double)(1 << (L - 1 - l));
    dduot_config c = *cfg;
    c.n1 = n1s[l];
    c.n2 = n2s[l];
    c.h = cfg->h * scale;
    const bool finest = l == L - 1;
    if (finest) {
      c.cell = cfg->cell;
    } else if (l == 0 && c.n1 == c.n2 && c.n1 % 2 == 0 && c.n1 <= kMaxTile) {
      // the coarsest layer is one composite cell: partition A solves the
      // global problem (the role of the paper's global Sinkhorn warm start)
      c.cell = c.n1 / 2;
    } else {
      c.cell = std::min(cfg->cell, ms->coarse_cell);
    }
    if (!finest) {
      c.sinkhorn_max_iter = std::max(cfg->sinkhorn_max_iter, ms->coarse_max_iter);
      c.box_cap = std::max(c.box_cap, ms->coarse_box_cap);
      c.lenience = ms->coarse_lenience;
      // small layers: the whole grid fits the in-LDS layout
      if (std::max(c.n1, c.n2) <= 64) c.box_cap = std::max(c.box_cap, std::max(c.n1, c.n2));
    }
    const double h2 = c.h * c.h;
    c.eps = ms->eps_start_h2 * h2;
    dduot_handle* nh = nullptr;
    if (l == 0) {
      c.init = (c.box_cap >= c.n1 && c.box_cap >= c.n2) ? DDUOT_INIT_PRODUCT : DDUOT_INIT_BLOCK;
      CHK(dd_uot_init(&c, mus[l].data(), nus[l].data(), hip_stream, &nh));
    } else {
      const int r = dd_uot_refine(h, &c, mus[l].data(), nus[l].data(), hip_stream, &nh);
      halves_before += h->k;
      destroy_keep_error(h);
      h = nullptr;
      if (r != DDUOT_OK) return r;
    }
    h = nh;
    if (ms->verbose && ms->polish_iters > 0) {
      const int r = dd_uot_set_polish(h, ms->polish_iters);
      if (r != DDUOT_OK) {
        destroy_keep_error(h);
        return r;
      }
    }
    auto fail_out = [&](int r) {
      std::string keep = g_err;
      dd_uot_destroy(h);
      g_err = keep;
      return r;
    };
    // eps stages of this layer: halve from eps_start down to eps_end (the
    // finest layer continues to cfg->eps); each stage runs halves_per_stage
    // half-iterations, then more until the certificate's relative gap is
    // below stage_gap or stage_max_halves are done
    const double e_end = finest ? cfg->eps : ms->eps_end_h2 * h2;
    double e = c.eps;
    for (;;) {
      int done = 0;
      dduot_score sc{};
      bool have_sc = false;
      long long inner = 0, cells = 0, unconv = 0;
      for (;;) {
        dduot_iter_stats it{};
        int r = dd_uot_iterate(h, ms->halves_per_stage, ms->verbose ? &it : nullptr);
        if (r != DDUOT_OK) return fail_out(r);
        inner += it.inner_iters;
        cells += it.n_cells;
        unconv += it.n_unconverged;
        done += ms->halves_per_stage;
        have_sc = false;
        if (done + ms->halves_per_stage > ms->stage_max_halves) break;
        r = dd_uot_score(h, 0, &sc);
        if (r != DDUOT_OK) return fail_out(r);
        have_sc = true;
        if (sc.rel_pd_gap <= ms->stage_gap) break;
      }
      if (ms->verbose) {
        if (!have_sc) {
          const int r = dd_uot_score(h, 0, &sc);
          if (r != DDUOT_OK) return fail_out(r);
        }
        fprintf(stderr,
                "[multiscale] DD %dx%d cell %d eps %.3g h^2: %d half-iterations (%.1f inner "
                "iterations per cell, %lld unconverged), certificate gap %.3g, DD-plan gap %.3g, "
                "polished gap %.3g, %.0f ms\n",
                c.n1, c.n2, c.cell, e / h2, done, cells ? (double)inner / cells : 0.0, unconv,
                sc.rel_pd_gap, (sc.tracked - sc.dual) / fabs(sc.dual), sc.rel_gap_polished,
                now_ms() - t0);
      }
      if (e <= e_end * (1.0 + 1e-12)) break;
      e = std::max(e * 0.5, e_end);
      int r = dd_uot_set_eps(h, 0, e);
      if (r != DDUOT_OK) return fail_out(r);
    }
    if (finest) {
      // final stage: iterate, certificate every check_every half-iterations
      dduot_score sc;
      int r = dd_uot_set_polish(h, ms->polish_iters);
      if (r != DDUOT_OK) return fail_out(r);
      r = dd_uot_score(h, 0, &sc);
      if (r != DDUOT_OK) return fail_out(r);
      record(h, sc);
      int done = 0;
      auto gap = [&](const dduot_score& q) {
        return ms->polish_iters > 0 ? q.rel_gap_polished : q.rel_pd_gap;
      };
      while (!(gap(sc) <= ms->target_rel_gap) && done < ms->final_max_halves) {
        const int k = std::min(ms->check_every, ms->final_max_halves - done);
        r = dd_uot_iterate(h, k, nullptr);
        if (r != DDUOT_OK) return fail_out(r);
        done += k;
        r = dd_uot_score(h, 0, &sc);
        if (r != DDUOT_OK) return fail_out(r);
        record(h, sc);
        if (ms->final_err_ratio > 0.0) {
          const double cur = h->probs[0].err;
          const double want = std::max(ms->final_err_min, std::min(cur, ms->final_err_ratio * gap(sc)));
          if (want < cur) {
            r = dd_uot_set_err(h, 0, want);
            if (r != DDUOT_OK) return fail_out(r);
          }
        }
        if (ms->verbose)
          fprintf(stderr, "[multiscale] final %dx%d: %d half-iterations, certificate gap %.3g, "
                  "DD-plan gap %.3g, polished gap %.3g, Err %.3g, %.0f ms\n", c.n1, c.n2, done,
                  sc.rel_pd_gap, (sc.tracked - sc.dual) / fabs(sc.dual), sc.rel_gap_polished,
                  h->probs[0].err, now_ms() - t0);
      }
    }
  }
  if (trace_len) *trace_len = tl;
  *out = h;
  return DDUOT_OK;
}
