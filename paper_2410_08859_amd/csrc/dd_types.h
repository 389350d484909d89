// Device-side descriptors shared by the HIP kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dduot {

constexpr int kBlock = 256;        // threads per workgroup of the cell kernels
constexpr int kMaxTile = 16;       // maximal X tile side (2 * basic cell side)
constexpr int kHistFields = 12;    // doubles per half-iteration record

// One transport problem of a (possibly batched) handle.
struct Prob {
  int n1, n2, s, nb1, nb2;
  double h, eps, lam;
  double kappa;     // lam / (lam + eps)
  double K;         // lam / eps
  double ch;        // h^2 / eps: cost / eps = ch * |i - j|^2 in grid units
  double err, trunc, lenience;
  int getweights, fixed_iters, max_iter;
  int margin;
  int translate;
  int balance;         // 1: balancing step after every cell solve (Sec. 4.1)
  int support;         // 1: the cell problem lives on the support of nu_J (Sec. 4.1)
  int precision;
  int moved;           // 1: Y points displaced (dense, non-separable cost)
  int grid_off;     // offset of this problem's grid arrays
  int basic_off, nbasic;
  int cell_off[2][4], ncell[2][4];   // composite cells of partition A (0) / B (1)
                                     // in its four staggered batches
  int chunk_off, nchunk;       // reduction chunks over the grid
  double mass_mu, mass_nu;
};

// Composite cell: up to 4 basic cells and the X rectangle they cover.
struct Cell {
  int prob;
  int nb;
  int basic[4];
  int x1, x2, lx1, lx2;
};

struct Box { int o1, o2, l1, l2; };

// Device pointers of a handle (all problems concatenated).
struct Dev {
  const Prob* probs;
  const Cell* cells;          // A cells then B cells
  const int* basic_prob;      // problem of each basic cell
  const int2* basic_xy;       // X origin of each basic cell
  const int* basic_cell[2];   // composite cell (global index) of each basic cell per partition
  const double* mu;           // grids
  const double* nu;
  double* P;                  // aggregated Y-marginal of the state
  unsigned long long* fxacc;  // 2 per grid point: fixed-point sums of the aggregation
  double* Pg;                 // aggregated Y-marginal of the greedy candidate
  double* px;                 // X-marginal of the state plan
  double* pxc;                // X-marginal of the candidate cell plans
  double* abar;               // stitched alpha of the last cell solves
  int* awarm;                 // per basic cell: abar holds a potential on X_i
  // Basic-cell Y-marginals live in variable-size pools: no box size limit.
  // The state is double-buffered: every step writes the new state compactly
  // into the other pool and flips *sp (a device word, so captured graphs stay
  // valid).
  Box* box;                   // state box of each basic cell
  long* voff;                 // offset of each state box in the current pool
  double* pool0;              // state pools
  double* pool1;
  int* sp;                    // index of the current state pool
  long pool_cap;              // doubles per state pool
  Box* cbox;                  // candidate box of each basic cell
  long* coff;                 // offset of each candidate box in the candidate pool
  double* cand;               // candidate pool
  long cand_cap;              // doubles
  Box* nbox;                  // mix: the new state box of each basic cell
  int2* nsub;                 // mix: its origin inside the candidate box (-1: unchanged)
  long* nsize;                // mix: its area, then (scanned) its offset in the other pool
  long* nuse;                 // mix: total doubles of the new state
  // per composite cell of a step (prepared by k_cell_prep)
  Box* cellbox;               // Y-box
  long* csize;                // candidate doubles, then (scanned) candidate offset
  long* wsize;                // workspace bytes, then (scanned) workspace offset
  long* cuse;                 // [0] candidate doubles, [1] workspace bytes of the step
  unsigned char* ws;          // per-cell workspace pool (log nu, log r; large boxes:
                              // the potentials and pass buffers)
  long ws_cap;                // bytes
  long long* need;            // [0] state, [1] candidate, [2] workspace: largest
                              // need since the host last read it
  int* cap_fail;              // per problem: a pool was too small for a step
  double* hbar;               // tracked piece of each basic cell
  double* htil;               // candidate piece of each basic cell
  int* cell_iters;            // Y-halves of the last solve of each cell (-1: not solved)
  int* cell_conv;             // converged flag of the last solve
  double* cell_bytes;         // algorithmic bytes of the last solve
  double* cell_terms;         // log-sum-exp terms of the last solve
  double* cell_fall;          // pass outputs recomputed in FP64 (underflow) in the last solve
  const double* ydel;         // moved Y: (y'/h - j) per grid point, 2 doubles each
  long long* kstep;           // half-iterations done (history record index)
  double* chunk_part;         // 2 doubles per reduction chunk
  double* theta;              // per problem
  double* cell_theta;         // per cell: the weight of its last step (GetWeights)
  double* cell_dir;           // per cell: GetWeights opt direction
  double* cell_ddh;           // per cell: direction times the change of its pieces
  double* line;               // per problem, GetWeights line search: lo, a, b, z, dH,
                              // phase, active, opt lower bound (0: no opt rounds)
  double* line_part;          // 2 doubles per reduction chunk (line search sums)
  double* hist;               // per problem ring of records
  int* force_greedy;          // per problem: next GetWeights takes theta = 1
  int hist_cap;
  int lcap;                   // largest box side of the in-LDS cell layouts
  // gangs (several workgroups per wide cell; cell_kernel.hip)
  int* glist;                 // the step's wide cells, longest first
  int* gcount;                // their number, and how many of them are heavy
  double* gpart;              // per gang: [2][G][256] X pass 2 partials
  double* gxch;               // per gang: [2][G][16] partial reductions
  unsigned* gcnt;             // per gang (stride 64): barrier arrivals
  unsigned* gxcd;             // gang formation: [0, 16) slots taken per XCD, [16] arrivals
  double* gsolo;              // per workgroup of the gang kernel: its slots when alone
  int* gabort;                // a gang barrier timed out (sticky until read)
  int gumax;                  // set per launch: gangs solve the wide cells with at
                              // most gumax box columns (0: no gangs)
};

// Launch shape of the gangs that solve the wide cells (G = 0: one
// workgroup per wide cell): G workgroups per gang, nwg workgroups in all (a
// multiple of 8 G within the occupancy), the kernel variant, a barrier's
// wait limit in wall-clock ticks.
struct GangLaunch {
  int G, nwg;
  int minb;          // kernel variant: workgroups per CU its registers allow
  long long limit;
};

// Per-cell workspace in global memory (byte offsets from the cell's base):
// log r on the box (R), log nu (FP64 kernels: FP64), the list of the
// Y-domain's points (int32, at most the box); for a box wider than
// the in-LDS layouts also b, z, log nu (FP32 kernels), the pass buffers, the
// row / column maxima and the displacements.
struct WsLayout {
  size_t lrr, lnv, dom, bd, zp, lnvf, Tt, Ud, Mr, MU, d1, d2, total;
};
__host__ __device__ inline WsLayout cell_ws_layout(int rbytes, long ny, int cmax, bool moved,
                                                   bool big) {
  WsLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 15) & ~size_t(15);
    return o;
  };
  const size_t n = (size_t)ny;
  w.lrr = take((size_t)rbytes * n);
  w.lnv = take(rbytes == 8 ? 8 * n : 0);
  w.dom = take(4 * n);
  const size_t nb = big ? n : 0, nt = big ? (size_t)cmax * kMaxTile : 0, nc = big ? (size_t)cmax : 0;
  w.bd = take(8 * nb);
  w.zp = take((size_t)rbytes * nb);
  w.lnvf = take(rbytes == 4 ? 4 * nb : 0);
  w.Tt = take(8 * nt);
  w.Ud = take(8 * nt);
  w.Mr = take(8 * nc);
  w.MU = take(8 * nc);
  w.d1 = take(moved ? (size_t)rbytes * nb : 0);
  w.d2 = take(moved ? (size_t)rbytes * nb : 0);
  w.total = (off + 255) & ~size_t(255);
  return w;
}

// Y-box of composite cell J (Sec. 4.1: nu_{-J} is needed on the support of
// nu_J): the bounding box of its basic cells' boxes, dilated by the margin
// and clipped to the grid (the X rectangle of J when every basic box is
// empty).  Used by the step preparation, the pool bounds and the host.
__host__ __device__ inline Box cell_ybox(const Cell& C, const Prob& P, const Box* box) {
  int lo1 = 0x7fffffff, lo2 = 0x7fffffff, hi1 = -0x7fffffff, hi2 = -0x7fffffff;
  for (int k = 0; k < C.nb; ++k) {
    const Box b = box[C.basic[k]];
    if (b.l1 > 0 && b.l2 > 0) {
      lo1 = lo1 < b.o1 ? lo1 : b.o1;
      lo2 = lo2 < b.o2 ? lo2 : b.o2;
      hi1 = hi1 > b.o1 + b.l1 ? hi1 : b.o1 + b.l1;
      hi2 = hi2 > b.o2 + b.l2 ? hi2 : b.o2 + b.l2;
    }
  }
  if (lo1 == 0x7fffffff) {
    lo1 = C.x1; lo2 = C.x2; hi1 = C.x1 + C.lx1; hi2 = C.x2 + C.lx2;
  }
  const int m = P.margin;
  Box yb;
  yb.o1 = lo1 - m > 0 ? lo1 - m : 0;
  yb.o2 = lo2 - m > 0 ? lo2 - m : 0;
  yb.l1 = (hi1 + m < P.n1 ? hi1 + m : P.n1) - yb.o1;
  yb.l2 = (hi2 + m < P.n2 ? hi2 + m : P.n2) - yb.o2;
  return yb;
}

// The current state pool.
__device__ __forceinline__ const double* state_pool(const Dev& d) {
  return *d.sp ? d.pool1 : d.pool0;
}

// Basic-cell state from a pair of global potentials (warmstart.hip).
struct DualsArgs {
  const double* alpha;   // grid, cost units
  const double* beta;
  const double* mu;
  const double* nu;
  const int2* bxy;       // X origin of each basic cell
  const Box* win;        // Y scan window of each basic cell
  int n1, n2, s;
  int gcols;             // largest window width (LDS rows of G)
  int hrows;             // largest window height (LDS rows of H)
  double eps, lam, ch, trunc, mass_nu;
  Box* box;              // phase 0: written; phase 1: read
  const long* voff;      // phase 1: offset of each box in vals
  double* vals;          // the state pool
  double* px;
  double* hbar;
  int phase;
};

// Refinement of a single-problem state to the grid with twice the points per
// axis (multiscale.hip).
struct RefineArgs {
  // coarse problem (one problem, grid offset 0)
  const Box* cbox;
  const double* cvals;   // the coarse handle's current state pool
  const long* cvoff;
  const double* mu_c;
  const double* nu_c;
  const double* chbar;
  int cn2, cs, cnb2;
  // fine problem
  const int2* fxy;
  const double* mu_f;
  const double* nu_f;
  int fn2, fs;
  double trunc;
  Box* fbox;
  int* fwarm;            // stored-potential flags of the fine basic cells
  const int* cwarm;      // ... of the coarse ones
  const long* fvoff;     // phase 1: offsets of the fine boxes in fvals
  double* fvals;
  double* fhbar;
  int phase;             // 0: boxes, pieces, P_X; 1: values
};

}  // namespace dduot
