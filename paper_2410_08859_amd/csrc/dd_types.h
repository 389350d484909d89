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
  int margin, cap;
  int translate;
  int balance;         // 1: balancing step after every cell solve (Sec. 4.1)
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
  Box* box;                   // state box of each basic cell
  double* vals;               // state slots, cap2 doubles per basic cell
  Box* cbox;                  // candidate box of each basic cell
  double* cand;               // candidate slots
  double* hbar;               // tracked piece of each basic cell
  double* htil;               // candidate piece of each basic cell
  int* cell_iters;            // Y-halves of the last solve of each cell (-1: skipped)
  int* cell_conv;             // converged flag of the last solve
  double* cell_bytes;         // algorithmic bytes of the last solve
  double* cell_terms;         // log-sum-exp terms of the last solve
  double* cell_fall;          // pass outputs recomputed in FP64 (underflow) in the last solve
  double* ws_lnv;             // per cell: log nu on the Y-box (cap2 entries)
  double* ws_lrr;             // per cell: log(nu_{-J}/nu) on the Y-box (cap2 entries)
  const double* ydel;         // moved Y: (y'/h - j) per grid point, 2 doubles each
  long long* kstep;           // half-iterations done (history record index)
  double* chunk_part;         // 2 doubles per reduction chunk
  double* theta;              // per problem
  double* line;               // per problem, GetWeights line search: lo, a, b, z, dH, phase, active, -
  double* line_part;          // 2 doubles per reduction chunk (line search sums)
  double* hist;               // per problem ring of records
  int* overflow_any;          // per problem
  int* force_greedy;          // per problem: next GetWeights takes theta = 1
  int hist_cap;
  long cap2;                  // doubles per slot
};

// Basic-cell state from a pair of global potentials (warmstart.hip).
struct DualsArgs {
  const double* alpha;   // grid, cost units
  const double* beta;
  const double* mu;
  const double* nu;
  const int2* bxy;       // X origin of each basic cell
  const Box* win;        // Y scan window of each basic cell
  int n1, n2, s, cap;
  int gcols;             // largest window width (LDS rows of G)
  long cap2;
  double eps, lam, ch, trunc, mass_nu;
  Box* box;
  double* vals;
  double* px;
  double* hbar;
  int* nclip;
};

}  // namespace dduot
