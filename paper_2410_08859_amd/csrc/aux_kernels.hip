// Kernels around the cell solve: aggregation of basic Y-marginals, the
// GetWeights decision, the convex-combination update with truncation, and the
// global primal-dual certificate.
#include "dd_types.h"

#include <limits.h>
#include <math.h>

namespace dduot {

__global__ void k_fill(double* p, long n, double v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Deterministic sums for the aggregation: a value v is added as the
// fixed-point pair (floor(v 2^50), round(frac(v 2^50) 2^50)) to two 64-bit
// integer sums per grid point, so the result (exact to 2^-100 absolute) does
// not depend on the order of the atomic adds.  The pair holds any point sum
// below 2^13 (masses are limited to 2^10) and 2^13 terms.
__device__ __forceinline__ void fx_add(unsigned long long* acc, double v) {
  const double s = v * 0x1p50;
  const double fh = floor(s);
  atomicAdd(acc, (unsigned long long)(long long)fh);
  atomicAdd(acc + 1, (unsigned long long)(long long)rint((s - fh) * 0x1p50));
}

__global__ void k_fx_zero(unsigned long long* acc, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc[i] = 0ull;
}

__global__ void k_fx_finish(const unsigned long long* acc, double* P, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    P[i] = (double)(long long)acc[2 * i] * 0x1p-50 + (double)(long long)acc[2 * i + 1] * 0x1p-100;
}

// P_Y pi = sum_i nu_i (Sec. 4.1): one workgroup per basic cell scatters its box.
__global__ __launch_bounds__(kBlock) void k_aggregate(Dev d) {
  const int b = blockIdx.x;
  const Box bx = d.box[b];
  if (bx.l1 <= 0 || bx.l2 <= 0) return;
  const Prob& p = d.probs[d.basic_prob[b]];
  const long n = (long)bx.l1 * bx.l2;
  const double* v = state_pool(d) + d.voff[b];
  unsigned long long* out = d.fxacc + 2 * (long)p.grid_off;
  for (long o = threadIdx.x; o < n; o += kBlock) {
    const int j1 = (int)(o / bx.l2), j2 = (int)(o - (long)j1 * bx.l2);
    const double x = v[o];
    if (x != 0.0) fx_add(out + 2 * ((long)(bx.o1 + j1) * p.n2 + (bx.o2 + j2)), x);
  }
}

// Candidate P_Y for GetWeights: the candidate marginal of every basic cell
// whose composite cell (in partition `part`) lies in [glo, ghi) and was
// solved, the state marginal of every other basic cell.
__global__ __launch_bounds__(kBlock) void k_aggregate_sel(Dev d, int part, int glo, int ghi) {
  const int b = blockIdx.x;
  const int J = d.basic_cell[part][b];
  const bool in = J >= glo && J < ghi && d.cell_iters[J] >= 0;
  const Box bx = in ? d.cbox[b] : d.box[b];
  if (bx.l1 <= 0 || bx.l2 <= 0) return;
  const Prob& p = d.probs[d.basic_prob[b]];
  const long n = (long)bx.l1 * bx.l2;
  const double* v = in ? d.cand + d.coff[b] : state_pool(d) + d.voff[b];
  unsigned long long* out = d.fxacc + 2 * (long)p.grid_off;
  for (long o = threadIdx.x; o < n; o += kBlock) {
    const int j1 = (int)(o / bx.l2), j2 = (int)(o - (long)j1 * bx.l2);
    const double x = v[o];
    if (x != 0.0) fx_add(out + 2 * ((long)(bx.o1 + j1) * p.n2 + (bx.o2 + j2)), x);
  }
}

__device__ __forceinline__ double kl_term(double p, double q) {
  return p > 0.0 ? p * (log(p) - log(q)) - p + q : q;
}

template <int N>
__device__ __forceinline__ void block_sum_aux(double (&v)[N], double* red) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[k] = x;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < N; ++k) red[w * N + k] = v[k];
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int ww = 0; ww < kBlock / 64; ++ww) s += red[ww * N + k];
    v[k] = s;
  }
  __syncthreads();
}

// KL(P|nu) and KL(Pg|nu) per reduction chunk (fixed order, deterministic).
__global__ __launch_bounds__(kBlock) void k_kl_chunks(const int* chunk_prob, const int* chunk_start,
                                                      const int* chunk_len, const Prob* probs,
                                                      const double* P, const double* Pg,
                                                      const double* nu, double* part) {
  __shared__ double red[4 * 2];
  const int c = blockIdx.x;
  const Prob& p = probs[chunk_prob[c]];
  const long base = p.grid_off + (long)chunk_start[c];
  double acc[2] = {0.0, 0.0};
  for (int o = threadIdx.x; o < chunk_len[c]; o += kBlock) {
    const double q = nu[base + o];
    acc[0] += kl_term(P[base + o], q);
    acc[1] += kl_term(Pg[base + o], q);
  }
  block_sum_aux<2>(acc, red);
  if (threadIdx.x == 0) {
    part[2 * c] = acc[0];
    part[2 * c + 1] = acc[1];
  }
}

// GetWeights (Proposition converging-getweights) with tracked scores:
// E_cur = sum Hbar + lam KL(P|nu), E_greedy = sum Htil + lam KL(Pg|nu);
// greedy theta = 1, safe theta = 1/n (n = cells updated), swift = greedy iff
// E_greedy <= E_cur + lenience |E_cur|; line: set up the search of
// k_line_partials / k_line_update / k_line_finish.  One workgroup per problem.
__global__ __launch_bounds__(kBlock) void k_getweights(Dev d, int part, int blo, int bhi, int glo,
                                                       int ghi, int last) {
  const long long rec = d.kstep[0];
  __shared__ double red[4 * 10];
  const int pi = blockIdx.x;
  const Prob p = d.probs[pi];
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // [0] sum hbar, [1] sum of the candidate pieces (htil for the step's solved
  // basic cells, hbar elsewhere), [2] cells updated, [3] point iters,
  // [4] unconverged, [5] cells not solved (a pool too small), [6] inner
  // iters, [7] bytes, [8] log-sum-exp terms, [9] exact recomputations
  for (int b = threadIdx.x; b < p.nbasic; b += kBlock) {
    const int gb = p.basic_off + b;
    const int J = d.basic_cell[part][gb];
    acc[0] += d.hbar[gb];
    acc[1] += (J >= glo && J < ghi && d.cell_iters[J] >= 0) ? d.htil[gb] : d.hbar[gb];
  }
  int maxit = 0;
  for (int bt = blo; bt < bhi; ++bt) {
    const int c0 = p.cell_off[part][bt], nc = p.ncell[part][bt];
    for (int c = threadIdx.x; c < nc; c += kBlock) {
      const int it = d.cell_iters[c0 + c];
      const Cell C = d.cells[c0 + c];
      if (it >= 0) {
        acc[2] += 1.0;
        acc[3] += (double)it * C.lx1 * C.lx2;
        acc[4] += d.cell_conv[c0 + c] ? 0.0 : 1.0;
        acc[6] += it;
        acc[7] += d.cell_bytes[c0 + c];
        acc[8] += d.cell_terms[c0 + c];
        acc[9] += d.cell_fall[c0 + c];
        maxit = max(maxit, it);
      } else {
        acc[5] += 1.0;
      }
    }
  }
  block_sum_aux<10>(acc, red);
  __shared__ int mred[4];
  for (int o = 32; o > 0; o >>= 1) maxit = max(maxit, __shfl_down(maxit, o, 64));
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = maxit;
  __syncthreads();
  const double n = acc[2] > 0.0 ? acc[2] : 1.0;
  if (threadIdx.x == 0) {
    maxit = max(max(mred[0], mred[1]), max(mred[2], mred[3]));
    double kp = 0.0, kg = 0.0;
    for (int c = 0; c < p.nchunk; ++c) {
      kp += d.chunk_part[2 * (p.chunk_off + c)];
      kg += d.chunk_part[2 * (p.chunk_off + c) + 1];
    }
    const double ecur = acc[0] + p.lam * kp;
    const double egr = acc[1] + p.lam * kg;
    double th;
    if (d.force_greedy[pi] || p.getweights == 0) th = 1.0;
    else if (p.getweights == 1) th = 1.0 / n;
    else if (p.getweights >= 4) th = 1.0 / n;   // provisional: the line search sets it
    else th = (egr <= ecur + p.lenience * fabs(ecur)) ? 1.0 : 1.0 / n;
    // line search state (k_line_*): phase 0 evaluates f' at 1/n, 1 at 1, 2 inside
    // the bracket, 3 = done
    double* ls = d.line + 8 * pi;
    const bool line = p.getweights >= 4 && !d.force_greedy[pi];
    ls[0] = 1.0 / n;
    ls[1] = 1.0 / n;
    ls[2] = 1.0;
    ls[3] = 1.0 / n;
    ls[4] = acc[1] - acc[0];
    ls[5] = line ? 0.0 : 3.0;
    ls[6] = line ? 1.0 : 0.0;
    ls[7] = (line && p.getweights == 5) ? 1.0 / n : 0.0;   // opt: per-cell rounds follow
    if (last) d.force_greedy[pi] = 0;   // a forced greedy half-iteration covers every batch
    d.theta[pi] = th;
    double* r = d.hist + ((long)pi * d.hist_cap + (rec % d.hist_cap)) * kHistFields;
    r[0] = th;
    r[1] = ecur;
    r[2] = egr;
    r[3] = acc[2];
    r[4] = acc[3];
    r[5] = (double)maxit;
    r[6] = acc[4];
    r[7] = acc[5];
    r[8] = acc[6];
    r[9] = acc[7];
    r[10] = acc[8];
    r[11] = acc[9];
  }
}

// GetWeights line: the minimiser over [1/n, 1] of the tracked score of the
// mixture, f(z) = E_cur + z dH + lam (KL(P_z|nu) - KL(P|nu)), P_z = (1 - z) P
// + z Pg, dH = sum (Htil - Hbar): an endpoint or the root of
// f'(z) = dH + lam sum (Pg - P) log(P_z / nu), found by Newton steps on f'
// (f'' = lam sum (Pg - P)^2 / P_z > 0) kept inside a bisection bracket.
// Every round sums over all reduction chunks of the grid (one workgroup per
// chunk, fixed order), then advances each problem's search by one step.
__global__ __launch_bounds__(kBlock) void k_line_partials(Dev d, const int* chunk_prob,
                                                          const int* chunk_start,
                                                          const int* chunk_len) {
  __shared__ double red[4 * 2];
  const int c = blockIdx.x;
  const int pi = chunk_prob[c];
  const double* ls = d.line + 8 * pi;
  if (ls[5] == 3.0) return;   // uniform across the workgroup
  const Prob& p = d.probs[pi];
  const double z = ls[3];
  const long base = p.grid_off + chunk_start[c];
  double s[2] = {0.0, 0.0};
  for (int o = threadIdx.x; o < chunk_len[c]; o += kBlock) {
    const double P0 = d.P[base + o], D = d.Pg[base + o] - P0;
    if (D == 0.0) continue;
    const double Pz = P0 + z * D;
    s[0] += D * (log(Pz) - log(d.nu[base + o]));
    s[1] += D * D / Pz;
  }
  block_sum_aux<2>(s, red);
  if (threadIdx.x == 0) {
    d.line_part[2 * c] = s[0];
    d.line_part[2 * c + 1] = s[1];
  }
}

__global__ void k_line_update(Dev d) {
  if (threadIdx.x != 0) return;
  const int pi = blockIdx.x;
  double* ls = d.line + 8 * pi;
  if (ls[5] == 3.0) return;
  const Prob& p = d.probs[pi];
  double s0 = 0.0, s1 = 0.0;
  for (int c = 0; c < p.nchunk; ++c) {
    s0 += d.line_part[2 * (p.chunk_off + c)];
    s1 += d.line_part[2 * (p.chunk_off + c) + 1];
  }
  const double f1 = ls[4] + p.lam * s0, f2 = p.lam * s1;
  const double lo = ls[0];
  if (ls[5] == 0.0) {   // f' at 1/n
    if (lo >= 1.0 || f1 >= 0.0) {
      ls[3] = lo;
      ls[5] = 3.0;
    } else {
      ls[3] = 1.0;
      ls[5] = 1.0;
    }
  } else if (ls[5] == 1.0) {   // f' at 1
    if (f1 <= 0.0) {
      ls[3] = 1.0;
      ls[5] = 3.0;
    } else {
      ls[1] = lo;
      ls[2] = 1.0;
      ls[3] = 0.5 * (lo + 1.0);
      ls[5] = 2.0;
    }
  } else {   // inside the bracket
    const double z = ls[3];
    if (f1 == 0.0) {
      ls[5] = 3.0;
      return;
    }
    double a = ls[1], b = ls[2];
    if (f1 < 0.0) a = z; else b = z;
    double zn = f2 > 0.0 ? z - f1 / f2 : 0.5 * (a + b);
    if (!(zn > a && zn < b)) zn = 0.5 * (a + b);
    const bool stop = fabs(zn - z) <= 1e-15 * z || b - a <= 1e-15 * b;
    ls[1] = a;
    ls[2] = b;
    ls[3] = zn;
    if (stop) ls[5] = 3.0;
  }
}

__global__ void k_line_finish(Dev d) {
  if (threadIdx.x != 0) return;
  const int pi = blockIdx.x;
  if (d.line[8 * pi + 6] != 1.0) return;   // not searched in this step
  const double th = d.line[8 * pi + 3];
  d.theta[pi] = th;
  const long long rec = d.kstep[0];
  d.hist[((long)pi * d.hist_cap + (rec % d.hist_cap)) * kHistFields] = th;
}

hipError_t launch_line_search(const Dev& d, const int* chunk_prob, const int* chunk_start,
                              const int* chunk_len, int nchunk, int nprob, int rounds,
                              hipStream_t st) {
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_line_partials, dim3(nchunk), dim3(kBlock), 0, st, d, chunk_prob,
                       chunk_start, chunk_len);
    hipLaunchKernelGGL(k_line_update, dim3(nprob), dim3(64), 0, st, d);
  }
  hipLaunchKernelGGL(k_line_finish, dim3(nprob), dim3(64), 0, st, d);
  return hipGetLastError();
}

// Weight of every cell of the step: its problem's weight (GetWeights opt
// then refines it per cell).
__global__ void k_cell_theta(Dev d, int glo, int ghi) {
  for (int J = glo + blockIdx.x * blockDim.x + threadIdx.x; J < ghi; J += gridDim.x * blockDim.x)
    d.cell_theta[J] = d.theta[d.cells[J].prob];
}

// ---- GetWeights opt (eq. opt-weights-problem) on the tracked score ----------
// One weight theta_J in [1/n, 1] per cell of the step, minimising
//   f(theta) = sum_J theta_J dH_J + lam KL(P + sum_J theta_J Delta_J | nu),
// Delta_J = sum_{i in J} (nu~_i - nu_i), dH_J = sum_{i in J} (H~_i - Hbar_i)
// (the pieces are linear in the weights, the KL term convex).  Starting from
// the line-search weight, every round takes the projected diagonal Newton
// direction d_J = clamp(theta_J - g_J / h_J, 1/n, 1) - theta_J (g the
// gradient, h the diagonal of the Hessian of f) and minimises f exactly along
// theta + t d, t in [0, 1], with the line-search kernels (P := P_theta,
// Pg := P_{theta + d}).  line[7] = 1/n marks a problem under opt.
__device__ __forceinline__ bool opt_active(const Dev& d, int pi) { return d.line[8 * pi + 7] > 0.0; }

// P_w = sum over basic cells of the mixture with weight w_J = theta_J (+ d_J
// when with_d) for the step's solved cells, the state elsewhere (fixed point).
__global__ __launch_bounds__(kBlock) void k_opt_mixture(Dev d, int part, int glo, int ghi,
                                                        int with_d) {
  const int b = blockIdx.x;
  const int J = d.basic_cell[part][b];
  const bool in = J >= glo && J < ghi && d.cell_iters[J] >= 0;
  const Prob& p = d.probs[d.basic_prob[b]];
  unsigned long long* out = d.fxacc + 2 * (long)p.grid_off;
  const Box ob = d.box[b];
  const double* sv = state_pool(d) + d.voff[b];
  if (!in) {
    const long n = (long)ob.l1 * ob.l2;
    for (long o = threadIdx.x; o < n; o += kBlock) {
      const int j1 = (int)(o / ob.l2), j2 = (int)(o - (long)j1 * ob.l2);
      const double x = sv[o];
      if (x != 0.0) fx_add(out + 2 * ((long)(ob.o1 + j1) * p.n2 + (ob.o2 + j2)), x);
    }
    return;
  }
  double w = d.cell_theta[J];
  const int pi = d.basic_prob[b];
  if (with_d && opt_active(d, pi) && d.line[8 * pi + 6] != 0.0) w += d.cell_dir[J];
  const Box cb = d.cbox[b];
  const double* cv = d.cand + d.coff[b];
  const long n = (long)cb.l1 * cb.l2;
  for (long o = threadIdx.x; o < n; o += kBlock) {
    const int j1 = (int)(o / cb.l2), j2 = (int)(o - (long)j1 * cb.l2);
    const int a1 = cb.o1 + j1 - ob.o1, a2 = cb.o2 + j2 - ob.o2;
    const double old = (a1 >= 0 && a1 < ob.l1 && a2 >= 0 && a2 < ob.l2) ? sv[(long)a1 * ob.l2 + a2] : 0.0;
    const double x = (1.0 - w) * old + w * cv[o];
    if (x != 0.0) fx_add(out + 2 * ((long)(cb.o1 + j1) * p.n2 + (cb.o2 + j2)), x);
  }
}

// Per cell of an opt problem: gradient and Hessian diagonal of f at theta
// (P_theta in d.Pg), the projected Newton direction and d_J dH_J.
__global__ __launch_bounds__(kBlock) void k_opt_direction(Dev d, int glo) {
  __shared__ double red[4 * 2];
  const int J = glo + blockIdx.x;
  const Cell C = d.cells[J];
  const int pi = C.prob;
  if (!opt_active(d, pi) || d.line[8 * pi + 6] == 0.0) return;   // not opt, or converged
  const Prob& p = d.probs[pi];
  double dH = 0.0;
  for (int k = 0; k < C.nb; ++k) dH += d.htil[C.basic[k]] - d.hbar[C.basic[k]];
  double s[2] = {0.0, 0.0};
  const bool solved = d.cell_iters[J] >= 0;
  if (solved) {
    const Box yb = d.cellbox[J];
    const long n = (long)yb.l1 * yb.l2;
    const double* pool = state_pool(d);
    for (long o = threadIdx.x; o < n; o += kBlock) {
      const int j1 = (int)(o / yb.l2), j2 = (int)(o - (long)j1 * yb.l2);
      const int y1 = yb.o1 + j1, y2 = yb.o2 + j2;
      double dl = 0.0;
      for (int k = 0; k < C.nb; ++k) {
        const int b = C.basic[k];
        dl += d.cand[d.coff[b] + o];
        const Box ob = d.box[b];
        const int a1 = y1 - ob.o1, a2 = y2 - ob.o2;
        if (a1 >= 0 && a1 < ob.l1 && a2 >= 0 && a2 < ob.l2) dl -= pool[d.voff[b] + (long)a1 * ob.l2 + a2];
      }
      if (dl == 0.0) continue;
      const long g = p.grid_off + (long)y1 * p.n2 + y2;
      const double pt = d.Pg[g];
      if (!(pt > 0.0)) continue;
      s[0] += dl * (log(pt) - log(d.nu[g]));
      s[1] += dl * dl / pt;
    }
  }
  block_sum_aux<2>(s, red);
  if (threadIdx.x != 0) return;
  const double lo = d.line[8 * pi + 7];
  const double th = d.cell_theta[J];
  double dir = 0.0;
  if (solved) {
    const double g = dH + p.lam * s[0], hh = p.lam * s[1];
    double tn;
    if (hh > 0.0) tn = th - g / hh;
    else tn = g < 0.0 ? 1.0 : (g > 0.0 ? lo : th);
    tn = fmin(1.0, fmax(lo, tn));
    dir = tn - th;
  }
  d.cell_dir[J] = dir;
  d.cell_ddh[J] = dir * dH;
}

// Per opt problem: the line-search state for t in [0, 1] along d (dH = sum
// d_J dH_J in a fixed order), or converged when d = 0.
__global__ __launch_bounds__(kBlock) void k_opt_line_init(Dev d, int part, int blo, int bhi) {
  __shared__ double red[4 * 2];
  const int pi = blockIdx.x;
  if (!opt_active(d, pi) || d.line[8 * pi + 6] == 0.0) return;
  const Prob& p = d.probs[pi];
  double s[2] = {0.0, 0.0};
  for (int bt = blo; bt < bhi; ++bt) {
    const int c0 = p.cell_off[part][bt], nc = p.ncell[part][bt];
    for (int c = threadIdx.x; c < nc; c += kBlock) {
      s[0] += d.cell_ddh[c0 + c];
      s[1] = fmax(s[1], fabs(d.cell_dir[c0 + c]));
    }
  }
  // s[1] is a maximum: combine it apart from the sum
  double m = s[1];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  __shared__ double mred[4];
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = m;
  s[1] = 0.0;
  block_sum_aux<2>(s, red);
  if (threadIdx.x != 0) return;
  m = fmax(fmax(mred[0], mred[1]), fmax(mred[2], mred[3]));
  double* ls = d.line + 8 * pi;
  if (!(m > 1e-15)) {
    ls[5] = 3.0;
    ls[6] = 0.0;
    return;
  }
  ls[0] = 0.0;
  ls[1] = 0.0;
  ls[2] = 1.0;
  ls[3] = 0.0;
  ls[4] = s[0];
  ls[5] = 0.0;
}

// theta_J += t d_J for the cells of opt problems still searching.
__global__ void k_opt_step(Dev d, int glo, int ghi) {
  for (int J = glo + blockIdx.x * blockDim.x + threadIdx.x; J < ghi; J += gridDim.x * blockDim.x) {
    const int pi = d.cells[J].prob;
    if (!opt_active(d, pi) || d.line[8 * pi + 6] == 0.0) continue;
    const double lo = d.line[8 * pi + 7];
    d.cell_theta[J] = fmin(1.0, fmax(lo, d.cell_theta[J] + d.line[8 * pi + 3] * d.cell_dir[J]));
  }
}

// Per opt problem: the record's weight is the mean of the cells' weights.
__global__ __launch_bounds__(kBlock) void k_opt_finish(Dev d, int part, int blo, int bhi) {
  __shared__ double red[4 * 2];
  const int pi = blockIdx.x;
  if (!opt_active(d, pi)) return;
  const Prob& p = d.probs[pi];
  double s[2] = {0.0, 0.0};
  for (int bt = blo; bt < bhi; ++bt) {
    const int c0 = p.cell_off[part][bt], nc = p.ncell[part][bt];
    for (int c = threadIdx.x; c < nc; c += kBlock)
      if (d.cell_iters[c0 + c] >= 0) {
        s[0] += d.cell_theta[c0 + c];
        s[1] += 1.0;
      }
  }
  block_sum_aux<2>(s, red);
  if (threadIdx.x != 0) return;
  const double th = s[1] > 0.0 ? s[0] / s[1] : 1.0;
  d.theta[pi] = th;
  d.hist[((long)pi * d.hist_cap + (d.kstep[0] % d.hist_cap)) * kHistFields] = th;
}

// Algorithm 4 update: nu_i <- (1 - theta) nu_i + theta nu~_i on the cell box,
// truncation below `trunc`, shrink to the bbox of the nonzeros; the tracked
// piece and the X-marginal are mixed with the same weight.  Three kernels:
// k_mix_values mixes into the candidate box in place and finds the new box,
// the sizes are scanned, and k_mix_copy writes every basic cell's new state
// compactly into the other state pool (k_flip then makes it the current one).
__device__ __forceinline__ bool mix_updated(const Dev& d, int part, int glo, int ghi, int b) {
  const int J = d.basic_cell[part][b];
  return J >= glo && J < ghi && d.cell_iters[J] >= 0;
}

__global__ __launch_bounds__(kBlock) void k_mix_values(Dev d, int part, int glo, int ghi) {
  __shared__ int ired[4 * 4];
  const int b = blockIdx.x;
  if (!mix_updated(d, part, glo, ghi, b)) {   // not in this step, or not solved
    if (threadIdx.x == 0) {
      const Box ob = d.box[b];
      d.nbox[b] = ob;
      d.nsub[b] = make_int2(-1, -1);
      d.nsize[b] = (long)ob.l1 * ob.l2;
    }
    return;
  }
  const Prob& p = d.probs[d.basic_prob[b]];
  const double th = d.cell_theta[d.basic_cell[part][b]];
  const Box cb = d.cbox[b];
  const Box ob = d.box[b];
  const long n = (long)cb.l1 * cb.l2;
  double* cv = d.cand + d.coff[b];
  const double* sv = state_pool(d) + d.voff[b];
  int lo1 = INT_MAX, lo2 = INT_MAX, hi1 = INT_MIN, hi2 = INT_MIN;
  for (long o = threadIdx.x; o < n; o += kBlock) {
    const int j1 = (int)(o / cb.l2), j2 = (int)(o - (long)j1 * cb.l2);
    double v = cv[o];
    if (th != 1.0) {
      const int a1 = cb.o1 + j1 - ob.o1, a2 = cb.o2 + j2 - ob.o2;
      double old = 0.0;
      if (a1 >= 0 && a1 < ob.l1 && a2 >= 0 && a2 < ob.l2) old = sv[(long)a1 * ob.l2 + a2];
      v = (1.0 - th) * old + th * v;
    }
    if (v < p.trunc) v = 0.0;
    cv[o] = v;
    if (v > 0.0) {
      lo1 = min(lo1, j1); hi1 = max(hi1, j1 + 1);
      lo2 = min(lo2, j2); hi2 = max(hi2, j2 + 1);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo1 = min(lo1, __shfl_down(lo1, o, 64));
    lo2 = min(lo2, __shfl_down(lo2, o, 64));
    hi1 = max(hi1, __shfl_down(hi1, o, 64));
    hi2 = max(hi2, __shfl_down(hi2, o, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    ired[w * 4 + 0] = lo1; ired[w * 4 + 1] = lo2; ired[w * 4 + 2] = hi1; ired[w * 4 + 3] = hi2;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  lo1 = INT_MAX; lo2 = INT_MAX; hi1 = INT_MIN; hi2 = INT_MIN;
  for (int ww = 0; ww < kBlock / 64; ++ww) {
    lo1 = min(lo1, ired[ww * 4 + 0]); lo2 = min(lo2, ired[ww * 4 + 1]);
    hi1 = max(hi1, ired[ww * 4 + 2]); hi2 = max(hi2, ired[ww * 4 + 3]);
  }
  Box nb;
  if (lo1 == INT_MAX) {
    nb.o1 = cb.o1; nb.o2 = cb.o2; nb.l1 = 0; nb.l2 = 0;
    lo1 = lo2 = 0;
  } else {
    nb.o1 = cb.o1 + lo1; nb.o2 = cb.o2 + lo2; nb.l1 = hi1 - lo1; nb.l2 = hi2 - lo2;
  }
  d.nbox[b] = nb;
  d.nsub[b] = make_int2(lo1, lo2);
  d.nsize[b] = (long)nb.l1 * nb.l2;
}

// After the scan: nsize holds each new box's offset, nuse[0] the total.  A
// total beyond the pool leaves the state as it was (reported per problem).
__global__ __launch_bounds__(kBlock) void k_mix_copy(Dev d, int part, int glo, int ghi) {
  const int b = blockIdx.x;
  const int pi = d.basic_prob[b];
  if (d.nuse[0] > d.pool_cap) {
    if (threadIdx.x == 0) d.cap_fail[pi] = 1;
    return;
  }
  const bool upd = mix_updated(d, part, glo, ghi, b);
  const int cur = *d.sp;
  double* dst = (cur ? d.pool0 : d.pool1) + d.nsize[b];
  const Box nb = d.nbox[b];
  const long n = (long)nb.l1 * nb.l2;
  const double* src;
  long stride;
  if (upd) {
    const int2 sub = d.nsub[b];
    stride = d.cbox[b].l2;
    src = d.cand + d.coff[b] + (long)sub.x * stride + sub.y;
  } else {
    stride = nb.l2;
    src = (cur ? d.pool1 : d.pool0) + d.voff[b];
  }
  for (long o = threadIdx.x; o < n; o += kBlock) {
    const int a1 = (int)(o / nb.l2), a2 = (int)(o - (long)a1 * nb.l2);
    dst[o] = src[(long)a1 * stride + a2];
  }
  __syncthreads();   // every thread has read voff[b] before it changes
  if (threadIdx.x == 0) {
    d.box[b] = nb;
    d.voff[b] = d.nsize[b];
  }
  if (!upd) return;
  const Prob& p = d.probs[pi];
  const double th = d.cell_theta[d.basic_cell[part][b]];
  if (threadIdx.x == 0) d.hbar[b] = (1.0 - th) * d.hbar[b] + th * d.htil[b];
  const int2 xy = d.basic_xy[b];
  for (int o = threadIdx.x; o < p.s * p.s; o += kBlock) {
    const int i1 = o / p.s, i2 = o - i1 * p.s;
    const long g = p.grid_off + (long)(xy.x + i1) * p.n2 + (xy.y + i2);
    d.px[g] = th == 1.0 ? d.pxc[g] : (1.0 - th) * d.px[g] + th * d.pxc[g];
  }
}

__global__ void k_flip(int* sp, const long* nuse, long cap) {
  if (threadIdx.x == 0 && nuse[0] <= cap) *sp ^= 1;
}

// ---- certificate: separable global log-sum-exp on one problem's grid --------
// out[r, k] = LSE_c in[r, c] - ch (c - k)^2, one workgroup per row r.
__global__ __launch_bounds__(kBlock) void k_lse_rows(const double* in, double* out, int n2, double ch) {
  extern __shared__ __align__(16) double row[];
  const int r = blockIdx.x;
  for (int c = threadIdx.x; c < n2; c += kBlock) row[c] = in[(long)r * n2 + c];
  __syncthreads();
  for (int k = threadIdx.x; k < n2; k += kBlock) {
    double m = -INFINITY;
    for (int c = 0; c < n2; ++c) {
      const double dd = double(c - k);
      const double t = row[c] - ch * dd * dd;
      m = t > m ? t : m;
    }
    double s = 0.0;
    for (int c = 0; c < n2; ++c) {
      const double dd = double(c - k);
      s += exp(row[c] - ch * dd * dd - m);
    }
    out[(long)r * n2 + k] = m + log(s);
  }
}

__global__ void k_transpose(const double* in, double* out, int n1, int n2) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int r = by + j, c = bx + threadIdx.x;
    if (r < n1 && c < n2) tile[j][threadIdx.x] = in[(long)r * n2 + c];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += blockDim.y) {
    const int c = bx + j, r = by + threadIdx.x;
    if (r < n1 && c < n2) out[(long)c * n1 + r] = tile[threadIdx.x][j];
  }
}

// a(x) = alpha(x)/eps + log mu(x)
__global__ void k_prep_alpha(const double* alpha, const double* mu, double* a, long n, double inv_eps) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = alpha[i] * inv_eps + log(mu[i]);
}

// beta_hat = -eps kappa z ; b(y) = beta_hat/eps + log nu(y)
__global__ void k_prep_beta(const double* z, const double* nu, double* bhat, double* b, long n,
                            double eps, double kappa) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    bhat[i] = -eps * kappa * z[i];
    b[i] = bhat[i] / eps + log(nu[i]);
  }
}

// Per-point certificate terms and gradients.  Partial sums per workgroup:
// [0] PD/lam terms, [1] |pi_hat|, [2] sum lam (e^{-a/lam} - 1) mu,
// [3] sum lam (e^{-b/lam} - 1) nu, [4] l1 X error (state), [5] l1 Y error (state),
// [6] |P_X pi| (state), [7] |P_Y pi| (state)
__global__ __launch_bounds__(kBlock) void k_cert_terms(const double* alpha, const double* bhat,
                                                       const double* S, const double* z,
                                                       const double* mu, const double* nu,
                                                       const double* px, const double* P, long n,
                                                       double eps, double lam, double mass_mu,
                                                       double mass_nu, double* dmu, double* dnu,
                                                       double* part) {
  __shared__ double red[4 * 8];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long i = blockIdx.x * (long)kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double a = alpha[i], m = mu[i];
    const double lp = a / eps + S[i];
    const double pxh = m * exp(lp);
    const double aol = a / lam;
    const double ea = exp(-aol);
    acc[0] += pxh * (lp + aol) - pxh + m * ea;
    acc[1] += pxh;
    acc[2] += lam * (ea - 1.0) * m;
    const double b = bhat[i], v = nu[i];
    const double eb = exp(-b / lam);
    const double pyh = v * exp(b / eps + z[i]);
    acc[3] += lam * (eb - 1.0) * v;
    acc[4] += fabs(px[i] - ea * m);
    acc[5] += fabs(P[i] - eb * v);
    acc[6] += px[i];
    acc[7] += P[i];
    dmu[i] = eps * mass_nu - eps * pxh / m - lam * (ea - 1.0);
    dnu[i] = eps * mass_mu - eps * pyh / v - lam * (eb - 1.0);
  }
  block_sum_aux<8>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) part[blockIdx.x * 8 + k] = acc[k];
}

// The half-iteration counter lives on the device, so a captured step graph
// writes every replay's history record to its own slot.
__global__ void k_advance(long long* kstep) {
  if (threadIdx.x == 0) kstep[0] += 1;
}

hipError_t launch_advance(long long* kstep, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, kstep);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_fill(double* p, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

static int grid_blocks(long n) { return (int)min((n + 255) / 256, (long)8192); }

// dst = a * src over n doubles (the gradient times the caller's seed).
__global__ void k_scale_copy(double* dst, const double* src, long n, double a) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = a * src[i];
}

// *flag = 1 if some mass is not finite and > 0 or some beta is not finite
// (the flag is cleared before; every offender writes the same value).
__global__ void k_check_grids(const double* mu, const double* nu, const double* beta, long n,
                              double* flag) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!(mu[i] > 0.0) || !isfinite(mu[i]) || !(nu[i] > 0.0) || !isfinite(nu[i]) || !isfinite(beta[i]))
      *flag = 1.0;
}

hipError_t launch_check_grids(const double* mu, const double* nu, const double* beta, long n,
                              double* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_grids, dim3(grid_blocks(n)), dim3(256), 0, st, mu, nu, beta, n, flag);
  return hipGetLastError();
}

hipError_t launch_scale_copy(double* dst, const double* src, long n, double a, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_blocks(n)), dim3(256), 0, st, dst, src, n, a);
  return hipGetLastError();
}

// P over all problems' grids (ngrid points) from the candidate marginals of
// the cells in [glo, ghi) and the state marginals of every other cell.
hipError_t launch_aggregate_sel(const Dev& d, int part, int glo, int ghi, double* P, int nbasic,
                                long ngrid, hipStream_t st) {
  hipLaunchKernelGGL(k_fx_zero, dim3(grid_blocks(2 * ngrid)), dim3(256), 0, st, d.fxacc, 2 * ngrid);
  if (nbasic > 0)
    hipLaunchKernelGGL(k_aggregate_sel, dim3(nbasic), dim3(kBlock), 0, st, d, part, glo, ghi);
  hipLaunchKernelGGL(k_fx_finish, dim3(grid_blocks(ngrid)), dim3(256), 0, st, d.fxacc, P, ngrid);
  return hipGetLastError();
}

// P = sum of the state marginals over all problems' grids (ngrid points).
hipError_t launch_aggregate(const Dev& d, double* P, int nbasic, long ngrid, hipStream_t st) {
  hipLaunchKernelGGL(k_fx_zero, dim3(grid_blocks(2 * ngrid)), dim3(256), 0, st, d.fxacc, 2 * ngrid);
  if (nbasic > 0) hipLaunchKernelGGL(k_aggregate, dim3(nbasic), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_fx_finish, dim3(grid_blocks(ngrid)), dim3(256), 0, st, d.fxacc, P, ngrid);
  return hipGetLastError();
}

hipError_t launch_kl_chunks(const int* cp, const int* cs, const int* cl, const Prob* probs,
                            const double* P, const double* Pg, const double* nu, double* part,
                            int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_kl_chunks, dim3(nchunk), dim3(kBlock), 0, st, cp, cs, cl, probs, P, Pg, nu,
                     part);
  return hipGetLastError();
}

hipError_t launch_getweights(const Dev& d, int part, int blo, int bhi, int glo, int ghi, bool last,
                             int nprob, hipStream_t st) {
  hipLaunchKernelGGL(k_getweights, dim3(nprob), dim3(kBlock), 0, st, d, part, blo, bhi, glo, ghi,
                     last ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scan2(long* a, long* b, int n, long* tot, long long* need, int ia, int ib,
                        hipStream_t st);

hipError_t launch_cell_theta(const Dev& d, int glo, int ghi, hipStream_t st) {
  const int n = ghi - glo;
  if (n > 0) hipLaunchKernelGGL(k_cell_theta, dim3((n + 255) / 256), dim3(256), 0, st, d, glo, ghi);
  return hipGetLastError();
}

// GetWeights opt: `rounds` rounds of direction + exact search after the line
// search set the uniform weight (k_cell_theta must have run).  Pt: a grid
// for P_theta; the line kernels see P := Pt and Pg := P_{theta + d}.
hipError_t launch_opt_weights(const Dev& d, int part, int blo, int bhi, int glo, int ghi,
                              int nbasic, long ngrid, int nprob, const int* chunk_prob,
                              const int* chunk_start, const int* chunk_len, int nchunk,
                              int rounds, int line_rounds, double* Pt, double* Pd,
                              hipStream_t st) {
  Dev dt = d;
  dt.Pg = Pt;   // k_opt_direction reads P_theta from Pg
  Dev dl = d;
  dl.P = Pt;
  dl.Pg = Pd;
  const int ncell = ghi - glo;
  for (int r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_fx_zero, dim3(grid_blocks(2 * ngrid)), dim3(256), 0, st, d.fxacc, 2 * ngrid);
    hipLaunchKernelGGL(k_opt_mixture, dim3(nbasic), dim3(kBlock), 0, st, d, part, glo, ghi, 0);
    hipLaunchKernelGGL(k_fx_finish, dim3(grid_blocks(ngrid)), dim3(256), 0, st, d.fxacc, Pt, ngrid);
    if (ncell > 0) hipLaunchKernelGGL(k_opt_direction, dim3(ncell), dim3(kBlock), 0, st, dt, glo);
    hipLaunchKernelGGL(k_opt_line_init, dim3(nprob), dim3(kBlock), 0, st, d, part, blo, bhi);
    hipLaunchKernelGGL(k_fx_zero, dim3(grid_blocks(2 * ngrid)), dim3(256), 0, st, d.fxacc, 2 * ngrid);
    hipLaunchKernelGGL(k_opt_mixture, dim3(nbasic), dim3(kBlock), 0, st, d, part, glo, ghi, 1);
    hipLaunchKernelGGL(k_fx_finish, dim3(grid_blocks(ngrid)), dim3(256), 0, st, d.fxacc, Pd, ngrid);
    for (int q = 0; q < line_rounds; ++q) {
      hipLaunchKernelGGL(k_line_partials, dim3(nchunk), dim3(kBlock), 0, st, dl, chunk_prob,
                         chunk_start, chunk_len);
      hipLaunchKernelGGL(k_line_update, dim3(nprob), dim3(64), 0, st, dl);
    }
    if (ncell > 0)
      hipLaunchKernelGGL(k_opt_step, dim3((ncell + 255) / 256), dim3(256), 0, st, d, glo, ghi);
  }
  hipLaunchKernelGGL(k_opt_finish, dim3(nprob), dim3(kBlock), 0, st, d, part, blo, bhi);
  return hipGetLastError();
}

hipError_t launch_mix(const Dev& d, int part, int glo, int ghi, int nbasic, hipStream_t st) {
  if (nbasic <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mix_values, dim3(nbasic), dim3(kBlock), 0, st, d, part, glo, ghi);
  hipError_t e = launch_scan2(d.nsize, nullptr, nbasic, d.nuse, d.need, 0, -1, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mix_copy, dim3(nbasic), dim3(kBlock), 0, st, d, part, glo, ghi);
  hipLaunchKernelGGL(k_flip, dim3(1), dim3(64), 0, st, d.sp, d.nuse, d.pool_cap);
  return hipGetLastError();
}

// out = LSE over the grid of in(x) - ch |x - y|^2 (two separable passes).
static hipError_t gauss_lse2d(const double* in, double* out, double* tmp, int n1, int n2, double ch,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_lse_rows, dim3(n1), dim3(kBlock), sizeof(double) * n2, st, in, tmp, n2, ch);
  dim3 tb(32, 8);
  hipLaunchKernelGGL(k_transpose, dim3((n2 + 31) / 32, (n1 + 31) / 32), tb, 0, st, tmp, out, n1, n2);
  hipLaunchKernelGGL(k_lse_rows, dim3(n2), dim3(kBlock), sizeof(double) * n1, st, out, tmp, n1, ch);
  hipLaunchKernelGGL(k_transpose, dim3((n1 + 31) / 32, (n2 + 31) / 32), tb, 0, st, tmp, out, n2, n1);
  return hipGetLastError();
}

hipError_t dense_lse(const double* v, const double* qdel, const double* pdel, int n1, int n2,
                     double ch, double* info, double* out, double* mom, hipStream_t st);

// Certificate of one problem; scratch holds 5 grids.  Partial sums go to part
// (nblk x 8 doubles).  ydel (moved Y points, else NULL): the cost is not
// separable and both global log-sum-exps are dense (pruned exactly).
hipError_t launch_certificate(const Prob& p, const double* alpha, const double* mu, const double* nu,
                              const double* px, const double* P, const double* ydel, double* bhat,
                              double* dmu, double* dnu, double* scratch, double* part, int nblk,
                              hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  double* a = scratch;
  double* z = scratch + n;
  double* tmp = scratch + 2 * n;
  double* b = scratch + 3 * n;
  double* S = scratch + 4 * n;
  const int eb = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_prep_alpha, dim3(eb), dim3(256), 0, st, alpha, mu, a, n, 1.0 / p.eps);
  double* info = scratch + 5 * n;   // block table of the dense sums
  hipError_t e = ydel ? dense_lse(a, nullptr, ydel, p.n1, p.n2, p.ch, info, z, nullptr, st)
                      : gauss_lse2d(a, z, tmp, p.n1, p.n2, p.ch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep_beta, dim3(eb), dim3(256), 0, st, z, nu, bhat, b, n, p.eps, p.kappa);
  e = ydel ? dense_lse(b, ydel, nullptr, p.n1, p.n2, p.ch, info, S, nullptr, st)
           : gauss_lse2d(b, S, tmp, p.n1, p.n2, p.ch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cert_terms, dim3(nblk), dim3(kBlock), 0, st, alpha, bhat, S, z, mu, nu, px, P,
                     n, p.eps, p.lam, p.mass_mu, p.mass_nu, dmu, dnu, part);
  return hipGetLastError();
}

// ---- global Sinkhorn (Definition sinkhorn; eq. sinkhorn-iters-ot) ---------
// One iteration on one problem's grid, all in FP64 with the separable
// log-sum-exp of the certificate:
//   beta  = -eps kappa LSE_x [alpha/eps + log mu - ch |x - y|^2]   (Y-update)
//   S     =            LSE_y [beta/eps + log nu - ch |x - y|^2]
//   PD/lam terms of the pair (alpha, beta): log P_X pi = alpha/eps + log mu + S,
//   then (when continuing) alpha = -eps kappa S                      (X-update)
__global__ void k_gs_alpha(const double* S, double* alpha, long n, double f) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    alpha[i] = f * S[i];
}

__global__ __launch_bounds__(kBlock) void k_gs_pd(const double* alpha, const double* S,
                                                  const double* mu, long n, double eps, double lam,
                                                  double* part) {
  __shared__ double red[4];
  double acc[1] = {0.0};
  for (long i = blockIdx.x * (long)kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double a = alpha[i], m = mu[i];
    const double lp = a / eps + S[i];
    const double pxh = m * exp(lp);
    const double aol = a / lam;
    acc[0] += pxh * (lp + aol) - pxh + m * exp(-aol);
  }
  block_sum_aux<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// alpha = -eps kappa LSE_y [beta/eps + log nu - c/eps] (scratch: 3 grids)
hipError_t gs_x_update(const Prob& p, const double* beta, const double* nu, double* alpha,
                       double* scratch, hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  double* b = scratch;
  double* S = scratch + n;
  double* tmp = scratch + 2 * n;
  const int eb = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_prep_alpha, dim3(eb), dim3(256), 0, st, beta, nu, b, n, 1.0 / p.eps);
  hipError_t e = gauss_lse2d(b, S, tmp, p.n1, p.n2, p.ch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gs_alpha, dim3(eb), dim3(256), 0, st, S, alpha, n, -p.eps * p.kappa);
  return hipGetLastError();
}

// Y-update, then S and the PD partial sums (nblk doubles) of the pair
// (alpha, beta).  scratch: 5 grids; S stays in scratch + n.
hipError_t gs_iteration(const Prob& p, const double* alpha, const double* mu, const double* nu,
                        double* beta, double* scratch, double* part, int nblk, hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  double* b = scratch;
  double* S = scratch + n;
  double* tmp = scratch + 2 * n;
  double* a = scratch + 3 * n;
  double* z = scratch + 4 * n;
  const int eb = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_prep_alpha, dim3(eb), dim3(256), 0, st, alpha, mu, a, n, 1.0 / p.eps);
  hipError_t e = gauss_lse2d(a, z, tmp, p.n1, p.n2, p.ch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_prep_beta, dim3(eb), dim3(256), 0, st, z, nu, beta, b, n, p.eps, p.kappa);
  e = gauss_lse2d(b, S, tmp, p.n1, p.n2, p.ch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gs_pd, dim3(nblk), dim3(kBlock), 0, st, alpha, S, mu, n, p.eps, p.lam, part);
  return hipGetLastError();
}

// Dual and gap terms of a global pair (alpha, beta) with S = LSE_y[beta/eps +
// log nu - c/eps] (Definition unbalanced-entropic-transport with nu_- = 0):
// [0] PD/lam terms (eq. PD-gap-KL), [1] |pi|, [2] sum lam (e^{-alpha/lam} - 1) mu,
// [3] sum lam (e^{-beta/lam} - 1) nu; 4 partial sums per workgroup.
__global__ __launch_bounds__(kBlock) void k_pair_terms(const double* alpha, const double* beta,
                                                       const double* S, const double* mu,
                                                       const double* nu, long n, double eps,
                                                       double lam, double* part) {
  __shared__ double red[4 * 4];
  double acc[4] = {0, 0, 0, 0};
  for (long i = blockIdx.x * (long)kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double a = alpha[i], m = mu[i];
    const double lp = a / eps + S[i];
    const double pxh = m * exp(lp);
    const double aol = a / lam;
    const double ea = exp(-aol);
    acc[0] += pxh * (lp + aol) - pxh + m * ea;
    acc[1] += pxh;
    acc[2] += lam * (ea - 1.0) * m;
    acc[3] += lam * (exp(-beta[i] / lam) - 1.0) * nu[i];
  }
  block_sum_aux<4>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[blockIdx.x * 4 + k] = acc[k];
}

hipError_t launch_pair_terms(const Prob& p, const double* alpha, const double* beta,
                             const double* scratch, const double* mu, const double* nu,
                             double* part, int nblk, hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  hipLaunchKernelGGL(k_pair_terms, dim3(nblk), dim3(kBlock), 0, st, alpha, beta, scratch + n, mu, nu,
                     n, p.eps, p.lam, part);
  return hipGetLastError();
}

// Stored entries above `thr` of the basic cells [b0, b0 + nb) (the sparsity
// measure of Sec. 4.2); one workgroup per basic cell, one count each.
__global__ __launch_bounds__(kBlock) void k_count_nnz(Dev d, int b0, double thr,
                                                      unsigned long long* count) {
  __shared__ unsigned long long red[kBlock / 64];
  const int b = b0 + blockIdx.x;
  const Box bx = d.box[b];
  const long n = (long)bx.l1 * bx.l2;
  const double* v = state_pool(d) + d.voff[b];
  unsigned long long c = 0;
  for (long o = threadIdx.x; o < n; o += kBlock) c += v[o] > thr ? 1ull : 0ull;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    count[blockIdx.x] = t;
  }
}

hipError_t launch_count_nnz(const Dev& d, int b0, int nb, double thr, unsigned long long* count,
                            hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_count_nnz, dim3(nb), dim3(kBlock), 0, st, d, b0, thr, count);
  return hipGetLastError();
}

// alpha = -eps kappa S with S from the last gs_iteration
hipError_t gs_alpha_from_s(const Prob& p, const double* scratch, double* alpha, hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  const int eb = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_gs_alpha, dim3(eb), dim3(256), 0, st, scratch + n, alpha, n, -p.eps * p.kappa);
  return hipGetLastError();
}

// dW/dy' = sum_x pi_hat(x, y) 2 (y' - x) = 2 h P_Y pi_hat(y) (y'/h - E[x | y]) with
// the conditional mean E[x | y] (pixel units) from the moments of the Y-update sum.
__global__ void k_grad_ypos(const double* mom, const double* z, const double* bhat, const double* nu,
                            const double* ydel, int n1, int n2, double eps, double h, double gout,
                            double* out) {
  const long n = (long)n1 * n2;
  for (long g = blockIdx.x * (long)blockDim.x + threadIdx.x; g < n; g += (long)gridDim.x * blockDim.x) {
    const int j1 = (int)(g / n2), j2 = (int)(g - (long)j1 * n2);
    const double y1 = ydel ? j1 + ydel[2 * g] : (double)j1;
    const double y2 = ydel ? j2 + ydel[2 * g + 1] : (double)j2;
    const double py = nu[g] * exp(bhat[g] / eps + z[g]);
    out[2 * g] = gout * 2.0 * h * py * (y1 - mom[2 * g]);
    out[2 * g + 1] = gout * 2.0 * h * py * (y2 - mom[2 * g + 1]);
  }
}

// Gradient with respect to the Y positions at the certificate pair (after
// launch_certificate: bhat set); scratch as above, mom 2 grids.
hipError_t launch_grad_ypos(const Prob& p, const double* alpha, const double* mu, const double* nu,
                            const double* ydel, const double* bhat, double gout, double* scratch,
                            double* mom, double* out, hipStream_t st) {
  const long n = (long)p.n1 * p.n2;
  double* a = scratch;
  double* z = scratch + n;
  double* info = scratch + 5 * n;
  const int eb = (int)min((n + 255) / 256, (long)4096);
  hipLaunchKernelGGL(k_prep_alpha, dim3(eb), dim3(256), 0, st, alpha, mu, a, n, 1.0 / p.eps);
  hipError_t e = dense_lse(a, nullptr, ydel, p.n1, p.n2, p.ch, info, z, mom, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_ypos, dim3(eb), dim3(256), 0, st, mom, z, bhat, nu, ydel, p.n1, p.n2,
                     p.eps, p.h, gout, out);
  return hipGetLastError();
}

hipError_t set_rows_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void*)k_lse_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace dduot
