// Batched cell solve of one composite partition (the hot path).
//
// One workgroup solves one composite cell J of partition A or B (Algorithm 4:
// all cells of a partition in one launch, cells of every problem of the
// handle included).  Per cell:
//   * Y-box of J from the basic boxes (bbox of the union, dilated, clipped);
//   * nu_{-J} = P_Y pi - nu_J on the box (Sec. 4.1, "Computing nu_{-J}");
//   * warm start beta^0 = -lam log(P_Y pi / nu), the Y optimality condition of
//     eq. optimality-conditions-KL for the current plan;
//   * Sinkhorn: X-half eq. sinkhorn-X-iteration, Y-half eq. sinkhorn-Y-iteration
//     through eq. proxdiv-problem solved per point by Newton, stopping rule
//     PD/lam <= Err |mu_J| with PD from eq. PD-gap-KL;
//   * re-split of the cell plan eq. sinkhorn-primal into the Y-marginals of its
//     basic cells, X-marginal, and the cell-restricted score pieces
//     H_i = <alpha, P_X> + <beta, nu_i> - eps |nu_i| + eps |mu_i||nu| + lam KL(P_X|mu_i).
//
// Numerics.  The potentials live in LDS in FP64 as b(y) = beta/eps + log nu
// and a(x) = alpha/eps + log mu.  Near the optimum beta/eps ~ -(lam/eps)
// log(P_Y pi / nu) has magnitude and curvature scaled by lam/eps (~1e6 on
// fine grids), far beyond what FP32 can hold, so FP32 never sees them.  The
// cost |x - y|^2/eps = ch |i - j|^2 is separable: each log-sum-exp over the
// tile (lx1 x lx2) or the box (L1 x L2) is two 1-D passes.  Every pass output
// is evaluated as
//     out = s + log sum_k exp(R(base_k - s - ch (k - c)^2))
// with an FP64 shift s equal to the same output's value at the previous
// Sinkhorn iteration (so the sum is O(1)), the exponent in FP64 (base and
// cost can both be large and cancel) and exp / accumulation in the kernel
// precision R.  Terms provably below
// e^-W of the shift are skipped (window from the row maximum).  When the sum
// leaves [e^-22, e^60] it is redone once with the shift corrected by its log;
// when it is not representable (first iteration, very large change) the
// output is recomputed exactly by a max pass and a sum pass.
// The Newton solve works in R on the log cell share relative to the FP64
// reference z/(1+K) (the root when nu_{-J} = 0).  FP32 kernels keep log nu in
// LDS as FP32 (a relative perturbation of nu below 1e-6) and log r in a
// per-cell FP32 workspace in global memory; FP64 kernels keep both in a
// per-cell FP64 workspace.
#include "dd_types.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace dduot {

template <typename R>
struct M;
template <>
struct M<float> {
  static constexpr float kScale = 1.4426950408889634f;   // log2(e): exp(x) = 2^(x log2 e)
  static constexpr double kScale64 = 1.4426950408889634;  // the same in FP64
  static __device__ __forceinline__ float ex2s(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float ex(float x) { return __expf(x); }
  // hardware log2 times ln 2: the arguments are normal floats (shifted sums
  // accepted in [1.8e-35, 5.5e34], exact sums >= 1, 1 + x in [1, 2]); a
  // subnormal retry sum gives -inf, which sends that output to the exact path
  static __device__ __forceinline__ float lg(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
  }
  // log(1 + x) for x in [0, 1]: the series below 1e-4 (error < x^3/3), the
  // hardware logarithm above (absolute error ~1e-7, the level of the FP32
  // rounding of the Newton variables anyway)
  static __device__ __forceinline__ float lg1p(float x) {
    return x < 1e-4f ? x * (1.0f - 0.5f * x) : lg(1.0f + x);
  }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};
template <>
struct M<double> {
  static constexpr double kScale = 1.0;
  static constexpr double kScale64 = 1.0;
  static __device__ __forceinline__ double ex2s(double x) { return exp(x); }
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double lg(double x) { return log(x); }
  static __device__ __forceinline__ double lg1p(double x) { return log1p(x); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
};

// Sum N doubles over the workgroup in a fixed order (deterministic).
template <int NT, int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[k] = x;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[w * N + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int ww = 0; ww < NT / 64; ++ww) s += red[ww * N + k];
    v[k] = s;
  }
  __syncthreads();
}

// out[r] = max_c a[r*rs + c*cs] for r < rows, c < cols: G consecutive lanes
// share a row and combine by butterfly shuffles (G divides 64).
template <int NT, int G>
__device__ __forceinline__ void seg_max(const double* a, int rows, int cols, int rs, int cs,
                                        double* out) {
  const int g = threadIdx.x % G;
  for (int r0 = 0; r0 < rows; r0 += NT / G) {
    const int r = r0 + threadIdx.x / G;
    double m = -INFINITY;
    if (r < rows)
      for (int c = g; c < cols; c += G) m = fmax(m, a[r * rs + c * cs]);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (g == 0 && r < rows) out[r] = m;
  }
}

// Y-update, eq. proxdiv-problem, at one point.  With q = -beta/lam,
// q_ref = z/(1+K) (the root when nu_{-J} = 0), a = log r - q_ref and the unknown
// v = -K (q - q_ref) (log of the cell's share of P_Y at the point, up to q_ref),
// the equation reads  G(v) = v + K logaddexp(a, v) = 0;  G is increasing and
// convex, so Newton from any start converges (a step from the left lands right
// of the root, from where the iterates decrease monotonically).  v is O(10), so
// its R rounding is harmless: beta/eps = -K q_ref + v.  The R rounding of a
// and v puts a floor of about K ulp on G, i.e. 1/(1 + K sigma) ulp on v where
// sigma is the cell's share: the error of the plan at a point is inversely
// proportional to the share, its mass proportional to it.
template <typename R>
__device__ __forceinline__ double newton_v(double a, double v0, double K, R tol, int maxit) {
  if (!(a > -INFINITY)) return 0.0;
  const R aR = R(a), KR = R(K);
  R v = R(v0);
  R gprev = R(INFINITY);
  for (int it = 0; it < maxit; ++it) {
    // logaddexp(a, v) = max(a, v) + log1p(e), e = e^{-|a - v|}, without a
    // branch (lanes on both sides of a would run both); the share
    // sig = e^v / (e^a + e^v) is 1/(1 + e) right of a and e/(1 + e) left of
    // it, and G' (1 + e) = 1 + e + K (1 or e): one reciprocal per step
    const bool right = v >= aR;
    const R e = M<R>::ex(-fabs(aR - v));
    const R la = (right ? v : aR) + M<R>::lg1p(e);
    const R e1 = R(1) + e;
    const R den = e1 + KR * (right ? R(1) : e);
    const R g = v + KR * la;
    // Right of the root (G > 0) the Newton iterates of a convex increasing G
    // decrease monotonically and so does G; a residual that stops decreasing
    // is the rounding floor of K logaddexp, inside which steps only move v
    // around.  (Step lengths need not shrink: they grow where G' drops.)
    if (g > R(0)) {
      if (!(g < gprev)) break;
      gprev = g;
    }
    const R dv = g * e1 * M<R>::rcp(den);
    v -= dv;
    // Near the root the error after a step is at most (G''/2G') dv^2, and
    // G''/G' = K sig (1 - sig) / (1 + K sig) <= 1: stop once dv^2/2 is below
    // the tolerance (the step just taken then meets it).
    if (!(R(0.5) * dv * dv > tol * (R(1) + fabs(v)))) break;
  }
  return (double)v;
}

// One pass output: LSE over k in [k0, k1) of base[k*stride] - ch (k - c)^2.
// `shift` is an FP64 estimate of the result (have_shift false: none); `bmax`
// bounds base over [k0, k1) from above (window).  Counts exact recomputations
// in nfall.
template <typename R>
__device__ __forceinline__ double lse_pass(const double* base, int stride, int k0, int k1, double c,
                                           double ch, float ichf, const double* qc, int qlim,
                                           bool have_shift, double shift, double bmax,
                                           double& nfall) {
  // Terms more than W below the shift are skipped; an output is accepted when
  // its shifted sum stays above e^-22, so every skipped term is below e^-(W-22)
  // of the output (e^-18 in FP32, e^-38 in FP64), i.e. under the R rounding.
  constexpr double W = sizeof(R) == 8 ? 60.0 : 40.0;
  // every base value -inf (a row outside the cell's Y-domain): no terms
  if (!(bmax > -INFINITY)) return -INFINITY;
  // A sum outside the accepted range but still representable says where the
  // output moved: one more windowed pass with the shift corrected by its log.
  for (int attempt = 0; have_shift && attempt < 2; ++attempt) {
    int a = k0, b = k1;
    if (ch > 0.0) {
      // window in FP32 (1/ch precomputed), widened by 1e-3 of a point
      const float r2 = (float)(bmax - shift + W) * ichf;
      if (r2 < 0.0f) {
        a = b = k0;   // every term is below e^-W of the shift: recompute
      } else {
        const float rr = fminf(__fsqrt_rn(r2), 1e6f) + 1e-3f, cf = (float)c;
        a = max(k0, (int)ceilf(cf - rr));
        b = min(k1, (int)floorf(cf + rr) + 1);
      }
    }
    // Terms are exp(base_k - shift - ch d^2) (d = k - c an integer): the
    // exponent in FP64, since base_k - shift and the cost ch d^2 can both be
    // large and cancel (a potential that pays for a long transport), then
    // rounded to R for the exponential and the sum.  FP32 kernels use the
    // base-2 exponential: the exponent times log2 e, one FP64 fused
    // multiply-add with the table qc[d] = -sc ch d^2 (sc = log2 e; 1 in FP64
    // kernels); four terms per trip with their reads issued together.
    constexpr double sc = M<R>::kScale64;
    R acc0 = R(0), acc1 = R(0);
    const int ci = (int)c;
    if (a - ci >= -qlim && b - 1 - ci <= qlim) {
      const double* q = qc + (a - ci);
      const double* p = base + (long)a * stride;
      int k = a;
      for (; k + 4 <= b; k += 4, p += 4 * stride, q += 4) {
        const double v0 = p[0], v1 = p[stride], v2 = p[2 * stride], v3 = p[3 * stride];
        acc0 += M<R>::ex2s(R(fma(v0 - shift, sc, q[0])));
        acc1 += M<R>::ex2s(R(fma(v1 - shift, sc, q[1])));
        acc0 += M<R>::ex2s(R(fma(v2 - shift, sc, q[2])));
        acc1 += M<R>::ex2s(R(fma(v3 - shift, sc, q[3])));
      }
      for (; k < b; ++k, p += stride, ++q) acc0 += M<R>::ex2s(R(fma(p[0] - shift, sc, q[0])));
    } else {
      // offsets beyond the table (a Y-box far from its tile): costs computed
      double dk = (double)(a - ci);
      const double* p = base + (long)a * stride;
      for (int k = a; k < b; ++k, p += stride, dk += 1.0)
        acc0 += M<R>::ex2s(R(((p[0] - shift) - ch * dk * dk) * sc));
    }
    const R acc = acc0 + acc1;
    if (acc > R(2.8e-10) && acc < R(1.1e26)) return shift + (double)M<R>::lg(acc);   // e^-22 .. e^60
    if (!(acc > R(0)) || !(acc < R(INFINITY))) break;
    shift += (double)M<R>::lg(acc);
  }
  nfall += 1.0;
  // exact: max pass in FP64, then sum pass with R exponentials of FP64 differences
  double m = -INFINITY;
  for (int k = k0; k < k1; ++k) {
    const double d = k - c;
    const double t = base[k * stride] - ch * d * d;
    m = t > m ? t : m;
  }
  if (!(m > -INFINITY)) return m;
  int a = k0, b = k1;
  if (ch > 0.0) {
    const float rr = fminf(__fsqrt_rn((float)(bmax - m + W) * ichf), 1e6f) + 1e-3f, cf = (float)c;
    a = max(k0, (int)ceilf(cf - rr));
    b = min(k1, (int)floorf(cf + rr) + 1);
  }
  R acc = R(0);
  for (int k = a; k < b; ++k) {
    const double d = k - c;
    acc += M<R>::ex(R(base[k * stride] - ch * d * d - m));
  }
  return m + (double)M<R>::lg(acc);
}

// One pass output over a short range (the tile's extent, at most 16 terms):
// every term is summed, so no window is needed, and a shifted sum anywhere in
// [e^-80, e^80] (FP32; e^-700 .. e^700 in FP64) is accurate to R rounding.
// Otherwise one retry with the corrected shift, then the exact two passes.
template <typename R>
__device__ __forceinline__ double lse_full(const double* base, int stride, int k0, int k1, double c,
                                           double ch, const double* qc, int qlim, bool have_shift,
                                           double shift, double& nfall) {
  constexpr R lo = sizeof(R) == 8 ? R(1e-304) : R(1.8e-35);
  constexpr R hi = sizeof(R) == 8 ? R(1e304) : R(5.5e34);
  constexpr double sc = M<R>::kScale64;   // exponents and table as in lse_pass
  const int ci = (int)c;
  const bool tab = k0 - ci >= -qlim && k1 - 1 - ci <= qlim;
  for (int attempt = 0; have_shift && attempt < 2; ++attempt) {
    R acc0 = R(0), acc1 = R(0);
    const double* p = base + (long)k0 * stride;
    int k = k0;
    if (tab) {
      const double* q = qc + (k0 - ci);
      for (; k + 4 <= k1; k += 4, p += 4 * stride, q += 4) {
        const double v0 = p[0], v1 = p[stride], v2 = p[2 * stride], v3 = p[3 * stride];
        acc0 += M<R>::ex2s(R(fma(v0 - shift, sc, q[0])));
        acc1 += M<R>::ex2s(R(fma(v1 - shift, sc, q[1])));
        acc0 += M<R>::ex2s(R(fma(v2 - shift, sc, q[2])));
        acc1 += M<R>::ex2s(R(fma(v3 - shift, sc, q[3])));
      }
      for (; k < k1; ++k, p += stride, ++q) acc0 += M<R>::ex2s(R(fma(p[0] - shift, sc, q[0])));
    } else {
      double dk = (double)(k0 - ci);
      for (; k < k1; ++k, p += stride, dk += 1.0)
        acc0 += M<R>::ex2s(R(((p[0] - shift) - ch * dk * dk) * sc));
    }
    const R acc = acc0 + acc1;
    if (acc > lo && acc < hi) return shift + (double)M<R>::lg(acc);
    if (!(acc > R(0)) || !(acc < R(INFINITY))) break;
    shift += (double)M<R>::lg(acc);
  }
  nfall += 1.0;
  double m = -INFINITY;
  for (int k = k0; k < k1; ++k) {
    const double d = k - c;
    m = fmax(m, base[k * stride] - ch * d * d);
  }
  if (!(m > -INFINITY)) return m;
  R acc = R(0);
  for (int k = k0; k < k1; ++k) {
    const double d = k - c;
    acc += M<R>::ex(R(base[k * stride] - ch * d * d - m));
  }
  return m + (double)M<R>::lg(acc);
}

template <typename R>
struct CellLds {
  double* bd;    // b(y) = beta/eps + log nu                      [cmax^2]
  R* zp;         // z(y) of the last Y-half (a shift estimate)    [cmax^2]
  double* Tt;    // X pass 1 output / re-split half 1             [16*cmax]
  double* Ud;    // Y pass 1 output                               [16*cmax]
  double* Mr;    // row maxima of b                               [cmax]
  double* MU;    // column maxima of Ud                           [cmax]
  double* Mc;    // column maxima of Tt                           [16]
  double* adr;   // a(x) = alpha/eps + log mu                     [256]
  double* Ma;    // row maxima of adr                             [16]
  double* red;   // reductions                                    [4*16]
  float* lnvf;   // FP32 kernels: log nu on the box                [cmax^2]

  R* dl1;        // moved Y: displacement (pixels) on the box      [cmax^2]
  R* dl2;
  double* mx;    // moved Y: partial sums, shifts, flags           [3*256]
  double* qtab;  // -sc ch d^2 for d = -cmax .. cmax (pass costs)   [2*cmax+1]
};

// cmax: largest box side of the launch; qmax: the largest box side of the
// in-LDS layouts, which sizes the cost table (every launch reads the same
// table entries).  big: the box arrays (b, z, the pass buffers, log nu and
// the displacements) live in the cell's global workspace (cell_ws_layout)
// and only the tile-sized arrays and the cost table stay in LDS.
template <typename R>
__host__ __device__ inline size_t cell_lds_layout(int cmax, int qmax, bool moved, bool big,
                                                  CellLds<R>* L, unsigned char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 15) & ~size_t(15);
    return o;
  };
  const size_t n2 = big ? 0 : (size_t)cmax * cmax, nt = big ? 0 : (size_t)cmax * kMaxTile;
  const size_t nc = big ? 0 : (size_t)cmax;
  size_t o_bd = take(8 * n2), o_zp = take(sizeof(R) * n2), o_Tt = take(8 * nt), o_Ud = take(8 * nt);
  size_t o_Mr = take(8 * nc), o_MU = take(8 * nc), o_Mc = take(8 * kMaxTile);
  size_t o_adr = take(8 * kMaxTile * kMaxTile), o_Ma = take(8 * kMaxTile), o_red = take(8 * 4 * 16);
  // FP32 kernels keep log nu in LDS (FP64 kernels use the global per-cell
  // workspace, whose full precision the FP64 parity needs)
  const size_t o_lnv = sizeof(R) == 4 ? take(4 * n2) : 0;
  const size_t o_d1 = moved ? take(sizeof(R) * n2) : 0, o_d2 = moved ? take(sizeof(R) * n2) : 0;
  const size_t o_mx = moved ? take(8 * 3 * kMaxTile * kMaxTile) : 0;
  const size_t o_q = take(8 * (2 * (size_t)qmax + 1));
  if (L) {
    L->bd = (double*)(base + o_bd);
    L->zp = (R*)(base + o_zp);
    L->Tt = (double*)(base + o_Tt);
    L->Ud = (double*)(base + o_Ud);
    L->Mr = (double*)(base + o_Mr);
    L->MU = (double*)(base + o_MU);
    L->Mc = (double*)(base + o_Mc);
    L->adr = (double*)(base + o_adr);
    L->Ma = (double*)(base + o_Ma);
    L->red = (double*)(base + o_red);
    L->lnvf = sizeof(R) == 4 ? (float*)(base + o_lnv) : nullptr;
    L->dl1 = moved ? (R*)(base + o_d1) : nullptr;
    L->dl2 = moved ? (R*)(base + o_d2) : nullptr;
    L->mx = moved ? (double*)(base + o_mx) : nullptr;
    L->qtab = (double*)(base + o_q);
  }
  return off;
}

// ---- moved Y points: the cost ch |(x - j) - delta_j|^2 is not separable ----
// Dense sums over explicit (x, y) pairs, FP64 argument, R exponential.

// sum over box points j in [ja, jb) (row-major, row length L2) of
// exp(b_j - shift - ch |c - j - delta_j|^2) for one tile point c (box coordinates)
template <typename R>
__device__ __forceinline__ R dense_x_sum(const double* bd, const R* dl1, const R* dl2, int L2, int ja,
                                         int jb, double c1, double c2, double ch, double shift) {
  const R sc = M<R>::kScale;
  R acc0 = R(0), acc1 = R(0);
  int r = ja / L2, c = ja - r * L2;
  int j = ja;
  for (; j + 2 <= jb; j += 2) {
    const double e1 = (c1 - r) - (double)dl1[j], e2 = (c2 - c) - (double)dl2[j];
    acc0 += M<R>::ex2s(R((bd[j] - shift) - ch * (e1 * e1 + e2 * e2)) * sc);
    if (++c == L2) { c = 0; ++r; }
    const double f1 = (c1 - r) - (double)dl1[j + 1], f2 = (c2 - c) - (double)dl2[j + 1];
    acc1 += M<R>::ex2s(R((bd[j + 1] - shift) - ch * (f1 * f1 + f2 * f2)) * sc);
    if (++c == L2) { c = 0; ++r; }
  }
  if (j < jb) {
    const double e1 = (c1 - r) - (double)dl1[j], e2 = (c2 - c) - (double)dl2[j];
    acc0 += M<R>::ex2s(R((bd[j] - shift) - ch * (e1 * e1 + e2 * e2)) * sc);
  }
  return acc0 + acc1;
}

template <typename R>
__device__ __forceinline__ double dense_x_max(const double* bd, const R* dl1, const R* dl2, int L2,
                                              int ja, int jb, double c1, double c2, double ch) {
  double m = -INFINITY;
  int r = ja / L2, c = ja - r * L2;
  for (int j = ja; j < jb; ++j) {
    const double e1 = (c1 - r) - (double)dl1[j], e2 = (c2 - c) - (double)dl2[j];
    m = fmax(m, bd[j] - ch * (e1 * e1 + e2 * e2));
    if (++c == L2) { c = 0; ++r; }
  }
  return m;
}

// sum over tile points x in [xa1, xb1) x [xa2, xb2) (row length lx2) of
// exp(a_x - shift - ch |(D + x) - y|^2) for one moved point y (box coordinates)
template <typename R>
__device__ __forceinline__ R dense_y_sum(const double* adr, const double* Ma, int lx2, int xa1,
                                         int xb1, int xa2, int xb2, double D1, double D2, double y1,
                                         double y2, double ch, double shift, double W) {
  const R sc = M<R>::kScale;
  R acc = R(0);
  for (int x1 = xa1; x1 < xb1; ++x1) {
    const double e1 = (D1 + x1) - y1;
    const double q1 = ch * e1 * e1;
    if (Ma[x1] - shift - q1 < -W) continue;   // every term of the row is below e^-W
    const double* row = adr + x1 * lx2;
    for (int x2 = xa2; x2 < xb2; ++x2) {
      const double e2 = (D2 + x2) - y2;
      acc += M<R>::ex2s(R((row[x2] - shift) - q1 - ch * e2 * e2) * sc);
    }
  }
  return acc;
}

template <typename R>
__device__ __forceinline__ double dense_y_max(const double* adr, int lx2, int xa1, int xb1, int xa2,
                                              int xb2, double D1, double D2, double y1, double y2,
                                              double ch) {
  double m = -INFINITY;
  for (int x1 = xa1; x1 < xb1; ++x1) {
    const double e1 = (D1 + x1) - y1;
    for (int x2 = xa2; x2 < xb2; ++x2) {
      const double e2 = (D2 + x2) - y2;
      m = fmax(m, adr[x1 * lx2 + x2] - ch * (e1 * e1 + e2 * e2));
    }
  }
  return m;
}

// z(y) over the whole tile: shifted sum, else exact max + sum
template <typename R>
__device__ __forceinline__ double dense_y_lse(const double* adr, const double* Ma, int lx1, int lx2,
                                              double D1, double D2, double y1, double y2, double ch,
                                              bool have, double shift, double& nfall) {
  constexpr double W = sizeof(R) == 8 ? 60.0 : 40.0;
  if (have) {
    const R acc = dense_y_sum<R>(adr, Ma, lx2, 0, lx1, 0, lx2, D1, D2, y1, y2, ch, shift, W);
    if (acc > R(2.8e-10) && acc < R(1.1e26)) return shift + (double)M<R>::lg(acc);
  }
  nfall += 1.0;
  const double m = dense_y_max<R>(adr, lx2, 0, lx1, 0, lx2, D1, D2, y1, y2, ch);
  if (!(m > -INFINITY)) return m;
  const R acc = dense_y_sum<R>(adr, Ma, lx2, 0, lx1, 0, lx2, D1, D2, y1, y2, ch, m, 745.0);
  return m + (double)M<R>::lg(acc);
}

// NT threads per cell (64, 128 or 256; at least the tile's point count,
// since thread t owns tile point t).  Launch tiers (same arithmetic; a cell's
// Y-box never depends on the tier): see k_cell_solve.  The FP32 separable
// kernel asks for three waves per SIMD (its LDS at box side 48 allows three
// workgroups per CU; the register limit costs a few spills outside the hot
// loops, and the extra wave hides more latency: measured 7 % faster at
// 1024^2).
// Balancing step of Sec. 4.1 ("Balancing") for one composite cell J, after
// its solve and before the re-split marginals are truncated.  On entry
// candJ holds log nu_k(y) = log nu + beta/eps + z_k(y) of every basic cell k
// of J on the Y-box (untruncated), pxb the thread's P_X pi, lmb = -alpha'/lam
// at the thread's point with alpha' the X-half of the final beta.  Basic cell
// k should carry m_k = mubar(X_k) |pi| / |mubar| of the mass, mubar =
// e^{-alpha'/lam} mu.  Mass moves along X only (every y keeps its total): a
// donor (|pi_k| > m_k) keeps the fraction m_k / |pi_k| of its plan; what the
// donors give up, R(y), goes to the receivers in proportion to their
// deficits, spread over X_k at every y like the cell kernel
// k(x, y) = e^{(alpha(x) - c(x, y))/eps} mu(x) normalised on X_k.  The
// balanced plan on X_k is again k(x, y) g_k(y), so its piece keeps the closed
// form with eps log(g_k/nu) = eps (log nu'_k - z_k - log nu) in place of
// beta.  A receiver's P_X needs sum_y R(y) e^{-z_k(y)} k(x, y), one more
// separable pass (FP64, exact maximum then sum) over the rows of X_k.  On
// exit the candidates hold the balanced, truncated marginals; accy the Y
// sums (<eps log(g_k/nu), nu'_k>, |nu'_k|), pxb and lpb the balanced P_X and
// log(P_X/mu) of the thread's point.  candJ: the candidate marginals of the
// cell's basic cells (NY doubles each, in basic order); wlR: per-cell
// workspace for log R.
template <typename R, int NT>
__device__ void balance_cell(double* candJ, const Cell& C, const Prob& P, const CellLds<R>& S,
                             int ti1, int ti2, int lx, int L1, int L2, int NY, int D1, int D2,
                             int nc, const int* kr, const int* kc, double mux, double lmb,
                             const double* wlnv, R* wlR, double (&accy)[8], double& pxb,
                             double& lpb) {
  const int t = threadIdx.x;
  const int nb = C.nb, s = P.s;
  const double eps = P.eps, ch = P.ch;
  const int kt = t < lx ? (ti1 / s) * nc + (ti2 / s) : -1;   // basic cell of the thread's point
  double ms[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) ms[q] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q != kt) continue;
    ms[q] = pxb;
    ms[4 + q] = mux * exp(lmb);
  }
  block_sum<NT, 8>(ms, S.red);
  double tot = 0.0, mtot = 0.0;
  for (int k = 0; k < nb; ++k) {
    tot += ms[k];
    mtot += ms[4 + k];
  }
  // per basic cell: role (1 donor, -1 receiver, 0 neither), donor factor
  // m/M and share e/M of its plan given away, receiver share -e/E
  int role[4] = {0, 0, 0, 0};
  double fac[4] = {1.0, 1.0, 1.0, 1.0}, give[4] = {0.0, 0.0, 0.0, 0.0},
         rcv[4] = {0.0, 0.0, 0.0, 0.0};
  if (tot > 0.0 && mtot > 0.0) {
    double ex[4] = {0.0, 0.0, 0.0, 0.0}, mk[4] = {0.0, 0.0, 0.0, 0.0}, E = 0.0;
    for (int k = 0; k < nb; ++k) {
      mk[k] = ms[4 + k] * tot / mtot;
      ex[k] = ms[k] - mk[k];
      if (ex[k] > 0.0) E += ex[k];
    }
    if (E > 0.0) {
      for (int k = 0; k < nb; ++k) {
        if (ex[k] > 0.0) {
          role[k] = 1;
          fac[k] = mk[k] / ms[k];
          give[k] = ex[k] / ms[k];
        } else if (ex[k] < 0.0) {
          role[k] = -1;
          rcv[k] = -ex[k] / E;
        }
      }
    }
  }
  bool anyr = false;
  for (int k = 0; k < nb; ++k) anyr = anyr || role[k] < 0;
  auto removed = [&](int o) {   // R(y) at box point o
    double r = 0.0;
    for (int k = 0; k < nb; ++k)
      if (role[k] > 0) r += give[k] * exp(candJ[(long)k * NY + o]);
    return r;
  };
  if (anyr) {
    for (int o = t; o < NY; o += NT) {
      const double r = removed(o);
      wlR[o] = r > 0.0 ? R(log(r)) : R(-INFINITY);
    }
    __syncthreads();
    const double pxold = pxb;
    double add = 0.0;
    for (int k = 0; k < nb; ++k) {
      if (role[k] >= 0) continue;
      const double* lk = candJ + (long)k * NY;
      // pass 1 over y2 for the columns of X_k: T(j1, i) =
      // LSE_j2 [log R - z_k - ch (D2 + kc s + i - j2)^2]
      for (int o = t; o < L1 * s; o += NT) {
        const int j1 = o / s, il = o - j1 * s;
        const double c2 = (double)(D2 + kc[k] * s + il);
        const int row = j1 * L2;
        double m = -INFINITY;
        for (int j2 = 0; j2 < L2; ++j2) {
          if (!(S.bd[row + j2] > -INFINITY)) continue;   // outside the Y-domain
          const double dd = c2 - j2;
          m = fmax(m, (double)wlR[row + j2] - lk[row + j2] + S.bd[row + j2] - ch * dd * dd);
        }
        double v = -INFINITY;
        if (m > -INFINITY) {
          double a = 0.0;
          for (int j2 = 0; j2 < L2; ++j2) {
            if (!(S.bd[row + j2] > -INFINITY)) continue;
            const double dd = c2 - j2;
            a += exp((double)wlR[row + j2] - lk[row + j2] + S.bd[row + j2] - ch * dd * dd - m);
          }
          v = m + log(a);
        }
        S.Tt[o] = v;
      }
      __syncthreads();
      // pass 2 over y1 for the points of X_k
      if (kt == k) {
        const int il = ti2 - kc[k] * s;
        const double c1 = (double)(D1 + ti1);
        double m = -INFINITY;
        for (int j1 = 0; j1 < L1; ++j1) {
          const double dd = c1 - j1;
          m = fmax(m, S.Tt[j1 * s + il] - ch * dd * dd);
        }
        if (m > -INFINITY) {
          double a = 0.0;
          for (int j1 = 0; j1 < L1; ++j1) {
            const double dd = c1 - j1;
            a += exp(S.Tt[j1 * s + il] - ch * dd * dd - m);
          }
          add = rcv[k] * exp(S.adr[t] + m + log(a));
        }
      }
      __syncthreads();
    }
    if (kt >= 0 && role[kt] < 0) pxb = pxold + add;
  }
  if (kt >= 0 && role[kt] > 0) pxb *= fac[kt];
  if (kt >= 0 && role[kt] != 0) lpb = pxb > 0.0 ? log(pxb / mux) : -INFINITY;
  // balanced marginals, their Y sums, truncation
  for (int o = t; o < NY; o += NT) {
    double lnv;
    if constexpr (sizeof(R) == 4)
      lnv = (double)S.lnvf[o];
    else
      lnv = wlnv[o];
    const double bo = S.bd[o];
    const double r = anyr ? removed(o) : 0.0;
    for (int k = 0; k < nb; ++k) {
      double* ck = candJ + (long)k * NY;
      const double lnk = ck[o];
      double lv = lnk;
      if (role[k] > 0) {
        lv = lnk + log(fac[k]);
      } else if (role[k] < 0) {
        const double nv = exp(lnk) + rcv[k] * r;
        lv = nv > 0.0 ? log(nv) : -INFINITY;
      }
      const double nt = exp(lv);
      if (nt > 0.0) {
        accy[k] += eps * (lv - lnk + bo - lnv) * nt;
        accy[4 + k] += nt;
      }
      ck[o] = nt < P.trunc ? 0.0 : nt;
    }
  }
  __syncthreads();
}

// ---- gangs: one wide cell solved by G co-resident workgroups --------------
// Member m of a gang owns the box rows [L1 m / G, L1 (m + 1) / G) (b, z, the
// X pass 1 rows, the Newton updates, the re-split candidates) and the box
// columns [L2 m / G, L2 (m + 1) / G) of the Y pass 1 outputs, which every
// member reads.  Tile-sized work (the X potential, the stopping rule, the
// translation step) is done by every member on identical data, so all
// members take the same branches and meet at the same barriers.  Partial
// results cross workgroups through the gang's slots, double-buffered by
// barrier parity: a slot written for barrier e is read after it, and the
// next write to it comes after barrier e + 1, which no member passes before
// every member has finished reading.
//
// Coherence.  The members of a gang sit on one XCD (k_cell_gang forms the
// gangs from the XCD id register), so they share one L2, which is the point
// of coherence among them: a member's
// stores reach that L2 before it arrives at a barrier (every wave waits for
// its stores), and every read of another member's data after a barrier
// bypasses the CU's L1 (agent-scope loads).  No L2 writeback or invalidate
// is needed, which other gangs on the XCD would pay for.
constexpr int kGangUmax = 512;   // widest box (columns) a gang solves: its LDS copy

struct Gang {
  int G, m;
  double* part;      // [2][G][256]: X pass 2 partial sums or maxima per tile point
  double* xch;       // [2][G][16]: partial reductions
  unsigned* cnt;     // arrivals at this gang's barriers (zero at launch)
  int* abort_flag;   // launch-wide: some wait timed out
  int* lflag;        // LDS: the last barrier's outcome
  long long limit;   // wall-clock ticks a barrier may wait
  unsigned epoch;    // barriers passed
};

// Load of data another member of the gang wrote before the last barrier:
// an agent-scope load, which misses the CU's L1 and reads the XCD's L2.
__device__ __forceinline__ double gang_ld(const double* p) {
  const unsigned long long v =
      __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

// dst[q] = src[q] for q < n, from global memory into LDS (kAgent: loads
// as gang_ld).  Eight loads per thread are issued before the first write,
// so their latencies overlap instead of adding up.
template <int NT, bool kAgent>
__device__ __forceinline__ void load_to_lds(double* dst, const double* src, int n) {
  auto ld = [&](int i) { return kAgent ? gang_ld(src + i) : src[i]; };
  int q = threadIdx.x;
  for (; q + 7 * NT < n; q += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld(q + u * NT);
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[q + u * NT] = v[u];
  }
  if (q < n) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = q + u * NT < n ? ld(q + u * NT) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q + u * NT < n) dst[q + u * NT] = v[u];
  }
}

// Barrier of the G workgroups of one gang.  The launch keeps every workgroup
// resident (grid within the occupancy), so every wait ends; the wait is
// still bounded: past `limit` ticks it flags the launch and returns false,
// and so does every later wait, so every workgroup leaves (the host reports
// the failed step).
__device__ __forceinline__ bool gang_sync(Gang& g) {
  __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
  __syncthreads();
  if (g.G == 1) {   // a workgroup on its own: its waves only
    g.epoch += 1u;
    return true;
  }
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned target = (g.epoch + 1u) * (unsigned)g.G;
    __hip_atomic_fetch_add(g.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(g.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(g.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          wall_clock64() - t0 > g.limit) {
        __hip_atomic_store(g.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *g.lflag = ok;
  }
  __syncthreads();
  g.epoch += 1u;
  return *g.lflag != 0;
}

// v[lo, N) summed over the gang's members in member order (every member
// gets the same bits).  Call with identical N and lo in every member.
template <int N>
__device__ bool gang_sum(Gang& g, double (&v)[N], int lo) {
  static_assert(N <= 16, "gang_sum: at most 16 values");
  double* slot = g.xch + (size_t)(g.epoch & 1u) * g.G * 16;
  if (threadIdx.x == 0)
    for (int k = lo; k < N; ++k) slot[g.m * 16 + k] = v[k];
  if (!gang_sync(g)) return false;
  for (int k = lo; k < N; ++k) {
    double a = 0.0;
    for (int q = 0; q < g.G; ++q) a += gang_ld(slot + q * 16 + k);
    v[k] = a;
  }
  return true;
}

// X pass 2 partial over the rows [k0, k1): sum of exp(base_k - shift -
// ch (k - c)^2) in R, terms below e^-W of the shift skipped (window from the
// rows' maximum bmax); 0 when there is none.
template <typename R>
__device__ __forceinline__ R lse_partial(const double* base, int stride, int k0, int k1, double c,
                                         double ch, float ichf, const double* qc, int qlim,
                                         double shift, double bmax) {
  constexpr double W = sizeof(R) == 8 ? 60.0 : 40.0;
  if (!(bmax > -INFINITY) || k1 <= k0) return R(0);
  int a = k0, b = k1;
  if (ch > 0.0) {
    const float r2 = (float)(bmax - shift + W) * ichf;
    if (r2 < 0.0f) return R(0);
    const float rr = fminf(__fsqrt_rn(r2), 1e6f) + 1e-3f, cf = (float)c;
    a = max(k0, (int)ceilf(cf - rr));
    b = min(k1, (int)floorf(cf + rr) + 1);
  }
  constexpr double sc = M<R>::kScale64;   // exponents and table as in lse_pass
  R acc0 = R(0), acc1 = R(0);
  const int ci = (int)c;
  if (a < b && a - ci >= -qlim && b - 1 - ci <= qlim) {
    const double* q = qc + (a - ci);
    const double* p = base + (long)a * stride;
    int k = a;
    for (; k + 2 <= b; k += 2, p += 2 * stride, q += 2) {
      acc0 += M<R>::ex2s(R(fma(p[0] - shift, sc, q[0])));
      acc1 += M<R>::ex2s(R(fma(p[stride] - shift, sc, q[1])));
    }
    if (k < b) acc0 += M<R>::ex2s(R(fma(p[0] - shift, sc, q[0])));
  } else {
    double dk = (double)(a - ci);
    const double* p = base + (long)a * stride;
    for (int k = a; k < b; ++k, p += stride, dk += 1.0)
      acc0 += M<R>::ex2s(R(((p[0] - shift) - ch * dk * dk) * sc));
  }
  return acc0 + acc1;
}

// Exact pieces of the X pass 2 over the rows [k0, k1): the maximum of
// base_k - ch (k - c)^2 in FP64, and the sum of exp of the terms minus m.
__device__ __forceinline__ double rows_max(const double* base, int stride, int k0, int k1, double c,
                                           double ch) {
  double m = -INFINITY;
  for (int k = k0; k < k1; ++k) {
    const double d = k - c;
    m = fmax(m, base[k * stride] - ch * d * d);
  }
  return m;
}
template <typename R>
__device__ __forceinline__ double rows_sum(const double* base, int stride, int k0, int k1, double c,
                                           double ch, double m) {
  R acc = R(0);
  for (int k = k0; k < k1; ++k) {
    const double d = k - c;
    acc += M<R>::ex(R(base[k * stride] - ch * d * d - m));
  }
  return (double)acc;
}

// The solve of composite cell ci by one workgroup, or (kGang) by member
// g->m of a gang.  kBal: the variant with the balancing step (separable cost
// only); the plain variant keeps its own register allocation.  kBig: the
// variant for boxes wider than the in-LDS layouts (box arrays in the cell's
// workspace).  tier 0: every cell whose box fits d.lcap, LDS layout of
// d.lcap; tier 1: the cells whose box fits tcap, layout of tcap; tier 2: the
// cells between tcap and d.lcap, layout of d.lcap; tier 3 (kBig): the cells
// wider than d.lcap.  Returns false only when a gang barrier failed.
template <typename R, bool kMoved, int NT, bool kBal, bool kBig, bool kGang>
__device__ __forceinline__ bool cell_body(const Dev& d, int ci, int tcap, int tier, Gang* g,
                                          unsigned char* smem_raw) {
  static_assert(!kGang || (kBig && !kMoved && !kBal), "gangs solve plain separable wide cells");
  const int t = threadIdx.x;
  const Cell C = d.cells[ci];
  const Prob P = d.probs[C.prob];
  const int lcap = d.lcap;

  // ---- Y-box of the cell (k_cell_prep) and its tier --------------------------
  const Box yb = d.cellbox[ci];
  const int o1 = yb.o1, o2 = yb.o2, L1 = yb.l1, L2 = yb.l2;
  const int NY = L1 * L2;
  const int side = max(L1, L2);
  if (kBig ? (side <= lcap || (!kGang && L2 <= d.gumax))
           : (side > lcap || (tier == 1 && side > tcap) || (tier == 2 && side <= tcap)))
    return true;
  // this workgroup's box rows [r0, r1) and Y pass 1 columns [c0, c1)
  const int gG = kGang ? g->G : 1, gm = kGang ? g->m : 0;
  const int r0 = L1 * gm / gG, r1 = L1 * (gm + 1) / gG;
  const int c0 = L2 * gm / gG, c1 = L2 * (gm + 1) / gG;
  const int ya = r0 * L2, yz = r1 * L2;   // box points of the rows
  const bool lead = gm == 0;              // writes the cell's outputs
  const int lx1 = C.lx1, lx2 = C.lx2, lx = lx1 * lx2;
  const int s = P.s;
  // candidate marginals and workspace from the step's pools; a step whose
  // pools are too small solves no cell that does not fit (reported)
  const long coff = d.csize[ci];
  const long woff = d.wsize[ci];
  const WsLayout wl = cell_ws_layout((int)sizeof(R), NY, side, kMoved, kBig);
  if (coff + (long)C.nb * NY > d.cand_cap || woff + (long)wl.total > d.ws_cap) {
    if (t == 0 && lead) {
      d.cell_iters[ci] = -1;
      d.cell_conv[ci] = 0;
      d.cell_bytes[ci] = 0.0;
      d.cell_terms[ci] = 0.0;
      d.cell_fall[ci] = 0.0;
      d.cap_fail[C.prob] = 1;
    }
    return true;
  }
  double* candJ = d.cand + coff;
  unsigned char* wsc = d.ws + woff;
  const double* vals = state_pool(d);

  CellLds<R> S;
  cell_lds_layout<R>(kBig ? 0 : (tier == 1 ? tcap : lcap), lcap, kMoved, kBig, &S, smem_raw);
  if constexpr (kBig) {
    S.bd = (double*)(wsc + wl.bd);
    S.zp = (R*)(wsc + wl.zp);
    S.Tt = (double*)(wsc + wl.Tt);
    S.Ud = (double*)(wsc + wl.Ud);
    S.Mr = (double*)(wsc + wl.Mr);
    S.MU = (double*)(wsc + wl.MU);
    if constexpr (sizeof(R) == 4) S.lnvf = (float*)(wsc + wl.lnvf);
    if constexpr (kMoved) {
      S.dl1 = (R*)(wsc + wl.d1);
      S.dl2 = (R*)(wsc + wl.d2);
    }
  }
  double* red = S.red;

  const double eps = P.eps, lam = P.lam, kap = P.kappa, K = P.K, ch = P.ch;
  const float ichf = ch > 0.0 ? (float)(1.0 / ch) : 0.0f;   // window: 1/ch (unused for ch = 0)
  // cost table of the separable passes, centred: qc[d] = -sc ch d^2 (sc =
  // log2 e in FP32 kernels, 1 in FP64 ones), |d| <= lcap
  const double* qc = S.qtab + lcap;
  for (int i = t; i <= 2 * lcap; i += NT) {
    const double dd = (double)(i - lcap);
    S.qtab[i] = -M<R>::kScale64 * ch * dd * dd;
  }
  const int D1 = C.x1 - o1, D2 = C.x2 - o2;      // tile origin in box coordinates
  const double* nu = d.nu + P.grid_off;
  const double* mu = d.mu + P.grid_off;
  const double* Pst = d.P + P.grid_off;
  double* wlnv = (double*)(wsc + wl.lnv);   // FP64 kernels
  double* wlrr = (double*)(wsc + wl.lrr);
  float* wlrf = (float*)(wsc + wl.lrr);     // FP32 kernels

  // ---- X tile inputs (thread t owns tile point t) --------------------------
  const int ti1 = t < lx ? t / lx2 : 0, ti2 = t < lx ? t - ti1 * lx2 : 0;
  const long gx = (long)(C.x1 + ti1) * P.n2 + (C.x2 + ti2);
  double mux = 0.0, lmux = 0.0;
  if (t < lx) {
    mux = mu[gx];
    lmux = log(mux);
  }

  // ---- Y box inputs: nu_{-J}, r, log nu, warm start -------------------------
  // The cell's Y-domain is the support of nu_J in the box (P.support; Sec.
  // 4.1), or the whole box: points outside it carry b = -inf (no plan mass,
  // excluded from every sum), and Newton skips them.  An empty support falls
  // back to the whole box.  acc0: |mu_J|, then |nu_{-J}| and the sum of
  // e^{-beta0/lam} nu over the support, the same over the box, support size.
  double acc0[6] = {mux, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int o = ya + t; o < yz; o += NT) {
    const int j1 = o / L2, j2 = o - j1 * L2;
    const int y1 = o1 + j1, y2 = o2 + j2;
    const long g = (long)y1 * P.n2 + y2;
    const double pv = Pst[g], nv = nu[g];
    double nj = 0.0;
    for (int k = 0; k < C.nb; ++k) {
      const Box b = d.box[C.basic[k]];
      const int a1 = y1 - b.o1, a2 = y2 - b.o2;
      if (a1 >= 0 && a1 < b.l1 && a2 >= 0 && a2 < b.l2)
        nj += vals[d.voff[C.basic[k]] + (long)a1 * b.l2 + a2];
    }
    const double r = fmax(pv - nj, 0.0) / nv;
    const bool in = !P.support || nj > 0.0;
    const double b0 = pv > 0.0 ? pv : nv;
    acc0[3] += r * nv;
    acc0[4] += b0;
    if (in) {
      acc0[1] += r * nv;
      acc0[2] += b0;
      acc0[5] += 1.0;
    }
    double lnv = log(nv);
    const double lr = r > 0.0 ? log(r) : -INFINITY;
    if constexpr (sizeof(R) == 4) {
      S.lnvf[o] = (float)lnv;
      wlrf[o] = (float)lr;
      lnv = (double)(float)lnv;   // b carries the same rounded log nu
    } else {
      wlrr[o] = lr;
      wlnv[o] = lnv;
    }
    // beta^0/eps = -K log(P/nu); b = beta/eps + log nu
    S.bd[o] = in ? (pv > 0.0 ? -K * log(pv / nv) : 0.0) + lnv : -INFINITY;
    if constexpr (kMoved) {
      S.dl1[o] = R(d.ydel[2 * (P.grid_off + g)]);
      S.dl2[o] = R(d.ydel[2 * (P.grid_off + g) + 1]);
    }
  }
  block_sum<NT, 6>(acc0, red);
  if constexpr (kGang)
    if (!gang_sum(*g, acc0, 1)) return false;
  if (!(acc0[5] > 0.0) && P.support) {
    // empty support: the whole box
    for (int o = ya + t; o < yz; o += NT) {
      const long g = (long)(o1 + o / L2) * P.n2 + (o2 + o % L2);
      const double pv = Pst[g], nv = nu[g];
      const double lnv = sizeof(R) == 4 ? (double)S.lnvf[o] : wlnv[o];
      S.bd[o] = (pv > 0.0 ? -K * log(pv / nv) : 0.0) + lnv;
    }
    acc0[1] = acc0[3];
    acc0[2] = acc0[4];
    __syncthreads();
  }
  // The Y-domain's points of the rows [r0, r1), in order, at dom[ya ..
  // ya + ndom): the domain is fixed for the solve (b = -inf outside it), and
  // the Y-updates run over this list, so that every lane of a trip has a
  // point.  Per trip of NT points: wave counts by ballot, offsets from the
  // counts of the lower waves.
  int* dom = (int*)(wsc + wl.dom);
  int ndom = 0;
  {
    int* cnt = (int*)red;   // free until the first sum of the loop
    const int lane = t & 63, wv = t >> 6;
    for (int ob = ya; ob < yz; ob += NT) {
      const int o = ob + t;
      const bool in = o < yz && S.bd[o] > -INFINITY;
      const unsigned long long m = __ballot(in);
      if (lane == 0) cnt[wv] = __popcll(m);
      __syncthreads();
      int before = ndom, tot = ndom;
      for (int w = 0; w < NT / 64; ++w) {
        before += w < wv ? cnt[w] : 0;
        tot += cnt[w];
      }
      if (in) dom[ya + before + __popcll(m & ((1ull << lane) - 1ull))] = o;
      ndom = tot;
      __syncthreads();
    }
  }
  const double muJ = acc0[0];
  const double Rmass = acc0[1];    // |nu_{-J}| on the domain
  const double B0mass = acc0[2];   // sum of e^{-beta0/lam} nu on the domain
  double pxsum = 0.0;              // |P_X pi| of the last evaluated pair
  double nfall = 0.0;             // pass outputs recomputed exactly

  // ---- X-half: S(i) = LSE_j [b(j) - ch |j - (D + i)|^2], in place over Tt ----
  // Returns S for the thread's point; sprev is that point's previous S.
  // a gang member's LDS buffer of 16 x L2 doubles (L2 <= kGangUmax): the copy
  // of the Y pass 1 outputs, and the staged rows of the X pass 1
  double* Ul = nullptr;
  if constexpr (kGang)
    Ul = (double*)(smem_raw + cell_lds_layout<R>(0, lcap, false, true, nullptr, nullptr));
  bool have_x = false;
  double xext = 0.0;   // expected move of the X-half outputs since the last X-half
  bool gfail = false;  // a gang barrier failed (the cell is abandoned)
  auto x_half = [&](double sprev) -> double {
    if constexpr (kMoved) {
      // dense: tile point xi summed over the box by np threads, each over a
      // contiguous part of the box; partial sums, shifts and flags meet in mx
      const int np = max(1, NT / lx);
      const int xi = t % lx, part = t / lx;
      const bool act = part < np;
      const int ja = (int)((long)NY * part / np), jb = (int)((long)NY * (part + 1) / np);
      const double c1 = D1 + xi / lx2, c2 = D2 + xi % lx2;
      double* pt = S.mx;                  // [np * lx] partial sums / maxima
      double* sh = S.mx + kMaxTile * kMaxTile;        // [lx] shift, then result
      double* need = S.mx + 2 * kMaxTile * kMaxTile;  // [lx] exact recomputation flag
      const double sprev_x = sprev + xext;
      if (t < lx) sh[t] = sprev_x;
      __syncthreads();
      if (have_x) {
        if (act)
          pt[part * lx + xi] =
              (double)dense_x_sum<R>(S.bd, S.dl1, S.dl2, L2, ja, jb, c1, c2, ch, sh[xi]);
        __syncthreads();
        if (t < lx) {
          double a = 0.0;
          for (int q = 0; q < np; ++q) a += pt[q * lx + t];
          const bool ok = a > 2.8e-10 && a < 1.1e26;
          need[t] = ok ? 0.0 : 1.0;
          if (ok) sh[t] = sprev_x + log(a);
        }
      } else if (t < lx) {
        need[t] = 1.0;
      }
      __syncthreads();
      int any = 0;
      if (t < lx) any = need[t] != 0.0;
      if (__syncthreads_or(any)) {
        // exact: maximum over the parts, then the shifted sum
        const bool my = act && need[xi] != 0.0;
        if (my) pt[part * lx + xi] = dense_x_max<R>(S.bd, S.dl1, S.dl2, L2, ja, jb, c1, c2, ch);
        __syncthreads();
        double m = -INFINITY;
        if (my)
          for (int q = 0; q < np; ++q) m = fmax(m, pt[q * lx + xi]);
        __syncthreads();
        if (my)
          pt[part * lx + xi] =
              m > -INFINITY ? (double)dense_x_sum<R>(S.bd, S.dl1, S.dl2, L2, ja, jb, c1, c2, ch, m)
                            : 0.0;
        __syncthreads();
        if (t < lx && need[t] != 0.0) {
          double a = 0.0, mm = -INFINITY;
          for (int q = 0; q < np; ++q) a += pt[q * lx + t];
          mm = m;   // thread t is part 0 of tile point t
          sh[t] = mm > -INFINITY ? mm + log(a) : mm;
          nfall += 1.0;
        }
      }
      __syncthreads();
      const double sv = t < lx ? sh[t] : 0.0;
      have_x = true;
      xext = 0.0;
      __syncthreads();
      return sv;
    } else {
      // pass 1 over the rows [r0, r1) (a gang member's rows; all rows otherwise)
      if constexpr (kGang) {
        // 16 rows at a time through LDS (the Y pass 1 copy is not needed
        // again before the next Y-half): each b value is read from global
        // memory once, then by every window that covers it from LDS
        // (row maxima of the staged rows in Mc, free until pass 2)
        for (int jb = r0; jb < r1; jb += kMaxTile) {
          const int nr = min(kMaxTile, r1 - jb);
          // the thread's first output's previous value, loaded with the rows
          const double tp = t < nr * lx2 ? S.Tt[jb * lx2 + t] : 0.0;
          load_to_lds<NT, false>(Ul, S.bd + (long)jb * L2, nr * L2);
          __syncthreads();
          seg_max<NT, 8>(Ul, nr, L2, L2, 1, S.Mc);
          __syncthreads();
          for (int q = t; q < nr * lx2; q += NT) {
            const int jl = q / lx2, i2 = q - jl * lx2;
            const int o = jb * lx2 + q;
            S.Tt[o] = lse_pass<R>(Ul + jl * L2, 1, 0, L2, (double)(D2 + i2), ch, ichf, qc, lcap,
                                  have_x, (q == t ? tp : S.Tt[o]) + xext, S.Mc[jl], nfall);
          }
          __syncthreads();
        }
      } else {
        seg_max<NT, 8>(S.bd + ya, r1 - r0, L2, L2, 1, S.Mr + r0);
        __syncthreads();
        for (int o = r0 * lx2 + t; o < r1 * lx2; o += NT) {
          const int j1 = o / lx2, i2 = o - j1 * lx2;
          S.Tt[o] = lse_pass<R>(S.bd + j1 * L2, 1, 0, L2, (double)(D2 + i2), ch, ichf, qc, lcap,
                                have_x, S.Tt[o] + xext, S.Mr[j1], nfall);
        }
        __syncthreads();
      }
      seg_max<NT, 16>(S.Tt + r0 * lx2, lx2, r1 - r0, 1, lx2, S.Mc);
      __syncthreads();
      double sv = 0.0;
      if constexpr (kGang) {
        // pass 2: the members' shifted partial sums over their rows, added in
        // member order; outputs whose sum leaves [e^-22, e^60] (or without a
        // shift) are recomputed exactly from the maximum over all rows
        const double shift = sprev + xext;
        double* pb = g->part + (size_t)(g->epoch & 1u) * gG * 256;
        if (t < lx)
          pb[gm * 256 + t] = have_x ? (double)lse_partial<R>(S.Tt + ti2, lx2, r0, r1, (double)(D1 + ti1),
                                                             ch, ichf, qc, lcap, shift, S.Mc[ti2])
                                    : 0.0;
        if (!gang_sync(*g)) {
          gfail = true;
          return 0.0;
        }
        int need = 0;
        if (t < lx) {
          double a = 0.0;
          for (int q = 0; q < gG; ++q) a += gang_ld(pb + q * 256 + t);
          if (have_x && a > 2.8e-10 && a < 1.1e26)
            sv = shift + log(a);
          else
            need = 1;
        }
        if (__syncthreads_or(need)) {
          double* pm = g->part + (size_t)(g->epoch & 1u) * gG * 256;
          if (t < lx)
            pm[gm * 256 + t] = need ? rows_max(S.Tt + ti2, lx2, r0, r1, (double)(D1 + ti1), ch) : -INFINITY;
          if (!gang_sync(*g)) {
            gfail = true;
            return 0.0;
          }
          double mx = -INFINITY;
          if (t < lx && need)
            for (int q = 0; q < gG; ++q) mx = fmax(mx, gang_ld(pm + q * 256 + t));
          double* ps = g->part + (size_t)(g->epoch & 1u) * gG * 256;
          if (t < lx)
            ps[gm * 256 + t] = (need && mx > -INFINITY)
                                   ? rows_sum<R>(S.Tt + ti2, lx2, r0, r1, (double)(D1 + ti1), ch, mx)
                                   : 0.0;
          if (!gang_sync(*g)) {
            gfail = true;
            return 0.0;
          }
          if (t < lx && need) {
            double a = 0.0;
            for (int q = 0; q < gG; ++q) a += gang_ld(ps + q * 256 + t);
            sv = mx > -INFINITY ? mx + log(a) : mx;
            if (lead) nfall += 1.0;
          }
        }
      } else {
        if (t < lx)
          sv = lse_pass<R>(S.Tt + ti2, lx2, 0, L1, (double)(D1 + ti1), ch, ichf, qc, lcap, have_x,
                           sprev + xext, S.Mc[ti2], nfall);
      }
      have_x = true;
      xext = 0.0;
      __syncthreads();
      return sv;
    }
  };

  // warm start: the stored potential alpha on X_J when every basic cell of J
  // has one (the loop then starts with a Y-half), else the X-half of beta^0
  bool warm = true;
  for (int k = 0; k < C.nb; ++k) warm = warm && d.awarm[C.basic[k]] != 0;
  double Sx = 0.0;
  double aeps = 0.0;   // alpha/eps of the thread's point
  if (warm) {
    if (t < lx) aeps = d.abar[P.grid_off + gx] / eps;
  } else {
    Sx = x_half(0.0);
    if (gfail) return false;
    aeps = -kap * Sx;
  }

  const double tol = P.err * muJ;
  const double iK1 = 1.0 / (K + 1.0);   // q_ref = z / (1 + K), one divide per cell
  // Newton stops when its error bound reaches the rounding of v (R epsilon)
  const R newton_tol = sizeof(R) == 8 ? R(1.1e-16) : R(6e-8);
  const int newton_max = sizeof(R) == 8 ? 100 : 60;
  double pxv = 0.0, lpv = 0.0;
  double Sfin = 0.0;   // X-half output of the final beta (balancing)
  int it = 0;
  bool conv = false;
  bool have_y = false;
  double ushift = 0.0;   // shift applied to alpha since the last Y-half (eps units)
  double Anext = 0.0;    // translation: sum of e^{-alpha/lam} mu for the current alpha

  // ---- Y-half pieces -------------------------------------------------------
  auto y_prepare = [&]() {
    if (t < lx) S.adr[t] = aeps + lmux;
    __syncthreads();
    if constexpr (kMoved) {   // row maxima prune the dense sums
      seg_max<NT, 16>(S.adr, lx1, lx2, lx2, 1, S.Ma);
      __syncthreads();
    }
  };
  // Y pass 1 over tile columns [ib, ie): Uo(i1, j2) = LSE_i2 [a - ch (i2 - (j2 - D2))^2]
  // for the box columns [c0, c1) (a gang member's columns; all otherwise);
  // false when a gang barrier failed
  auto y_pass1 = [&](double* Uo, int ib, int ie, bool have, double extra) -> bool {
    const int w = c1 - c0;
    // each output's previous value (its shift) is loaded one trip ahead
    auto at = [&](int q) { return (q / w) * L2 + c0 + q % w; };
    double un = t < lx1 * w ? Uo[at(t)] : 0.0;
    for (int q = t; q < lx1 * w; q += NT) {
      const int i1 = q / w, j2 = c0 + (q - i1 * w);
      const int o = i1 * L2 + j2;
      const double uo = un;
      if (q + NT < lx1 * w) un = Uo[at(q + NT)];
      Uo[o] = lse_full<R>(S.adr + i1 * lx2, 1, ib, ie, (double)(j2 - D2), ch, qc, lcap, have,
                          uo + extra, nfall);
    }
    if constexpr (kGang) {
      // every member reads all columns: a copy in LDS (agent-scope loads)
      if (!gang_sync(*g)) return false;
      load_to_lds<NT, true>(Ul, Uo, lx1 * L2);
      __syncthreads();
      return true;
    } else {
      __syncthreads();
      return true;
    }
  };

  for (;;) {
    ++it;
    double ysh = 0.0;   // translation of b in this iteration (eps units)
    if (P.translate) {
      // exact maximisation of the cell dual along (alpha + s, beta - s):
      // e^{s/lam} = (R + sqrt(R^2 + 4AB)) / (2B), A = sum e^{-alpha/lam} mu,
      // B = sum e^{-beta/lam} nu.  After a Y-update e^{-beta/lam} nu =
      // P_Y pi + nu_{-J} pointwise, so B = |P_X pi of the last pair| + R (and
      // B = |P_Y pi| of the state before the first Y-half, where
      // e^{-beta0/lam} nu = P_Y pi).  The plan is invariant along this
      // direction, so R-level relative accuracy of w suffices.
      // (A of the next alpha is summed with the PD terms of the previous
      // iteration, saving a reduction)
      if (it == 1) {
        double ab[1] = {0.0};
        if (t < lx) ab[0] = mux * exp(-aeps / K);
        block_sum<NT, 1>(ab, red);
        Anext = ab[0];
      }
      const double Bsum = it == 1 ? B0mass : pxsum + Rmass;
      const double w = (Rmass + sqrt(Rmass * Rmass + 4.0 * Anext * Bsum)) / (2.0 * Bsum);
      const double sh = K * log(w);   // s/eps
      aeps += sh;
      ushift += sh;
      xext -= sh;   // b = beta/eps + log nu moves by about -s/eps through the Y-half
      // b itself moves by -s/eps; the Y-update below rewrites b at every
      // point of the Y-domain, and the translated value enters only its
      // Newton warm start, which takes ysh instead of a pass over the box
      ysh = sh;
    }
    // ---- Y-half: z by two passes, Newton per point --------------------------
    y_prepare();
    if constexpr (!kMoved)
      if (!y_pass1(S.Ud, 0, lx2, have_y, ushift)) return false;
    // over the Y-domain's points (outside it b = -inf for the whole solve:
    // no plan mass, and z is never read); each point's index is loaded a
    // trip ahead
    int onext = t < ndom ? dom[ya + t] : 0;
    for (int i = t; i < ndom; i += NT) {
      const int o = onext;
      if (i + NT < ndom) onext = dom[ya + i + NT];
      const int j1 = o / L2, j2 = o - j1 * L2;
      // the point's inputs, loaded before the sum so that their latency
      // (global memory in the wide kernels, and log r in every kernel)
      // overlaps it
      const double bo = S.bd[o];
      const double zo = (double)S.zp[o];
      double lnv, lrr;
      if constexpr (sizeof(R) == 4) {
        lnv = (double)S.lnvf[o];
        lrr = (double)wlrf[o];
      } else {
        lnv = wlnv[o];
        lrr = wlrr[o];
      }
      double z;
      if constexpr (kMoved)
        z = dense_y_lse<R>(S.adr, S.Ma, lx1, lx2, (double)D1, (double)D2, j1 + (double)S.dl1[o],
                           j2 + (double)S.dl2[o], ch, have_y, zo + ushift, nfall);
      else
        z = lse_full<R>((kGang ? Ul : S.Ud) + j2, L2, 0, lx1, (double)(j1 - D1), ch, qc, lcap, have_y,
                        zo + ushift, nfall);
      S.zp[o] = R(z);
      const double qref = z * iK1;
      // warm start: the previous beta/eps (translated) = bd - ysh - log nu,
      // i.e. v0 = bd - ysh - lnv + K qref
      const double v0 = (bo - ysh) - lnv + K * qref;
      const double v = newton_v<R>(lrr - qref, v0, K, newton_tol, newton_max);
      S.bd[o] = -K * qref + v + lnv;
    }
    have_y = true;
    ushift = 0.0;
    __syncthreads();

    // ---- next X-half (gives P_X of the pair for the stopping rule) ----------
    const double Sn = x_half(Sx);
    if (gfail) return false;
    Sfin = Sn;
    double term = 0.0;
    if (t < lx) {
      lpv = aeps + Sn;               // log(P_X / mu)
      const double aol = aeps / K;   // alpha/lam
      pxv = mux * exp(lpv);
      term = pxv * (lpv + aol) - pxv + mux * exp(-aol);
    }
    // A = sum e^{-alpha/lam} mu of the next iteration's alpha, for its
    // translation step
    double pdv[3] = {term, pxv, (P.translate && t < lx) ? mux * exp(kap * Sn / K) : 0.0};
    block_sum<NT, 3>(pdv, red);
    conv = pdv[0] <= tol;
    pxsum = pdv[1];
    Anext = pdv[2];
    const bool done = P.fixed_iters > 0 ? (it >= P.fixed_iters) : (conv || it >= P.max_iter);
    if (done) break;
    Sx = Sn;
    aeps = -kap * Sn;
  }

  // ---- re-split into the basic cells of J ----------------------------------
  // The final pair is (alpha of the last Y-half, beta = eps (b - log nu)); adr,
  // Ma and zp still hold that alpha's values.
  const int nc = lx2 / s;
  int kr[4], kc[4];
  for (int k = 0; k < C.nb; ++k) {
    const int2 bx = d.basic_xy[C.basic[k]];
    kr[k] = (bx.x - C.x1) / s;
    kc[k] = (bx.y - C.x2) / s;
  }
  // balancing (Sec. 4.1): the loop below then stores log nu_k untruncated
  // and the balanced marginals replace them afterwards
  const bool bal = kBal && !kMoved && P.balance && C.nb > 1;
  // Y sums per basic cell k: <beta, nu_k>, |nu_k|
  double accy[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) accy[k] = 0.0;
  for (int c = 0; c < nc; ++c) {
    double* Uo = c == 0 ? S.Ud : S.Tt;
    if constexpr (!kMoved)
      if (!y_pass1(Uo, c * s, (c + 1) * s, false, 0.0)) return false;
    for (int o = ya + t; o < yz; o += NT) {
      const int j1 = o / L2, j2 = o - j1 * L2;
      const double beta =
          eps * (S.bd[o] - (sizeof(R) == 4 ? (double)S.lnvf[o] : wlnv[o]));
      const bool dom = S.bd[o] > -INFINITY;   // in the cell's Y-domain (z defined)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k >= C.nb || kc[k] != c) continue;
        if (!dom) {
          candJ[(long)k * NY + o] = bal ? -INFINITY : 0.0;
          continue;
        }
        double zk;
        if constexpr (kMoved) {
          const R a = dense_y_sum<R>(S.adr, S.Ma, lx2, kr[k] * s, (kr[k] + 1) * s, kc[k] * s,
                                     (kc[k] + 1) * s, (double)D1, (double)D2,
                                     j1 + (double)S.dl1[o], j2 + (double)S.dl2[o], ch, S.zp[o],
                                     sizeof(R) == 8 ? 60.0 : 40.0);
          zk = a > R(0) ? S.zp[o] + (double)M<R>::lg(a) : -INFINITY;
        } else {
          zk = lse_full<R>((kGang ? Ul : Uo) + j2, L2, kr[k] * s, (kr[k] + 1) * s, (double)(j1 - D1), ch, qc, lcap,
                           true, S.zp[o], nfall);
        }
        if (bal) {
          candJ[(long)k * NY + o] = S.bd[o] + zk;
          continue;
        }
        const double nt = exp(S.bd[o] + zk);   // nu e^{beta/eps} e^{z_k}
        if (nt > 0.0) {   // 0 outside the cell's Y-domain (b = -inf)
          accy[k] += beta * nt;
          accy[4 + k] += nt;
        }
        candJ[(long)k * NY + o] = nt < P.trunc ? 0.0 : nt;
      }
    }
    __syncthreads();
  }
  double pxb = pxv, lpb = lpv;   // P_X of the (balanced) plan at the thread's point
  if constexpr (kBal && !kMoved) {
    if (bal) {
      R* wlR = sizeof(R) == 4 ? reinterpret_cast<R*>(wlrf) : reinterpret_cast<R*>(wlrr);
      balance_cell<R, NT>(candJ, C, P, S, ti1, ti2, lx, L1, L2, NY, D1, D2, nc, kr, kc, mux,
                          kap * Sfin / K, wlnv, wlR, accy, pxb, lpb);
    }
  }
  block_sum<NT, 8>(accy, red);
  // X sums per basic cell k: <alpha, px>, KL terms, |mu_k|; then the count of
  // exact recomputations
  double accx[13];
#pragma unroll
  for (int k = 0; k < 12; ++k) accx[k] = 0.0;
  if (t < lx) {
    const int k = (ti1 / s) * nc + (ti2 / s);
    const double alpha = eps * aeps;
    const double e = exp(lpb);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q != k) continue;
      accx[q] = alpha * pxb;
      accx[4 + q] = pxb > 0.0 ? mux * (e * lpb - e + 1.0) : mux;
      accx[8 + q] = mux;
    }
    if (lead) {
      d.pxc[P.grid_off + gx] = pxb;
      d.abar[P.grid_off + gx] = alpha;
    }
  }
  accx[12] = nfall;
  block_sum<NT, 13>(accx, red);
  if constexpr (kGang) {
    // the members' Y sums (their rows) and recomputation counts
    double gx9[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) gx9[k] = accy[k];
    gx9[8] = accx[12];
    if (!gang_sum(*g, gx9, 0)) return false;
#pragma unroll
    for (int k = 0; k < 8; ++k) accy[k] = gx9[k];
    accx[12] = gx9[8];
  }
  if (t == 0 && lead) {
    double bytes = 8.0 * (2.0 * NY + 3.0 * lx + (double)C.nb * NY);
    for (int k = 0; k < C.nb; ++k) {
      const int b = C.basic[k];
      const Box ob = d.box[b];
      bytes += 8.0 * ob.l1 * ob.l2;
      d.htil[b] = accx[k] + accy[k] - eps * accy[4 + k] + eps * accx[8 + k] * P.mass_nu +
                  lam * accx[4 + k];
      d.cbox[b] = yb;
      d.coff[b] = coff + (long)k * NY;
      d.awarm[b] = 1;
    }
    // log-sum-exp terms of the separable passes: every Y-half and X-half of
    // the loop, the first X-half, and the re-split passes
    const double xh = kMoved ? (double)lx * NY : (double)L1 * lx2 * L2 + (double)lx * L1;
    const double yh = kMoved ? (double)NY * lx : (double)lx1 * L2 * lx2 + (double)NY * lx1;
    const double rs = kMoved ? (double)NY * lx : (double)lx1 * L2 * lx2 + (double)NY * s * C.nb;
    d.cell_iters[ci] = it;
    d.cell_conv[ci] = conv ? 1 : 0;
    d.cell_bytes[ci] = bytes;
    d.cell_terms[ci] = it * (xh + yh) + xh + rs;
    d.cell_fall[ci] = accx[12];
  }
  return true;
}

template <typename R, bool kMoved, int NT, bool kBal = false, bool kBig = false>
__global__ __launch_bounds__(NT, (sizeof(R) == 4 && !kMoved && !kBig) ? 3 : 1) void k_cell_solve(
    Dev d, int cell_base, int tcap, int tier) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cell_body<R, kMoved, NT, kBal, kBig, false>(d, cell_base + blockIdx.x, tcap, tier, nullptr, smem_raw);
}

// Gangs of G workgroups solve the heavy wide cells of the list (k_gang_list),
// gang k the cells k, k + ngang, ...; then every workgroup alone solves the
// light ones, taking the next from a queue (no waits on other workgroups).
// A gang's members must share an XCD (its L2 is their point of coherence),
// and the dispatcher's placement of workgroups on XCDs is not assumed: every
// workgroup reads its XCD id and takes the next slot on that XCD; once all
// workgroups have arrived (the grid is within the kernel's occupancy, so all
// are resident at once; the wait is bounded like a gang barrier), each XCD's
// slots form floor(count / G) gangs of consecutive slots, numbered XCD after
// XCD, and the workgroups left over only take light cells.
// MINB: workgroups per CU the register allocation must allow (1: no
// spills; 2: twice the workgroups, a few spills).
template <typename R, int MINB>
__global__ __launch_bounds__(256, MINB) void k_cell_gang(Dev d, int G, long long limit) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int lflag, sh_gang, sh_m, sh_ngang;
  const int nwg = (int)gridDim.x;
  if (threadIdx.x == 0) {
    const int xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)) & 15;   // HW_REG_XCC_ID
    const unsigned slot = atomicAdd(&d.gxcd[xcc], 1u);
    __hip_atomic_fetch_add(&d.gxcd[16], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(&d.gxcd[16], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)nwg) {
      if (__hip_atomic_load(d.gabort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          wall_clock64() - t0 > limit) {
        __hip_atomic_store(d.gabort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    int gang = -1, m = 0, ngang = 0;
    if (ok) {
      for (int x = 0; x < 16; ++x) {
        const int full = (int)__hip_atomic_load(&d.gxcd[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / G;
        if (x == xcc && (int)slot < full * G) {
          gang = ngang + (int)slot / G;
          m = (int)slot % G;
        }
        ngang += full;
      }
    }
    lflag = ok;
    sh_gang = gang;
    sh_m = m;
    sh_ngang = ngang;
  }
  __syncthreads();
  if (!lflag) return;
  const int gang = sh_gang, m = sh_m, ngang = sh_ngang;
  const int n = d.gcount[0], nheavy = ngang > 0 ? d.gcount[1] : 0;
  if (gang >= 0) {
    Gang g;
    g.G = G;
    g.m = m;
    g.part = d.gpart + (size_t)gang * 2 * G * 256;
    g.xch = d.gxch + (size_t)gang * 2 * G * 16;
    g.cnt = d.gcnt + (size_t)gang * 64;
    g.abort_flag = d.gabort;
    g.lflag = &lflag;
    g.limit = limit;
    g.epoch = 0u;
    for (int q = gang; q < nheavy; q += ngang)
      if (!cell_body<R, false, 256, false, true, true>(d, d.glist[q], 0, 3, &g, smem_raw)) return;
  }
  Gang solo;
  solo.G = 1;
  solo.m = 0;
  solo.part = d.gsolo + (size_t)blockIdx.x * (2 * 256 + 2 * 16);
  solo.xch = solo.part + 2 * 256;
  solo.cnt = nullptr;
  solo.abort_flag = d.gabort;
  solo.lflag = &lflag;
  solo.limit = limit;
  solo.epoch = 0u;
  __shared__ int qnext;
  for (;;) {   // the light cells from a queue, heaviest first
    if (threadIdx.x == 0) qnext = nheavy + atomicAdd(&d.gcount[2], 1);
    __syncthreads();
    const int q = qnext;
    __syncthreads();
    if (q >= n) break;
    if (!cell_body<R, false, 256, false, true, true>(d, d.glist[q], 0, 3, &solo, smem_raw)) return;
  }
}

// The wide cells of [cell_base, cell_base + ncell) for the gang kernel (at
// most kGangUmax box columns; wider ones keep one workgroup each), heaviest
// first: keyed by the work estimate w = box points x the iterations of the
// cell's previous solve, in half-octave buckets (the order inside a bucket
// is arbitrary; no cell's result depends on it).  The heavy cells, solved by
// whole gangs, are the buckets down to the one holding the even share
// sum(w) / nwg of one workgroup: a lighter cell alone does not lengthen the
// launch.  gcount[0]: cells, gcount[1]: heavy cells, gcount[2]: the light
// cells' queue head.  Also clears the gangs' barrier counters and the XCD
// slot counters of the gang formation.
__global__ __launch_bounds__(1024) void k_gang_list(Dev d, int cell_base, int ncell, int ngang,
                                                    int nwg) {
  __shared__ int hist[64], off[64];
  __shared__ double wsum[16];
  const int t = threadIdx.x;
  for (int i = t; i < ngang; i += 1024) d.gcnt[(size_t)i * 64] = 0u;
  if (t < 32) d.gxcd[t] = 0u;
  if (t < 64) hist[t] = 0;
  __syncthreads();
  auto work = [&](int ci) -> double {
    const Box yb = d.cellbox[ci];
    if (max(yb.l1, yb.l2) <= d.lcap || yb.l2 > kGangUmax) return -1.0;
    return (double)yb.l1 * yb.l2 * (double)max(d.cell_iters[ci], 1);
  };
  auto bucket_of = [](double w) { return 63 - min(63, (int)(2.0 * log2(w))); };
  double mine = 0.0;
  for (int j = t; j < ncell; j += 1024) {
    const double w = work(cell_base + j);
    if (w < 0.0) continue;
    atomicAdd(&hist[bucket_of(w)], 1);
    mine += w;
  }
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
  if ((t & 63) == 0) wsum[t >> 6] = mine;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int k = 0; k < 16; ++k) tot += wsum[k];
    const int kthr = tot > 0.0 ? bucket_of(fmax(tot / nwg, 1.0)) : 63;
    int a = 0, heavy = 0;
    for (int k = 0; k < 64; ++k) {
      off[k] = a;
      a += hist[k];
      if (k <= kthr) heavy = a;
    }
    d.gcount[0] = a;
    d.gcount[1] = heavy;
    d.gcount[2] = 0;
  }
  __syncthreads();
  for (int j = t; j < ncell; j += 1024) {
    const double w = work(cell_base + j);
    if (w >= 0.0) d.glist[atomicAdd(&off[bucket_of(w)], 1)] = cell_base + j;
  }
}


size_t cell_lds_bytes(int lcap, int cap, int precision, bool moved, bool big) {
  if (precision == 64) return cell_lds_layout<double>(lcap, cap, moved, big, nullptr, nullptr);
  return cell_lds_layout<float>(lcap, cap, moved, big, nullptr, nullptr);
}

// ---- per-step preparation of the composite cells --------------------------
// Y-box of every composite cell of the step (cell_ybox), its candidate size
// (one box per basic cell) and its workspace size.
__global__ void k_cell_prep(Dev d, int cell_base, int ncell, int rbytes) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncell) return;
  const int ci = cell_base + j;
  const Cell C = d.cells[ci];
  const Prob& P = d.probs[C.prob];
  const Box yb = cell_ybox(C, P, d.box);
  d.cellbox[ci] = yb;
  const long ny = (long)yb.l1 * yb.l2;
  const int side = max(yb.l1, yb.l2);
  d.csize[ci] = (long)C.nb * ny;
  d.wsize[ci] = (long)cell_ws_layout(rbytes, ny, side, P.moved != 0, side > d.lcap).total;
}

// ---- upper bounds of the pool needs of the coming steps --------------------
// A step's basic boxes end inside their cell's Y-box (truncation and mixing
// only shrink or keep them), so replaying the Y-box rule on bound boxes tb,
// step after step, bounds every step's candidate, workspace and new-state
// sizes.  acc: [0] candidate doubles, [1] workspace bytes, [2] state doubles.
__global__ void k_bound_cells(Dev d, Box* tb, int cell_base, int ncell, int rbytes,
                              unsigned long long* acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncell) return;
  const Cell C = d.cells[cell_base + j];
  const Prob& P = d.probs[C.prob];
  const Box yb = cell_ybox(C, P, tb);   // reads only the basic boxes of this cell
  const long ny = (long)yb.l1 * yb.l2;
  const int side = max(yb.l1, yb.l2);
  atomicAdd(acc, (unsigned long long)((long)C.nb * ny));
  atomicAdd(acc + 1,
            (unsigned long long)cell_ws_layout(rbytes, ny, side, P.moved != 0, side > d.lcap).total);
  for (int k = 0; k < C.nb; ++k) tb[C.basic[k]] = yb;
}

__global__ void k_bound_state(const Box* tb, int nbasic, unsigned long long* acc) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbasic; b += gridDim.x * blockDim.x)
    atomicAdd(acc + 2, (unsigned long long)((long)tb[b].l1 * tb[b].l2));
}

// bound[0..2] = max(bound, (state, candidate, workspace) of acc); acc = 0.
__global__ void k_bound_fold(unsigned long long* acc, long long* bound) {
  if (threadIdx.x != 0) return;
  const long long v[3] = {(long long)acc[2], (long long)acc[0], (long long)acc[1]};
  for (int k = 0; k < 3; ++k) bound[k] = bound[k] > v[k] ? bound[k] : v[k];
  acc[0] = acc[1] = acc[2] = 0ull;
}

__global__ void k_bound_zero(unsigned long long* acc, long long* bound) {
  if (threadIdx.x < 3) {
    acc[threadIdx.x] = 0ull;
    bound[threadIdx.x] = 0;
  }
}

hipError_t launch_bound_begin(unsigned long long* acc, long long* bound, hipStream_t st) {
  hipLaunchKernelGGL(k_bound_zero, dim3(1), dim3(64), 0, st, acc, bound);
  return hipGetLastError();
}

// One coming step over the cells [cell_base, cell_base + ncell).
hipError_t launch_bound_step(const Dev& d, Box* tb, int cell_base, int ncell, int nbasic,
                             int precision, unsigned long long* acc, long long* bound,
                             hipStream_t st) {
  if (ncell > 0)
    hipLaunchKernelGGL(k_bound_cells, dim3((ncell + 255) / 256), dim3(256), 0, st, d, tb, cell_base,
                       ncell, precision == 64 ? 8 : 4, acc);
  const int blocks = (nbasic + 255) / 256 < 1024 ? (nbasic + 255) / 256 : 1024;
  if (nbasic > 0) hipLaunchKernelGGL(k_bound_state, dim3(blocks), dim3(256), 0, st, tb, nbasic, acc);
  hipLaunchKernelGGL(k_bound_fold, dim3(1), dim3(64), 0, st, acc, bound);
  return hipGetLastError();
}

// In-place exclusive prefix sums of a[0, n) and (if b) b[0, n) in a fixed
// order, one workgroup of 1024 threads; totals to tot[0], tot[1], and the
// largest total seen so far to need[ia], need[ib].
__global__ __launch_bounds__(1024) void k_scan2(long* a, long* b, int n, long* tot,
                                                 long long* need, int ia, int ib) {
  __shared__ long sa[1024], sb[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  long ta = 0, tb = 0;
  for (int i = lo; i < hi; ++i) {
    ta += a[i];
    if (b) tb += b[i];
  }
  sa[t] = ta;
  sb[t] = tb;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan of the chunk sums
    const long va = t >= o ? sa[t - o] : 0, vb = t >= o ? sb[t - o] : 0;
    __syncthreads();
    sa[t] += va;
    sb[t] += vb;
    __syncthreads();
  }
  long ra = sa[t] - ta, rb = sb[t] - tb;
  for (int i = lo; i < hi; ++i) {
    const long va = a[i];
    a[i] = ra;
    ra += va;
    if (b) {
      const long vb = b[i];
      b[i] = rb;
      rb += vb;
    }
  }
  if (t == 1023) {
    tot[0] = sa[1023];
    if (b) tot[1] = sb[1023];
    if (ia >= 0 && (long long)sa[1023] > need[ia]) need[ia] = sa[1023];
    if (b && ib >= 0 && (long long)sb[1023] > need[ib]) need[ib] = sb[1023];
  }
}

hipError_t launch_scan2(long* a, long* b, int n, long* tot, long long* need, int ia, int ib,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(1024), 0, st, a, b, n, tot, need, ia, ib);
  return hipGetLastError();
}

hipError_t launch_cell_prep(const Dev& d, int cell_base, int ncells, int precision, hipStream_t st) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_prep, dim3((ncells + 255) / 256), dim3(256), 0, st, d, cell_base, ncells,
                     precision == 64 ? 8 : 4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan2(d.csize + cell_base, d.wsize + cell_base, ncells, d.cuse, d.need, 1, 2, st);
}

// The wide-box variant always runs 256 threads per cell.
template <typename R, bool kMoved, bool kBal, bool kBig>
static void launch_nt(const Dev& d, int cell_base, int ncells, size_t lds, int nt, int tcap, int tier,
                      hipStream_t st) {
  if constexpr (kBig)
    hipLaunchKernelGGL((k_cell_solve<R, kMoved, 256, kBal, true>), dim3(ncells), dim3(256), lds, st,
                       d, cell_base, tcap, tier);
  else if (nt == 64)
    hipLaunchKernelGGL((k_cell_solve<R, kMoved, 64, kBal, false>), dim3(ncells), dim3(64), lds, st, d,
                       cell_base, tcap, tier);
  else if (nt == 128)
    hipLaunchKernelGGL((k_cell_solve<R, kMoved, 128, kBal, false>), dim3(ncells), dim3(128), lds, st,
                       d, cell_base, tcap, tier);
  else
    hipLaunchKernelGGL((k_cell_solve<R, kMoved, 256, kBal, false>), dim3(ncells), dim3(256), lds, st,
                       d, cell_base, tcap, tier);
}

template <bool kBig>
static void launch_kind(const Dev& d, int cell_base, int ncells, size_t lds, int precision,
                        bool moved, bool balance, int nt, int tcap, int tier, hipStream_t st) {
  if (precision == 64) {
    if (moved) launch_nt<double, true, false, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
    else if (balance) launch_nt<double, false, true, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
    else launch_nt<double, false, false, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
  } else {
    if (moved) launch_nt<float, true, false, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
    else if (balance) launch_nt<float, false, true, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
    else launch_nt<float, false, false, kBig>(d, cell_base, ncells, lds, nt, tcap, tier, st);
  }
}

// LDS of the gang kernel: the wide-cell layout, then the copy of the Y pass 1
// outputs (16 x kGangUmax doubles).
size_t gang_lds_bytes(int precision, int lcap) {
  return cell_lds_bytes(0, lcap, precision, false, true) + (size_t)kMaxTile * kGangUmax * 8;
}

// Workgroups of the gang kernel (variant minb) that fit one CU at once.
hipError_t gang_occupancy(int precision, int minb, size_t lds, int* occ) {
  if (precision == 64)
    return minb >= 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_cell_gang<double, 2>, 256, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_cell_gang<double, 1>, 256, lds);
  return minb >= 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_cell_gang<float, 2>, 256, lds)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_cell_gang<float, 1>, 256, lds);
}

// The cell solves of [cell_base, cell_base + ncells) after k_cell_prep: the
// cells wider than the in-LDS layouts (lcap) first, with their arrays in the
// workspace (by gangs of gl.G workgroups when gl.G > 0, else one workgroup
// each); then, when tcap < lcap, the cells between tcap and lcap with the
// layout of lcap, and last those that fit tcap (more workgroups per CU).
hipError_t launch_cell_solve(const Dev& d, int cell_base, int ncells, int lcap, int tcap,
                             int precision, bool moved, bool balance, int nt, const GangLaunch& gl,
                             hipStream_t st) {
  if (ncells <= 0) return hipSuccess;
  const size_t lds_wide = cell_lds_bytes(0, lcap, precision, moved, true);
  Dev dw = d;
  dw.gumax = 0;
  if (gl.G > 0 && !moved && !balance) {
    // gangs for the wide cells up to kGangUmax columns, then one workgroup
    // for each wider one
    dw.gumax = kGangUmax;
    const size_t lds_g = gang_lds_bytes(precision, lcap);
    hipLaunchKernelGGL(k_gang_list, dim3(1), dim3(1024), 0, st, dw, cell_base, ncells, gl.nwg / gl.G,
                       gl.nwg);
    if (precision == 64) {
      if (gl.minb >= 2)
        hipLaunchKernelGGL((k_cell_gang<double, 2>), dim3(gl.nwg), dim3(256), lds_g, st, dw, gl.G, gl.limit);
      else
        hipLaunchKernelGGL((k_cell_gang<double, 1>), dim3(gl.nwg), dim3(256), lds_g, st, dw, gl.G, gl.limit);
    } else {
      if (gl.minb >= 2)
        hipLaunchKernelGGL((k_cell_gang<float, 2>), dim3(gl.nwg), dim3(256), lds_g, st, dw, gl.G, gl.limit);
      else
        hipLaunchKernelGGL((k_cell_gang<float, 1>), dim3(gl.nwg), dim3(256), lds_g, st, dw, gl.G, gl.limit);
    }
  }
  launch_kind<true>(dw, cell_base, ncells, lds_wide, precision, moved, balance, nt, tcap, 3, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t big = cell_lds_bytes(lcap, lcap, precision, moved, false);
  if (tcap >= lcap) {
    launch_kind<false>(d, cell_base, ncells, big, precision, moved, balance, nt, lcap, 0, st);
  } else {
    launch_kind<false>(d, cell_base, ncells, big, precision, moved, balance, nt, tcap, 2, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_kind<false>(d, cell_base, ncells, cell_lds_bytes(tcap, lcap, precision, moved, false),
                       precision, moved, balance, nt, tcap, 1, st);
  }
  return hipGetLastError();
}

template <typename R, bool kMoved, bool kBal, bool kBig>
static hipError_t set_lds_nt(size_t bytes) {
  const void* fns[3] = {(const void*)k_cell_solve<R, kMoved, 256, kBal, kBig>, nullptr, nullptr};
  if constexpr (!kBig) {
    fns[1] = (const void*)k_cell_solve<R, kMoved, 64, kBal, false>;
    fns[2] = (const void*)k_cell_solve<R, kMoved, 128, kBal, false>;
  }
  for (const void* f : fns) {
    if (!f) continue;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool kBig>
static hipError_t set_lds_kind(size_t bytes) {
  hipError_t e = set_lds_nt<double, false, false, kBig>(bytes);
  if (e == hipSuccess) e = set_lds_nt<double, true, false, kBig>(bytes);
  if (e == hipSuccess) e = set_lds_nt<float, false, false, kBig>(bytes);
  if (e == hipSuccess) e = set_lds_nt<float, true, false, kBig>(bytes);
  if (e == hipSuccess) e = set_lds_nt<double, false, true, kBig>(bytes);
  if (e == hipSuccess) e = set_lds_nt<float, false, true, kBig>(bytes);
  return e;
}

hipError_t set_cell_lds_limit(size_t bytes, size_t gang_bytes) {
  hipError_t e = set_lds_kind<false>(bytes);
  if (e == hipSuccess) e = set_lds_kind<true>(bytes);
  const void* gk[4] = {(const void*)k_cell_gang<float, 1>, (const void*)k_cell_gang<float, 2>,
                       (const void*)k_cell_gang<double, 1>, (const void*)k_cell_gang<double, 2>};
  for (const void* f : gk)
    if (e == hipSuccess)
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gang_bytes);
  return e;
}



}  // namespace dduot
